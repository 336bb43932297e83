"""The learned filter's training labels: truth matching of peak cells
against the generator's track parameters (no refinement involved)."""
import numpy as np

from paper_1309_6275_amd import configs as CF
from paper_1309_6275_amd import eventgen as G
from paper_1309_6275_amd.peakfilter import truth_labels


def _lin(g, i, j, k):
    return (k * g["n_qpt"] + j) * g["n_phi"] + i


def test_truth_labels_cells_near_the_truth():
    g = CF.GRID_3D
    # one track at known parameters; its true cell from the bin edges
    phi0, qpt, d0 = 3.1, 0.31, 2.2
    ev = G.make_tracks_event([(phi0, qpt, d0)], seed=1)
    it = int(np.floor((phi0 + np.pi) * g["n_phi"] / (2 * np.pi))) % g["n_phi"]
    jt = int((qpt - g["qpt_lo"]) / ((g["qpt_hi"] - g["qpt_lo"]) / g["n_qpt"]))
    kt = int((d0 - g["d0_lo"]) / ((g["d0_hi"] - g["d0_lo"]) / g["n_d0"]))
    cells = [(it, jt, kt, 1), ((it + 2) % g["n_phi"], jt + 1, kt - 1, 1),
             ((it + 3) % g["n_phi"], jt, kt, 0), (it, jt + 2, kt, 0), (it, jt, kt + 2, 0),
             ((it - 2) % g["n_phi"], jt - 1, kt + 1, 1)]
    y = truth_labels(ev, g, 7, [_lin(g, i, j, k) for i, j, k, _ in cells])
    assert list(y) == [c[3] for c in cells]


def test_truth_labels_phi_wrap_and_acceptance():
    g = CF.GRID_3D
    # phi0 just below pi: the true bin is the last one; a peak in bin 0 is
    # one bin away through the wrap
    ev = G.make_tracks_event([(np.pi - 1e-4, -0.5, 0.4)], seed=2)
    jt = int((-0.5 - g["qpt_lo"]) / ((g["qpt_hi"] - g["qpt_lo"]) / g["n_qpt"]))
    kt = int((0.4 - g["d0_lo"]) / ((g["d0_hi"] - g["d0_lo"]) / g["n_d0"]))
    y = truth_labels(ev, g, 7, [_lin(g, 0, jt, kt), _lin(g, g["n_phi"] - 1, jt, kt)])
    assert list(y) == [1.0, 1.0]
    # a track outside the q/pT range labels nothing
    ev2 = G.make_tracks_event([(0.5, 1.5, 0.0)], seed=3)
    assert truth_labels(ev2, g, 7, np.arange(0, g["n_phi"] * g["n_qpt"] * g["n_d0"], 997)).sum() == 0


def _labels_by_track(ev, g, min_layers, lins, dphi=2, dq=1, dd=1):
    """The rule read literally: for every track in acceptance, mark the peaks
    whose periodic phi0 distance and q/pT, d0 distances to its true cell are
    within the tolerances."""
    from paper_1309_6275_amd import metrics as M
    nphi, nq, nd = g["n_phi"], g["n_qpt"], g["n_d0"]
    lins = np.asarray(lins, np.int64)
    i, col = lins % nphi, lins // nphi
    j, k = col % nq, col // nq
    y = np.zeros(lins.size, np.float32)
    for t in np.flatnonzero(M.in_acceptance(ev, g, min_layers)):
        ti = int(np.floor((ev.trk_phi0[t] + np.pi) * nphi / (2 * np.pi))) % nphi
        tj = min(max(int(np.floor((ev.trk_qpt[t] - g["qpt_lo"]) / ((g["qpt_hi"] - g["qpt_lo"]) / nq))), 0), nq - 1)
        tk = 0
        if nd > 1:
            tk = min(max(int(np.floor((ev.trk_d0[t] - g["d0_lo"]) / ((g["d0_hi"] - g["d0_lo"]) / nd))), 0), nd - 1)
        dphi_t = np.minimum((i - ti) % nphi, (ti - i) % nphi)
        y[(dphi_t <= dphi) & (np.abs(j - tj) <= dq) & (np.abs(k - tk) <= dd)] = 1.0
    return y


def test_truth_labels_equal_the_rule_per_track():
    """On whole events of both grids, against random cells and cells next to
    the tracks: the cell lookup equals the track-by-track rule."""
    rng = np.random.default_rng(3)
    for w, seed in ((2, 5_000_123), (1, 1_000_321)):
        W = CF.WORKLOADS[w]
        g = W["grid"]
        ev = G.make_event(w, seed)
        ncell = g["n_phi"] * g["n_qpt"] * g["n_d0"]
        near = []
        for t in range(len(ev.trk_qpt)):
            i = int(np.floor((ev.trk_phi0[t] + np.pi) * g["n_phi"] / (2 * np.pi))) % g["n_phi"]
            j = int(np.clip((ev.trk_qpt[t] - g["qpt_lo"]) / (g["qpt_hi"] - g["qpt_lo"]) * g["n_qpt"], 0, g["n_qpt"] - 1))
            k = 0
            if g["n_d0"] > 1:
                k = int(np.clip((ev.trk_d0[t] - g["d0_lo"]) / (g["d0_hi"] - g["d0_lo"]) * g["n_d0"],
                                0, g["n_d0"] - 1))
            for di, dj, dk in ((-3, 0, 0), (-2, 1, 0), (0, 0, 1), (2, -1, -1), (3, 0, 0),
                               (0, 2, 0), (1, 0, 2)):
                jj, kk = j + dj, k + dk
                if 0 <= jj < g["n_qpt"] and 0 <= kk < g["n_d0"]:
                    near.append(_lin(g, (i + di) % g["n_phi"], jj, kk))
        lins = np.concatenate([rng.integers(0, ncell, 20000), np.array(near, np.int64)])
        mine = truth_labels(ev, g, W["cluster"]["min_layers"], lins)
        want = _labels_by_track(ev, g, W["cluster"]["min_layers"], lins)
        assert np.array_equal(mine, want)
        assert want.sum() > 50 and (want == 0).sum() > 1000
