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
