"""Pins of the oracle's tie and ordering rules that the noiseless-event pins
cannot see: the vertex-peak rule (theta wrap, rho clip, plateaus, ties),
the keys of duplicate cleaning, and the seed-sum key of the best seed.

Each rule is pinned by hand-worked fixtures (tests/golden/) or by a case
whose answer follows from the generator's geometry, and each test at the
end plants one plausible mistake in a copy of the oracle's C source and
shows that a pin fails with it.
"""
import json
import os

import numpy as np
import pytest

from paper_1309_6275_amd import configs as CF
from paper_1309_6275_amd import eventgen as G

from planted import planted

HERE = os.path.dirname(os.path.abspath(__file__))


def _load(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)["cases"]


# --------------------------------------------------------------------------
# vertex peaks (second transform; the paper reuses the first transform's
# local-maximum finder, section "Jet and Black Hole Detection")
def _vacc(case):
    nm, nt = case["dims"]
    v = np.full((nm, nt), case["background"], np.int32)
    for m, t, x in case["cells"]:
        v[m, t] = x
    return v


def _vertex_golden_failures(O):
    bad = []
    for case in _load("vertex_peaks_cases.json"):
        got = O.vertex_peaks(_vacc(case), case["threshold"]).tolist()
        if got != case["expected"]:
            bad.append((case["name"], got))
    return bad


def test_vertex_peaks_golden(oracle):
    assert _vertex_golden_failures(oracle) == []


def test_vertex_peaks_distinct_values_vs_maximum_filter(oracle):
    """Distinct values: the rule is a strict local maximum, which scipy's
    maximum filter finds by another route (theta wrapped, rho clipped)."""
    from scipy import ndimage
    rng = np.random.default_rng(21)
    for nm, nt in ((5, 8), (7, 16), (1, 12)):
        v = rng.permutation(nm * nt).astype(np.int32).reshape(nm, nt)
        pad = np.pad(v.astype(np.int64), ((1, 1), (0, 0)), constant_values=-1)
        mx = ndimage.maximum_filter(pad, size=3, mode=("constant", "wrap"), cval=-1)
        thr = nm * nt // 3
        want = np.flatnonzero((mx[1:-1] == v) & (v >= thr))
        assert np.array_equal(oracle.vertex_peaks(v, thr), want)


def test_vertex_near_theta_wrap_gives_one_object(oracle):
    """A noiseless vertex half a theta bin inside -pi: one object, in the
    cell of the vertex or next to it through the wrap, with every track."""
    cl = CF.CLUSTER_3D
    W = CF.WORKLOADS[2]
    rng = np.random.default_rng(6)
    nt = cl["n_theta"]
    theta = -np.pi + 0.5 * (2 * np.pi / nt)
    psis = theta + rng.uniform(-0.3, 0.3, 10)
    qpts = rng.choice([-1, 1], 10) * rng.uniform(0.3, 0.9, 10)
    ev = G.make_vertex_event(12.0, theta, psis, qpts, seed=6, smear=0.0)
    acc, _ = oracle.hough_vote(W["grid"], ev.r, ev.phi)
    pk, _ = oracle.hough_peaks(W["grid"], acc, W["min_votes"])
    res = oracle.assoc_cluster(W["grid"], ev.r, ev.phi, ev.layer, pk, cl)
    obj = res["objects"]
    near = []
    for o in obj:
        dth = abs((o["theta"] - theta + np.pi) % (2 * np.pi) - np.pi)
        if dth <= 3 * (2 * np.pi / nt) and abs(o["rho"] - 12.0) <= 3.0:
            near.append(o)
    assert len(near) == 1, obj
    assert near[0]["n_tracks"] == res["counts"][1] == 10


# --------------------------------------------------------------------------
# duplicate cleaning keys (section "Current Tracker and Tracking Algorithm")
def _ownership_failures(O):
    bad = []
    for case in _load("ownership_cases.json"):
        c = case["cands"]
        hits = np.full((len(c), 16), -1, np.int32)
        for p, x in enumerate(c):
            hits[p, :len(x["hits"])] = x["hits"]
        owner, n_owned = O.ownership([x["n_in"] for x in c], [x["ss"] for x in c],
                                     [x["lin"] for x in c], hits, case["n_hits"])
        if owner.tolist() != case["owner"] or n_owned.tolist() != case["n_owned"]:
            bad.append((case["name"], owner.tolist(), n_owned.tolist()))
    return bad


def test_ownership_golden(oracle):
    assert _ownership_failures(oracle) == []


# --------------------------------------------------------------------------
# best seed: equal inlier counts are decided by the smaller sum of squared
# distances (then by the first combination)
def _two_seed_event(oracle):
    """A noiseless track plus one extra hit on the outermost seed layer, 30 um
    off the track and nearer the cell centre than the track's own hit, so
    its seed combination comes first and reaches the same inlier count."""
    W = CF.WORKLOADS[2]
    g = W["grid"]
    np_, nq, nd = g["n_phi"], g["n_qpt"], g["n_d0"]
    i, j, k = 100, 170, 37
    wphi = 2 * np.pi / np_
    wq = (g["qpt_hi"] - g["qpt_lo"]) / nq
    wd = (g["d0_hi"] - g["d0_lo"]) / nd
    phi0 = -np.pi + (i + 0.8) * wphi
    qpt = g["qpt_lo"] + (j + 0.3) * wq
    d0 = g["d0_lo"] + (k + 0.6) * wd
    ev = G.make_tracks_event([(phi0, qpt, d0)], smear=0.0, seed=1, shuffle=False)
    true9 = int(np.flatnonzero((ev.layer == 9) & (ev.hit_track == 0))[0])
    jj = np.array([j], np.int32)
    kk = np.array([k], np.int32)
    x_true = oracle.phi0_coord(g, ev.r[true9:true9 + 1], ev.phi[true9:true9 + 1], jj, kk)[0][0]
    side = -1.0 if x_true > i + 0.5 else 1.0
    extra_phi = np.float32(ev.phi[true9] + side * 30e-4 / ev.r[true9])
    r = np.append(ev.r, ev.r[true9]).astype(np.float32)
    phi = np.append(ev.phi, extra_phi).astype(np.float32)
    layer = np.append(ev.layer, np.uint8(9))
    x_extra = oracle.phi0_coord(g, r[-1:], phi[-1:], jj, kk)[0][0]
    assert abs(x_extra - (i + 0.5)) < abs(x_true - (i + 0.5))
    lin = (k * nq + j) * np_ + i
    return g, W["cluster"], r, phi, layer, lin, true9, ev.n_hits


def _best_seed_failure(O):
    g, cl, r, phi, layer, lin, true9, extra = _two_seed_event(O)
    res = O.refine_one(g, r, phi, layer, lin, cl)
    if res["status"] != 0 or res["n_inliers"] != 10:
        return ("not refined", res["status"], res["n_inliers"])
    if res["hits"][9] != true9 or not res["ss"] < 1e-10:
        return ("wrong seed", int(res["hits"][9]), res["ss"])
    return None


def test_best_seed_prefers_smaller_sum(oracle):
    # the extra hit's circle also reaches every layer: the key decides
    g, cl, r, phi, layer, lin, true9, extra = _two_seed_event(oracle)
    keep = np.ones(r.size, bool)
    keep[true9] = False
    alone = oracle.refine_one(g, r[keep], phi[keep], layer[keep], lin, cl)
    assert alone["status"] == 0 and alone["n_inliers"] == 10 and alone["ss"] > 1e-8
    assert _best_seed_failure(oracle) is None


# --------------------------------------------------------------------------
# planted mistakes: each must make a pin above (or the 3D peak fixtures) fail
PEAK2 = "static int is_peak2("
PEAK3 = "static int is_peak3("
KEY = "static int key_greater("
REFINE = "static void refine("

MISTAKES = {
    "vpeak_strict_sides_swapped": (PEAK2, "negative ? !(c > w) : !(c >= w)",
                                   "negative ? !(c >= w) : !(c > w)", "vertex"),
    "vpeak_no_theta_wrap": (PEAK2, "int tt = ((t + dt) % nt + nt) % nt;",
                            "int tt = t + dt; if (tt < 0 || tt >= nt) continue;", "vertex"),
    "vpeak_rho_wraps": (PEAK2, "if (mm < 0 || mm >= nm) continue;",
                        "mm = (mm + nm) % nm;", "vertex"),
    "vpeak_threshold_exclusive": (PEAK2, "if (c < thr) return 0;", "if (c <= thr) return 0;",
                                  "vertex"),
    "vpeak_theta_before_rho": (PEAK2, "int negative = dm < 0 || (dm == 0 && dt < 0);",
                               "int negative = dt < 0 || (dt == 0 && dm < 0);", "vertex"),
    "peak3_strict_sides_swapped": (PEAK3, "negative ? !(v > w) : !(v >= w)",
                                   "negative ? !(v >= w) : !(v > w)", "peaks3"),
    "peak3_no_phi_wrap": (PEAK3, "int ii = ((i + di) % np + np) % np;",
                          "int ii = i + di; if (ii < 0 || ii >= np) continue;", "peaks3"),
    "peak3_dj_before_dk": (PEAK3, "int negative = dk < 0 || (dk == 0 && (dj < 0 || (dj == 0 && di < 0)));",
                           "int negative = dj < 0 || (dj == 0 && (dk < 0 || (dk == 0 && di < 0)));",
                           "peaks3"),
    "own_more_inliers_lose": (KEY, "return n_a > n_b;", "return n_a < n_b;", "ownership"),
    "own_sum_key_reversed": (KEY, "return ss_a < ss_b;", "return ss_a > ss_b;", "ownership"),
    "own_sum_key_dropped": (KEY, "if (ss_a != ss_b) return ss_a < ss_b;", "", "ownership"),
    "own_cell_key_reversed": (KEY, "return lin_a < lin_b;", "return lin_a > lin_b;", "ownership"),
    "seed_sum_key_reversed": (REFINE, "(n_in == best_n && ss < best_ss)",
                              "(n_in == best_n && ss > best_ss)", "seed"),
    "seed_sum_key_dropped": (REFINE, "(n_in == best_n && ss < best_ss)", "(0)", "seed"),
}


def _peaks3_failures(O):
    bad = []
    for case in _load("peaks_cases.json"):
        nd, nq, np_ = case["dims"]
        acc = np.zeros((nd, nq, np_), np.int32)
        for k, j, i, v in case["cells"]:
            acc[k, j, i] = v
        g = dict(n_phi=np_, n_qpt=nq, n_d0=nd, qpt_lo=-1.0, qpt_hi=1.0,
                 d0_lo=-20.0 if nd > 1 else 0.0, d0_hi=20.0 if nd > 1 else 0.0, bfield=3.8)
        pk, _ = O.hough_peaks(g, acc, case["threshold"])
        got = [[int(a), int(b)] for a, b in zip(pk["lin"], pk["votes"])]
        if got != case["expected"]:
            bad.append(case["name"])
    return bad


CHECKS = {"vertex": _vertex_golden_failures, "peaks3": _peaks3_failures,
          "ownership": _ownership_failures, "seed": _best_seed_failure}


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_planted_mistake_is_caught(oracle, tmp_path, name):
    head, old, new, check = MISTAKES[name]
    assert not CHECKS[check](oracle), "the pin fails on the real oracle"
    with planted(tmp_path, head, old, new) as mutant:
        assert CHECKS[check](mutant), f"planted mistake {name} passes the {check} pins"
