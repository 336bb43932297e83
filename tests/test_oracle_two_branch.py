"""Pins of the two-branch vertex vote (vtx_two_branch = 1): a track also
votes on the part of its circle before the perigee, which a track sent from
its vertex towards the beam line follows.  The truth comes from the
generator's geometry (a track produced at a known vertex), not from the
oracle's own crossing formula; a planted mistake (the incoming crossing
taken on the outgoing side) fails the first pin."""
import numpy as np

from paper_1309_6275_amd import configs as CF
from paper_1309_6275_amd import eventgen as G

from planted import planted

RHO, THETA = 10.0, -1.1


def _cfg(two):
    W = CF.WORKLOADS[2]
    return W, dict(W["cluster"], member_cap=512, vtx_two_branch=two)


def _cell(cl, rho, theta):
    rw = (cl["rho_hi"] - cl["rho_lo"]) / cl["n_rho"]
    m = int((rho - cl["rho_lo"]) // rw)
    t = int(np.floor((theta + np.pi) / (2 * np.pi / cl["n_theta"]))) % cl["n_theta"]
    return m, t


def _inward_event(n=10, seed=3):
    rng = np.random.default_rng(seed)
    # directions pointing towards the beam line (radial component < 0)
    psis = THETA + np.pi + rng.uniform(-0.9, 0.9, n)
    qpts = rng.choice([-1, 1], n) * rng.uniform(0.3, 0.9, n)
    return G.make_vertex_event(RHO, THETA, np.sort(psis), qpts, smear=0.0)


def _incoming_votes_at_vertex(O):
    """Votes near the true vertex cell from a decay whose tracks all head
    for the beam line, without and with the incoming branch."""
    W, _ = _cfg(0)
    ev = _inward_event()
    acc, _ = O.hough_vote(W["grid"], ev.r, ev.phi)
    pk, _ = O.hough_peaks(W["grid"], acc, W["min_votes"])
    out = []
    for two in (0, 1):
        _, cl = _cfg(two)
        res = O.assoc_cluster(W["grid"], ev.r, ev.phi, ev.layer, pk, cl)
        m, t = _cell(cl, RHO, THETA)
        v = res["vacc"]
        nt = cl["n_theta"]
        near = max(int(v[mm, (t + dt) % nt]) for mm in (m - 1, m, m + 1) for dt in (-1, 0, 1))
        out.append((near, int(res["counts"][1])))
    return out


def test_incoming_branch_votes_at_the_vertex(oracle):
    (off, n0), (on, n1) = _incoming_votes_at_vertex(oracle)
    assert n0 == n1 >= 8, (n0, n1)  # the tracks are found either way
    assert off == 0, off              # none of them reaches its vertex going outward
    assert on >= 8, on                # each passes through its vertex going inward


def test_isotropic_decay_shows_both_hemispheres(oracle):
    """60 tracks in all directions from a vertex 10 cm out: with both
    branches the object at the vertex has members of both hemispheres and a
    mean direction near zero (black-hole-like); with the outgoing branch
    only, it sees the outward half."""
    W = CF.WORKLOADS[2]
    rng = np.random.default_rng(21)
    psis = np.sort(THETA + rng.uniform(-np.pi, np.pi, 60))
    qpts = rng.choice([-1, 1], 60) * rng.uniform(0.3, 0.9, 60)
    ev = G.make_vertex_event(RHO, THETA, psis, qpts, smear=0.0)
    acc, _ = oracle.hough_vote(W["grid"], ev.r, ev.phi)
    pk, _ = oracle.hough_peaks(W["grid"], acc, W["min_votes"])
    outward = np.cos(psis - THETA) > 0  # truth track t has direction psis[t]
    found = {}
    for two in (0, 1):
        _, cl = _cfg(two)
        res = oracle.assoc_cluster(W["grid"], ev.r, ev.phi, ev.layer, pk, cl)
        obj, mem, trk = res["objects"], res["members"], res["tracks"]
        rw = (cl["rho_hi"] - cl["rho_lo"]) / cl["n_rho"]
        tw = 2 * np.pi / cl["n_theta"]
        dth = np.abs((obj["theta"] - THETA + np.pi) % (2 * np.pi) - np.pi)
        near = np.flatnonzero((np.abs(obj["rho"] - RHO) <= 2 * rw) & (dth <= 2 * tw))
        assert near.size, two
        o = obj[near[np.argmax(obj["n_tracks"][near])]]
        ids = mem[o["member_begin"]:o["member_begin"] + o["n_tracks"]]
        # truth track of each member: the generated track owning most of its hits
        truth = []
        for t in ids:
            h = trk["hits"][t]
            h = h[h >= 0]
            vals, cnt = np.unique(ev.hit_track[h], return_counts=True)
            truth.append(vals[np.argmax(cnt)])
        truth = np.array(truth)
        found[two] = (o, outward[truth].sum(), (~outward[truth]).sum())
    o0, out0, in0 = found[0]
    o1, out1, in1 = found[1]
    assert in0 <= 2 and out0 >= 20, (out0, in0)
    assert in1 >= 20 and out1 >= 20, (out1, in1)
    assert o1["kind"] == 1 and o1["isotropy"] <= 0.3, o1
    assert o0["isotropy"] > 0.5, o0


def test_planted_branch_sign_mistake_is_caught(oracle, tmp_path):
    assert _incoming_votes_at_vertex(oracle)[1][0] >= 8
    with planted(tmp_path, "static double crossing_theta(", "if (branch < 0) h = -h;",
                 "(void)branch;") as mutant:
        (off, _), (on, _) = _incoming_votes_at_vertex(mutant)
        assert on < 8, on
