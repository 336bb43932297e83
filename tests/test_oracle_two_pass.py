"""Pins of the oracle's iterative hit removal (section "Current Tracker and
Tracking Algorithm": a prompt pass, removal of its hits, a displaced pass).

On noiseless events the truth fixes the outcome: the prompt pass finds
exactly the beam-line tracks, the kept hits are exactly the others, and the
displaced pass finds the vertex tracks with their own hits."""
import numpy as np

from paper_1309_6275_amd import configs as CF
from paper_1309_6275_amd import eventgen as G
from paper_1309_6275_amd import metrics as M


def test_compact_keeps_unowned_hits_in_order(oracle):
    rng = np.random.default_rng(5)
    n = 1000
    r = rng.uniform(4, 100, n).astype(np.float32)
    phi = rng.uniform(-3, 3, n).astype(np.float32)
    layer = rng.integers(0, 10, n).astype(np.uint8)
    owner = np.where(rng.random(n) < 0.6, rng.integers(0, 50, n), -1).astype(np.int32)
    r2, phi2, l2, idx = oracle.compact_hits(r, phi, layer, owner)
    want = [h for h in range(n) if owner[h] < 0]
    assert idx.tolist() == want
    assert np.array_equal(r2, r[want]) and np.array_equal(phi2, phi[want])
    assert np.array_equal(l2, layer[want])
    # empty and all-owned events
    assert oracle.compact_hits(r[:0], phi[:0], layer[:0], owner[:0])[3].size == 0
    assert oracle.compact_hits(r, phi, layer, np.zeros(n, np.int32))[3].size == 0


def test_two_pass_separates_prompt_and_displaced_tracks(oracle):
    rng = np.random.default_rng(17)
    prompt = [(rng.uniform(-np.pi, np.pi), rng.choice([-1, 1]) * rng.uniform(0.3, 0.95))
              for _ in range(25)]
    rho, theta = 14.0, 1.1
    psis = theta + rng.uniform(-0.5, 0.5, 10)
    qpts = rng.choice([-1, 1], 10) * rng.uniform(0.4, 0.9, 10)
    ev = G.make_vertex_event(rho, theta, psis, qpts, smear=0.0, seed=3, prompt=prompt)
    P, D = CF.TWO_PASS["prompt"], CF.TWO_PASS["displaced"]
    first, keep, second = oracle.two_pass(P["grid"], P["min_votes"], P["cluster"], D["grid"],
                                          D["min_votes"], D["cluster"], ev.r, ev.phi, ev.layer)
    is_prompt = ev.trk_vertex < 0
    m1 = M.match_tracks(first["tracks"]["hits"], ev.hit_track, 8)
    assert (m1 >= 0).all() and is_prompt[m1].all()
    assert sorted(m1.tolist()) == sorted(np.flatnonzero(is_prompt & (ev.trk_nhits >= 8)).tolist())
    # kept hits: every hit of a track the prompt pass did not find
    found = np.zeros(len(is_prompt), bool)
    found[m1] = True
    assert keep.tolist() == np.flatnonzero(~found[ev.hit_track]).tolist()
    # displaced pass: the vertex tracks, with their own event hits
    t2 = second["tracks"]
    m2 = M.match_tracks(t2["hits"], ev.hit_track, D["cluster"]["min_layers"])
    assert (m2 >= 0).all() and (~is_prompt[m2]).all()
    assert len(m2) >= 8
    for ti, tt in enumerate(m2):
        own = np.sort(t2["hits"][ti][t2["hits"][ti] >= 0])
        assert np.array_equal(own, np.sort(np.flatnonzero(ev.hit_track == tt)))
    # the vertex is found among the displaced tracks
    ob = second["objects"]
    assert len(ob) >= 1
    near = np.abs(ob["rho"] - rho) <= 2.0
    assert near.any()
