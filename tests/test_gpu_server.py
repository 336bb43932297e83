"""The trigger serving loop (ht_server_*): results equal the oracle's for
events of two grid kinds submitted in a mix; an event gives bit-identical
results alone and inside a mix; graph replay equals direct launches across
events of different sizes; admission by HBM budget and queue bound."""
from types import SimpleNamespace

import numpy as np
import pytest

from paper_1309_6275_amd import configs as CF
from paper_1309_6275_amd import eventgen as G

from test_gpu_assoc import compare

pytestmark = pytest.mark.gpu

KINDS = [dict(grid=CF.WORKLOADS[1]["grid"], cluster=CF.WORKLOADS[1]["cluster"],
              min_votes=CF.WORKLOADS[1]["min_votes"], peak_cap=1 << 16),
         dict(grid=CF.WORKLOADS[2]["grid"], cluster=CF.WORKLOADS[2]["cluster"],
              min_votes=CF.WORKLOADS[2]["min_votes"], peak_cap=1 << 19)]
SERVER_ARGS = dict(max_hits=8192, track_cap=2048, object_cap=128, member_cap=4096,
                   hbm_budget=24 << 30, max_slots=3, queue_cap=64)


@pytest.fixture(scope="module")
def ht():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1309_6275_amd import houghtrig
    houghtrig.lib()
    return houghtrig


def oracle_result(oracle, kind, ev):
    K = KINDS[kind]
    acc, _ = oracle.hough_vote(K["grid"], ev.r, ev.phi)
    pk, _ = oracle.hough_peaks(K["grid"], acc, K["min_votes"])
    pk = pk[:K["peak_cap"]]
    return oracle.assoc_cluster(K["grid"], ev.r, ev.phi, ev.layer, pk, K["cluster"],
                                track_cap=SERVER_ARGS["track_cap"],
                                object_cap=SERVER_ARGS["object_cap"],
                                member_cap=SERVER_ARGS["member_cap"])


def as_got(res):
    return dict(counts=res["counts"], hit_owner=res["hit_owner"], tracks=res["tracks"],
                objects=res["objects"], members=res["members"], vacc=np.zeros(1, np.int32))


def mixed_events():
    evs = []
    for s in range(3):
        evs.append((0, G.make_event(1, CF.WORKLOADS[1]["seed0"] + 40 + s)))
    for s in range(2):
        evs.append((1, G.make_event(2, CF.WORKLOADS[2]["seed0"] + 40 + s)))
    order = [0, 3, 1, 4, 2]
    return [evs[i] for i in order]


def run_all(srv, events, tag0=0):
    for i, (kind, ev) in enumerate(events):
        assert srv.submit(kind, ev.r, ev.phi, ev.layer, tag0 + i)
    got = {}
    for d in srv.drain():
        got[d["tag"]] = d
    assert len(got) == len(events)
    return got


def test_server_matches_oracle(ht, oracle):
    srv = ht.Server(KINDS, **SERVER_ARGS)
    print(f"slots {srv.n_slots} bytes/slot {srv.slot_bytes}", flush=True)
    events = mixed_events()
    got = run_all(srv, events)
    for i, (kind, ev) in enumerate(events):
        d = got[i]
        assert d["status"] == 0
        want = oracle_result(oracle, kind, ev)
        want = dict(want, vacc=np.zeros(1, np.int32))
        compare(as_got(d), want, f"server event {i} kind {kind}")
    srv.close()


def test_server_alone_vs_mix_bitexact(ht):
    """An event's results do not depend on what else is in flight."""
    kind, ev = 1, G.make_event(2, CF.WORKLOADS[2]["seed0"] + 77)
    srv = ht.Server(KINDS, **SERVER_ARGS)
    alone = run_all(srv, [(kind, ev)])[0]
    rng = np.random.default_rng(5)
    mix = []
    for i in range(12):
        k = int(rng.integers(0, 2))
        n = int(rng.integers(0, 8000))
        r, phi, layer = G.random_hits(n, seed=1000 + i, r_lo=3.0, r_hi=105.0)
        mix.append((k, SimpleNamespace(r=r, phi=phi, layer=layer, n_hits=n)))
    mix.insert(5, (kind, ev))
    got = run_all(srv, mix, tag0=100)
    inmix = got[105]
    for key in ("counts", "hit_owner", "tracks", "objects", "members"):
        assert inmix[key].tobytes() == alone[key].tobytes(), key
    assert inmix["n_peaks"] == alone["n_peaks"]
    srv.close()


def test_server_graph_replay_equals_direct(ht):
    """Graph replays with the hit count in device memory give the results of
    direct launches, for events of different sizes in a row (and the empty
    event)."""
    rng = np.random.default_rng(9)
    events = []
    for i, n in enumerate([3000, 17, 0, 8192, 500, 4096, 1]):
        r, phi, layer = G.random_hits(n, seed=2000 + i, r_lo=3.0, r_hi=105.0,
                                      bad_fraction=0.03 if n > 100 else 0.0)
        events.append((i % 2, SimpleNamespace(r=r, phi=phi, layer=layer, n_hits=n)))
    events.append((1, G.make_event(2, CF.WORKLOADS[2]["seed0"] + 78)))
    events.append((0, G.make_event(1, CF.WORKLOADS[1]["seed0"] + 78)))
    res = []
    for graphs in (True, False):
        srv = ht.Server(KINDS, use_graphs=graphs, **SERVER_ARGS)
        res.append(run_all(srv, events + events, tag0=0))
        srv.close()
    for t in range(2 * len(events)):
        a, b = res[0][t], res[1][t]
        for key in ("counts", "hit_owner", "tracks", "objects", "members"):
            assert a[key].tobytes() == b[key].tobytes(), (t, key)
        assert a["n_peaks"] == b["n_peaks"]
        # the second pass replays the same events on reused slots: same results
        if t >= len(events):
            c = res[0][t - len(events)]
            assert a["counts"].tobytes() == c["counts"].tobytes(), t


def test_server_admission_and_shedding(ht):
    args = dict(SERVER_ARGS, max_slots=8, queue_cap=0)
    one = ht.Server(KINDS, **dict(args, max_slots=1))
    per_slot = one.slot_bytes
    one.close()
    srv = ht.Server(KINDS, **dict(args, hbm_budget=int(per_slot * 2.5)))
    assert srv.n_slots == 2
    ev = G.make_event(1, CF.WORKLOADS[1]["seed0"] + 5)
    assert srv.submit(0, ev.r, ev.phi, ev.layer, 1)
    assert srv.submit(0, ev.r, ev.phi, ev.layer, 2)
    assert not srv.submit(0, ev.r, ev.phi, ev.layer, 3)  # both slots busy until polled, no queue
    done = srv.drain()
    assert sorted(d["tag"] for d in done) == [1, 2]
    assert done[0]["counts"].tobytes() == done[1]["counts"].tobytes()
    srv.close()
    with pytest.raises(ht.HoughError) as e:
        ht.Server(KINDS, **dict(args, hbm_budget=per_slot // 4))
    assert e.value.code == ht.HT_ENOMEM


def test_server_work_budget(ht, oracle):
    """With a work budget of one 3D event of 8192 hits (hits x q/pT x d0
    columns), 3D events of 5000-8192 hits run one after another: an event
    starts only once the one before has been seen done.  Small 2D events
    still overlap.  Results equal the plain server's and the oracle's."""
    g3 = KINDS[1]["grid"]
    budget = 8192 * g3["n_qpt"] * g3["n_d0"]
    heavy = []
    for i, n in enumerate([8192, 5000, 7000, 6000]):
        r, phi, layer = G.random_hits(n, seed=3000 + i, r_lo=3.0, r_hi=105.0)
        heavy.append((1, SimpleNamespace(r=r, phi=phi, layer=layer, n_hits=n)))
    light = [(0, G.make_event(1, CF.WORKLOADS[1]["seed0"] + 60 + i)) for i in range(6)]
    budgeted = ht.Server(KINDS, work_budget=budget, **SERVER_ARGS)
    plain = ht.Server(KINDS, **SERVER_ARGS)
    got_h = run_all(budgeted, heavy)
    ref_h = run_all(plain, heavy)
    spans = sorted((d["t_start"], d["t_done"]) for d in got_h.values())
    for (s0, e0), (s1, e1) in zip(spans, spans[1:]):
        assert s1 >= e0  # no two heavy events in flight together
    got_l = run_all(budgeted, light, tag0=100)
    # light ones overlap: each of the first light events was put on a slot
    # inside its own submit call (the server stamps t_start there), before
    # the next event was submitted, while the events before it were still
    # in flight (completion is only taken in poll, after all the submits);
    # an order of host calls, not a race of clocks
    first = min(budgeted.n_slots, len(light))
    assert first >= 2
    for i in range(first - 1):
        assert got_l[100 + i]["t_start"] <= got_l[101 + i]["t_submit"], i
    assert got_l[100]["t_done"] >= got_l[99 + first]["t_start"]
    for t, d in got_h.items():
        for key in ("counts", "hit_owner", "tracks", "objects", "members"):
            assert d[key].tobytes() == ref_h[t][key].tobytes(), (t, key)
    kind, ev = light[2]
    want = dict(oracle_result(oracle, kind, ev), vacc=np.zeros(1, np.int32))
    compare(as_got(got_l[102]), want, "budgeted light event")
    budgeted.close()
    plain.close()
    with pytest.raises(ht.HoughError) as e:
        ht.Server(KINDS, work_budget=-1, **SERVER_ARGS)
    assert e.value.code == ht.HT_EINVAL
