"""The serving loop's batched launches and its learned peak filter.

Batches: with one slot, every event submitted while the slot is busy waits,
and the waiting events start in batches of up to four of a kind (the
oldest, then later small ones of its kind); each event's results are
bit-identical to those of the same event run alone by a server without
batching, with graph replay and with direct launches, and events above the
batch hit bound run alone.  Filter: a kind with filter parameters gives the
results of hough_vote, hough_peaks, cnn_score, cnn_keep and assoc_cluster
called one by one, alone and in batches."""
from types import SimpleNamespace

import numpy as np
import pytest

from paper_1309_6275_amd import configs as CF
from paper_1309_6275_amd import eventgen as G
from paper_1309_6275_amd import peakfilter as PF

from test_gpu_server import KINDS, SERVER_ARGS, run_all

pytestmark = pytest.mark.gpu

KEYS = ("counts", "hit_owner", "tracks", "objects", "members")


@pytest.fixture(scope="module")
def ht():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1309_6275_amd import houghtrig
    houghtrig.lib()
    return houghtrig


def _hits(n, seed):
    r, phi, layer = G.random_hits(n, seed=seed, r_lo=3.0, r_hi=105.0)
    return SimpleNamespace(r=r, phi=phi, layer=layer, n_hits=n)


def _stream():
    """Kinds and sizes mixed: real events of both workloads, random hits of
    0 to 8192 (two above the batch bound of 6000)."""
    ev = []
    W1, W2 = CF.WORKLOADS[1], CF.WORKLOADS[2]
    for i in range(5):
        ev.append((0, G.make_event(1, W1["seed0"] + 300 + i)))
        ev.append((1, G.make_event(2, W2["seed0"] + 300 + i)))
    for i, (k, n) in enumerate([(0, 0), (1, 1), (0, 7000), (1, 5999), (1, 8192), (0, 6000),
                                (1, 17), (0, 4000)]):
        ev.append((k, _hits(n, 6100 + i)))
    rng = np.random.default_rng(11)
    return [ev[i] for i in rng.permutation(len(ev))]


def _same(a, b, what):
    for key in KEYS:
        assert a[key].tobytes() == b[key].tobytes(), (what, key)
    assert a["n_peaks"] == b["n_peaks"], what
    assert a["n_kept"] == b["n_kept"], what


def test_server_batches_equal_events_alone(ht):
    events = _stream()
    print(f"server batches: {len(events)} events, one slot", flush=True)
    plain = ht.Server(KINDS, **dict(SERVER_ARGS, max_slots=1))
    alone = {}
    for i, e in enumerate(events):  # one at a time: never batched, never overlapped
        alone.update(run_all(plain, [e], tag0=i))
    plain.close()
    for graphs in (True, False):
        srv = ht.Server(KINDS, use_graphs=graphs, batch_max=4, batch_max_hits=6000,
                        **dict(SERVER_ARGS, max_slots=1))
        got = run_all(srv, events)
        srv.close()
        sizes = [d["batch"] for d in got.values()]
        assert max(sizes) == 4, sizes
        for t, (k, ev) in enumerate(events):
            d = got[t]
            assert d["status"] == 0 and d["kind"] == k
            assert alone[t]["batch"] == 1
            if ev.n_hits > 6000:
                assert d["batch"] == 1, t
            _same(d, alone[t], f"event {t} ({ev.n_hits} hits, batch {d['batch']}, graphs {graphs})")
            assert d["n_kept"] == d["n_peaks"]


def test_server_batch_order_and_poll_bound(ht):
    """The oldest waiting event leads each batch; a poll that cannot take a
    whole batch is refused."""
    ev = [(0, G.make_event(1, CF.WORKLOADS[1]["seed0"] + 320 + i)) for i in range(6)]
    ev.insert(3, (1, G.make_event(2, CF.WORKLOADS[2]["seed0"] + 320)))
    srv = ht.Server(KINDS, batch_max=4, batch_max_hits=6000, **dict(SERVER_ARGS, max_slots=1))
    with pytest.raises(ht.HoughError) as e:
        srv.poll(max_results=3)
    assert e.value.code == ht.HT_EINVAL
    got = run_all(srv, ev)
    # tag 0 starts at submit; tags 1, 2, 4, 5 (kind 0) then form one batch;
    # tag 3 (kind 1) and tag 6 follow
    assert got[0]["batch"] == 1
    assert [got[t]["batch"] for t in (1, 2, 4, 5)] == [4] * 4
    assert len({got[t]["t_start"] for t in (1, 2, 4, 5)}) == 1
    assert got[3]["batch"] == 1 and got[6]["batch"] == 1
    assert got[3]["t_start"] >= got[1]["t_start"]
    srv.close()


def _filter_kind(ht, torch, ev0):
    """Kind 1 with seeded filter weights and the median logit of an event's
    peaks as its threshold (about half of the peaks kept)."""
    K = dict(KINDS[1])
    params = PF.init_params(7)
    g = K["grid"]
    plan = ht.Plan(g, max_hits=SERVER_ARGS["max_hits"], max_peaks=K["peak_cap"],
                   max_member_cap=K["cluster"]["member_cap"], max_tracks=SERVER_ARGS["track_cap"])
    acc = torch.empty(plan.acc_shape, dtype=torch.int32, device="cuda")
    peaks = torch.empty((K["peak_cap"], 2), dtype=torch.int32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    logits = torch.empty(K["peak_cap"], dtype=torch.float32, device="cuda")
    ws = ht.cnn_workspace(K["peak_cap"])
    d = dict(r=torch.from_numpy(ev0.r).cuda(), phi=torch.from_numpy(ev0.phi).cuda())
    ht.hough_vote(plan, d["r"], d["phi"], acc)
    ht.hough_peaks(plan, acc, K["min_votes"], peaks, nf)
    ht.cnn_score(plan, torch.from_numpy(params).cuda(), acc, peaks, nf, logits, ws)
    torch.cuda.synchronize()
    n = int(nf.item())
    thr = float(np.median(logits[:n].cpu().numpy()))
    plan.close()
    return dict(K, cnn_params=params, cnn_threshold=thr)


def _calls(ht, torch, K, ev):
    """The filtered chain called one by one."""
    g, cl, cap = K["grid"], K["cluster"], K["peak_cap"]
    plan = ht.Plan(g, max_hits=SERVER_ARGS["max_hits"], max_peaks=cap,
                   max_member_cap=cl["member_cap"], max_tracks=SERVER_ARGS["track_cap"])
    acc = torch.empty(plan.acc_shape, dtype=torch.int32, device="cuda")
    peaks = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    kept = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    nk = torch.zeros(1, dtype=torch.int32, device="cuda")
    logits = torch.empty(cap, dtype=torch.float32, device="cuda")
    ws = ht.cnn_workspace(cap)
    bufs = ht.ClusterBuffers(max(ev.n_hits, 1), SERVER_ARGS["track_cap"], SERVER_ARGS["object_cap"],
                             SERVER_ARGS["member_cap"], cl["n_rho"], cl["n_theta"])
    r = torch.from_numpy(ev.r).cuda()
    phi = torch.from_numpy(ev.phi).cuda()
    layer = torch.from_numpy(ev.layer).cuda()
    params = torch.from_numpy(K["cnn_params"]).cuda()
    ht.hough_vote(plan, r, phi, acc)
    ht.hough_peaks(plan, acc, K["min_votes"], peaks, nf)
    ht.cnn_score(plan, params, acc, peaks, nf, logits, ws)
    ht.cnn_keep(plan, logits, peaks, nf, K["cnn_threshold"], kept, nk)
    ht.assoc_cluster(plan, r, phi, layer, kept, nk, cl, bufs, with_vacc=False, acc=acc)
    torch.cuda.synchronize()
    out = bufs.to_host(ev.n_hits)
    out.update(n_peaks=int(nf.item()), n_kept=int(nk.item()))
    plan.close()
    return out


def test_server_filter_equals_calls(ht):
    import torch
    W2 = CF.WORKLOADS[2]
    events = [(1, G.make_event(2, W2["seed0"] + 340 + i)) for i in range(5)]
    events.insert(2, (0, G.make_event(1, CF.WORKLOADS[1]["seed0"] + 340)))
    K1 = _filter_kind(ht, torch, events[0][1])
    print(f"server filter: threshold {K1['cnn_threshold']:.4f}", flush=True)
    kinds = [KINDS[0], K1]
    srv = ht.Server(kinds, batch_max=4, batch_max_hits=6000, **dict(SERVER_ARGS, max_slots=1))
    got = run_all(srv, events)
    srv.close()
    assert max(d["batch"] for d in got.values()) == 4
    for t, (k, ev) in enumerate(events):
        d = got[t]
        assert d["status"] == 0
        if k == 0:
            assert d["n_kept"] == d["n_peaks"]
            continue
        want = _calls(ht, torch, K1, ev)
        assert 0 < d["n_kept"] < d["n_peaks"], (d["n_kept"], d["n_peaks"])
        assert d["n_kept"] == want["n_kept"] and d["n_peaks"] == want["n_peaks"], t
        assert np.array_equal(d["counts"], want["counts"]), (t, d["counts"], want["counts"])
        assert np.array_equal(d["hit_owner"], want["hit_owner"]), t
        for key in ("tracks", "objects"):
            assert d[key].tobytes() == want[key].tobytes(), (t, key)
        assert np.array_equal(d["members"], want["members"]), t
