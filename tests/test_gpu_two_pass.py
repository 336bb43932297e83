"""GPU parity of iterative hit removal (prompt pass, ht_compact_hits,
displaced pass, ht_remap_track_hits) against the oracle's two-pass chain.

The oracle runs its own vote and peaks on both passes; kept-hit indices and
every integer output must match exactly, refits within the tolerance of the
assoc_cluster parity tests."""
import numpy as np
import pytest

from paper_1309_6275_amd import configs as CF
from paper_1309_6275_amd import eventgen as G

from test_gpu_assoc import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def tp(torch):
    from paper_1309_6275_amd import iterative
    t = iterative.TwoPass(max_hits=65535, track_cap=4096, object_cap=512)
    yield t
    t.close()


def _event(label):
    if label.startswith("cfg2"):
        W = CF.WORKLOADS[2]
        return G.make_event(2, W["seed0"] + int(label[-1]))
    rng = np.random.default_rng(17)
    prompt = [(rng.uniform(-np.pi, np.pi), rng.choice([-1, 1]) * rng.uniform(0.3, 0.95))
              for _ in range(40)]
    psis = 1.1 + rng.uniform(-0.5, 0.5, 10)
    qpts = rng.choice([-1, 1], 10) * rng.uniform(0.4, 0.9, 10)
    return G.make_vertex_event(14.0, 1.1, psis, qpts, n_noise=200, seed=3, prompt=prompt)


@pytest.mark.parametrize("label", ["cfg2_0", "cfg2_1", "cfg2_2", "vertex"])
def test_two_pass_parity(torch, tp, oracle, label):
    ev = _event(label)
    print(f"two-pass {label} hits {ev.n_hits}", flush=True)
    r = torch.from_numpy(ev.r).cuda()
    phi = torch.from_numpy(ev.phi).cuda()
    layer = torch.from_numpy(ev.layer).cuda()
    tp.run(r, phi, layer)
    first, keep, second = tp.to_host(ev.n_hits)
    P, D = CF.TWO_PASS["prompt"], CF.TWO_PASS["displaced"]
    w1, wkeep, w2 = oracle.two_pass(P["grid"], P["min_votes"], P["cluster"], D["grid"],
                                    D["min_votes"], D["cluster"], ev.r, ev.phi, ev.layer,
                                    peak_cap=None, track_cap=4096, object_cap=512,
                                    member_cap=1 << 15)
    # the prompt pass (its vertex outputs are not asked for)
    assert np.array_equal(first["counts"][:2], w1["counts"][:2]), label
    assert np.array_equal(first["hit_owner"], w1["hit_owner"]), label
    w1t = w1["tracks"]
    for f in ("lin", "n_inliers", "n_owned", "seed_ss", "hits", "status"):
        assert np.array_equal(first["tracks"][f], w1t[f]), (label, f)
    assert keep.size == wkeep.size and np.array_equal(keep, wkeep), label
    compare(second, w2, f"{label} displaced pass")
    assert second["tracks"].size > 0


def test_compact_hits_edge_cases(torch):
    from paper_1309_6275_amd import houghtrig as H
    rng = np.random.default_rng(9)
    for n in (0, 1, 1023, 1024, 1025, 65535):
        print(f"compact n={n}", flush=True)
        r = torch.from_numpy(rng.uniform(4, 100, n).astype(np.float32)).cuda()
        phi = torch.from_numpy(rng.uniform(-3, 3, n).astype(np.float32)).cuda()
        layer = torch.from_numpy(rng.integers(0, 10, n).astype(np.uint8)).cuda()
        own_h = np.where(rng.random(n) < 0.5, rng.integers(0, 9, n), -1).astype(np.int32)
        if n == 1025:
            own_h[:] = -1
        if n == 1023:
            own_h[:] = 3
        owner = torch.from_numpy(own_h).cuda()
        outs = [torch.full((max(n, 1),), v, dtype=d, device="cuda")
                for v, d in ((-7, torch.float32), (-7, torch.float32), (250, torch.uint8),
                             (-7, torch.int32))]
        n_out = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        H.compact_hits(r, phi, layer, owner, outs[0][:n], outs[1][:n], outs[2][:n], outs[3][:n],
                       n_out)
        torch.cuda.synchronize()
        want = np.flatnonzero(own_h < 0)
        k = int(n_out.item())
        assert k == want.size
        assert np.array_equal(outs[3][:k].cpu().numpy(), want)
        assert np.array_equal(outs[0][:k].cpu().numpy(), r.cpu().numpy()[want])
        assert np.array_equal(outs[1][:k].cpu().numpy(), phi.cpu().numpy()[want])
        assert np.array_equal(outs[2][:k].cpu().numpy(), layer.cpu().numpy()[want])
        # nothing beyond the kept hits is written
        if k < n:
            assert (outs[3][k:n].cpu().numpy() == -7).all()


def test_device_count_calls_match_host_count(torch, oracle):
    """hough_vote_n and assoc_cluster_n over buffers of n hits with a device
    count k < n equal hough_vote and assoc_cluster on the first k hits."""
    from paper_1309_6275_amd import houghtrig as H
    W = CF.WORKLOADS[2]
    g, cl = W["grid"], W["cluster"]
    ev = G.make_event(2, W["seed0"] + 9)
    k = ev.n_hits - 1000
    print(f"device count {k} of {ev.n_hits}", flush=True)
    plan = H.Plan(g, max_peaks=1 << 20, max_tracks=1 << 13)
    r = torch.from_numpy(ev.r).cuda()
    phi = torch.from_numpy(ev.phi).cuda()
    layer = torch.from_numpy(ev.layer).cuda()
    nk = torch.tensor([k], dtype=torch.int32, device="cuda")
    outs = []
    for dev in (True, False):
        acc = torch.full(plan.acc_shape, -1, dtype=torch.int32, device="cuda")
        nv = torch.zeros(1, dtype=torch.int64, device="cuda")
        peaks = torch.full((1 << 20, 2), -1, dtype=torch.int32, device="cuda")
        nf = torch.zeros(1, dtype=torch.int32, device="cuda")
        bufs = H.ClusterBuffers(ev.n_hits, 4096, 512, 1 << 15, cl["n_rho"], cl["n_theta"])
        if dev:
            H.hough_vote_n(plan, r, phi, nk, acc, nv)
            H.hough_peaks(plan, acc, W["min_votes"], peaks, nf)
            H.assoc_cluster_n(plan, r, phi, layer, nk, peaks, nf, cl, bufs)
        else:
            H.hough_vote(plan, r[:k], phi[:k], acc, nv)
            H.hough_peaks(plan, acc, W["min_votes"], peaks, nf)
            H.assoc_cluster(plan, r[:k], phi[:k], layer[:k], peaks, nf, cl, bufs)
        torch.cuda.synchronize()
        outs.append((acc.cpu().numpy(), int(nv.item()), bufs.to_host(k)))
    (a1, v1, o1), (a2, v2, o2) = outs
    assert v1 == v2 and np.array_equal(a1, a2)
    compare(o1, o2, "device count")
    assert np.array_equal(o1["tracks"]["phi0"], o2["tracks"]["phi0"])
    plan.close()
