"""GPU parity of the hit-sliced launches (point and band votes, member
sweep) and of candidates dropped over member_cap, through the C-ABI.

Grids with few 64-column tiles (the 2D grid has four) split the hits into
slices: the vote adds each slice's tile into a cleared accumulator, and the
member sweep shares global slot counters between slices.  A candidate that
goes over member_cap is dropped; the sweep stops testing it from then on.
Accumulators, vote totals and every integer output must stay bit-exact
against the oracle."""
from types import SimpleNamespace

import numpy as np
import pytest

from paper_1309_6275_amd import configs as CF
from paper_1309_6275_amd import eventgen as G

from test_gpu_assoc import compare, run_gpu, run_oracle
from test_gpu_vote_peaks import ODD_GRIDS, gpu_vote, plan_for

pytestmark = pytest.mark.gpu

SLICE_GRIDS = [CF.GRID_2D] + ODD_GRIDS


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def ht(torch):
    from paper_1309_6275_amd import houghtrig
    houghtrig.lib()
    return houghtrig


def _same(got, want):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{bad.shape[0]} cells differ, first {bad[:5].tolist()}")


@pytest.mark.parametrize("gi", range(len(SLICE_GRIDS)))
@pytest.mark.parametrize("n_hits", [2047, 2048, 4099, 20000, 65535])
def test_sliced_vote_parity(torch, ht, oracle, gi, n_hits):
    """Random hits (5% invalid) on grids of 1 to 64 tiles, from just below
    the slicing bound to the largest event."""
    g = SLICE_GRIDS[gi]
    print(f"sliced vote grid {gi} hits {n_hits}", flush=True)
    r, phi, _ = G.random_hits(n_hits, seed=500 + gi * 11 + n_hits, r_lo=0.5, r_hi=120.0,
                              bad_fraction=0.05)
    acc_d, nv = gpu_vote(torch, ht, g, r, phi)
    want, nv_w = oracle.hough_vote(g, r, phi)
    assert nv == nv_w
    _same(acc_d.cpu().numpy(), want)


def test_sliced_vote_serving_event(torch, ht, oracle):
    """A 2D trigger event of ~40k hits (prompt tracks, 20% noise)."""
    ev = G.make_serving_event(0, 8101, h_lo=40000, h_hi=40001)
    print(f"serving 2D hits {ev.n_hits}", flush=True)
    acc_d, nv = gpu_vote(torch, ht, CF.GRID_2D, ev.r, ev.phi)
    want, nv_w = oracle.hough_vote(CF.GRID_2D, ev.r, ev.phi)
    assert nv == nv_w
    _same(acc_d.cpu().numpy(), want)


@pytest.mark.parametrize("k", [0, 1, 2047, 5000, 65535])
def test_sliced_vote_device_count(torch, ht, oracle, k):
    """hough_vote_n with a 65535-hit bound (63 slices) and a device count k:
    the slices divide k, and the result is the vote of the first k hits."""
    g = CF.GRID_2D
    plan = plan_for(ht, g)
    r, phi, _ = G.random_hits(65535, seed=77, r_lo=3.0, r_hi=105.0, bad_fraction=0.02)
    print(f"device count {k}", flush=True)
    rd = torch.from_numpy(r).cuda()
    pd = torch.from_numpy(phi).cuda()
    nk = torch.tensor([k], dtype=torch.int32, device="cuda")
    acc = torch.full(plan.acc_shape, -7, dtype=torch.int32, device="cuda")
    nv = torch.zeros(1, dtype=torch.int64, device="cuda")
    ht.hough_vote_n(plan, rd, pd, nk, acc, nv)
    torch.cuda.synchronize()
    want, nv_w = oracle.hough_vote(g, r[:k], phi[:k])
    assert int(nv.item()) == nv_w
    _same(acc.cpu().numpy(), want)


@pytest.mark.parametrize("target", [20000, 45000])
def test_sliced_member_sweep_dense_2d(torch, ht, oracle, target):
    """Dense 2D trigger events: the member sweep runs in hit slices with
    shared slot counters, and many candidates go over member_cap (256)."""
    W = CF.WORKLOADS[1]
    ev = G.make_serving_event(0, 8200 + target, h_lo=target, h_hi=target + 1)
    print(f"dense 2D hits {ev.n_hits}", flush=True)
    got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], W["cluster"])
    want = run_oracle(oracle, W["grid"], ev, acc, pk, W["cluster"])
    compare(got, want, f"dense 2D {target}")
    assert want["counts"][4] > 0  # candidates dropped over member_cap
    if target == 20000:
        assert want["counts"][0] > 0  # and others refined


def test_sliced_member_sweep_device_count(torch, ht, oracle):
    """assoc_cluster_n on the 2D grid with a 65535-hit bound and a device
    count of 9000 equals the oracle on the first 9000 hits."""
    W = CF.WORKLOADS[1]
    g, cl = W["grid"], W["cluster"]
    ev = G.make_serving_event(0, 8300, h_lo=12000, h_hi=12001)
    k = 9000
    print(f"device count {k} of {ev.n_hits}", flush=True)
    plan = plan_for(ht, g)
    n = 65535
    pad = n - ev.n_hits
    r = np.concatenate([ev.r, np.full(pad, 50.0, np.float32)])
    phi = np.concatenate([ev.phi, np.zeros(pad, np.float32)])
    layer = np.concatenate([ev.layer, np.zeros(pad, np.uint8)])
    rd = torch.from_numpy(r).cuda()
    pd = torch.from_numpy(phi).cuda()
    ld = torch.from_numpy(layer).cuda()
    nk = torch.tensor([k], dtype=torch.int32, device="cuda")
    acc = torch.empty(plan.acc_shape, dtype=torch.int32, device="cuda")
    ht.hough_vote_n(plan, rd, pd, nk, acc)
    peaks = torch.full((1 << 20, 2), -1, dtype=torch.int32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    ht.hough_peaks(plan, acc, W["min_votes"], peaks, nf)
    bufs = ht.ClusterBuffers(n, 4096, 512, 1 << 15, cl["n_rho"], cl["n_theta"])
    ht.assoc_cluster_n(plan, rd, pd, ld, nk, peaks, nf, cl, bufs)
    torch.cuda.synchronize()
    got = bufs.to_host(k)
    pk = peaks[:int(nf.item())].cpu().numpy()
    sub = SimpleNamespace(r=ev.r[:k], phi=ev.phi[:k], layer=ev.layer[:k], n_hits=k)
    want = run_oracle(oracle, g, sub, None, pk, cl)
    compare(got, want, "device count 2D")


@pytest.mark.parametrize("cap", [8, 16])
def test_member_cap_overflow_3d(torch, ht, oracle, cap):
    """The displaced-jet workload with a member_cap below most candidates'
    member counts: the candidates dropped, the counts and the tracks of the
    rest match the oracle."""
    W = CF.WORKLOADS[2]
    ev = G.make_event(2, W["seed0"] + 21)
    cfg = dict(W["cluster"], member_cap=cap)
    print(f"member_cap {cap} hits {ev.n_hits}", flush=True)
    got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], cfg)
    want = run_oracle(oracle, W["grid"], ev, acc, pk, cfg)
    compare(got, want, f"member_cap {cap}")
    assert want["counts"][4] > pk.shape[0] // 2


@pytest.mark.parametrize("gi", range(len(SLICE_GRIDS)))
@pytest.mark.parametrize("n_hits", [2048, 20000, 65535])
def test_sliced_cell_vote_parity(torch, ht, oracle, gi, n_hits):
    """The band vote in hit slices on grids of 1 to 64 tiles."""
    g = SLICE_GRIDS[gi]
    print(f"sliced cell vote grid {gi} hits {n_hits}", flush=True)
    r, phi, _ = G.random_hits(n_hits, seed=900 + gi * 13 + n_hits, r_lo=0.5, r_hi=120.0,
                              bad_fraction=0.05)
    plan = plan_for(ht, g)
    rd = torch.from_numpy(r).cuda()
    pd = torch.from_numpy(phi).cuda()
    acc = torch.full(plan.acc_shape, -7, dtype=torch.int32, device="cuda")
    nv = torch.zeros(1, dtype=torch.int64, device="cuda")
    ht.hough_vote_cell(plan, rd, pd, acc, nv)
    torch.cuda.synchronize()
    want, nv_w = oracle.hough_vote_cell(g, r, phi)
    assert int(nv.item()) == nv_w
    _same(acc.cpu().numpy(), want)
