"""GPU parity of hough_vote_cell (the band variant of the vote) against the
oracle, through the C-ABI: accumulators and vote totals bit-exact, then the
peak finder and assoc_cluster on the band accumulator."""
import numpy as np
import pytest

from paper_1309_6275_amd import configs as CF
from paper_1309_6275_amd import eventgen as G

from test_gpu_assoc import compare, run_oracle
from test_gpu_vote_peaks import ODD_GRIDS, gpu_peaks, plan_for

pytestmark = pytest.mark.gpu


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


def gpu_cell_vote(torch, ht, grid, r, phi):
    plan = plan_for(ht, grid)
    rd = torch.from_numpy(np.ascontiguousarray(r, np.float32)).cuda()
    pd = torch.from_numpy(np.ascontiguousarray(phi, np.float32)).cuda()
    acc = torch.full(plan.acc_shape, -7, dtype=torch.int32, device="cuda")
    nv = torch.zeros(1, dtype=torch.int64, device="cuda")
    ht.hough_vote_cell(plan, rd, pd, acc, nv)
    torch.cuda.synchronize()
    return acc, int(nv.item())


def _same(got, want):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{bad.shape[0]} cells differ, first {bad[:5].tolist()}")


@pytest.mark.parametrize("cfg,seeds", [(1, range(3)), (2, range(2)), (3, range(1))])
def test_cell_vote_parity_workloads(torch, ht, oracle, cfg, seeds):
    W = CF.WORKLOADS[cfg]
    g = W["grid"]
    for s in seeds:
        ev = G.make_event(cfg, W["seed0"] + s)
        print(f"cell cfg{cfg} seed {W['seed0'] + s} hits {ev.n_hits}", flush=True)
        acc_d, nv = gpu_cell_vote(torch, ht, g, ev.r, ev.phi)
        want, nv_w = oracle.hough_vote_cell(g, ev.r, ev.phi)
        assert nv == nv_w
        _same(acc_d.cpu().numpy(), want)
        pk_w, n_w = oracle.hough_peaks(g, want, W["min_votes"], 1 << 21)
        pk, n = gpu_peaks(torch, ht, g, acc_d, W["min_votes"], min(n_w + 16, 1 << 21))
        assert n == n_w
        assert np.array_equal(pk[:, 0], pk_w["lin"]) and np.array_equal(pk[:, 1], pk_w["votes"])


@pytest.mark.parametrize("gi", range(len(ODD_GRIDS)))
@pytest.mark.parametrize("n_hits", [0, 1, 65, 1000])
def test_cell_vote_parity_odd_grids(torch, ht, oracle, gi, n_hits):
    """Odd phi sizes (37, 1024 with 16-bit LDS counters, 4), straight lines
    (one q/pT bin at 0), a one-plane prompt grid, hits inside |d0| and 5%
    invalid hits."""
    g = ODD_GRIDS[gi]
    print(f"cell odd grid {gi} hits {n_hits}", flush=True)
    r, phi, _ = G.random_hits(n_hits, seed=300 + gi * 7 + n_hits, r_lo=0.5, r_hi=120.0,
                              bad_fraction=0.05)
    acc_d, nv = gpu_cell_vote(torch, ht, g, r, phi)
    want, nv_w = oracle.hough_vote_cell(g, r, phi)
    assert nv == nv_w
    _same(acc_d.cpu().numpy(), want)


def test_cell_vote_max_hits_packed_counters(torch, ht, oracle):
    """65535 identical hits on a 1024-bin phi axis (16-bit LDS counters):
    every bin of the band holds 65535."""
    g = dict(n_phi=1024, n_qpt=8, n_d0=2, qpt_lo=-1.0, qpt_hi=1.0, d0_lo=-2.0, d0_hi=2.0,
             bfield=3.8)
    r = np.full(65535, 50.0, np.float32)
    phi = np.full(65535, 0.25, np.float32)
    acc_d, nv = gpu_cell_vote(torch, ht, g, r, phi)
    want, nv_w = oracle.hough_vote_cell(g, r, phi)
    assert nv == nv_w
    _same(acc_d.cpu().numpy(), want)
    assert want.max() == 65535


def test_cell_vote_rejects_too_many_hits(torch, ht):
    g = CF.GRID_2D
    plan = plan_for(ht, g)
    r = torch.ones(65536, dtype=torch.float32, device="cuda")
    acc = torch.zeros(plan.acc_shape, dtype=torch.int32, device="cuda")
    with pytest.raises(ht.HoughError) as e:
        ht.hough_vote_cell(plan, r, r, acc)
    assert e.value.code == ht.HT_EUNSUPPORTED


def test_cell_vote_then_assoc_parity(torch, ht, oracle):
    """Band accumulator -> peaks -> assoc_cluster on the displaced-jet
    workload, against the oracle given the same peaks."""
    W = CF.WORKLOADS[2]
    g, cl = W["grid"], W["cluster"]
    ev = G.make_event(2, W["seed0"] + 5)
    print(f"cell+assoc hits {ev.n_hits}", flush=True)
    plan = ht.Plan(g, max_peaks=1 << 21, max_member_cap=1024, max_tracks=1 << 15)
    r = torch.from_numpy(ev.r).cuda()
    phi = torch.from_numpy(ev.phi).cuda()
    layer = torch.from_numpy(ev.layer).cuda()
    acc = torch.empty(plan.acc_shape, dtype=torch.int32, device="cuda")
    ht.hough_vote_cell(plan, r, phi, acc)
    cap = 1 << 21
    peaks = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    ht.hough_peaks(plan, acc, W["min_votes"], peaks, nf)
    cfg = dict(cl, member_cap=1024)
    bufs = ht.ClusterBuffers(ev.n_hits, 4096, 512, 1 << 15, cl["n_rho"], cl["n_theta"])
    ht.assoc_cluster(plan, r, phi, layer, peaks, nf, cfg, bufs)
    torch.cuda.synchronize()
    got = bufs.to_host(ev.n_hits)
    pk = peaks[:int(nf.item())].cpu().numpy()
    want = run_oracle(oracle, g, ev, None, pk, cfg)
    compare(got, want, "cell vote + assoc")
    plan.close()
