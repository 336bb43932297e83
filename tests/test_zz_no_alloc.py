"""hough_peaks_noalloc (the entry point for callers that cannot allocate)
against hough_peaks with a plan: two calls in a row on the same GPU, the
second on a smaller grid, bit-exact peak lists and counts; the size limit is
refused on the host."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _peaks_both(H, grid, acc, min_votes, cap):
    plan = H.Plan(grid, max_hits=16, max_peaks=16, max_member_cap=8, max_tracks=16)
    try:
        out_p = torch.full((cap, 2), -7, dtype=torch.int32, device="cuda")
        nf_p = torch.zeros(1, dtype=torch.int32, device="cuda")
        H.hough_peaks(plan, acc, min_votes, out_p, nf_p)
        out_s = torch.full((cap, 2), -7, dtype=torch.int32, device="cuda")
        nf_s = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        H.hough_peaks_noalloc(grid, acc, min_votes, out_s, nf_s)
        torch.cuda.synchronize()
    finally:
        plan.close()
    return out_p.cpu().numpy(), int(nf_p.item()), out_s.cpu().numpy(), int(nf_s.item())


def test_noalloc_matches_plan_path_twice_second_smaller():
    from paper_1309_6275_amd import configs as CF
    from paper_1309_6275_amd import eventgen as G
    from paper_1309_6275_amd import houghtrig as H
    print("noalloc: workload 2 event, then workload 1 event", flush=True)
    cases = [(CF.WORKLOADS[2], G.make_event(2, 2_000_321), 1 << 19),
             (CF.WORKLOADS[1], G.make_event(1, 1_000_321), 1 << 12)]
    for W, ev, cap in cases:
        g = W["grid"]
        plan = H.Plan(g, max_hits=65535, max_peaks=16, max_member_cap=8, max_tracks=16)
        acc = torch.empty(plan.acc_shape, dtype=torch.int32, device="cuda")
        H.hough_vote(plan, torch.from_numpy(ev.r).cuda(), torch.from_numpy(ev.phi).cuda(), acc)
        torch.cuda.synchronize()
        plan.close()
        want, n_want, got, n_got = _peaks_both(H, g, acc, W["min_votes"], cap)
        assert n_got == n_want and n_want > 0
        k = min(n_want, cap)
        assert np.array_equal(got[:k], want[:k])
        assert (got[k:] == -7).all()


def test_noalloc_truncation_and_odd_grid():
    from paper_1309_6275_amd import houghtrig as H
    print("noalloc: truncated list, odd grid (one-cell lanes)", flush=True)
    rng = np.random.default_rng(11)
    for grid, cap in [(dict(n_phi=512, n_qpt=256, n_d0=64, qpt_lo=-1.0, qpt_hi=1.0, d0_lo=-20.0,
                            d0_hi=20.0, bfield=3.8), 1000),
                      (dict(n_phi=37, n_qpt=65, n_d0=3, qpt_lo=-1.0, qpt_hi=1.0, d0_lo=-2.0,
                            d0_hi=2.0, bfield=3.8), 50000)]:
        shape = (grid["n_d0"], grid["n_qpt"], grid["n_phi"])
        acc = torch.from_numpy(rng.integers(0, 12, size=shape).astype(np.int32)).cuda()
        want, n_want, got, n_got = _peaks_both(H, grid, acc, 7, cap)
        assert n_got == n_want
        k = min(n_want, cap)
        assert np.array_equal(got[:k], want[:k])


def test_noalloc_refuses_oversize_grid_on_host():
    from paper_1309_6275_amd import houghtrig as H
    big = dict(n_phi=1024, n_qpt=256, n_d0=128, qpt_lo=-1.0, qpt_hi=1.0, d0_lo=-20.0, d0_hi=20.0,
               bfield=3.8)
    acc = torch.zeros((128, 256, 1024), dtype=torch.int32, device="cuda")
    out = torch.zeros((4, 2), dtype=torch.int32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(H.HoughError) as e:
        H.hough_peaks_noalloc(big, acc, 7, out, nf)
    assert e.value.code == H.HT_EUNSUPPORTED
