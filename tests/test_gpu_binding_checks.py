"""The binding's size checks: buffers too small for the call raise ValueError
before anything is launched (the C ABI sees pointers only, so these checks
are the only guard against out-of-bounds device writes)."""
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_1309_6275_amd import configs as CF
    from paper_1309_6275_amd import houghtrig as H
    W = CF.WORKLOADS[2]
    plan = H.Plan(W["grid"], max_hits=1024, max_peaks=1 << 12, max_member_cap=128,
                  max_tracks=256)
    n = 100
    r = torch.full((n,), 30.0, device="cuda")
    phi = torch.zeros(n, device="cuda")
    layer = torch.zeros(n, dtype=torch.uint8, device="cuda")
    peaks = torch.zeros((16, 2), dtype=torch.int32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    yield H, W, plan, r, phi, layer, peaks, nf
    plan.close()


def test_assoc_cluster_rejects_small_buffers(setup):
    H, W, plan, r, phi, layer, peaks, nf = setup
    cl = W["cluster"]
    small_owner = H.ClusterBuffers(50, 64, 16, 64, cl["n_rho"], cl["n_theta"])
    with pytest.raises(ValueError, match="hit_owner"):
        H.assoc_cluster(plan, r, phi, layer, peaks, nf, cl, small_owner)
    small_vacc = H.ClusterBuffers(100, 64, 16, 64, 8, 8)
    with pytest.raises(ValueError, match="vacc"):
        H.assoc_cluster(plan, r, phi, layer, peaks, nf, cl, small_vacc)
    # without the vertex accumulator the small vacc is never written
    H.assoc_cluster(plan, r, phi, layer, peaks, nf, cl, small_vacc, with_vacc=False)
    ok = H.ClusterBuffers(100, 64, 16, 64, cl["n_rho"], cl["n_theta"])
    with pytest.raises(ValueError, match="peaks"):
        H.assoc_cluster(plan, r, phi, layer, peaks.reshape(-1), nf, cl, ok)
    with pytest.raises(ValueError, match="peaks"):
        H.assoc_cluster(plan, r, phi, layer, torch.zeros((16, 3), dtype=torch.int32,
                                                         device="cuda"), nf, cl, ok)
    with pytest.raises(ValueError, match="n_peaks"):
        H.assoc_cluster(plan, r, phi, layer, peaks, nf[:0], cl, ok)
    with pytest.raises(ValueError, match="hit_owner"):
        H.assoc_cluster_n(plan, r, phi, layer, torch.tensor([100], dtype=torch.int32,
                                                            device="cuda"),
                          peaks, nf, cl, small_owner)
    torch.cuda.synchronize()


def test_peaks_and_vote_reject_small_counts(setup):
    H, W, plan, r, phi, layer, peaks, nf = setup
    acc = torch.empty(plan.acc_shape, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError, match="n_found"):
        H.hough_peaks(plan, acc, 7, peaks, nf[:0])
    with pytest.raises(ValueError, match="n_votes"):
        H.hough_vote(plan, r, phi, acc, torch.zeros(0, dtype=torch.int64, device="cuda"))


def test_cnn_calls_reject_small_buffers(setup):
    H, W, plan, r, phi, layer, peaks, nf = setup
    win = torch.zeros((32, H.CNN_WINDOW), dtype=torch.bfloat16, device="cuda")
    params = torch.zeros(H.CNN_PARAMS, dtype=torch.float32, device="cuda")
    ws = H.cnn_workspace(32)
    with pytest.raises(ValueError, match="logits"):
        H.cnn_forward(params, win, torch.zeros(31, device="cuda"), ws)
    with pytest.raises(ValueError, match="win"):
        H.cnn_forward(params, torch.zeros((32, 64), dtype=torch.bfloat16, device="cuda"),
                      torch.zeros(32, device="cuda"), ws)
    with pytest.raises(ValueError, match="params"):
        H.cnn_forward(params[:100], win, torch.zeros(32, device="cuda"), ws)
    out = torch.zeros((16, 2), dtype=torch.int32, device="cuda")
    n_out = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError, match="logits"):
        H.cnn_keep(plan, torch.zeros(8, device="cuda"), peaks, nf, 0.0, out, n_out)
    torch.cuda.synchronize()
