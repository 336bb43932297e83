"""hough_batch (vote, peaks and assoc_cluster for several events, each
kernel launched once for all of them) against the same calls made event by
event: every output bit-exact, on 2D and 3D grids, events of different sizes
in one batch, an empty event, and batches of 1 to 4.  The event-by-event
path is itself held to the oracle by the other parity tests."""
import numpy as np
import pytest

from paper_1309_6275_amd import configs as CF
from paper_1309_6275_amd import eventgen as G

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


def _dev_event(torch, ev, n_max):
    def pad(a, dt):
        out = np.zeros(max(n_max, 1), dt)
        out[:a.size] = a
        return torch.from_numpy(out).cuda()
    return dict(r=pad(ev.r, np.float32), phi=pad(ev.phi, np.float32), layer=pad(ev.layer, np.uint8),
                n_dev=torch.tensor([ev.n_hits], dtype=torch.int32, device="cuda"), n=ev.n_hits)


def _buffers(torch, ht, plan, cap, n_max, cl):
    return dict(acc=torch.full(plan.acc_shape, -3, dtype=torch.int32, device="cuda"),
                peaks=torch.full((cap, 2), -3, dtype=torch.int32, device="cuda"),
                nf=torch.zeros(1, dtype=torch.int32, device="cuda"),
                bufs=ht.ClusterBuffers(n_max, 2048, 256, 1 << 14, cl["n_rho"], cl["n_theta"]))


def _host(torch, e, n):
    out = e["bufs"].to_host(n)
    nf = int(e["nf"].item())
    return dict(acc=e["acc"].cpu().numpy(), nf=nf,
                peaks=e["peaks"][:min(nf, e["peaks"].shape[0])].cpu().numpy(), **out)


def _check_batch(torch, ht, W, events, cap):
    g, cl = W["grid"], W["cluster"]
    n_max = max(ev.n_hits for ev in events)
    plans = [ht.Plan(g, max_hits=max(n_max, 1), max_peaks=cap, max_member_cap=cl["member_cap"],
                     max_tracks=2048) for _ in events]
    devs = [_dev_event(torch, ev, n_max) for ev in events]
    # one by one
    want = []
    for plan, d, ev in zip(plans, devs, events):
        b = _buffers(torch, ht, plan, cap, n_max, cl)
        r, phi, layer = d["r"][:ev.n_hits], d["phi"][:ev.n_hits], d["layer"][:ev.n_hits]
        ht.hough_vote(plan, r, phi, b["acc"])
        ht.hough_peaks(plan, b["acc"], W["min_votes"], b["peaks"], b["nf"])
        ht.assoc_cluster(plan, r, phi, layer, b["peaks"], b["nf"], cl, b["bufs"], acc=b["acc"])
        torch.cuda.synchronize()
        want.append(_host(torch, b, ev.n_hits))
    # batched
    bat = []
    for plan, d in zip(plans, devs):
        b = _buffers(torch, ht, plan, cap, n_max, cl)
        bat.append(dict(plan=plan, r=d["r"], phi=d["phi"], layer=d["layer"], n_dev=d["n_dev"], **b))
    ht.hough_batch(bat, n_max, W["min_votes"], cl)
    torch.cuda.synchronize()
    for i, (b, ev) in enumerate(zip(bat, events)):
        got = _host(torch, b, ev.n_hits)
        w = want[i]
        assert np.array_equal(got["acc"], w["acc"]), i
        assert got["nf"] == w["nf"] and np.array_equal(got["peaks"], w["peaks"]), i
        assert np.array_equal(got["counts"], w["counts"]), (i, got["counts"], w["counts"])
        assert np.array_equal(got["hit_owner"], w["hit_owner"]), i
        for key in ("tracks", "objects"):
            assert got[key].tobytes() == w[key].tobytes(), (i, key)
        assert np.array_equal(got["members"], w["members"]), i
        assert np.array_equal(got["vacc"], w["vacc"]), i
    for p in plans:
        p.close()
    return want


def test_batch_2d_events_of_different_sizes(torch, ht):
    W = CF.WORKLOADS[1]
    print("batch: 4 workload-1 events of 250 to 4000 hits", flush=True)
    events = [G.make_event(1, W["seed0"] + 500),
              G.make_event(1, W["seed0"] + 501, n_prompt=200, n_noise=500),
              G.make_event(1, W["seed0"] + 502, n_prompt=60),
              G.make_event(1, W["seed0"] + 503, n_prompt=350, n_noise=800)]
    want = _check_batch(torch, ht, W, events, 1 << 16)
    assert all(int(w["counts"][1]) > 0 for w in want)


@pytest.mark.parametrize("nb", [1, 2, 3])
def test_batch_3d_events(torch, ht, nb):
    W = CF.WORKLOADS[2]
    print(f"batch: {nb} workload-2 events", flush=True)
    events = [G.make_event(2, W["seed0"] + 600 + e) for e in range(nb)]
    _check_batch(torch, ht, W, events, 1 << 19)


def test_batch_with_an_empty_event(torch, ht):
    from types import SimpleNamespace
    W = CF.WORKLOADS[1]
    empty = SimpleNamespace(r=np.zeros(0, np.float32), phi=np.zeros(0, np.float32),
                            layer=np.zeros(0, np.uint8), n_hits=0)
    print("batch: workload-1 events with an empty one", flush=True)
    events = [G.make_event(1, W["seed0"] + 700), empty, G.make_event(1, W["seed0"] + 701)]
    want = _check_batch(torch, ht, W, events, 1 << 16)
    assert int(want[1]["counts"][0]) == 0 and want[1]["nf"] == 0
