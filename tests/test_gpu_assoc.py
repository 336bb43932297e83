"""GPU parity of assoc_cluster (refinement, ownership, refit, vertex
transform) against the CPU oracle through the C-ABI.

Integer results (counts, ownership, track hits, vertex accumulator, objects,
members) and float results computed by copying or by fixed-order float64
arithmetic (r_first, seed sums, isotropy) must be bit-exact; the refit uses
the device asin/atan2 and must agree within 1e-5 relative."""
from types import SimpleNamespace

import numpy as np
import pytest

from paper_1309_6275_amd import configs as CF
from paper_1309_6275_amd import eventgen as G

pytestmark = pytest.mark.gpu

EXACT_TRACK = ("peak", "lin", "votes", "n_layers", "n_inliers", "n_owned", "seed_ss", "r_first",
               "hits")
EXACT_OBJECT = ("lin", "votes", "n_tracks", "kind", "rho", "theta", "member_begin", "isotropy")


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


_plans = {}


def plan_for(ht, grid, member_cap=1024):
    key = tuple(sorted(grid.items()))
    if key not in _plans:
        _plans[key] = ht.Plan(grid, max_peaks=1 << 20, max_member_cap=member_cap,
                              max_tracks=1 << 15)
    return _plans[key]


def run_gpu(torch, ht, grid, ev, min_votes, cfg, peak_cap=None, track_cap=4096,
            object_cap=512, member_cap=1 << 15, with_vacc=True, use_acc=True, peak_stride=1):
    """Vote, peaks and assoc_cluster on the device; assoc_cluster gets the
    accumulator (member-count bound) unless use_acc is False.  peak_stride > 1
    hands assoc_cluster every peak_stride-th peak of the full list (still in
    cell order) instead of the first peak_cap."""
    plan = plan_for(ht, grid)
    r = torch.from_numpy(ev.r).cuda()
    phi = torch.from_numpy(ev.phi).cuda()
    layer = torch.from_numpy(ev.layer).cuda()
    acc = torch.empty(plan.acc_shape, dtype=torch.int32, device="cuda")
    ht.hough_vote(plan, r, phi, acc)
    cap = peak_cap if peak_cap is not None else (1 << 20)
    peaks = torch.full((max(cap, 1), 2), -1, dtype=torch.int32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    ht.hough_peaks(plan, acc, min_votes, peaks[:cap], nf)
    if peak_stride > 1:
        torch.cuda.synchronize()
        n_all = int(nf.item())
        assert n_all <= cap
        sub = peaks[:n_all:peak_stride].contiguous()
        cap = int(sub.shape[0])
        peaks = torch.full((max(cap, 1), 2), -1, dtype=torch.int32, device="cuda")
        peaks[:cap] = sub
        nf = torch.tensor([cap], dtype=torch.int32, device="cuda")
    bufs = ht.ClusterBuffers(max(ev.n_hits, 1), track_cap, object_cap, member_cap,
                             cfg["n_rho"], cfg["n_theta"])
    ht.assoc_cluster(plan, r, phi, layer, peaks[:cap], nf, cfg, bufs, with_vacc=with_vacc,
                     acc=acc if use_acc else None)
    torch.cuda.synchronize()
    got = bufs.to_host(ev.n_hits)
    return got, acc.cpu().numpy(), peaks[:min(int(nf.item()), cap)].cpu().numpy()


def run_oracle(oracle, grid, ev, acc, pk_gpu, cfg, track_cap=4096, object_cap=512,
               member_cap=1 << 15):
    pk = np.zeros(pk_gpu.shape[0], oracle.PEAK_DT)
    pk["lin"] = pk_gpu[:, 0]
    pk["votes"] = pk_gpu[:, 1]
    return oracle.assoc_cluster(grid, ev.r, ev.phi, ev.layer, pk, cfg, track_cap=track_cap,
                                object_cap=object_cap, member_cap=member_cap)


def compare(got, want, label=""):
    assert np.array_equal(got["counts"][:7], want["counts"][:7]), (label, got["counts"],
                                                                   want["counts"])
    assert np.array_equal(got["hit_owner"], want["hit_owner"]), label
    gt, wt = got["tracks"], want["tracks"]
    assert gt.shape == wt.shape, label
    for f in EXACT_TRACK:
        assert np.array_equal(gt[f], wt[f]), (label, f)
    assert np.array_equal(gt["status"], wt["status"]), label
    ok = wt["status"] == 0
    for f, floor in (("phi0", 1e-6), ("qpt", 1e-6), ("d0", 1e-5)):
        a, b = gt[f][ok].astype(np.float64), wt[f][ok].astype(np.float64)
        assert np.all(np.abs(a - b) <= 1e-5 * np.abs(b) + floor), (label, f)
    a, b = gt["chi2"][ok].astype(np.float64), wt["chi2"][ok].astype(np.float64)
    assert np.all(np.abs(a - b) <= 1e-4 * np.abs(b) + 1e-3), (label, "chi2")
    assert np.array_equal(got["vacc"], want["vacc"]), label
    go, wo = got["objects"], want["objects"]
    assert go.shape == wo.shape, label
    for f in EXACT_OBJECT:
        assert np.array_equal(go[f], wo[f]), (label, f)
    assert np.array_equal(got["members"], want["members"]), label


@pytest.mark.parametrize("cfgid,seeds", [(1, range(8)), (2, range(4))])
def test_assoc_parity_workloads(torch, ht, oracle, cfgid, seeds):
    W = CF.WORKLOADS[cfgid]
    for s in seeds:
        seed = W["seed0"] + s
        print(f"cfg{cfgid} seed {seed}", flush=True)
        ev = G.make_event(cfgid, seed)
        got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], W["cluster"])
        want = run_oracle(oracle, W["grid"], ev, acc, pk, W["cluster"])
        compare(got, want, f"cfg{cfgid}/{seed}")


def test_assoc_parity_dense_event_strided_peaks(torch, ht, oracle):
    """The 55k-hit workload with every 64th peak of its list (cell order, so
    the subset spans every d0 plane)."""
    W = CF.WORKLOADS[3]
    ev = G.make_event(3, W["seed0"])
    print(f"cfg3 hits {ev.n_hits}, every 64th peak", flush=True)
    got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], W["cluster"],
                           peak_stride=64)
    g = W["grid"]
    planes = np.unique(pk[:, 0] // (g["n_phi"] * g["n_qpt"]))
    assert planes.size == g["n_d0"], planes.size
    want = run_oracle(oracle, W["grid"], ev, acc, pk, W["cluster"])
    compare(got, want, "cfg3/stride 64")


def test_assoc_parity_dense_event_full_list(torch, ht, oracle):
    """The 55k-hit workload with its whole peak list (about 2.3e5 candidates;
    the oracle takes about half a minute on 16 cores)."""
    W = CF.WORKLOADS[3]
    ev = G.make_event(3, W["seed0"] + 2)
    print(f"cfg3 hits {ev.n_hits}, full peak list", flush=True)
    got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], W["cluster"],
                           track_cap=1 << 14, object_cap=1024)
    print(f"peaks {pk.shape[0]}, tracks {int(got['counts'][1])}", flush=True)
    assert pk.shape[0] > 100000
    want = run_oracle(oracle, W["grid"], ev, acc, pk, W["cluster"], track_cap=1 << 14,
                      object_cap=1024)
    compare(got, want, "cfg3/full")


def test_assoc_parity_many_peaks_per_workgroup(torch, ht, oracle):
    """Over 4096 peaks among one workgroup's 64 columns: the member sweep
    keeps the candidates' slot counters in global memory instead of LDS."""
    grid = dict(CF.GRID_2D, n_phi=1024, n_qpt=64)
    r, phi, layer = G.random_hits(3000, seed=41, r_lo=3.0, r_hi=105.0, bad_fraction=0.02)
    ev = SimpleNamespace(r=r, phi=phi, layer=layer, n_hits=int(r.size))
    cfg = dict(CF.CLUSTER_2D, min_layers=4, member_cap=1024)
    got, acc, pk = run_gpu(torch, ht, grid, ev, 1, cfg)
    print(f"peaks {pk.shape[0]}", flush=True)
    assert pk.shape[0] > 4096
    want = run_oracle(oracle, grid, ev, acc, pk, cfg)
    compare(got, want, "many peaks")


@pytest.mark.parametrize("kw", [dict(n_prompt=0, n_jets=1, jet_ntrk=10),
                                dict(n_prompt=0, n_jets=4, jet_ntrk=10),
                                dict(n_prompt=600, n_jets=2, jet_ntrk=10)])
def test_assoc_parity_paper_geometry(torch, ht, oracle, kw):
    """The paper's toy detector (layers every 11 cm to 110 cm, 0.4 mm in x
    and y, vertex grid from the 3.0 cm pipe)."""
    W = CF.PAPER_WORKLOAD
    ev = G.make_paper_event(W["seed0"] + 7 + kw["n_prompt"] + kw["n_jets"], **kw)
    print(f"paper {kw} hits {ev.n_hits}", flush=True)
    got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], W["cluster"])
    want = run_oracle(oracle, W["grid"], ev, acc, pk, W["cluster"])
    compare(got, want, f"paper {kw}")


@pytest.mark.parametrize("case", ["cfg1", "cfg2", "paper"])
def test_assoc_parity_kalman_refit(torch, ht, oracle, case):
    """fit_kind 1: the Kalman-filter refit instead of Gauss-Newton (2D grid
    with d0 fixed, 3D grid, the paper's geometry)."""
    if case == "paper":
        W = CF.PAPER_WORKLOAD
        ev = G.make_paper_event(W["seed0"] + 21, n_prompt=300, n_jets=3)
    else:
        cid = int(case[-1])
        W = CF.WORKLOADS[cid]
        ev = G.make_event(cid, W["seed0"] + 21)
    cfg = dict(W["cluster"], fit_kind=1, fit_iters=3)
    print(f"kalman {case} hits {ev.n_hits}", flush=True)
    got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], cfg)
    want = run_oracle(oracle, W["grid"], ev, acc, pk, cfg)
    compare(got, want, f"kalman {case}")
    assert (want["tracks"]["status"] == 0).mean() > 0.9


@pytest.mark.parametrize("kind", ["jet", "bh"])
def test_assoc_parity_vertex_events(torch, ht, oracle, kind):
    W = CF.WORKLOADS[2]
    rng = np.random.default_rng(31 if kind == "jet" else 32)
    if kind == "jet":
        rho, theta = 12.3, 2.1
        psis = theta + rng.uniform(-0.5, 0.5, 12)
        qpts = rng.choice([-1, 1], 12) * rng.uniform(0.2, 0.9, 12)
    else:
        rho, theta = 7.0, -0.4
        psis = theta + rng.uniform(-1.45, 1.45, 60)
        qpts = rng.choice([-1, 1], 60) * rng.uniform(0.3, 0.9, 60)
    ev = G.make_vertex_event(rho, theta, psis, qpts, n_noise=300, seed=5)
    cfg = dict(W["cluster"], member_cap=512)
    got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], cfg)
    want = run_oracle(oracle, W["grid"], ev, acc, pk, cfg)
    compare(got, want, kind)
    assert want["counts"][2] >= 1


@pytest.mark.parametrize("n_rho,n_theta", [(9, 150), (3, 101), (40, 333)])
def test_assoc_parity_vertex_grid_tiles(torch, ht, oracle, n_rho, n_theta):
    """Vertex grids that do not fill whole 1024-cell tiles (the vertex peaks
    are counted and placed per tile): one partial tile, two tiles with a
    ragged tail, and thirteen tiles on an odd theta axis."""
    W = CF.WORKLOADS[2]
    rng = np.random.default_rng(33)
    psis = -0.4 + rng.uniform(-1.45, 1.45, 60)
    qpts = rng.choice([-1, 1], 60) * rng.uniform(0.3, 0.9, 60)
    ev = G.make_vertex_event(7.0, -0.4, psis, qpts, n_noise=300, seed=6)
    cfg = dict(W["cluster"], member_cap=512, n_rho=n_rho, n_theta=n_theta)
    got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], cfg)
    want = run_oracle(oracle, W["grid"], ev, acc, pk, cfg)
    compare(got, want, f"vertex grid {n_rho}x{n_theta}")
    assert want["counts"][2] >= 1


def test_assoc_capacities_and_overflow(torch, ht, oracle):
    """Small track/object/member capacities truncate in order with full
    counts; a small member_cap drops candidates identically."""
    W = CF.WORKLOADS[2]
    ev = G.make_event(2, W["seed0"] + 9)
    for cfg, tc, oc, mc in ((W["cluster"], 7, 1, 3),
                            (dict(W["cluster"], member_cap=40), 4096, 512, 1 << 15),
                            (dict(W["cluster"], seed_k=2, win_bins=0), 4096, 512, 1 << 15)):
        got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], cfg, track_cap=tc,
                               object_cap=oc, member_cap=mc)
        want = run_oracle(oracle, W["grid"], ev, acc, pk, cfg, track_cap=tc, object_cap=oc,
                          member_cap=mc)
        compare(got, want, f"caps {tc}/{oc}/{mc}/{cfg['member_cap']}")


def test_assoc_empty_inputs(torch, ht):
    W = CF.WORKLOADS[1]
    ev = G.make_tracks_event([], n_noise=0)
    got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], W["cluster"])
    assert got["counts"][:5].tolist() == [0, 0, 0, 0, 0]
    ev = G.make_tracks_event([], n_noise=40, seed=3)
    got, acc, pk = run_gpu(torch, ht, W["grid"], ev, 1, W["cluster"])
    assert got["counts"][1] == 0 and (got["hit_owner"] == -1).all()


def test_assoc_deterministic(torch, ht):
    W = CF.WORKLOADS[2]
    ev = G.make_event(2, W["seed0"] + 4)
    a, _, _ = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], W["cluster"])
    b, _, _ = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], W["cluster"])
    for k in ("hit_owner", "tracks", "objects", "members", "vacc", "counts"):
        assert a[k].tobytes() == b[k].tobytes(), k


def test_assoc_rejects_bad_config(torch, ht):
    W = CF.WORKLOADS[1]
    plan = plan_for(ht, W["grid"])
    ev = G.make_event(1, W["seed0"])
    r = torch.from_numpy(ev.r).cuda()
    layer = torch.from_numpy(ev.layer).cuda()
    peaks = torch.zeros((4, 2), dtype=torch.int32, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    bufs = ht.ClusterBuffers(ev.n_hits, 16, 4, 16, 64, 256)
    for bad, code in ((dict(min_layers=2), ht.HT_EINVAL), (dict(seed_k=5), ht.HT_EUNSUPPORTED),
                      (dict(member_cap=4096), ht.HT_EUNSUPPORTED),
                      (dict(rho_lo=-1.0), ht.HT_EINVAL), (dict(fit_kind=2), ht.HT_EINVAL),
                      (dict(vtx_min_d0=-0.1), ht.HT_EINVAL)):
        with pytest.raises(ht.HoughError) as e:
            ht.assoc_cluster(plan, r, r, layer, peaks, nf, dict(W["cluster"], **bad), bufs)
        assert e.value.code == code, bad


@pytest.mark.parametrize("case", ["isotropic", "cfg2", "cfg3"])
def test_assoc_parity_two_branch_vertex_vote(torch, ht, oracle, case):
    """vtx_two_branch = 1: the vertex vote also runs along each track's
    incoming branch (an isotropic decay 10 cm out with noise; a workload-2
    event; every 64th peak of a 55k-hit event)."""
    if case == "isotropic":
        W = CF.WORKLOADS[2]
        rng = np.random.default_rng(31)
        psis = np.sort(-1.1 + rng.uniform(-np.pi, np.pi, 60))
        qpts = rng.choice([-1, 1], 60) * rng.uniform(0.3, 0.9, 60)
        ev = G.make_vertex_event(10.0, -1.1, psis, qpts, n_noise=300, seed=32)
        kw = {}
    elif case == "cfg2":
        W = CF.WORKLOADS[2]
        ev = G.make_event(2, W["seed0"] + 11)
        kw = {}
    else:
        W = CF.WORKLOADS[3]
        ev = G.make_event(3, W["seed0"] + 3)
        kw = dict(peak_stride=64)
    cfg = dict(W["cluster"], vtx_two_branch=1)
    print(f"two-branch {case}: hits {ev.n_hits}", flush=True)
    got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], cfg, **kw)
    want = run_oracle(oracle, W["grid"], ev, acc, pk, cfg)
    compare(got, want, f"two-branch {case}")
    if case == "isotropic":
        obj = want["objects"]
        assert obj.size and obj["kind"].max() == 1


@pytest.mark.parametrize("mixed", [False, True])
def test_assoc_parity_angle_bins(torch, ht, oracle, mixed):
    """Above member_cap 128 the seed search groups each layer's members by
    azimuth bins; when all members of a layer share one radius, a seed
    circle is tested only against the bins its road can reach.  Workload-2
    events at member_cap 256 (every layer on the binned path), and the same
    events with the radii of half of one layer's hits moved by one float32
    step (that layer is scanned whole, the others binned)."""
    W = CF.WORKLOADS[2]
    cfg = dict(W["cluster"], member_cap=256)
    for s in range(2):
        ev = G.make_event(2, W["seed0"] + 50 + s)
        if mixed:
            r = ev.r.copy()
            sel = np.flatnonzero(ev.layer == 4)[::2]
            r[sel] = np.nextafter(r[sel], np.float32(200.0))
            ev = SimpleNamespace(r=r, phi=ev.phi, layer=ev.layer, n_hits=ev.n_hits)
        print(f"angle bins: seed {W['seed0'] + 50 + s}, mixed radii {mixed}", flush=True)
        got, acc, pk = run_gpu(torch, ht, W["grid"], ev, W["min_votes"], cfg)
        want = run_oracle(oracle, W["grid"], ev, acc, pk, cfg)
        compare(got, want, f"angle bins {s} mixed {mixed}")
        assert int(got["counts"][1]) > 100


@pytest.mark.parametrize("extra_radii", [6, 7])
def test_assoc_parity_member_lists_both_paths(torch, ht, oracle, extra_radii):
    """Member lists are built by candidate (hits bucketed by radius and
    azimuth) when the member-eligible hits have at most 16 distinct radii,
    else by the sweep over (hit, column) pairs.  A workload-2 event (10
    radii) plus one hit on each of 6 new radii takes the first path, plus 7
    the second; both equal the oracle."""
    W = CF.WORKLOADS[2]
    ev = G.make_event(2, W["seed0"] + 90)
    rng = np.random.default_rng(90)
    new_r = np.float32(rng.uniform(12.0, 100.0, extra_radii))
    r = np.concatenate([ev.r, new_r]).astype(np.float32)
    phi = np.concatenate([ev.phi, rng.uniform(-np.pi, np.pi, extra_radii)]).astype(np.float32)
    layer = np.concatenate([ev.layer, rng.integers(0, 10, extra_radii)]).astype(np.uint8)
    ev2 = SimpleNamespace(r=r, phi=phi, layer=layer, n_hits=int(r.size))
    assert np.unique(r).size == 10 + extra_radii
    print(f"member lists: {10 + extra_radii} radii", flush=True)
    got, acc, pk = run_gpu(torch, ht, W["grid"], ev2, W["min_votes"], W["cluster"])
    want = run_oracle(oracle, W["grid"], ev2, acc, pk, W["cluster"])
    compare(got, want, f"{10 + extra_radii} radii")
    assert int(got["counts"][1]) > 100


@pytest.mark.parametrize("case", ["phi_beyond_pi", "odd_grid_2d", "odd_grid_3d"])
def test_assoc_parity_member_lists_edges(torch, ht, oracle, case):
    """Member lists by candidate on inputs that stress the azimuth buckets:
    azimuths outside [-pi, pi) (valid hits reach |phi| <= 4; the buckets use
    the wrapped azimuth, the member test the raw one), and grids whose phi0
    axis is not a power of two."""
    if case == "phi_beyond_pi":
        W = CF.WORKLOADS[2]
        grid, cfg = W["grid"], W["cluster"]
        ev = G.make_event(2, W["seed0"] + 91)
        phi = ev.phi.astype(np.float64)
        phi = np.where(phi > np.pi - 0.85, phi - 2 * np.pi, phi)
        phi = np.where(phi < -np.pi + 0.85, phi + 2 * np.pi, phi)
        ev = SimpleNamespace(r=ev.r, phi=phi.astype(np.float32), layer=ev.layer, n_hits=ev.n_hits)
        assert np.abs(ev.phi).max() > np.pi and np.abs(ev.phi).max() <= 4.0
        min_votes = W["min_votes"]
    elif case == "odd_grid_2d":
        W = CF.WORKLOADS[1]
        grid = dict(W["grid"], n_phi=250, n_qpt=200)
        cfg = W["cluster"]
        ev = G.make_event(1, W["seed0"] + 91, n_prompt=80, n_noise=200)
        min_votes = W["min_votes"]
    else:
        W = CF.WORKLOADS[2]
        grid = dict(W["grid"], n_phi=500, n_qpt=120, n_d0=24)
        cfg = dict(W["cluster"], member_cap=256)
        ev = G.make_event(2, W["seed0"] + 91)
        min_votes = W["min_votes"]
    print(f"member list edges: {case}", flush=True)
    got, acc, pk = run_gpu(torch, ht, grid, ev, min_votes, cfg)
    want = run_oracle(oracle, grid, ev, acc, pk, cfg)
    compare(got, want, case)
    assert int(got["counts"][1]) > 10
