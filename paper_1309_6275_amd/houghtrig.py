"""Thin ctypes binding of libhoughtrig.so (the gfx950 Hough trigger library).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Tensors must be contiguous device tensors of the stated dtype; the
calls are asynchronous on the current torch stream.  There is no fallback:
if the library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhoughtrig.so")
MAX_LAYERS = 16

HT_OK, HT_EINVAL, HT_ENOMEM, HT_EDEVICE, HT_EUNSUPPORTED = 0, -1, -2, -3, -4

PEAK_DTYPE = np.dtype([("lin", "<i4"), ("votes", "<i4")])
TRACK_DTYPE = np.dtype([
    ("peak", "<i4"), ("lin", "<i4"), ("votes", "<i4"), ("n_layers", "<i4"),
    ("n_inliers", "<i4"), ("n_owned", "<i4"), ("status", "<i4"), ("seed_ss", "<f4"),
    ("phi0", "<f4"), ("qpt", "<f4"), ("d0", "<f4"), ("chi2", "<f4"), ("r_first", "<f4"),
    ("hits", "<i4", (MAX_LAYERS,)),
])
OBJECT_DTYPE = np.dtype([
    ("lin", "<i4"), ("votes", "<i4"), ("n_tracks", "<i4"), ("kind", "<i4"),
    ("rho", "<f4"), ("theta", "<f4"), ("isotropy", "<f4"), ("member_begin", "<i4"),
])


class HoughError(RuntimeError):
    def __init__(self, what, code):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("n_phi", C.c_int32), ("n_qpt", C.c_int32), ("n_d0", C.c_int32),
                ("qpt_lo", C.c_float), ("qpt_hi", C.c_float),
                ("d0_lo", C.c_float), ("d0_hi", C.c_float), ("bfield", C.c_float)]


class Limits(C.Structure):
    _fields_ = [("max_hits", C.c_int32), ("max_peaks", C.c_int32),
                ("max_member_cap", C.c_int32), ("max_tracks", C.c_int32),
                ("max_vertex_cells", C.c_int32), ("max_n_rho", C.c_int32)]


class ClusterCfg(C.Structure):
    _fields_ = [("win_bins", C.c_int32), ("min_layers", C.c_int32), ("seed_k", C.c_int32),
                ("member_cap", C.c_int32), ("road_sigmas", C.c_float),
                ("box_margin", C.c_float), ("sigma_rphi", C.c_float),
                ("fit_iters", C.c_int32), ("n_rho", C.c_int32), ("n_theta", C.c_int32),
                ("rho_lo", C.c_float), ("rho_hi", C.c_float),
                ("vtx_min_votes", C.c_int32), ("bh_min_tracks", C.c_int32),
                ("bh_max_isotropy", C.c_float), ("vtx_min_d0", C.c_float),
                ("fit_kind", C.c_int32), ("vtx_two_branch", C.c_int32)]


class ClusterOut(C.Structure):
    _fields_ = [("hit_owner", C.c_void_p), ("tracks", C.c_void_p), ("track_cap", C.c_int32),
                ("objects", C.c_void_p), ("object_cap", C.c_int32),
                ("members", C.c_void_p), ("member_cap", C.c_int32),
                ("vacc", C.c_void_p), ("counts", C.c_void_p), ("work", C.c_void_p)]


class BatchEvent(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("r", C.c_void_p), ("phi", C.c_void_p),
                ("layer", C.c_void_p), ("n_hits_dev", C.c_void_p), ("acc", C.c_void_p),
                ("peaks", C.c_void_p), ("n_peaks", C.c_void_p), ("out", ClusterOut)]


MAX_BATCH = 4
SERVER_MAX_KINDS = 4
HT_EBUSY = -5


class ServerKind(C.Structure):
    _fields_ = [("grid", Grid), ("cluster", ClusterCfg), ("min_votes", C.c_int32),
                ("peak_cap", C.c_int32), ("cnn_params", C.c_void_p), ("cnn_threshold", C.c_float),
                ("reserved", C.c_int32)]


class ServerCfg(C.Structure):
    _fields_ = [("n_kinds", C.c_int32), ("kinds", ServerKind * SERVER_MAX_KINDS),
                ("max_hits", C.c_int32), ("track_cap", C.c_int32), ("object_cap", C.c_int32),
                ("member_cap", C.c_int32), ("hbm_budget", C.c_int64), ("max_slots", C.c_int32),
                ("queue_cap", C.c_int32), ("use_graphs", C.c_int32), ("reserved", C.c_int32),
                ("work_budget", C.c_int64), ("batch_max", C.c_int32),
                ("batch_max_hits", C.c_int32)]


class ServerOut(C.Structure):
    _fields_ = [("tracks", C.c_void_p), ("track_cap", C.c_int32), ("hit_owner", C.c_void_p),
                ("objects", C.c_void_p), ("object_cap", C.c_int32), ("members", C.c_void_p),
                ("member_cap", C.c_int32)]


class ServerResult(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("kind", C.c_int32), ("n_hits", C.c_int32),
                ("status", C.c_int32), ("n_peaks", C.c_int32), ("counts", C.c_int32 * 8),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("device_ms", C.c_double), ("n_kept", C.c_int32), ("batch", C.c_int32)]


_lib = None


def lib():
    """Load libhoughtrig.so (built by ``paper_1309_6275_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1309_6275_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.ht_strerror.argtypes = [C.c_int]
        L.ht_strerror.restype = C.c_char_p
        L.ht_plan_create.argtypes = [vp, vp, vp]
        L.ht_plan_destroy.argtypes = [vp]
        L.ht_plan_destroy.restype = None
        L.hough_vote.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.hough_vote_cell.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.hough_vote_n.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
        L.assoc_cluster_n.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, i32, vp, vp, vp, vp]
        L.hough_peaks.argtypes = [vp, vp, i32, vp, i32, vp, vp]
        L.hough_peaks_noalloc.argtypes = [vp, vp, i32, vp, i32, vp, vp]
        L.assoc_cluster.argtypes = [vp, vp, vp, vp, i32, vp, vp, i32, vp, vp, vp, vp]
        L.ht_asin_f32.argtypes = [vp, vp, i64, vp]
        L.ht_compact_hits.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.ht_remap_track_hits.argtypes = [vp, i32, vp, vp, i32, vp]
        L.ht_sqrt_f64.argtypes = [vp, vp, i64, vp]
        L.ht_cnn_workspace_bytes.argtypes = [i32, i32]
        L.ht_cnn_workspace_bytes.restype = C.c_size_t
        L.ht_cnn_windows.argtypes = [vp, vp, vp, vp, i32, vp, vp]
        L.ht_cnn_forward.argtypes = [vp, vp, vp, i32, vp, vp, C.c_size_t, vp]
        L.ht_cnn_train_step.argtypes = [vp, vp, vp, vp, i32, C.c_float, C.c_float, C.c_float, vp,
                                        vp, C.c_size_t, vp]
        L.ht_cnn_keep.argtypes = [vp, vp, vp, vp, i32, C.c_float, vp, i32, vp, vp]
        L.ht_cnn_score.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, C.c_size_t, vp]
        L.hough_batch.argtypes = [i32, vp, i32, i32, i32, vp, vp]
        L.ht_server_create.argtypes = [vp, vp]
        L.ht_server_destroy.argtypes = [vp]
        L.ht_server_info.argtypes = [vp, vp, vp]
        L.ht_server_submit.argtypes = [vp, i32, vp, vp, vp, i32, vp, C.c_uint64]
        L.ht_server_poll.argtypes = [vp, vp, i32, i32, vp]
        L.ht_profile_begin.argtypes = [vp, i32]
        L.ht_profile_read.argtypes = [vp, vp, vp]
        L.ht_profile_end.argtypes = [vp]
        for f in ("ht_plan_create", "hough_vote", "hough_peaks", "assoc_cluster", "ht_asin_f32",
                  "ht_sqrt_f64", "ht_profile_begin", "ht_profile_read", "ht_profile_end",
                  "ht_server_create", "ht_server_destroy", "ht_server_info", "ht_server_submit",
                  "ht_server_poll", "ht_cnn_windows", "ht_cnn_forward", "ht_cnn_train_step",
                  "ht_cnn_keep", "hough_vote_cell", "ht_compact_hits", "ht_remap_track_hits",
                  "hough_vote_n", "assoc_cluster_n", "hough_peaks_noalloc", "ht_cnn_score",
                  "hough_batch"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().ht_strerror(int(code)).decode()
    except Exception:  # library not loadable: still report the code
        return "error"


def _check(rc, what):
    if rc != HT_OK:
        raise HoughError(what, rc)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("houghtrig needs a ROCm GPU; none is available")
    return torch


def _ptr(t, dtype, what):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{what} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous {dtype} tensor")
    return C.c_void_p(t.data_ptr())


def _need(ok, what):
    """Size checks the C ABI cannot make (it sees pointers only): raise before
    anything is launched."""
    if not ok:
        raise ValueError(what)


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def grid_struct(g: dict) -> Grid:
    return Grid(int(g["n_phi"]), int(g["n_qpt"]), int(g["n_d0"]), float(g["qpt_lo"]),
                float(g["qpt_hi"]), float(g["d0_lo"]), float(g["d0_hi"]), float(g["bfield"]))


def cluster_struct(c: dict) -> ClusterCfg:
    return ClusterCfg(int(c["win_bins"]), int(c["min_layers"]), int(c["seed_k"]),
                      int(c["member_cap"]), float(c["road_sigmas"]), float(c["box_margin"]),
                      float(c["sigma_rphi"]), int(c["fit_iters"]), int(c["n_rho"]),
                      int(c["n_theta"]), float(c["rho_lo"]), float(c["rho_hi"]),
                      int(c["vtx_min_votes"]), int(c["bh_min_tracks"]),
                      float(c["bh_max_isotropy"]),
                      float(c.get("vtx_min_d0", 0.0)), int(c.get("fit_kind", 0)),
                      int(c.get("vtx_two_branch", 0)))


class Plan:
    """Owns an ht_plan (constant tables + scratch) for one grid on the
    current device."""

    def __init__(self, grid: dict, max_hits=65535, max_peaks=1 << 20, max_member_cap=256,
                 max_tracks=1 << 16, max_vertex_cells=64 * 256, max_n_rho=64):
        _torch()
        self.grid = dict(grid)
        self._g = grid_struct(grid)
        self._lim = Limits(int(max_hits), int(max_peaks), int(max_member_cap), int(max_tracks),
                           int(max_vertex_cells), int(max_n_rho))
        h = C.c_void_p()
        _check(lib().ht_plan_create(C.byref(self._g), C.byref(self._lim), C.byref(h)),
               "ht_plan_create")
        self._h = h
        self.limits = dict(max_hits=max_hits, max_peaks=max_peaks, max_member_cap=max_member_cap,
                           max_tracks=max_tracks, max_vertex_cells=max_vertex_cells,
                           max_n_rho=max_n_rho)

    @property
    def handle(self):
        return self._h

    @property
    def acc_shape(self):
        return (self.grid["n_d0"], self.grid["n_qpt"], self.grid["n_phi"])

    def close(self):
        if getattr(self, "_h", None):
            lib().ht_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hough_vote(plan: Plan, r, phi, acc, n_votes=None, stream=None):
    """acc[n_d0, n_qpt, n_phi] int32 <- votes of hits (r, phi) (float32)."""
    torch = _torch()
    n = int(r.numel())
    if phi.numel() != n or tuple(acc.shape) != plan.acc_shape:
        raise ValueError("shape mismatch")
    _need(n_votes is None or n_votes.numel() >= 1, "n_votes must hold one element")
    _check(lib().hough_vote(plan.handle, _ptr(r, torch.float32, "r"),
                            _ptr(phi, torch.float32, "phi"), n,
                            _ptr(acc, torch.int32, "acc"),
                            _ptr(n_votes, torch.int64, "n_votes"), _stream(stream)),
           "hough_vote")


def hough_vote_cell(plan: Plan, r, phi, acc, n_votes=None, stream=None):
    """Band variant of hough_vote: each hit votes for every phi0 bin its
    curve reaches over each column's (q/pT, d0) cell."""
    torch = _torch()
    n = int(r.numel())
    if phi.numel() != n or tuple(acc.shape) != plan.acc_shape:
        raise ValueError("shape mismatch")
    _need(n_votes is None or n_votes.numel() >= 1, "n_votes must hold one element")
    _check(lib().hough_vote_cell(plan.handle, _ptr(r, torch.float32, "r"),
                                 _ptr(phi, torch.float32, "phi"), n,
                                 _ptr(acc, torch.int32, "acc"),
                                 _ptr(n_votes, torch.int64, "n_votes"), _stream(stream)),
           "hough_vote_cell")


def hough_peaks(plan: Plan, acc, min_votes: int, out, n_found, stream=None):
    """out: int32 [capacity, 2] (lin, votes) rows; n_found: int32 [1]."""
    torch = _torch()
    if tuple(acc.shape) != plan.acc_shape or out.dim() != 2 or out.shape[1] != 2:
        raise ValueError("shape mismatch")
    _need(n_found.numel() >= 1, "n_found must hold one element")
    _check(lib().hough_peaks(plan.handle, _ptr(acc, torch.int32, "acc"), int(min_votes),
                             _ptr(out, torch.int32, "out"), int(out.shape[0]),
                             _ptr(n_found, torch.int32, "n_found"), _stream(stream)),
           "hough_peaks")


def hough_peaks_noalloc(grid: dict, acc, min_votes: int, out, n_found, stream=None):
    """hough_peaks without a plan and without allocating: the library's fixed
    device scratch array (grids of at most 2^24 cells)."""
    torch = _torch()
    g = grid_struct(grid)
    if tuple(acc.shape) != (g.n_d0, g.n_qpt, g.n_phi) or out.dim() != 2 or out.shape[1] != 2:
        raise ValueError("shape mismatch")
    _need(n_found.numel() >= 1, "n_found must hold one element")
    _check(lib().hough_peaks_noalloc(C.byref(g), _ptr(acc, torch.int32, "acc"), int(min_votes),
                                     _ptr(out, torch.int32, "out"), int(out.shape[0]),
                                     _ptr(n_found, torch.int32, "n_found"), _stream(stream)),
           "hough_peaks_noalloc")


class ClusterBuffers:
    """Device outputs of assoc_cluster."""

    def __init__(self, n_hits_max, track_cap, object_cap, member_cap, n_rho, n_theta,
                 device="cuda"):
        torch = _torch()
        self.hit_owner = torch.empty(max(n_hits_max, 1), dtype=torch.int32, device=device)
        self.tracks = torch.zeros((max(track_cap, 1), TRACK_DTYPE.itemsize // 4),
                                  dtype=torch.int32, device=device)
        self.objects = torch.zeros((max(object_cap, 1), OBJECT_DTYPE.itemsize // 4),
                                   dtype=torch.int32, device=device)
        self.members = torch.zeros(max(member_cap, 1), dtype=torch.int32, device=device)
        self.vacc = torch.zeros((n_rho, n_theta), dtype=torch.int32, device=device)
        self.counts = torch.zeros(8, dtype=torch.int32, device=device)
        # the seed search's 64-bit work totals: road tests defined, float64 distances computed
        self.work = torch.zeros(2, dtype=torch.int64, device=device)
        self.track_cap, self.object_cap, self.member_cap = track_cap, object_cap, member_cap

    def struct(self, with_vacc=True) -> ClusterOut:
        return ClusterOut(self.hit_owner.data_ptr(), self.tracks.data_ptr(), self.track_cap,
                          self.objects.data_ptr(), self.object_cap, self.members.data_ptr(),
                          self.member_cap, self.vacc.data_ptr() if with_vacc else None,
                          self.counts.data_ptr(), self.work.data_ptr())

    def to_host(self, n_hits):
        """Copy back as numpy (structured track/object arrays), trimmed."""
        counts = self.counts.cpu().numpy()
        nt = min(int(counts[1]), self.track_cap)
        no = min(int(counts[2]), self.object_cap)
        nm = min(int(counts[3]), self.member_cap)
        tr = self.tracks.cpu().numpy().view(TRACK_DTYPE).reshape(-1)[:nt].copy()
        ob = self.objects.cpu().numpy().view(OBJECT_DTYPE).reshape(-1)[:no].copy()
        return dict(hit_owner=self.hit_owner[:n_hits].cpu().numpy(), tracks=tr, objects=ob,
                    members=self.members[:nm].cpu().numpy(), vacc=self.vacc.cpu().numpy(),
                    counts=counts, work=self.work.cpu().numpy())


def compact_hits(r, phi, layer, hit_owner, out_r, out_phi, out_layer, out_index, n_out,
                 stream=None):
    """Keeps the hits with hit_owner < 0 in event order (ht_compact_hits);
    out_*: [n_hits] device tensors, n_out: int32 [1] device."""
    torch = _torch()
    n = int(r.numel())
    for t in (phi, layer, hit_owner, out_r, out_phi, out_layer, out_index):
        if t.numel() < n:
            raise ValueError("shape mismatch")
    _check(lib().ht_compact_hits(_ptr(r, torch.float32, "r"), _ptr(phi, torch.float32, "phi"),
                                 _ptr(layer, torch.uint8, "layer"),
                                 n, _ptr(hit_owner, torch.int32, "hit_owner"),
                                 _ptr(out_r, torch.float32, "out_r"),
                                 _ptr(out_phi, torch.float32, "out_phi"),
                                 _ptr(out_layer, torch.uint8, "out_layer"),
                                 _ptr(out_index, torch.int32, "out_index"),
                                 _ptr(n_out, torch.int32, "n_out"), _stream(stream)),
           "ht_compact_hits")


def remap_track_hits(bufs: "ClusterBuffers", index, stream=None):
    """Maps the hit indices of bufs' tracks through index (ht_remap_track_hits)."""
    torch = _torch()
    _check(lib().ht_remap_track_hits(bufs.tracks.data_ptr(), bufs.track_cap,
                                     _ptr(bufs.counts, torch.int32, "counts"),
                                     _ptr(index, torch.int32, "index"), int(index.numel()),
                                     _stream(stream)),
           "ht_remap_track_hits")


def _acc_ptr(plan: Plan, acc):
    if acc is None:
        return None
    if tuple(acc.shape) != plan.acc_shape:
        raise ValueError("shape mismatch")
    return _ptr(acc, _torch().int32, "acc")


def _check_cluster_args(plan: Plan, n, peaks, n_peaks, cfg: dict, bufs: ClusterBuffers,
                        with_vacc):
    _need(peaks.dim() == 2 and peaks.shape[1] == 2, "peaks must be int32 [cap, 2]")
    _need(n_peaks.numel() >= 1, "n_peaks must hold one element")
    _need(bufs.hit_owner.numel() >= n, "bufs.hit_owner holds fewer entries than there are hits")
    _need(bufs.counts.numel() >= 8, "bufs.counts must hold 8 entries")
    _need(bufs.tracks.shape[0] >= bufs.track_cap and bufs.objects.shape[0] >= bufs.object_cap
          and bufs.members.numel() >= bufs.member_cap, "bufs capacities exceed their tensors")
    if with_vacc:
        _need(bufs.vacc.numel() >= int(cfg["n_rho"]) * int(cfg["n_theta"]),
              "bufs.vacc holds fewer cells than n_rho * n_theta")


def assoc_cluster(plan: Plan, r, phi, layer, peaks, n_peaks, cfg: dict, bufs: ClusterBuffers,
                  with_vacc=True, stream=None, acc=None):
    """peaks: int32 [cap, 2] from hough_peaks; n_peaks: int32 [1] device;
    acc: optionally the hough_vote accumulator of these hits (candidates it
    proves to exceed member_cap skip the member search; same results)."""
    torch = _torch()
    n = int(r.numel())
    if phi.numel() != n or layer.numel() != n:
        raise ValueError("shape mismatch")
    _check_cluster_args(plan, n, peaks, n_peaks, cfg, bufs, with_vacc)
    c = cluster_struct(cfg)
    o = bufs.struct(with_vacc)
    _check(lib().assoc_cluster(plan.handle, _ptr(r, torch.float32, "r"),
                               _ptr(phi, torch.float32, "phi"),
                               _ptr(layer, torch.uint8, "layer"), n,
                               _ptr(peaks, torch.int32, "peaks"),
                               _ptr(n_peaks, torch.int32, "n_peaks"), int(peaks.shape[0]),
                               _acc_ptr(plan, acc), C.byref(c), C.byref(o), _stream(stream)),
           "assoc_cluster")


def hough_vote_n(plan: Plan, r, phi, n_hits_dev, acc, n_votes=None, stream=None):
    """hough_vote with the hit count read on the device from n_hits_dev
    (int32 [1]); r and phi hold at least that many hits."""
    torch = _torch()
    n = int(r.numel())
    if phi.numel() != n or tuple(acc.shape) != plan.acc_shape:
        raise ValueError("shape mismatch")
    _need(n_hits_dev.numel() >= 1, "n_hits_dev must hold one element")
    _need(n_votes is None or n_votes.numel() >= 1, "n_votes must hold one element")
    _check(lib().hough_vote_n(plan.handle, _ptr(r, torch.float32, "r"),
                              _ptr(phi, torch.float32, "phi"), n,
                              _ptr(n_hits_dev, torch.int32, "n_hits_dev"),
                              _ptr(acc, torch.int32, "acc"),
                              _ptr(n_votes, torch.int64, "n_votes"), _stream(stream)),
           "hough_vote_n")


def assoc_cluster_n(plan: Plan, r, phi, layer, n_hits_dev, peaks, n_peaks, cfg: dict,
                    bufs: ClusterBuffers, with_vacc=True, stream=None, acc=None):
    """assoc_cluster with the hit count read on the device from n_hits_dev."""
    torch = _torch()
    n = int(r.numel())
    if phi.numel() != n or layer.numel() != n:
        raise ValueError("shape mismatch")
    _need(n_hits_dev.numel() >= 1, "n_hits_dev must hold one element")
    _check_cluster_args(plan, n, peaks, n_peaks, cfg, bufs, with_vacc)
    c = cluster_struct(cfg)
    o = bufs.struct(with_vacc)
    _check(lib().assoc_cluster_n(plan.handle, _ptr(r, torch.float32, "r"),
                                 _ptr(phi, torch.float32, "phi"),
                                 _ptr(layer, torch.uint8, "layer"), n,
                                 _ptr(n_hits_dev, torch.int32, "n_hits_dev"),
                                 _ptr(peaks, torch.int32, "peaks"),
                                 _ptr(n_peaks, torch.int32, "n_peaks"), int(peaks.shape[0]),
                                 _acc_ptr(plan, acc), C.byref(c), C.byref(o), _stream(stream)),
           "assoc_cluster_n")


def hough_batch(events, n_hits_max: int, min_votes: int, cfg: dict, with_vacc=True,
                stream=None):
    """hough_vote, hough_peaks and assoc_cluster for up to MAX_BATCH events in
    one launch per kernel.  events: list of dicts with plan, r, phi, layer
    (device tensors holding at least n_hits_max hits), n_dev (int32 [1]
    device hit count), acc, peaks (int32 [peak_cap, 2]), nf (int32 [1]) and
    bufs (ClusterBuffers); every peaks tensor has the same capacity."""
    torch = _torch()
    nb = len(events)
    _need(1 <= nb <= MAX_BATCH, "1 .. 4 events")
    cap = int(events[0]["peaks"].shape[0])
    arr = (BatchEvent * nb)()
    keep = []
    for b, e in enumerate(events):
        plan = e["plan"]
        for t in (e["r"], e["phi"], e["layer"]):
            _need(t.numel() >= n_hits_max, "hits hold fewer entries than n_hits_max")
        _need(tuple(e["acc"].shape) == plan.acc_shape, "acc must have the plan's shape")
        _need(e["peaks"].dim() == 2 and e["peaks"].shape == (cap, 2), "peaks must be int32 [cap, 2]")
        _need(e["n_dev"].numel() >= 1 and e["nf"].numel() >= 1, "counts must hold one element")
        _check_cluster_args(plan, n_hits_max, e["peaks"], e["nf"], cfg, e["bufs"], with_vacc)
        o = e["bufs"].struct(with_vacc)
        keep.append(o)
        arr[b] = BatchEvent(plan.handle.value, _ptr(e["r"], torch.float32, "r").value,
                            _ptr(e["phi"], torch.float32, "phi").value,
                            _ptr(e["layer"], torch.uint8, "layer").value,
                            _ptr(e["n_dev"], torch.int32, "n_dev").value,
                            _ptr(e["acc"], torch.int32, "acc").value,
                            _ptr(e["peaks"], torch.int32, "peaks").value,
                            _ptr(e["nf"], torch.int32, "nf").value, o)
    c = cluster_struct(cfg)
    _check(lib().hough_batch(nb, C.cast(arr, C.c_void_p), int(n_hits_max), int(min_votes), cap,
                             C.byref(c), _stream(stream)), "hough_batch")


def asin_f32(u, out, stream=None):
    torch = _torch()
    _check(lib().ht_asin_f32(_ptr(u, torch.float32, "u"), _ptr(out, torch.float32, "out"),
                             int(u.numel()), _stream(stream)), "ht_asin_f32")


def sqrt_f64(x, out, stream=None):
    torch = _torch()
    _check(lib().ht_sqrt_f64(_ptr(x, torch.float64, "x"), _ptr(out, torch.float64, "out"),
                             int(x.numel()), _stream(stream)), "ht_sqrt_f64")


CNN_PARAMS = 8529
CNN_WINDOW = 128


def cnn_workspace(n_windows, training=False):
    """A device workspace (uint8 tensor) for the CNN calls on n_windows."""
    torch = _torch()
    nb = int(lib().ht_cnn_workspace_bytes(int(n_windows), int(bool(training))))
    return torch.empty(nb, dtype=torch.uint8, device="cuda")


def cnn_windows(plan: "Plan", acc, peaks, n_peaks, win, stream=None):
    """Windows (bfloat16 [cap, 128]) of the first min(n_peaks, cap) peaks."""
    torch = _torch()
    cap = int(peaks.shape[0])
    if tuple(win.shape) != (cap, CNN_WINDOW):
        raise ValueError("win must be [cap, 128]")
    _need(tuple(acc.shape) == plan.acc_shape, "acc must have the plan's shape")
    _need(peaks.dim() == 2 and peaks.shape[1] == 2, "peaks must be int32 [cap, 2]")
    _need(n_peaks.numel() >= 1, "n_peaks must hold one element")
    _check(lib().ht_cnn_windows(plan.handle, _ptr(acc, torch.int32, "acc"),
                                _ptr(peaks, torch.int32, "peaks"),
                                _ptr(n_peaks, torch.int32, "n_peaks"), cap,
                                _ptr(win, torch.bfloat16, "win"), _stream(stream)), "ht_cnn_windows")


def cnn_forward(params, win, logits, workspace, n_dev=None, stream=None):
    torch = _torch()
    _need(win.dim() == 2 and win.shape[1] == CNN_WINDOW, "win must be [n, 128]")
    n_max = int(win.shape[0])
    _need(logits.numel() >= n_max, "logits holds fewer entries than there are windows")
    _need(params.numel() >= CNN_PARAMS, "params must hold HT_CNN_PARAMS floats")
    _need(n_dev is None or n_dev.numel() >= 1, "n_dev must hold one element")
    _check(lib().ht_cnn_forward(_ptr(params, torch.float32, "params"),
                                _ptr(win, torch.bfloat16, "win"),
                                _ptr(n_dev, torch.int32, "n_dev") if n_dev is not None else None,
                                n_max, _ptr(logits, torch.float32, "logits"),
                                _ptr(workspace, torch.uint8, "workspace"), int(workspace.numel()),
                                _stream(stream)), "ht_cnn_forward")


def cnn_score(plan: "Plan", params, acc, peaks, n_peaks, logits, workspace, stream=None):
    """Logits of the first min(n_peaks, cap) peaks, windows built in LDS from
    the accumulator (ht_cnn_score)."""
    torch = _torch()
    cap = int(peaks.shape[0])
    _need(tuple(acc.shape) == plan.acc_shape, "acc must have the plan's shape")
    _need(peaks.dim() == 2 and peaks.shape[1] == 2, "peaks must be int32 [cap, 2]")
    _need(n_peaks.numel() >= 1, "n_peaks must hold one element")
    _need(logits.numel() >= cap, "logits holds fewer entries than there are peaks")
    _need(params.numel() >= CNN_PARAMS, "params must hold HT_CNN_PARAMS floats")
    _check(lib().ht_cnn_score(plan.handle, _ptr(params, torch.float32, "params"),
                              _ptr(acc, torch.int32, "acc"), _ptr(peaks, torch.int32, "peaks"),
                              _ptr(n_peaks, torch.int32, "n_peaks"), cap,
                              _ptr(logits, torch.float32, "logits"),
                              _ptr(workspace, torch.uint8, "workspace"), int(workspace.numel()),
                              _stream(stream)), "ht_cnn_score")


def cnn_train_step(params, mom, win, labels, lr, momentum, pos_weight, loss, workspace,
                   stream=None):
    torch = _torch()
    _need(win.dim() == 2 and win.shape[1] == CNN_WINDOW, "win must be [n, 128]")
    _need(labels.numel() >= win.shape[0], "labels holds fewer entries than there are windows")
    _need(params.numel() >= CNN_PARAMS and mom.numel() >= CNN_PARAMS,
          "params and mom must hold HT_CNN_PARAMS floats")
    _need(loss.numel() >= 1, "loss must hold one element")
    _check(lib().ht_cnn_train_step(_ptr(params, torch.float32, "params"),
                                   _ptr(mom, torch.float32, "mom"),
                                   _ptr(win, torch.bfloat16, "win"),
                                   _ptr(labels, torch.float32, "labels"), int(win.shape[0]),
                                   float(lr), float(momentum), float(pos_weight),
                                   _ptr(loss, torch.float32, "loss"),
                                   _ptr(workspace, torch.uint8, "workspace"),
                                   int(workspace.numel()), _stream(stream)), "ht_cnn_train_step")


def cnn_keep(plan: "Plan", logits, peaks, n_peaks, threshold, out, n_out, stream=None):
    torch = _torch()
    _need(peaks.dim() == 2 and peaks.shape[1] == 2, "peaks must be int32 [cap, 2]")
    _need(out.dim() == 2 and out.shape[1] == 2, "out must be int32 [out_cap, 2]")
    _need(logits.numel() >= peaks.shape[0], "logits holds fewer entries than there are peaks")
    _need(n_peaks.numel() >= 1 and n_out.numel() >= 1, "n_peaks and n_out must hold one element")
    _check(lib().ht_cnn_keep(plan.handle, _ptr(logits, torch.float32, "logits"),
                             _ptr(peaks, torch.int32, "peaks"), _ptr(n_peaks, torch.int32, "n_peaks"),
                             int(peaks.shape[0]), float(threshold), _ptr(out, torch.int32, "out"),
                             int(out.shape[0]), _ptr(n_out, torch.int32, "n_out"),
                             _stream(stream)), "ht_cnn_keep")


STAGES = ("vote", "peaks", "assoc", "members", "refine")  # HT_STAGE_* order


def profile_begin(plan: "Plan", depth: int = 1024):
    """Start timing the stages of later calls on ``plan`` with HIP events."""
    _check(lib().ht_profile_begin(plan.handle, int(depth)), "ht_profile_begin")


def profile_read(plan: "Plan", acc: dict | None = None) -> dict:
    """Add the stage times recorded since the last read to ``acc`` (a dict
    of stage -> [milliseconds, launches]) and return it."""
    ms = np.zeros(len(STAGES), np.float64)
    n = np.zeros(len(STAGES), np.int64)
    _check(lib().ht_profile_read(plan.handle, ms.ctypes.data_as(C.c_void_p),
                                 n.ctypes.data_as(C.c_void_p)), "ht_profile_read")
    acc = {} if acc is None else acc
    for name, t, c in zip(STAGES, ms, n):
        a = acc.setdefault(name, [0.0, 0])
        a[0] += float(t)
        a[1] += int(c)
    return acc


def profile_end(plan: "Plan"):
    _check(lib().ht_profile_end(plan.handle), "ht_profile_end")


class Server:
    """The trigger serving loop (ht_server_*): events of several grid kinds,
    submitted one by one from host arrays, processed on device-resident
    slots; results come back through poll().  kinds: list of dicts with
    grid, cluster, min_votes, peak_cap, and optionally the learned filter:
    cnn_params (host float32 [CNN_PARAMS]) and cnn_threshold.  batch_max > 1
    lets up to that many waiting events of one kind with at most
    batch_max_hits hits share a batch."""

    def __init__(self, kinds, max_hits=65535, track_cap=4096, object_cap=256, member_cap=4096,
                 hbm_budget=64 << 30, max_slots=4, queue_cap=256, use_graphs=True,
                 work_budget=0, batch_max=0, batch_max_hits=0):
        if not 1 <= len(kinds) <= SERVER_MAX_KINDS:
            raise ValueError("1..4 kinds")
        _torch()  # a GPU must be there
        cfg = ServerCfg()
        cfg.n_kinds = len(kinds)
        params = []  # held until the server has copied them
        for i, k in enumerate(kinds):
            cfg.kinds[i].grid = grid_struct(k["grid"])
            cfg.kinds[i].cluster = cluster_struct(k["cluster"])
            cfg.kinds[i].min_votes = int(k["min_votes"])
            cfg.kinds[i].peak_cap = int(k["peak_cap"])
            if k.get("cnn_params") is not None:
                w = np.ascontiguousarray(k["cnn_params"], np.float32).reshape(-1)
                _need(w.size == CNN_PARAMS, f"cnn_params needs {CNN_PARAMS} floats")
                params.append(w)
                cfg.kinds[i].cnn_params = w.ctypes.data
                cfg.kinds[i].cnn_threshold = float(k["cnn_threshold"])
        cfg.max_hits, cfg.track_cap = int(max_hits), int(track_cap)
        cfg.object_cap, cfg.member_cap = int(object_cap), int(member_cap)
        cfg.hbm_budget, cfg.max_slots = int(hbm_budget), int(max_slots)
        cfg.queue_cap, cfg.use_graphs = int(queue_cap), int(bool(use_graphs))
        cfg.work_budget = int(work_budget)
        cfg.batch_max, cfg.batch_max_hits = int(batch_max), int(batch_max_hits)
        self.cfg = cfg
        h = C.c_void_p()
        _check(lib().ht_server_create(C.byref(cfg), C.byref(h)), "ht_server_create")
        del params
        self._h = h
        self._keep = {}
        n, b = C.c_int32(), C.c_int64()
        _check(lib().ht_server_info(h, C.byref(n), C.byref(b)), "ht_server_info")
        self.n_slots, self.slot_bytes = int(n.value), int(b.value)

    def submit(self, kind, r, phi, layer, tag, want_outputs=True):
        """Submit one event (numpy float32 r, phi; uint8 layer).  Returns False
        when the event is shed (every slot busy, queue full)."""
        r = np.ascontiguousarray(r, np.float32)
        phi = np.ascontiguousarray(phi, np.float32)
        layer = np.ascontiguousarray(layer, np.uint8)
        out = ServerOut()
        bufs = None
        if want_outputs:
            c = self.cfg
            bufs = dict(tracks=np.zeros(c.track_cap, TRACK_DTYPE),
                        hit_owner=np.full(max(r.size, 1), -1, np.int32),
                        objects=np.zeros(c.object_cap, OBJECT_DTYPE),
                        members=np.zeros(c.member_cap, np.int32))
            out.tracks = bufs["tracks"].ctypes.data
            out.track_cap = c.track_cap
            out.hit_owner = bufs["hit_owner"].ctypes.data
            out.objects = bufs["objects"].ctypes.data
            out.object_cap = c.object_cap
            out.members = bufs["members"].ctypes.data
            out.member_cap = c.member_cap
        rc = lib().ht_server_submit(self._h, int(kind), r.ctypes.data, phi.ctypes.data,
                                    layer.ctypes.data, int(r.size), C.byref(out), int(tag))
        if rc == HT_EBUSY:
            return False
        _check(rc, "ht_server_submit")
        self._keep[int(tag)] = (bufs, r.size)
        return True

    def poll(self, wait=False, max_results=256):
        res = (ServerResult * max_results)()
        n = C.c_int32()
        _check(lib().ht_server_poll(self._h, res, int(max_results), int(bool(wait)), C.byref(n)),
               "ht_server_poll")
        out = []
        for i in range(n.value):
            x = res[i]
            bufs, nh = self._keep.pop(int(x.tag), (None, 0))
            d = dict(tag=int(x.tag), kind=int(x.kind), n_hits=int(x.n_hits), status=int(x.status),
                     n_peaks=int(x.n_peaks), counts=np.array(x.counts[:], np.int32),
                     t_submit=x.t_submit, t_start=x.t_start, t_done=x.t_done,
                     device_ms=x.device_ms, n_kept=int(x.n_kept), batch=int(x.batch))
            if bufs is not None:
                c = d["counts"]
                d["tracks"] = bufs["tracks"][:min(c[1], self.cfg.track_cap)].copy()
                d["hit_owner"] = bufs["hit_owner"][:nh].copy()
                d["objects"] = bufs["objects"][:min(c[2], self.cfg.object_cap)].copy()
                d["members"] = bufs["members"][:min(c[3], self.cfg.member_cap)].copy()
            out.append(d)
        return out

    def drain(self):
        done = []
        while self._keep:
            got = self.poll(wait=True)
            if not got:
                break
            done += got
        return done

    def close(self):
        if getattr(self, "_h", None):
            lib().ht_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


EXPORTS = ("ht_plan_create", "ht_plan_destroy", "ht_strerror", "hough_vote", "hough_vote_cell",
           "hough_peaks",
           "assoc_cluster", "ht_asin_f32", "ht_sqrt_f64", "ht_profile_begin", "ht_profile_read",
           "ht_profile_end", "ht_server_create", "ht_server_destroy", "ht_server_info",
           "ht_server_submit", "ht_server_poll", "ht_cnn_workspace_bytes", "ht_cnn_windows",
           "ht_cnn_forward", "ht_cnn_train_step", "ht_cnn_keep", "ht_compact_hits",
           "ht_remap_track_hits", "hough_vote_n", "assoc_cluster_n", "hough_peaks_noalloc",
           "ht_cnn_score", "hough_batch")
