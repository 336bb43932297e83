"""ctypes wrapper of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It does not import the GPU package and
the GPU package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HT_ORACLE_LIB selects another build of the same source (the sanitizer build)
LIB_PATH = os.environ.get("HT_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
MAX_LAYERS = 16

PEAK_DT = np.dtype([("lin", "<i4"), ("votes", "<i4")])
TRACK_DT = np.dtype([
    ("peak", "<i4"), ("lin", "<i4"), ("votes", "<i4"), ("n_layers", "<i4"),
    ("n_inliers", "<i4"), ("n_owned", "<i4"), ("status", "<i4"), ("seed_ss", "<f4"),
    ("phi0", "<f4"), ("qpt", "<f4"),
    ("d0", "<f4"), ("chi2", "<f4"), ("r_first", "<f4"), ("hits", "<i4", (MAX_LAYERS,)),
])
OBJECT_DT = np.dtype([
    ("lin", "<i4"), ("votes", "<i4"), ("n_tracks", "<i4"), ("kind", "<i4"),
    ("rho", "<f4"), ("theta", "<f4"), ("isotropy", "<f4"), ("member_begin", "<i4"),
])


class _Grid(C.Structure):
    _fields_ = [("n_phi", C.c_int32), ("n_qpt", C.c_int32), ("n_d0", C.c_int32),
                ("qpt_lo", C.c_float), ("qpt_hi", C.c_float),
                ("d0_lo", C.c_float), ("d0_hi", C.c_float), ("bfield", C.c_float)]


class _Cfg(C.Structure):
    _fields_ = [("win_bins", C.c_int32), ("min_layers", C.c_int32), ("seed_k", C.c_int32),
                ("member_cap", C.c_int32), ("road_sigmas", C.c_float),
                ("box_margin", C.c_float), ("sigma_rphi", C.c_float),
                ("fit_iters", C.c_int32), ("n_rho", C.c_int32), ("n_theta", C.c_int32),
                ("rho_lo", C.c_float), ("rho_hi", C.c_float),
                ("vtx_min_votes", C.c_int32), ("bh_min_tracks", C.c_int32),
                ("bh_max_isotropy", C.c_float), ("vtx_min_d0", C.c_float),
                ("fit_kind", C.c_int32), ("vtx_two_branch", C.c_int32)]


def _grid(g: dict) -> _Grid:
    return _Grid(int(g["n_phi"]), int(g["n_qpt"]), int(g["n_d0"]), float(g["qpt_lo"]),
                 float(g["qpt_hi"]), float(g["d0_lo"]), float(g["d0_hi"]), float(g["bfield"]))


def _cfg(c: dict) -> _Cfg:
    return _Cfg(int(c["win_bins"]), int(c["min_layers"]), int(c["seed_k"]),
                int(c["member_cap"]), float(c["road_sigmas"]), float(c["box_margin"]),
                float(c["sigma_rphi"]), int(c["fit_iters"]), int(c["n_rho"]),
                int(c["n_theta"]), float(c["rho_lo"]), float(c["rho_hi"]),
                int(c["vtx_min_votes"]), int(c["bh_min_tracks"]), float(c["bh_max_isotropy"]),
                float(c.get("vtx_min_d0", 0.0)), int(c.get("fit_kind", 0)),
                int(c.get("vtx_two_branch", 0)))


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build()
        _lib = _bind(LIB_PATH)
    return _lib


def use_library(path):
    """Binds this wrapper to another build of the oracle (the tests build
    copies with a planted mistake to show that a pin catches it).  Returns
    the previous binding, to be passed back to restore it."""
    global _lib
    prev = lib()
    _lib = path if isinstance(path, C.CDLL) else _bind(path)
    return prev


def _bind(path):
    so = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    so.oracle_asin_f.argtypes = [C.c_float]
    so.oracle_asin_f.restype = C.c_float
    so.oracle_asin_f_array.argtypes = [vp, vp, i64]
    so.oracle_asin_f_array.restype = None
    so.oracle_tables.argtypes = [vp, vp, vp, vp, vp]
    so.oracle_sincos_array.argtypes = [vp, vp, vp, i64]
    so.oracle_sincos_array.restype = None
    so.oracle_atan2_array.argtypes = [vp, vp, vp, i64]
    so.oracle_atan2_array.restype = None
    so.oracle_phi0_coord.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp]
    so.oracle_hough_vote.argtypes = [vp, vp, vp, i32, vp, vp]
    so.oracle_hough_vote_cell.argtypes = [vp, vp, vp, i32, vp, vp]
    so.oracle_hough_peaks.argtypes = [vp, vp, i32, vp, i32, vp]
    so.oracle_assoc_cluster.argtypes = [vp, vp, vp, vp, i32, vp, i32, vp, vp, vp, i32, vp,
                                        i32, vp, i32, vp, vp]
    so.oracle_set_threads.argtypes = [C.c_int]
    so.oracle_set_threads.restype = None
    so.oracle_refine_one.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp, vp]
    so.oracle_ownership.argtypes = [i32, vp, vp, vp, vp, i32, vp, vp]
    so.oracle_vertex_peaks.argtypes = [vp, i32, i32, i32, vp, i32, vp]
    for f in ("oracle_refine_one", "oracle_tables", "oracle_phi0_coord", "oracle_hough_vote",
              "oracle_hough_vote_cell", "oracle_hough_peaks", "oracle_assoc_cluster",
              "oracle_ownership", "oracle_vertex_peaks"):
        getattr(so, f).restype = C.c_int
    return so


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def asin_f(u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float32)
    out = np.empty_like(u)
    lib().oracle_asin_f_array(_p(u), _p(out), u.size)
    return out


def sincos(a):
    a = np.ascontiguousarray(a, np.float64)
    s = np.empty_like(a)
    c = np.empty_like(a)
    lib().oracle_sincos_array(_p(a), _p(s), _p(c), a.size)
    return s, c


def atan2(y, x):
    y = np.ascontiguousarray(y, np.float64)
    x = np.ascontiguousarray(np.broadcast_to(x, y.shape), np.float64)
    out = np.empty_like(y)
    lib().oracle_atan2_array(_p(y), _p(x), _p(out), y.size)
    return out


def tables(grid: dict):
    g = _grid(grid)
    nq, nd = grid["n_qpt"], grid["n_d0"]
    kap = np.empty(nq, np.float32)
    q = np.empty(nq * nd, np.float32)
    t = np.empty(nq * nd, np.float32)
    consts = np.empty(2, np.float32)
    _check(lib().oracle_tables(C.byref(g), _p(kap), _p(q), _p(t), _p(consts)), "tables")
    return kap, q.reshape(nd, nq), t.reshape(nd, nq), consts


def phi0_coord(grid: dict, r, phi, j, k):
    r = np.ascontiguousarray(r, np.float32)
    phi = np.ascontiguousarray(phi, np.float32)
    n = r.size
    j = np.ascontiguousarray(np.broadcast_to(j, (n,)), np.int32)
    k = np.ascontiguousarray(np.broadcast_to(k, (n,)), np.int32)
    x = np.empty(n, np.float32)
    b = np.empty(n, np.int32)
    v = np.empty(n, np.int32)
    g = _grid(grid)
    _check(lib().oracle_phi0_coord(C.byref(g), _p(r), _p(phi), n, _p(j), _p(k), _p(x), _p(b),
                                   _p(v)), "phi0_coord")
    return x, b, v.astype(bool)


def hough_vote(grid: dict, r, phi):
    r = np.ascontiguousarray(r, np.float32)
    phi = np.ascontiguousarray(phi, np.float32)
    acc = np.empty((grid["n_d0"], grid["n_qpt"], grid["n_phi"]), np.int32)
    nv = C.c_uint64(0)
    g = _grid(grid)
    _check(lib().oracle_hough_vote(C.byref(g), _p(r), _p(phi), r.size, _p(acc), C.byref(nv)),
           "hough_vote")
    return acc, int(nv.value)


def hough_vote_cell(grid: dict, r, phi):
    """Band vote: every phi0 bin the hit's curve reaches over each column's
    (q/pT, d0) cell."""
    r = np.ascontiguousarray(r, np.float32)
    phi = np.ascontiguousarray(phi, np.float32)
    acc = np.empty((grid["n_d0"], grid["n_qpt"], grid["n_phi"]), np.int32)
    nv = C.c_uint64(0)
    g = _grid(grid)
    _check(lib().oracle_hough_vote_cell(C.byref(g), _p(r), _p(phi), r.size, _p(acc),
                                        C.byref(nv)), "hough_vote_cell")
    return acc, int(nv.value)


def hough_peaks(grid: dict, acc, min_votes: int, capacity: int | None = None):
    acc = np.ascontiguousarray(acc, np.int32)
    if capacity is None:
        capacity = acc.size
    out = np.zeros(max(capacity, 1), PEAK_DT)
    nf = C.c_int32(0)
    g = _grid(grid)
    _check(lib().oracle_hough_peaks(C.byref(g), _p(acc), int(min_votes), _p(out), int(capacity),
                                    C.byref(nf)), "hough_peaks")
    n = int(nf.value)
    return out[:min(n, capacity)].copy(), n


def assoc_cluster(grid: dict, r, phi, layer, peaks, cfg: dict, track_cap=1 << 16,
                  object_cap=4096, member_cap=1 << 18):
    r = np.ascontiguousarray(r, np.float32)
    phi = np.ascontiguousarray(phi, np.float32)
    layer = np.ascontiguousarray(layer, np.uint8)
    peaks = np.ascontiguousarray(peaks, PEAK_DT)
    n = r.size
    owner = np.empty(max(n, 1), np.int32)
    tracks = np.zeros(max(track_cap, 1), TRACK_DT)
    objects = np.zeros(max(object_cap, 1), OBJECT_DT)
    members = np.zeros(max(member_cap, 1), np.int32)
    vacc = np.zeros((cfg["n_rho"], cfg["n_theta"]), np.int32)
    counts = np.zeros(8, np.int32)
    g = _grid(grid)
    c = _cfg(cfg)
    _check(lib().oracle_assoc_cluster(C.byref(g), _p(r), _p(phi), _p(layer), n, _p(peaks),
                                      peaks.size, C.byref(c), _p(owner), _p(tracks), track_cap,
                                      _p(objects), object_cap, _p(members), member_cap,
                                      _p(vacc), _p(counts)), "assoc_cluster")
    nt = min(int(counts[1]), track_cap)
    no = min(int(counts[2]), object_cap)
    nm = min(int(counts[3]), member_cap)
    return dict(hit_owner=owner[:n].copy(), tracks=tracks[:nt].copy(), objects=objects[:no].copy(),
                members=members[:nm].copy(), vacc=vacc, counts=counts.copy())


def refine_one(grid: dict, r, phi, layer, lin: int, cfg: dict):
    """Refinement of one candidate cell (diagnostics and tests)."""
    r = np.ascontiguousarray(r, np.float32)
    phi = np.ascontiguousarray(phi, np.float32)
    layer = np.ascontiguousarray(layer, np.uint8)
    oi = np.zeros(3 + MAX_LAYERS, np.int32)
    of = np.zeros(5, np.float64)
    g = _grid(grid)
    c = _cfg(cfg)
    _check(lib().oracle_refine_one(C.byref(g), _p(r), _p(phi), _p(layer), r.size, int(lin),
                                   C.byref(c), _p(oi), _p(of)), "refine_one")
    return dict(status=int(oi[0]), n_layers=int(oi[1]), n_inliers=int(oi[2]), hits=oi[3:].copy(),
                ss=float(of[0]), circle=of[1:].copy())


def ownership(n_inliers, ss, lin, hits, n_hits: int):
    """The duplicate-cleaning step alone: per candidate its inlier layer
    count (-1: not a candidate), seed sum (float32), cell and inlier hit per
    layer ([n, <=16], -1 none).  Returns (owner per hit, owned hits per
    candidate)."""
    n_in = np.ascontiguousarray(n_inliers, np.int32)
    n = n_in.size
    ss = np.ascontiguousarray(ss, np.float32)
    lin = np.ascontiguousarray(lin, np.int32)
    h = np.full((max(n, 1), MAX_LAYERS), -1, np.int32)
    hits = np.asarray(hits, np.int32).reshape(n, -1)
    h[:n, :hits.shape[1]] = hits
    owner = np.empty(max(n_hits, 1), np.int32)
    n_owned = np.empty(max(n, 1), np.int32)
    _check(lib().oracle_ownership(n, _p(n_in), _p(ss), _p(lin), _p(h), int(n_hits), _p(owner),
                                  _p(n_owned)), "ownership")
    return owner[:n_hits].copy(), n_owned[:n].copy()


def vertex_peaks(vacc, thr: int):
    """Cells of the vertex accumulator [n_rho, n_theta] that pass the vertex
    peak rule, in cell order."""
    v = np.ascontiguousarray(vacc, np.int32)
    nm, nt = v.shape
    out = np.empty(v.size, np.int32)
    nf = C.c_int32(0)
    _check(lib().oracle_vertex_peaks(_p(v), nm, nt, int(thr), _p(out), v.size, C.byref(nf)),
           "vertex_peaks")
    return out[:nf.value].copy()


def set_threads(n: int):
    lib().oracle_set_threads(int(n))


# --------------------------------------------------------------------------
# Iterative hit removal (section "Current Tracker and Tracking Algorithm":
# an earlier pass finds the easier, prompt tracks, their hits are removed,
# and a later pass searches the rest for displaced tracks).

def compact_hits(r, phi, layer, hit_owner):
    """The hits that no track owns (hit_owner < 0), in event order, and the
    event index of each."""
    keep = np.flatnonzero(np.asarray(hit_owner) < 0).astype(np.int32)
    return (np.asarray(r)[keep], np.asarray(phi)[keep], np.asarray(layer)[keep], keep)


def remap_track_hits(tracks, index):
    """Tracks of a pass over kept hits, with their hit indices mapped back
    to the event through index."""
    out = tracks.copy()
    h = out["hits"]
    m = h >= 0
    h[m] = np.asarray(index)[h[m]]
    return out


def two_pass(grid_prompt: dict, min_votes_prompt: int, cfg_prompt: dict, grid: dict,
             min_votes: int, cfg: dict, r, phi, layer, peak_cap=None, **caps):
    """Prompt pass (vote, peaks, association on grid_prompt), removal of its
    owned hits, displaced pass on the rest; the displaced pass's tracks name
    event hits.  Returns (prompt result, kept event indices, displaced
    result)."""
    acc, _ = hough_vote(grid_prompt, r, phi)
    pk, _ = hough_peaks(grid_prompt, acc, min_votes_prompt, peak_cap)
    first = assoc_cluster(grid_prompt, r, phi, layer, pk, cfg_prompt, **caps)
    r2, phi2, layer2, keep = compact_hits(r, phi, layer, first["hit_owner"])
    acc2, _ = hough_vote(grid, r2, phi2)
    pk2, _ = hough_peaks(grid, acc2, min_votes, peak_cap)
    second = assoc_cluster(grid, r2, phi2, layer2, pk2, cfg, **caps)
    second["tracks"] = remap_track_hits(second["tracks"], keep)
    return first, keep, second
