"""Physics figures of merit from the path's outputs plus generator truth.

Track efficiency, fake and duplicate rates and vertex efficiency (the paper's
jet efficiency is found jets over jets present, section "Preliminary
Results").  Host-side numpy over small arrays; not part of the GPU path.

Reading used for matching: a track matches truth track t when at least 75% of
its owned hits, and at least ``min_layers`` of them, are hits of t.  A truth
track is in acceptance when its q/pT and d0 lie inside the grid and it has at
least ``min_layers`` hits after its point of closest approach (the branch the
transform votes for).
"""
from __future__ import annotations

import numpy as np


def match_tracks(hits: np.ndarray, hit_track: np.ndarray, min_layers: int, frac: float = 0.75):
    """hits: int32 [n_tracks, L] owned hit per layer (-1 none).  Returns the
    matched truth index per track (-1 = fake)."""
    out = np.full(hits.shape[0], -1, np.int64)
    for t in range(hits.shape[0]):
        h = hits[t][hits[t] >= 0]
        if h.size == 0:
            continue
        tt = hit_track[h]
        tt = tt[tt >= 0]
        if tt.size == 0:
            continue
        vals, cnt = np.unique(tt, return_counts=True)
        b = int(np.argmax(cnt))
        if cnt[b] >= min_layers and cnt[b] >= frac * h.size:
            out[t] = vals[b]
    return out


def in_acceptance(ev, grid: dict, min_layers: int) -> np.ndarray:
    q = np.abs(ev.trk_qpt) <= max(abs(grid["qpt_lo"]), abs(grid["qpt_hi"]))
    q &= (ev.trk_qpt >= grid["qpt_lo"]) & (ev.trk_qpt <= grid["qpt_hi"])
    if grid["n_d0"] > 1:
        d = (ev.trk_d0 >= grid["d0_lo"]) & (ev.trk_d0 <= grid["d0_hi"])
    else:
        d = np.abs(ev.trk_d0) < 1e-9
    return q & d & (ev.trk_nfwd >= min_layers)


def track_metrics(ev, grid: dict, min_layers: int, track_hits: np.ndarray) -> dict:
    m = match_tracks(track_hits, ev.hit_track, min_layers)
    acc = in_acceptance(ev, grid, min_layers)
    found = np.zeros(len(ev.trk_qpt), bool)
    found[m[m >= 0]] = True
    n_acc = int(acc.sum())
    n_found = int((found & acc).sum())
    n_trk = int(track_hits.shape[0])
    n_fake = int((m < 0).sum())
    uniq, cnt = np.unique(m[m >= 0], return_counts=True)
    dup = int((cnt - 1).sum()) if cnt.size else 0
    return dict(n_truth_acc=n_acc, n_found=n_found,
                efficiency=(n_found / n_acc) if n_acc else float("nan"),
                n_tracks=n_trk, n_fake=n_fake,
                fake_rate=(n_fake / n_trk) if n_trk else 0.0,
                duplicate_rate=(dup / max(len(uniq), 1)))


def vertex_metrics(ev, objects: np.ndarray, members: np.ndarray, track_match: np.ndarray,
                   rho_bin: float, theta_bin: float, min_tracks: int) -> dict:
    """A true vertex is found when an object lies within 2 bins in rho and
    theta and at least half of its members match tracks of that vertex."""
    nv = len(ev.vtx_rho)
    found = np.zeros(nv, bool)
    findable = np.zeros(nv, bool)
    for v in range(nv):
        tr = np.where(ev.trk_vertex == v)[0]
        findable[v] = np.isin(tr, track_match[track_match >= 0]).sum() >= min_tracks
    for o in objects:
        mem = members[o["member_begin"]:o["member_begin"] + o["n_tracks"]]
        tm = track_match[mem] if mem.size else np.zeros(0, np.int64)
        for v in range(nv):
            dth = abs((o["theta"] - ev.vtx_theta[v] + np.pi) % (2 * np.pi) - np.pi)
            if abs(o["rho"] - ev.vtx_rho[v]) <= 2 * rho_bin and dth <= 2 * theta_bin:
                hv = (tm >= 0) & np.isin(tm, np.where(ev.trk_vertex == v)[0])
                if mem.size and hv.sum() >= 0.5 * mem.size:
                    found[v] = True
    return dict(n_vertices=nv, n_findable=int(findable.sum()),
                n_found=int((found & findable).sum()), n_objects=int(len(objects)))
