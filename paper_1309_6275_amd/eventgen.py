"""Seeded synthetic tracker events (transverse plane only).

This module is the one input source shared by the GPU path, its tests and the
CPU oracle.  It simulates hits geometrically -- each charged track is a circle
in the transverse plane and each barrel layer a circle around the beam line, so
a hit is a circle-circle intersection -- and it holds none of the Hough
method's arithmetic: it never evaluates a track-parameter formula of the vote,
never bins anything and never counts votes.  Because the hit positions come
from plane geometry and not from the helix relation the vote inverts, a
noiseless track generated here is an independent check of that relation.

The detector model follows the paper's toy Monte Carlo in spirit (section
"Hough Transform Algorithm": transverse plane only, concentric barrel layers,
a beam pipe of 3.0 cm) with the layer radii, field and smear of the workloads
measured here: 10 layers at r = 4, 7, 11, 22, 30, 38, 50, 60, 80, 100 cm,
B = 3.8 T along +z, 20 um Gaussian r-phi smear.  Event compositions follow the
displaced-jet studies of section "Preliminary Results" (jets of ~10 tracks with
a dispersion half-angle between 15 and 60 degrees, a few thousand prompt
tracks) and the black-hole-like object of section "Physics Motivation"
(a high-multiplicity, isotropic decay of soft particles a few cm from the
interaction point).

Conventions (all float64 until the final cast of hit coordinates to float32):

* curvature kappa is signed counter-clockwise positive; a positive charge in a
  field along +z turns clockwise, so kappa = -0.299792458e-2 * B * (q/pT)
  [cm^-1, B in T, q/pT in GeV^-1];
* a track is produced at point V with momentum azimuth psi and moves along its
  circle from V until it reaches its largest distance from the beam line (the
  first turn) or leaves the last layer; every layer crossing on that arc is a
  hit, in order of arc length;
* the perigee of a track is its point of closest approach (PCA) to the beam
  line, d0 * (-sin phi0, cos phi0), with direction of motion phi0 there.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

RADII = (4.0, 7.0, 11.0, 22.0, 30.0, 38.0, 50.0, 60.0, 80.0, 100.0)
B_TESLA = 3.8
SMEAR_CM = 20e-4          # 20 um r-phi resolution
C_LIGHT = 0.299792458e-2  # cm^-1 per (T * GeV^-1)


def kappa_of(qpt, bfield=B_TESLA):
    """Signed curvature [1/cm] of a track with charge/transverse momentum qpt."""
    return -C_LIGHT * bfield * np.asarray(qpt, dtype=np.float64)


@dataclass
class Event:
    """One event: hit SoA (float32/uint8) plus Monte Carlo truth."""

    r: np.ndarray            # float32 [H], cm
    phi: np.ndarray          # float32 [H], rad in [-pi, pi)
    layer: np.ndarray        # uint8  [H]
    hit_track: np.ndarray    # int32  [H], -1 for noise
    hit_forward: np.ndarray  # bool   [H], crossing lies after the track's PCA
    trk_phi0: np.ndarray     # float64 [T] perigee azimuth
    trk_qpt: np.ndarray      # float64 [T] q/pT, GeV^-1
    trk_d0: np.ndarray       # float64 [T] signed impact parameter, cm
    trk_vertex: np.ndarray   # int32  [T], -1 = prompt
    trk_nhits: np.ndarray    # int32  [T]
    trk_nfwd: np.ndarray     # int32  [T], hits after the PCA
    vtx_rho: np.ndarray      # float64 [V]
    vtx_theta: np.ndarray    # float64 [V]
    vtx_kind: np.ndarray     # int32  [V], 0 = displaced jet, 1 = black-hole-like
    vtx_ntrk: np.ndarray     # int32  [V]
    meta: dict = field(default_factory=dict)

    @property
    def n_hits(self) -> int:
        return int(self.r.shape[0])


def _wrap(a):
    return (np.asarray(a) + np.pi) % (2.0 * np.pi) - np.pi


def perigee(vx, vy, psi, kappa):
    """Perigee (phi0, d0) of the circle through V=(vx,vy) with direction psi.

    Plane geometry only: the centre is C = V + (1/kappa) * left-normal(psi);
    the PCA is the circle point nearest the origin, C - R*C/|C| with
    R = 1/|kappa|, and the left normal at the PCA is sign(kappa)*C/|C|.
    """
    if kappa == 0.0:
        nx, ny = -np.sin(psi), np.cos(psi)
        return float(_wrap(psi)), float(vx * nx + vy * ny)
    cx = vx - np.sin(psi) / kappa
    cy = vy + np.cos(psi) / kappa
    dc = np.hypot(cx, cy)
    s = 1.0 if kappa > 0 else -1.0
    n0x, n0y = s * cx / dc, s * cy / dc
    d0 = s * dc - 1.0 / kappa
    phi0 = np.arctan2(-n0x, n0y)
    return float(phi0), float(d0)


def crossings(vx, vy, psi, kappa, radii=RADII):
    """Layer crossings of one track in arc-length order.

    Returns a list of (layer index, x, y, after_pca) for every intersection of
    the track circle with a layer circle that lies on the path from V to the
    first turn (largest distance from the origin).
    """
    out = []
    if kappa == 0.0:
        tx, ty = np.cos(psi), np.sin(psi)
        vt = vx * tx + vy * ty
        vv = vx * vx + vy * vy
        for li, rl in enumerate(radii):
            disc = vt * vt - (vv - rl * rl)
            if disc < 0:
                continue
            sq = np.sqrt(disc)
            for s_arc in (-vt - sq, -vt + sq):
                if s_arc > 0:
                    out.append((s_arc, li, vx + s_arc * tx, vy + s_arc * ty, s_arc + vt > 0))
        out.sort()
        return [(li, x, y, f) for _, li, x, y, f in out]
    rad = 1.0 / abs(kappa)
    sgn = 1.0 if kappa > 0 else -1.0
    cx = vx - np.sin(psi) / kappa
    cy = vy + np.cos(psi) / kappa
    dc = np.hypot(cx, cy)
    ux, uy = cx / dc, cy / dc
    th_v = np.arctan2(vy - cy, vx - cx)

    def arc(px, py):
        return (sgn * (np.arctan2(py - cy, px - cx) - th_v)) % (2.0 * np.pi)

    # first turn: the farthest circle point from the origin, C + R*C/|C|;
    # the PCA is the nearest one, C - R*C/|C|.
    apex = arc(cx + rad * ux, cy + rad * uy)
    pca = arc(cx - rad * ux, cy - rad * uy)
    for li, rl in enumerate(radii):
        a = (rl * rl - rad * rad + dc * dc) / (2.0 * dc)
        h2 = rl * rl - a * a
        if h2 < 0:
            continue
        h = np.sqrt(h2)
        for sign in (1.0, -1.0):
            px = a * ux - sign * h * uy
            py = a * uy + sign * h * ux
            t = arc(px, py)
            if 0.0 < t <= apex:
                # after the PCA iff the PCA was passed before reaching it (or
                # the production point already lies beyond the PCA)
                after = (pca >= apex) or (t > pca)
                out.append((t, li, px, py, bool(after)))
    out.sort()
    return [(li, x, y, f) for _, li, x, y, f in out]


class _Builder:
    def __init__(self, rng, bfield=B_TESLA, radii=RADII, smear=SMEAR_CM, smear_xy=0.0):
        self.rng = rng
        self.bfield = bfield
        self.radii = radii
        self.smear = smear
        self.smear_xy = smear_xy  # Gaussian smear of x and y each (then r moves too)
        self.hits = []          # (r, phi, layer, track, forward)
        self.trk = []           # (phi0, qpt, d0, vertex, nhits, nfwd)
        self.vtx = []           # (rho, theta, kind, ntrk)

    def add_track(self, vx, vy, psi, qpt, vertex=-1):
        kap = float(kappa_of(qpt, self.bfield))
        phi0, d0 = perigee(vx, vy, psi, kap)
        tid = len(self.trk)
        nh = nf = 0
        for li, x, y, fwd in crossings(vx, vy, psi, kap, self.radii):
            rl = self.radii[li]
            if self.smear_xy > 0:
                x = x + self.rng.normal(0.0, self.smear_xy)
                y = y + self.rng.normal(0.0, self.smear_xy)
                rl = float(np.hypot(x, y))
            ph = np.arctan2(y, x)
            if self.smear > 0:
                ph += self.rng.normal(0.0, self.smear / rl)
            self.hits.append((rl, float(_wrap(ph)), li, tid, fwd))
            nh += 1
            nf += int(fwd)
        self.trk.append((phi0, float(qpt), d0, vertex, nh, nf))
        return tid

    def add_perigee_track(self, phi0, qpt, d0, vertex=-1):
        """Track produced at its own PCA (so every hit is after the PCA)."""
        vx, vy = -d0 * np.sin(phi0), d0 * np.cos(phi0)
        return self.add_track(vx, vy, phi0, qpt, vertex)

    def add_noise(self, n):
        li = self.rng.integers(0, len(self.radii), size=n)
        ph = self.rng.uniform(-np.pi, np.pi, size=n)
        for a, b in zip(li, ph):
            rl = self.radii[int(a)]
            if self.smear_xy > 0:
                rl = float(rl + self.rng.normal(0.0, self.smear_xy))
            self.hits.append((rl, float(b), int(a), -1, False))

    def add_vertex(self, rho, theta, kind, ntrk):
        self.vtx.append((rho, theta, kind, ntrk))
        return len(self.vtx) - 1

    def build(self, shuffle=True, meta=None) -> Event:
        n = len(self.hits)
        order = self.rng.permutation(n) if shuffle else np.arange(n)
        h = [self.hits[i] for i in order]
        r = np.array([x[0] for x in h], dtype=np.float64)
        ph = np.array([x[1] for x in h], dtype=np.float64)
        phi32 = ph.astype(np.float32)
        # keep the float32 azimuth inside [-pi, pi)
        phi32 = np.where(phi32 >= np.float32(np.pi), np.float32(-np.pi), phi32).astype(np.float32)
        t = self.trk
        v = self.vtx
        return Event(
            r=r.astype(np.float32),
            phi=phi32,
            layer=np.array([x[2] for x in h], dtype=np.uint8),
            hit_track=np.array([x[3] for x in h], dtype=np.int32),
            hit_forward=np.array([x[4] for x in h], dtype=bool),
            trk_phi0=np.array([x[0] for x in t], dtype=np.float64),
            trk_qpt=np.array([x[1] for x in t], dtype=np.float64),
            trk_d0=np.array([x[2] for x in t], dtype=np.float64),
            trk_vertex=np.array([x[3] for x in t], dtype=np.int32),
            trk_nhits=np.array([x[4] for x in t], dtype=np.int32),
            trk_nfwd=np.array([x[5] for x in t], dtype=np.int32),
            vtx_rho=np.array([x[0] for x in v], dtype=np.float64),
            vtx_theta=np.array([x[1] for x in v], dtype=np.float64),
            vtx_kind=np.array([x[2] for x in v], dtype=np.int32),
            vtx_ntrk=np.array([x[3] for x in v], dtype=np.int32),
            meta=dict(meta or {}),
        )


def _qpt_uniform(rng, lo=0.1, hi=1.0):
    return float(rng.choice((-1.0, 1.0)) * rng.uniform(lo, hi))


def _displaced_jet(b, rng, ntrk, rho_lo=5.0, rho_hi=50.0, d0_max=20.0,
                   dmin_deg=15.0, dmax_deg=60.0):
    """A neutral decaying at radius U[rho_lo, rho_hi] into ntrk charged tracks
    spread uniformly within a half-angle U[dmin, dmax] of its flight azimuth."""
    theta = rng.uniform(-np.pi, np.pi)
    rho = rng.uniform(rho_lo, rho_hi)
    vid = b.add_vertex(rho, theta, 0, ntrk)
    vx, vy = rho * np.cos(theta), rho * np.sin(theta)
    delta = np.deg2rad(rng.uniform(dmin_deg, dmax_deg))
    for _ in range(ntrk):
        for _attempt in range(1000):
            psi = theta + rng.uniform(-delta, delta)
            qpt = _qpt_uniform(rng)
            _, d0 = perigee(vx, vy, psi, float(kappa_of(qpt, b.bfield)))
            if abs(d0) <= d0_max:
                break
        b.add_track(vx, vy, psi, qpt, vid)
    return vid


def _black_hole(b, rng, ntrk, rho_lo=5.0, rho_hi=15.0, pt_lo=0.5, pt_hi=2.0):
    """High-multiplicity isotropic decay of soft particles a few cm out."""
    theta = rng.uniform(-np.pi, np.pi)
    rho = rng.uniform(rho_lo, rho_hi)
    vid = b.add_vertex(rho, theta, 1, ntrk)
    vx, vy = rho * np.cos(theta), rho * np.sin(theta)
    for _ in range(ntrk):
        psi = rng.uniform(-np.pi, np.pi)
        qpt = float(rng.choice((-1.0, 1.0)) / rng.uniform(pt_lo, pt_hi))
        b.add_track(vx, vy, psi, qpt, vid)
    return vid


def make_event(config: int, seed: int, **kw) -> Event:
    """Seeded event of one of the standard workloads.

    config 1: 20 prompt tracks (d0=0, q/pT = +-U[0.1, 1]) + 50 noise hits.
    config 2: 300 prompt + 2 displaced neutrals x 8 tracks (|d0| <= 20 cm)
              + 500 noise hits.
    config 3: 5000 prompt tracks with pT ~ pT^-3 above 0.5 GeV, 4 displaced
              jets x 10 tracks, one black-hole-like vertex of 60 isotropic soft
              tracks, 5000 noise hits (pile-up z spread is irrelevant in the
              transverse plane).
    Keyword overrides: n_prompt, n_noise, n_jets, jet_ntrk, n_bh, bh_ntrk.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    b = _Builder(rng)
    if config == 1:
        n_prompt, n_noise, n_jets, jet_ntrk, n_bh, bh_ntrk = 20, 50, 0, 8, 0, 60
        soft = False
    elif config == 2:
        n_prompt, n_noise, n_jets, jet_ntrk, n_bh, bh_ntrk = 300, 500, 2, 8, 0, 60
        soft = False
    elif config == 3:
        n_prompt, n_noise, n_jets, jet_ntrk, n_bh, bh_ntrk = 5000, 5000, 4, 10, 1, 60
        soft = True
    else:
        raise ValueError(f"unknown config {config}")
    n_prompt = kw.get("n_prompt", n_prompt)
    n_noise = kw.get("n_noise", n_noise)
    n_jets = kw.get("n_jets", n_jets)
    jet_ntrk = kw.get("jet_ntrk", jet_ntrk)
    n_bh = kw.get("n_bh", n_bh)
    bh_ntrk = kw.get("bh_ntrk", bh_ntrk)
    for _ in range(n_prompt):
        phi0 = rng.uniform(-np.pi, np.pi)
        if soft:
            # pT = 0.5 * U^(-1/2) has density proportional to pT^-3 above 0.5
            pt = 0.5 * (1.0 - rng.uniform(0.0, 1.0)) ** -0.5
            qpt = float(rng.choice((-1.0, 1.0)) / pt)
        else:
            qpt = _qpt_uniform(rng)
        b.add_perigee_track(phi0, qpt, 0.0)
    for _ in range(n_jets):
        _displaced_jet(b, rng, jet_ntrk)
    for _ in range(n_bh):
        _black_hole(b, rng, bh_ntrk)
    b.add_noise(n_noise)
    return b.build(meta=dict(config=config, seed=seed))


def make_tracks_event(tracks, n_noise=0, seed=0, smear=SMEAR_CM, shuffle=True,
                      radii=RADII, bfield=B_TESLA) -> Event:
    """Event from explicit perigee tracks [(phi0, qpt, d0), ...] (test helper)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = _Builder(rng, bfield=bfield, radii=radii, smear=smear)
    for phi0, qpt, d0 in tracks:
        b.add_perigee_track(float(phi0), float(qpt), float(d0))
    b.add_noise(n_noise)
    return b.build(shuffle=shuffle)


def make_vertex_event(rho, theta, psis, qpts, n_noise=0, seed=0, smear=SMEAR_CM,
                      radii=RADII, bfield=B_TESLA, prompt=()) -> Event:
    """Event with tracks produced at one vertex, after prompt tracks
    [(phi0, qpt), ...] from the beam line (test helper)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = _Builder(rng, bfield=bfield, radii=radii, smear=smear)
    for phi0, q in prompt:
        b.add_perigee_track(float(phi0), float(q), 0.0)
    vid = b.add_vertex(rho, theta, 0, len(psis))
    vx, vy = rho * np.cos(theta), rho * np.sin(theta)
    for psi, q in zip(psis, qpts):
        b.add_track(vx, vy, float(psi), float(q), vid)
    b.add_noise(n_noise)
    return b.build()


def random_hits(n, seed, r_lo=1.0, r_hi=110.0, bad_fraction=0.0):
    """Unstructured hits (uniform r, phi) for parity sweeps; optionally a
    fraction of invalid values (NaN, r <= 0, |phi| > 4) that cast no votes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.uniform(r_lo, r_hi, size=n).astype(np.float32)
    phi = rng.uniform(-np.pi, np.pi, size=n).astype(np.float32)
    layer = rng.integers(0, 10, size=n).astype(np.uint8)
    if bad_fraction > 0 and n:
        nb = max(1, int(n * bad_fraction))
        idx = rng.choice(n, size=nb, replace=False)
        kinds = rng.integers(0, 5, size=nb)
        for i, kd in zip(idx, kinds):
            if kd == 0:
                r[i] = np.nan
            elif kd == 1:
                r[i] = -abs(r[i])
            elif kd == 2:
                phi[i] = np.float32(4.5)
            elif kd == 3:
                phi[i] = np.nan
            else:
                r[i] = 0.0
    return r, phi, layer


def make_serving_event(kind: int, seed: int, h_lo: int = 2000, h_hi: int = 60000) -> Event:
    """Event of a mixed trigger stream: kind 0 is a prompt-only event of the
    2D workload's composition (20% noise hits), kind 1 an event of the 3D
    workload's composition (two displaced neutrals, 14% noise hits); the
    prompt and noise counts are scaled so the hit count is close to a target
    drawn from U[h_lo, h_hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    target = int(rng.uniform(h_lo, h_hi))
    if kind == 0:
        n_noise = int(0.2 * target)
        return make_event(1, seed, n_prompt=max(1, round((target - n_noise) / 10.0)),
                          n_noise=n_noise)
    n_noise = int(0.14 * target)
    return make_event(2, seed, n_prompt=max(1, round((target - n_noise - 160) / 9.7)),
                      n_noise=n_noise)


# The paper's toy detector (section "Hough Transform Algorithm", sample input
# data): transverse plane, 3.0 cm beam pipe, ten evenly spaced layers out to
# 110 cm (here at 11, 22, ..., 110 cm), 0.4 mm resolution in x and in y.
PAPER_RADII = tuple(11.0 * (i + 1) for i in range(10))
PAPER_SMEAR_XY = 0.04


def make_paper_event(seed: int, n_prompt: int = 0, n_jets: int = 1, jet_ntrk: int = 10,
                     rho_lo: float = 4.0, rho_hi: float = 10.0) -> Event:
    """Event of the paper's efficiency studies on its toy detector: n_prompt
    tracks from the interaction point and n_jets displaced jets of jet_ntrk
    tracks each, dispersion half-angles U[15, 60] degrees; jet vertices at
    radius U[rho_lo, rho_hi], inside the first layer so that their tracks
    have ten hits, as in the studies."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = _Builder(rng, radii=PAPER_RADII, smear=0.0, smear_xy=PAPER_SMEAR_XY)
    for _ in range(n_prompt):
        b.add_perigee_track(rng.uniform(-np.pi, np.pi), _qpt_uniform(rng), 0.0)
    for _ in range(n_jets):
        _displaced_jet(b, rng, jet_ntrk, rho_lo=rho_lo, rho_hi=rho_hi)
    return b.build(meta=dict(paper=True, seed=seed, n_prompt=n_prompt, n_jets=n_jets,
                             jet_ntrk=jet_ntrk))

