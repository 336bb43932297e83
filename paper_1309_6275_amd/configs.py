"""Workload definitions: accumulator grids, thresholds and clustering settings.

Numbers only -- no arithmetic of the method lives here.

* ``GRID_2D``: 256 phi0 x 256 q/pT, q/pT in [-1, 1] GeV^-1, d0 fixed at 0
  (the prompt, "2D tracking" transform of the paper's section "Hough
  Transform Algorithm"), peaks need 8 votes.
* ``GRID_3D``: 512 phi0 x 256 q/pT x 64 d0, d0 in [-20, 20] cm, peaks need 7
  votes (the paper tunes its peak finder for tracks of 7 or more hits,
  section "Preliminary Results").
* vertex grid for the second transform: 64 rho x 256 theta over rho in
  [4, 68) cm.  Its lower bound is the paper's filter of features near the
  interaction point (sections "Jet and Black Hole Detection", "Preliminary
  Results": a 3.0 cm beam pipe), placed at the innermost layer (4 cm): a
  vertex inside the first layer cannot be told from the beam line by the
  first hits of its tracks.
* black-hole-like objects: at least 20 member tracks and a mean member
  direction of length at most 0.75.  Only tracks leaving the vertex outward
  can vote for it (a vertex lies inside the first hit of its tracks), so an
  isotropic decay shows the outward hemisphere, length about 0.64; a jet of
  half-angle 60 degrees, the widest generated, has 0.83.
"""

B_TESLA = 3.8

GRID_2D = dict(n_phi=256, n_qpt=256, n_d0=1, qpt_lo=-1.0, qpt_hi=1.0, d0_lo=0.0, d0_hi=0.0,
               bfield=B_TESLA)
GRID_3D = dict(n_phi=512, n_qpt=256, n_d0=64, qpt_lo=-1.0, qpt_hi=1.0, d0_lo=-20.0, d0_hi=20.0,
               bfield=B_TESLA)

CLUSTER_2D = dict(win_bins=1, min_layers=8, seed_k=4, member_cap=256, road_sigmas=5.0,
                  box_margin=16.0, sigma_rphi=20e-4, fit_iters=3, n_rho=64, n_theta=256,
                  rho_lo=4.0, rho_hi=68.0, vtx_min_votes=5, bh_min_tracks=20,
                  bh_max_isotropy=0.75, vtx_min_d0=0.0, fit_kind=0)
CLUSTER_3D = dict(CLUSTER_2D, min_layers=7, member_cap=128)
# ~55k hits: about 700 hits fall in a cell's member window
CLUSTER_3D_DENSE = dict(CLUSTER_3D, member_cap=1024)

WORKLOADS = {
    1: dict(name="2D Hough, 20 prompt tracks + 50 noise hits, 256x256", grid=GRID_2D,
            min_votes=8, cluster=CLUSTER_2D, seed0=1_000_000),
    2: dict(name="displaced-jet event, 3D Hough 512x256x64, ~3.6k hits", grid=GRID_3D,
            min_votes=7, cluster=CLUSTER_3D, seed0=2_000_000),
    3: dict(name="high-pileup event, 3D Hough 512x256x64, ~55k hits", grid=GRID_3D,
            min_votes=7, cluster=CLUSTER_3D_DENSE, seed0=3_000_000),
}

# The paper's toy detector (evenly spaced layers to 110 cm, 0.4 mm
# resolution, 3.0 cm beam pipe): road and fit resolution 0.4 mm, vertex grid
# from the beam pipe radius (the paper's IP filter), peaks at 7 votes as in
# its studies.
CLUSTER_PAPER = dict(CLUSTER_3D, sigma_rphi=0.04, rho_lo=3.0, rho_hi=67.0, vtx_min_d0=0.2)
PAPER_WORKLOAD = dict(name="paper toy detector, 3D Hough 512x256x64", grid=GRID_3D,
                      min_votes=7, cluster=CLUSTER_PAPER, seed0=5_100_000)

# Iterative hit removal (the paper's tracker practice, section "Current
# Tracker and Tracking Algorithm"): a prompt pass on the 2D grid (beam-line
# seed), then the displaced-jet pass on the hits it leaves.
TWO_PASS = dict(name="prompt pass 2D 256x256, then displaced pass 3D 512x256x64",
                prompt=dict(grid=GRID_2D, min_votes=8, cluster=dict(CLUSTER_2D, member_cap=512)),
                displaced=dict(grid=GRID_3D, min_votes=7, cluster=CLUSTER_3D))
