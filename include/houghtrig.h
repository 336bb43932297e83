/*
 * houghtrig -- Hough-transform track trigger for displaced jets and
 * black-hole-like vertices on AMD Instinct MI355X (gfx950).
 *
 * The method is that of Halyo, LeGresley and Lujan, "Massively Parallel
 * Computing and the Search for Jets and Black Holes at the LHC" (arXiv
 * 1309.6275):
 *   - section "Hough Transform Algorithm": every track instance starts with
 *     zero votes, each hit adds one vote to every instance that would contain
 *     it, and local maxima of the vote space are track candidates;
 *   - section "Jet and Black Hole Detection": candidates are refined and a
 *     second Hough transform over the tracks finds the vertices they share;
 *     features close to the interaction point are filtered out by a lower
 *     bound on the radius; the same local-maximum finder serves both
 *     transforms.
 *
 * Conventions shared by every call:
 *   - All array arguments are DEVICE pointers owned by the caller, except the
 *     small configuration structs, which are host pointers read during the
 *     call.  No call allocates device memory; a plan owns its constant
 *     tables and scratch.
 *   - Every compute call is asynchronous on `stream` (a hipStream_t; NULL is
 *     the default stream).  Counts are written to device memory, so the
 *     caller synchronises only when it reads them.
 *   - Argument errors are detected on the host before anything is launched
 *     and return HT_EINVAL (HT_EUNSUPPORTED for sizes beyond the kernels'
 *     limits); a failing HIP call returns HT_EDEVICE.
 *   - Invalid hit values (r outside (0, 1e4) cm, |phi| > 4 rad, NaN) are not
 *     errors: such hits cast no votes and are never associated.
 *   - Output lists that exceed their capacity are truncated in order; the
 *     reported count is the full count.
 *   - A plan's scratch is shared by the calls made with it: calls with one
 *     plan must be ordered (one stream, or synchronised streams).  Use one
 *     plan per concurrent stream.
 */
#ifndef HOUGHTRIG_H
#define HOUGHTRIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HT_OK = 0,
  HT_EINVAL = -1,        /* bad argument (null pointer, size out of range) */
  HT_ENOMEM = -2,        /* device allocation failed (plan creation only) */
  HT_EDEVICE = -3,       /* a HIP runtime call failed */
  HT_EUNSUPPORTED = -4,  /* valid request beyond the library's kernel limits */
  HT_EBUSY = -5          /* serving loop: every slot busy and the wait queue full */
};

#define HT_MAX_LAYERS 16

/* Accumulator grid.  Cells (i, j, k) are phi0 x q/pT x d0 bins at the bin
 * centres; the accumulator is int32 [n_d0][n_qpt][n_phi] with phi0 fastest,
 * cell index lin = (k * n_qpt + j) * n_phi + i.  phi0 covers [-pi, pi)
 * periodically; bins are [lo + n w, lo + (n+1) w).  n_d0 = 1 with
 * d0_lo = d0_hi = 0 is the prompt ("2D") transform; n_qpt = 1 with
 * qpt_lo = qpt_hi = 0 is the straight-line transform. */
typedef struct {
  int32_t n_phi, n_qpt, n_d0;
  float qpt_lo, qpt_hi;   /* q/pT [GeV^-1] */
  float d0_lo, d0_hi;     /* signed transverse impact parameter [cm] */
  float bfield;           /* solenoid field [T], > 0 */
} ht_grid;

/* Sizes the plan's scratch is allocated for. */
typedef struct {
  int32_t max_hits;        /* hits per call, <= 65535 */
  int32_t max_peaks;       /* peak-list capacity assoc_cluster accepts, <= 2^26 */
  int32_t max_member_cap;  /* largest ht_cluster_cfg.member_cap used */
  int32_t max_tracks;      /* largest track capacity used */
  int32_t max_vertex_cells;/* largest n_rho * n_theta used */
  int32_t max_n_rho;       /* largest n_rho used */
} ht_limits;

typedef struct { int32_t lin, votes; } ht_peak;

/* Candidate refinement and second-transform settings (see assoc_cluster). */
typedef struct {
  int32_t win_bins;        /* phi0 bins added to the cell-compatible member window */
  int32_t min_layers;      /* inlier layers a candidate needs, owned hits a track needs */
  int32_t seed_k;          /* members per seed layer tried, 1..4 */
  int32_t member_cap;      /* candidates with more member hits are dropped */
  float road_sigmas;       /* inlier road half-width in units of sigma_rphi */
  float box_margin;        /* seed circle must lie in the cell widened by this many bins */
  float sigma_rphi;        /* hit r-phi resolution [cm] */
  int32_t fit_iters;       /* Gauss-Newton iterations of the refit */
  int32_t n_rho, n_theta;  /* vertex accumulator extent, theta fastest */
  float rho_lo, rho_hi;    /* vertex radius range [cm]; rho_lo is the IP filter */
  int32_t vtx_min_votes;   /* vertex peak threshold */
  int32_t bh_min_tracks;   /* black-hole-like: at least this many member tracks */
  float bh_max_isotropy;   /* ... and |mean member direction| at most this */
  float vtx_min_d0;        /* tracks with seed |d0| below this [cm] cast no vertex votes (0: all vote) */
  int32_t fit_kind;        /* refit: 0 Gauss-Newton least squares, 1 extended Kalman filter */
  int32_t vtx_two_branch;  /* 0: vertex votes on the outgoing branch only; 1: also on the
                              incoming branch (see assoc_cluster) */
} ht_cluster_cfg;

typedef struct {
  int32_t peak;            /* index into the peak list */
  int32_t lin, votes;      /* the peak cell and its votes */
  int32_t n_layers;        /* layers with a member hit */
  int32_t n_inliers;       /* layers with a hit on the seed road */
  int32_t n_owned;         /* inlier hits this track owns */
  int32_t status;          /* refit: 0 ok, 1 |u| >= 1 on a hit, 2 singular normal matrix */
  float seed_ss;           /* sum of squared seed distances of the inliers [cm^2] */
  float phi0, qpt, d0, chi2;  /* refit perigee parameters and chi2 (-1 if status != 0) */
  float r_first;           /* smallest radius among owned hits [cm] */
  int32_t hits[HT_MAX_LAYERS]; /* owned hit on each layer, -1 if none */
} ht_track;

typedef struct {
  int32_t lin, votes;      /* vertex cell (m * n_theta + t) and its votes */
  int32_t n_tracks, kind;  /* members; kind 0 displaced jet, 1 black-hole-like */
  float rho, theta, isotropy; /* cell centre [cm, rad]; |mean member direction| */
  int32_t member_begin;    /* offset of this object's members in the member list */
} ht_object;

/* Outputs of assoc_cluster (device pointers; vacc may be NULL). */
typedef struct {
  int32_t* hit_owner;      /* [n_hits] track owning the hit, -1 if none */
  ht_track* tracks;        /* [track_cap] surviving tracks in peak order */
  int32_t track_cap;
  ht_object* objects;      /* [object_cap] vertex objects in cell order */
  int32_t object_cap;
  int32_t* members;        /* [member_cap] member track indices, object by object */
  int32_t member_cap;
  int32_t* vacc;           /* [n_rho * n_theta] vertex accumulator, or NULL */
  int32_t* counts;         /* [8]: candidates, tracks, objects, object members, candidates
                              over member_cap, (candidate, member) pairs of the others,
                              road tests of the seed search ((admissible seed circle,
                              member) pairs), 0; a count above INT32_MAX reads INT32_MAX */
  unsigned long long* work;/* [2] device, or NULL: the seed search's work as 64-bit totals:
                              [0] road tests the method defines (as counts[6], unclamped),
                              [1] float64 circle distances actually computed (members that
                              pass the float32 pre-filter on lanes still able to reach
                              min_layers, plus the tied lanes' distance sums) */
} ht_cluster_out;

typedef struct ht_plan ht_plan;

/* Create a plan for `grid` on the current HIP device: builds the constant
 * tables (bin centres computed in float64, rounded once to float32) and
 * allocates scratch for `limits`.  Host-synchronous; may allocate. */
int ht_plan_create(const ht_grid* grid, const ht_limits* limits, ht_plan** out);
void ht_plan_destroy(ht_plan* plan);
const char* ht_strerror(int status);

/* hough_vote -- the first transform (paper, section "Hough Transform
 * Algorithm": each datum adds a vote to every instance that would include
 * it).  For every valid hit and every column (q/pT_j, d0_k) the hit votes
 * once, for the phi0 bin of
 *   u = ((KAP_j * r^2 + Q_jk) * (1/r)) * T_jk,   phi0 = phi - asin_f(u)
 * (no vote unless |u| <= 1), with KAP_j = -0.299792458e-2 B q/pT_j,
 * Q_jk = KAP_j d0_k^2 + 2 d0_k, T_jk = 0.5 / (1 + KAP_j d0_k): the outgoing
 * branch of the circle through the perigee (d0, phi0) with curvature KAP_j.
 * asin_f is Abramowitz & Stegun 4.4.46 in float32; every operation is one
 * IEEE float32 rounding, no fused multiply-add.
 *   r, phi   [n_hits] float32 hit radius [cm] and azimuth [rad]
 *   acc      [n_d0 * n_qpt * n_phi] int32, fully overwritten
 *   n_votes  device uint64 receiving the total vote count, or NULL
 * n_hits may be 0 (acc is zeroed).  Returns HT_EUNSUPPORTED when n_hits
 * exceeds 65535 or the plan's max_hits. */
int hough_vote(const ht_plan* plan, const float* r, const float* phi, int32_t n_hits,
               int32_t* acc, unsigned long long* n_votes, void* stream);

/* hough_vote_cell -- band (cell) variant of hough_vote (the paper's feature
 * instances are cells of the parameter space, section "Hough Transform
 * Algorithm"): a valid hit votes once for every phi0 bin its curve reaches
 * while (kappa, d0) range over the column's cell, instead of the point at
 * the column centre.  u is increasing in kappa and d0 over the cell (for
 * r > |d0| and kappa^2 r^2 < (1 + kappa d0)^2 + 1), so the band lies between
 * the coordinates of two corners, each from the float32 formula of
 * hough_vote with that corner's tables (float64, rounded once):
 *   u_lo at (KAP = -c_B qpt_edge[j+1], d0_edge[k]),
 *   u_hi at (KAP = -c_B qpt_edge[j],   d0_edge[k+1]);
 * no vote when u_lo > 1 or u_hi < -1, else u clipped to [-1, 1],
 *   x_a = (phi - asin_f(u_hi) - PHI_LO) * INVW,
 *   x_b = (phi - asin_f(u_lo) - PHI_LO) * INVW,
 * and one vote in every bin from floor(min(x_a, x_b)) to floor(max(x_a,
 * x_b)), periodic (a band of n_phi or more bins votes once in every bin).
 * Arguments, layout, errors and n_votes (the total of band widths) as for
 * hough_vote.  The peak finder and assoc_cluster take its accumulator
 * unchanged. */
int hough_vote_cell(const ht_plan* plan, const float* r, const float* phi, int32_t n_hits,
                    int32_t* acc, unsigned long long* n_votes, void* stream);

/* hough_peaks -- local maxima of the accumulator (paper, section "Hough
 * Transform Algorithm"; reused for the second transform).  Cell c is a peak
 * iff acc[c] >= min_votes and for each of its 26 neighbours c+o inside the
 * q/pT and d0 range (phi0 periodic) acc[c] > acc[c+o] when o = (dk,dj,di) is
 * lexicographically negative and acc[c] >= acc[c+o] otherwise (a plateau
 * keeps its first cell).  Peaks are written sorted by lin.
 *   acc      accumulator of this plan's grid
 *   out      [capacity] peaks; the first `capacity` in lin order are written
 *   n_found  device int32 receiving the full peak count */
int hough_peaks(const ht_plan* plan, const int32_t* acc, int32_t min_votes, ht_peak* out,
                int32_t capacity, int32_t* n_found, void* stream);

/* hough_peaks_noalloc -- hough_peaks for callers that cannot allocate
 * device memory or create a plan: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same kernels, same
 * results (peaks, order, count) as hough_peaks with a plan of `grid`; no
 * allocation of any kind, no hipMemset.  The scratch (peak ballots and tile
 * counts) is a fixed device array inside the library, one copy per GPU, held
 * until the process ends; its device address is looked up once per GPU on
 * the first call there.  Every call on one GPU shares that copy: calls that
 * overlap on one GPU (concurrent streams) race and must be ordered by the
 * caller.  Nothing in it needs clearing between calls (every word read is
 * written first by the same call).
 *   grid     host pointer, the accumulator's grid (as for ht_plan_create)
 *   acc, min_votes, out, capacity, n_found  as for hough_peaks
 * Returns HT_EINVAL for a bad grid or pointer, HT_EUNSUPPORTED when the grid
 * has more than 2^24 cells (the array's size: 2 MiB of ballots, 256 KiB of
 * tile counts and 256 KiB of tile offsets), HT_EDEVICE when the array's
 * address cannot be found. */
int hough_peaks_noalloc(const ht_grid* grid, const int32_t* acc, int32_t min_votes, ht_peak* out,
                        int32_t capacity, int32_t* n_found, void* stream);

/* assoc_cluster -- candidate refinement, duplicate cleaning, refit and the
 * second transform (paper, section "Jet and Black Hole Detection").
 *   members    valid hits whose phi0 coordinate x in the peak's column lies
 *              within 0.5 + win_bins + 1.5 INVW (hd0/r + hk r/2) / sqrt(1-u^2)
 *              bins of the cell centre (hd0, hk: half column widths in d0
 *              and curvature; u as in hough_vote);
 *              more than member_cap members drops the candidate;
 *   seed       over the outer min(n, min_layers) member layers, circles
 *              through the seed_k nearest-centre members of the innermost,
 *              middle and outermost of them (through the beam line and two
 *              hits on the prompt grid), inliers = per layer the member
 *              within road_sigmas * sigma_rphi of the circle; best seed =
 *              most inlier layers, then smallest squared distance sum;
 *              candidates need min_layers inlier layers;
 *   ownership  each inlier hit goes to the candidate with the most inlier
 *              layers, then the smallest seed sum (float32), then the lowest
 *              cell; tracks own at least min_layers of their hits;
 *   refit      float64 Gauss-Newton of (phi0, kappa, d0) from the seed, or
 *              (fit_kind 1) a Kalman filter over the hits in increasing
 *              radius of the deviation from a reference state (the seed,
 *              then the previous pass), the azimuth model linearised at the
 *              reference: weak prior diag(0.1^2, 0.01^2, 10^2), no process
 *              noise, fit_iters passes;
 *   vertices   each track votes for the (rho, theta) cells its seed circle
 *              crosses between |d0| and its first hit radius, rho >= rho_lo;
 *              vertex peaks by the local-maximum rule; members are tracks
 *              within one cell; black-hole-like when >= bh_min_tracks members
 *              and |mean perigee direction| <= bh_max_isotropy; tracks whose seed
 *              circle passes within vtx_min_d0 of the beam line are
 *              features at the interaction point and cast no vertex votes.
 *              With vtx_two_branch = 1 each track also votes for the cells
 *              its circle crosses before the perigee (the path of a track
 *              sent from its vertex towards the beam line, as half of an
 *              isotropic decay's are), from |d0| to rho_hi; a cell covered
 *              by both arcs of a row gets one vote, and membership counts
 *              either arc.
 *   r, phi, layer  [n_hits] hits (layer index increasing with radius)
 *   peaks, n_peaks peak list and device count from hough_peaks (sorted by
 *                  lin, no cell twice); entries beyond min(*n_peaks,
 *                  peak_cap) are ignored; entries with lin outside the grid
 *                  are no candidates; any other list gives unspecified
 *                  results (memory accesses stay in bounds)
 *   acc            NULL, or the accumulator hough_vote (or hough_vote_n)
 *                  wrote for these hits with this plan (device, read only).
 *                  Results are the same either way; with it, a candidate
 *                  whose member count provably exceeds member_cap is dropped
 *                  before the member search: every valid hit with a layer
 *                  below HT_MAX_LAYERS that votes within win_bins bins of
 *                  the cell in its column is a member, so the votes of those
 *                  2 win_bins + 1 cells, less the valid hits of higher
 *                  layers, bound the count from below.  Used on grids with
 *                  a d0 axis (half d0 width >= 1e-20 cm) and
 *                  n_phi >= 4 (win_bins + 1); ignored otherwise.  Any other
 *                  accumulator (the band vote's included) gives unspecified
 *                  results.
 *   out            outputs (device pointers) */
int assoc_cluster(const ht_plan* plan, const float* r, const float* phi, const uint8_t* layer,
                  int32_t n_hits, const ht_peak* peaks, const int32_t* n_peaks,
                  int32_t peak_cap, const int32_t* acc, const ht_cluster_cfg* cfg,
                  const ht_cluster_out* out, void* stream);

/* hough_vote_n, assoc_cluster_n -- hough_vote and assoc_cluster with the
 * event's hit count read on the device from *n_hits_dev (clamped to
 * [0, n_hits_max]), for hit counts that are produced on the device (the
 * kept hits of ht_compact_hits) so that no host synchronisation sits
 * between two passes.  n_hits_max bounds the buffers and takes the limits
 * n_hits has in the plain calls; hit_owner entries beyond the device count
 * are not written.  n_hits_dev must not be NULL (HT_EINVAL). */
int hough_vote_n(const ht_plan* plan, const float* r, const float* phi, int32_t n_hits_max,
                 const int32_t* n_hits_dev, int32_t* acc, unsigned long long* n_votes,
                 void* stream);
int assoc_cluster_n(const ht_plan* plan, const float* r, const float* phi, const uint8_t* layer,
                    int32_t n_hits_max, const int32_t* n_hits_dev, const ht_peak* peaks,
                    const int32_t* n_peaks, int32_t peak_cap, const int32_t* acc,
                    const ht_cluster_cfg* cfg, const ht_cluster_out* out, void* stream);

/* ---- Batched launches ----------------------------------------------------
 * hough_batch -- hough_vote, hough_peaks and assoc_cluster for n_events
 * (1 .. HT_MAX_BATCH) events of one grid kind, each kernel launched once for
 * all of them (the event is a grid dimension of every launch), for events
 * too small to fill the chip alone (the trigger's many small events, section
 * "Physics Motivation").  Results are exactly those of the three calls made
 * event by event.  Event b uses its own plan (its scratch); the plans share
 * the grid; the events share the hit bound n_hits_max, the peak threshold and
 * capacity, the cluster configuration and the output capacities.
 *   plan        this event's plan (created for the shared grid)
 *   r, phi, layer, n_hits_dev   device hits and device hit count (<= n_hits_max)
 *   acc         device accumulator of the grid (written)
 *   peaks, n_peaks  device peak list [peak_cap] and count (written)
 *   out         outputs as for assoc_cluster (the accumulator bound of
 *               assoc_cluster is used with each event's accumulator)
 * Returns HT_EINVAL for a null pointer or mismatched plans or capacities,
 * HT_EUNSUPPORTED for sizes beyond a plan's limits. */
#define HT_MAX_BATCH 4
typedef struct {
  const ht_plan* plan;
  const float* r;
  const float* phi;
  const uint8_t* layer;
  const int32_t* n_hits_dev;
  int32_t* acc;
  ht_peak* peaks;
  int32_t* n_peaks;
  ht_cluster_out out;
} ht_batch_event;
int hough_batch(int32_t n_events, const ht_batch_event* events, int32_t n_hits_max,
                int32_t min_votes, int32_t peak_cap, const ht_cluster_cfg* cfg, void* stream);

/* Iterative hit removal (paper, section "Current Tracker and Tracking
 * Algorithm": earlier passes find the easier, prompt tracks, whose hits are
 * then removed so that later passes search for displaced tracks among far
 * fewer combinations).  Typical use: a prompt pass (hough_vote,
 * hough_peaks, assoc_cluster on a one-column d0 grid), ht_compact_hits on
 * its hit_owner, a displaced pass on the kept hits (hough_vote_n,
 * hough_peaks, assoc_cluster_n with n_out as the hit count), then
 * ht_remap_track_hits so that that pass's tracks name hits of the event.
 *
 * ht_compact_hits -- keeps the hits with hit_owner < 0, in event order.
 *   r, phi, layer  [n_hits] device hits of the event
 *   hit_owner      [n_hits] device owner array of assoc_cluster
 *   out_r, out_phi, out_layer, out_index
 *                  [n_hits] device outputs; out_index[i] is the event index
 *                  of kept hit i
 *   n_out          device int32 receiving the number of kept hits
 * n_hits is 0..65535 (HT_EUNSUPPORTED above); outputs must not overlap the
 * inputs.  Allocates nothing; one kernel on `stream`.
 *
 * ht_remap_track_hits -- replaces every hit index h >= 0 of the first
 * min(counts[1], track_cap) tracks by index[h] (h < n_index; others are
 * left alone).
 *   tracks, track_cap  device track array of an assoc_cluster call
 *   counts             that call's device counts
 *   index              [n_index] device out_index of ht_compact_hits */
int ht_compact_hits(const float* r, const float* phi, const uint8_t* layer, int32_t n_hits,
                    const int32_t* hit_owner, float* out_r, float* out_phi, uint8_t* out_layer,
                    int32_t* out_index, int32_t* n_out, void* stream);
int ht_remap_track_hits(ht_track* tracks, int32_t track_cap, const int32_t* counts,
                        const int32_t* index, int32_t n_index, void* stream);

/* Stage timing, for measurement.  After ht_profile_begin, each later call
 * on the plan records HIP events on its stream around its stages:
 *   HT_STAGE_VOTE     the vote kernel of hough_vote,
 *   HT_STAGE_PEAKS    the kernels of hough_peaks,
 *   HT_STAGE_ASSOC    all of assoc_cluster,
 *   HT_STAGE_MEMBERS  its member sweep (inside HT_STAGE_ASSOC),
 *   HT_STAGE_REFINE   its seed search (inside HT_STAGE_ASSOC).
 * At most `depth` launches per stage are recorded between two reads; later
 * ones are not timed.  ht_profile_read waits for the recorded events, ADDS
 * each stage's total milliseconds to ms[HT_STAGES] and its timed launches to
 * launches[HT_STAGES], and starts a new interval.  ht_profile_end stops
 * timing and frees the events.  Host calls; ht_profile_begin creates
 * 2 * depth * HT_STAGES events (HT_ENOMEM if that fails), the compute calls
 * still allocate nothing.  depth is 1..65536. */
enum { HT_STAGE_VOTE = 0, HT_STAGE_PEAKS = 1, HT_STAGE_ASSOC = 2, HT_STAGE_MEMBERS = 3,
       HT_STAGE_REFINE = 4, HT_STAGES = 5 };
int ht_profile_begin(ht_plan* plan, int32_t depth);
int ht_profile_read(ht_plan* plan, double* ms, int64_t* launches);
int ht_profile_end(ht_plan* plan);

/* ---- Learned peak filter ---------------------------------------------------
 * A 3D CNN scores each threshold peak from the 5 x 5 x 5 votes around it;
 * peaks scoring below a threshold are dropped before assoc_cluster (the
 * paper's call for efficiency and purity improvements of the peak finding,
 * section "Summary").  Network: conv3d 1->16 (3x3x3, valid), ReLU,
 * conv3d 16->16 (3x3x3, valid), ReLU, linear 16->64, ReLU, linear 64->1
 * (a logit).  Parameters: HT_CNN_PARAMS float32 in the order
 *   W1[16][27] b1[16] W2[16][16][27] b2[16] W3[64][16] b3[64] W4[64] b4
 * (tap t = (dk * 3 + dj) * 3 + di).  Arithmetic: bfloat16 inputs, weights
 * and activations (round to nearest even), float32 accumulation, bias after
 * the sum.  Windows: HT_CNN_WINDOW bfloat16 per peak, cell (dk, dj, di) in
 * -2..2 at index (dk+2)*25 + (dj+2)*5 + (di+2), votes * 1/16, phi0 periodic,
 * cells outside the q/pT and d0 range 0, entries 125..127 zero. */
#define HT_CNN_PARAMS 8529
#define HT_CNN_WINDOW 128

/* Device bytes of the workspace the CNN calls below need for max_windows
 * windows (training != 0: a training step; else inference). */
size_t ht_cnn_workspace_bytes(int32_t max_windows, int32_t training);
/* Windows of the first min(*n_peaks, cap) peaks (device count) of a peak
 * list of this plan's grid into win [cap][HT_CNN_WINDOW] (bfloat16 bits).
 * cap <= the plan's max_peaks. */
int ht_cnn_windows(const ht_plan* plan, const int32_t* acc, const ht_peak* peaks,
                   const int32_t* n_peaks, int32_t cap, uint16_t* win, void* stream);
/* Logits of n windows: n = min(*n_dev, n_max) when n_dev is not NULL (a
 * device count), else n_max.  params: device float32 [HT_CNN_PARAMS]. */
int ht_cnn_forward(const float* params, const uint16_t* win, const int32_t* n_dev, int32_t n_max,
                   float* logits, void* workspace, size_t workspace_bytes, void* stream);
/* One SGD step on n labelled windows (labels 0/1 as float): loss = mean over
 * the windows of w (softplus(z) - y z), w = pos_weight for y = 1, else 1;
 * mom <- momentum mom + grad; params <- params - lr mom.  *loss (device)
 * receives the loss before the step.  Gradients are summed with float32
 * atomics, so the last bits vary from run to run. */
int ht_cnn_train_step(float* params, float* mom, const uint16_t* win, const float* labels,
                      int32_t n, float lr, float momentum, float pos_weight, float* loss,
                      void* workspace, size_t workspace_bytes, void* stream);
/* Logits of the first min(*n_peaks, cap) peaks of a peak list of this
 * plan's grid, with each window built in LDS straight from the accumulator
 * (the windows of ht_cnn_windows, never written to device memory), in one
 * launch after the weights' packing.  Same logits as ht_cnn_windows followed
 * by ht_cnn_forward.  workspace as for ht_cnn_forward (inference);
 * cap <= the plan's max_peaks. */
int ht_cnn_score(const ht_plan* plan, const float* params, const int32_t* acc,
                 const ht_peak* peaks, const int32_t* n_peaks, int32_t cap, float* logits,
                 void* workspace, size_t workspace_bytes, void* stream);
/* Ordered compaction: the peaks among the first min(*n_peaks, cap) whose
 * logit is >= threshold, in their order, into out [out_cap]; *n_out (device)
 * receives their full count.  cap <= the plan's max_peaks. */
int ht_cnn_keep(const ht_plan* plan, const float* logits, const ht_peak* peaks,
                const int32_t* n_peaks, int32_t cap, float threshold, ht_peak* out,
                int32_t out_cap, int32_t* n_out, void* stream);

/* ---- Trigger serving loop --------------------------------------------------
 * Events of any size arrive one by one (the paper's trigger setting: each
 * event must be processed within the latency the trigger allows, section
 * "Physics Motivation"; copying the data to the GPU is part of the cost,
 * section "Preliminary Results").  The server owns a fixed set of slots;
 * each slot has its own stream and room for a batch of up to batch_max
 * events of one kind: per event a plan per grid kind and a resident
 * accumulator, peak list and outputs.  A slot runs one batch at a time:
 * copies of the hits to the device, one launch of the vote, of each peak
 * finder stage and of each assoc_cluster kernel for the whole batch (the
 * batched form of hough_batch), copies of the results to pinned host
 * memory.  A kind may carry the learned peak filter: its parameters
 * (HT_CNN_PARAMS float32, host memory, copied at creation) and threshold;
 * then ht_cnn_score and ht_cnn_keep run on each event's threshold peaks and
 * assoc_cluster refines the kept ones (the peak search improvement the
 * paper's summary names as future work).  With use_graphs the device part
 * of a slot is one HIP graph per kind and batch size, captured at creation
 * and replayed for every batch (hit counts travel in device memory).
 *
 * Admission.  The number of slots is the largest that fits hbm_budget (at
 * most max_slots).  An event submitted while nothing waits and a slot is
 * free starts at once, alone.  Otherwise it waits in a FIFO of queue_cap
 * (beyond it ht_server_submit returns HT_EBUSY: the event is shed).  When a
 * slot frees, the oldest waiting event starts; if it has at most
 * batch_max_hits hits, up to batch_max - 1 later waiting events of its kind
 * with at most batch_max_hits hits join it, oldest first (continuous
 * batching: batches form only while events wait).  With a work budget, the
 * events in flight share the device by their work (hits times the
 * q/pT x d0 columns of their kind): a batch starts only while the work in
 * flight plus its own stays within work_budget, or when nothing else runs
 * (an event too large for the budget runs alone).  Results are exactly
 * those of hough_vote, hough_peaks, (ht_cnn_score, ht_cnn_keep,)
 * assoc_cluster called one by one for the same event.  Single-threaded: one
 * thread calls submit and poll.  Host pointers throughout. */
#define HT_SERVER_MAX_KINDS 4

typedef struct {
  ht_grid grid;            /* accumulator grid of this kind of event */
  ht_cluster_cfg cluster;  /* refinement and vertex settings */
  int32_t min_votes;       /* peak threshold */
  int32_t peak_cap;        /* peak-list capacity per event */
  const float* cnn_params; /* NULL: no filter; else host float32 [HT_CNN_PARAMS] */
  float cnn_threshold;     /* peaks with a logit >= this are kept */
  int32_t reserved;        /* 0 */
} ht_server_kind;

typedef struct {
  int32_t n_kinds;                              /* 1 .. HT_SERVER_MAX_KINDS */
  ht_server_kind kinds[HT_SERVER_MAX_KINDS];
  int32_t max_hits;        /* hits per event, <= 65535 */
  int32_t track_cap;       /* tracks copied back per event */
  int32_t object_cap;      /* vertex objects copied back per event */
  int32_t member_cap;      /* object members copied back per event */
  int64_t hbm_budget;      /* device bytes the slots may use */
  int32_t max_slots;       /* concurrent batches at most, >= 1 */
  int32_t queue_cap;       /* events waiting for a slot at most, >= 0 */
  int32_t use_graphs;      /* 1: replay a captured HIP graph per slot, kind and batch size */
  int32_t reserved;        /* 0 */
  int64_t work_budget;     /* hit-columns in flight at most, 0: no limit */
  int32_t batch_max;       /* events per batch at most, 0 or 1 (no batching) .. HT_MAX_BATCH */
  int32_t batch_max_hits;  /* hits of an event that may share a batch at most, 1 .. max_hits
                              (ignored without batching); the slot's further event places are
                              sized for this many hits */
} ht_server_cfg;

/* Where the results of one event go (host memory, any pointer may be NULL;
 * at most the given capacities are written). */
typedef struct {
  ht_track* tracks;
  int32_t track_cap;
  int32_t* hit_owner;      /* [n_hits of the event] */
  ht_object* objects;
  int32_t object_cap;
  int32_t* members;
  int32_t member_cap;
} ht_server_out;

typedef struct {
  uint64_t tag;            /* as given to ht_server_submit */
  int32_t kind, n_hits;
  int32_t status;          /* HT_OK, or the error of a failed launch */
  int32_t n_peaks;         /* full peak count */
  int32_t counts[8];       /* as assoc_cluster's counts */
  double t_submit, t_start, t_done; /* host steady clock [s]: submitted, on a slot, seen done */
  double device_ms;        /* device time of the event's batch on its slot (HIP events) */
  int32_t n_kept;          /* peaks handed to assoc_cluster (n_peaks without a filter) */
  int32_t batch;           /* events in the event's batch */
} ht_server_result;

typedef struct ht_server ht_server;

/* Creates the slots (allocates device and pinned host memory, captures the
 * graphs).  HT_ENOMEM when not even one slot fits hbm_budget. */
int ht_server_create(const ht_server_cfg* cfg, ht_server** out);
/* Waits for the events on the device, then frees everything. */
int ht_server_destroy(ht_server* server);
/* Slot count and device bytes per slot. */
int ht_server_info(const ht_server* server, int32_t* n_slots, int64_t* slot_bytes);
/* Submits one event: r, phi, layer are host arrays of n_hits (copied before
 * the call returns); out says where its results go (the pointers must stay
 * valid until the event is returned by ht_server_poll).  Returns HT_EBUSY
 * when every slot is busy and the queue is full. */
int ht_server_submit(ht_server* server, int32_t kind, const float* r, const float* phi,
                     const uint8_t* layer, int32_t n_hits, const ht_server_out* out,
                     uint64_t tag);
/* Collects finished events into results (in completion order, whole
 * batches: max must be 0 or at least the batch size, else HT_EINVAL),
 * copies their outputs to the places given at submit, starts waiting events
 * on the freed slots.  wait != 0 blocks until at least one event is done or
 * none is pending. */
int ht_server_poll(ht_server* server, ht_server_result* results, int32_t max, int32_t wait,
                   int32_t* n_results);

/* ht_asin_f32 -- the canonical float32 arcsine of hough_vote, elementwise
 * over n device floats (for checking the formula on the device). */
int ht_asin_f32(const float* u, float* out, int64_t n, void* stream);

/* ht_sqrt_f64 -- the correctly rounded float64 square root the refinement's
 * seed circles use, elementwise over n device doubles (for checking it on
 * the device against an IEEE square root). */
int ht_sqrt_f64(const double* x, double* out, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif
#endif
