/*
 * Plain CPU oracle of the Hough trigger path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the package smoke check and the benchmark's CPU
 * baseline leg may load this library.  It shares no source with the GPU
 * library: every table, formula and loop below is written out again here from
 * the method's definition so that the two can be compared.
 *
 * Method (paper, section "Hough Transform Algorithm"): every track instance
 * starts with zero votes; each hit adds one vote to every instance it could
 * belong to; local maxima of the vote space are track candidates.  Section
 * "Jet and Black Hole Detection" refines candidates and feeds them to a second
 * Hough transform whose local maxima, away from the interaction point, are
 * displaced vertices (jets or black-hole-like objects).
 *
 * All functions take host pointers, are synchronous and return 0 on success or
 * a negative value on an argument error.
 */
#ifndef HOUGH_ORACLE_H
#define HOUGH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_LAYERS 16

typedef struct {
  int32_t n_phi, n_qpt, n_d0; /* accumulator extent: phi0 fastest, then q/pT, then d0 */
  float qpt_lo, qpt_hi;       /* q/pT range [GeV^-1]; bins are [lo + n w, lo + (n+1) w) */
  float d0_lo, d0_hi;         /* d0 range [cm]; n_d0 = 1 with [0,0] is the 2D prompt grid */
  float bfield;               /* tesla, > 0 */
} or_grid;

typedef struct { int32_t lin, votes; } or_peak;

typedef struct {
  int32_t win_bins;        /* phi0 bins added to the cell-compatible member window */
  int32_t min_layers;      /* inlier layers a candidate needs (and owned hits a track needs) */
  int32_t seed_k;          /* members per seed layer tried, nearest the cell centre first */
  int32_t member_cap;      /* candidates with more members are dropped */
  float road_sigmas;       /* inlier road half-width in units of sigma_rphi */
  float box_margin;        /* seed circle must lie in the cell widened by this many bins */
  float sigma_rphi;        /* hit r-phi resolution [cm] */
  int32_t fit_iters;       /* Gauss-Newton iterations */
  int32_t n_rho, n_theta;  /* vertex accumulator extent (rho slow, theta fast) */
  float rho_lo, rho_hi;    /* vertex radius range [cm]; rho_lo is the IP filter */
  int32_t vtx_min_votes;   /* vertex peak threshold */
  int32_t bh_min_tracks;   /* black-hole-like: at least this many member tracks */
  float bh_max_isotropy;   /* ... and |mean member direction| at most this */
  float vtx_min_d0;        /* tracks with seed |d0| below this cast no vertex votes */
  int32_t fit_kind;        /* refit: 0 Gauss-Newton least squares, 1 extended Kalman filter */
  int32_t vtx_two_branch;  /* 0: vertex votes on the outgoing branch only; 1: also the incoming branch */
} or_cluster_cfg;

typedef struct {
  int32_t peak;            /* index into the peak list */
  int32_t lin, votes;      /* the peak cell and its votes */
  int32_t n_layers;        /* layers with a member hit */
  int32_t n_inliers;       /* layers with a hit on the seed road */
  int32_t n_owned;         /* inlier hits this track owns */
  int32_t status;          /* fit: 0 ok, 1 |u| >= 1 on a hit, 2 singular normal matrix */
  float seed_ss;           /* sum of squared seed distances of the inliers [cm^2] */
  float phi0, qpt, d0, chi2;
  float r_first;           /* smallest radius among owned hits */
  int32_t hits[OR_MAX_LAYERS]; /* owned hit on each layer, -1 if none */
} or_track;

typedef struct {
  int32_t lin, votes;      /* vertex cell (m * n_theta + t) and its votes */
  int32_t n_tracks, kind;  /* members; kind 0 displaced jet, 1 black-hole-like */
  float rho, theta, isotropy;
  int32_t member_begin;    /* offset of this object's members in the member list */
} or_object;

/* Canonical float32 arcsine (Abramowitz & Stegun 4.4.46 form). */
float oracle_asin_f(float u);
void oracle_asin_f_array(const float* u, float* out, int64_t n);

/* Canonical float64 sine and cosine (|a| <= 4) used for hit coordinates. */
void oracle_sincos_array(const double* a, double* s, double* c, int64_t n);

/* Canonical float64 atan2 used by the vertex transform. */
void oracle_atan2_array(const double* y, const double* x, double* out, int64_t n);

/* Per-grid constant tables: kap[n_qpt], q[n_d0*n_qpt], t[n_d0*n_qpt]
 * (k-major: index k*n_qpt + j), consts[0] = PHI_LO, consts[1] = INVW. */
int oracle_tables(const or_grid* g, float* kap, float* q, float* t, float* consts);

/* Unfloored phi0 bin coordinate of hit h at column (j[h], k[h]);
 * valid[h] = 0 when the hit is invalid or |u| > 1. */
int oracle_phi0_coord(const or_grid* g, const float* r, const float* phi, int32_t n,
                      const int32_t* j, const int32_t* k, float* x, int32_t* bin,
                      int32_t* valid);

int oracle_hough_vote(const or_grid* g, const float* r, const float* phi, int32_t n_hits,
                      int32_t* acc, uint64_t* n_votes);
int oracle_hough_vote_cell(const or_grid* g, const float* r, const float* phi, int32_t n_hits,
                           int32_t* acc, uint64_t* n_votes);

int oracle_hough_peaks(const or_grid* g, const int32_t* acc, int32_t min_votes,
                       or_peak* out, int32_t capacity, int32_t* n_found);

/* One candidate's refinement, for diagnostics and tests. */
int oracle_refine_one(const or_grid* g, const float* r, const float* phi, const uint8_t* layer,
                      int32_t n_hits, int32_t lin, const or_cluster_cfg* cfg, int32_t* out_i32,
                      double* out_f64);

/* counts[0] candidates (seed with >= min_layers inlier layers), counts[1]
 * surviving tracks, counts[2] vertex objects, counts[3] object members,
 * counts[4] candidates dropped for exceeding member_cap, counts[5] (candidate,
 * member) pairs of the other candidates, counts[6] road tests of the seed
 * search: (admissible seed circle, member) pairs, summed over candidates,
 * counts[7] 0.  Counts above INT32_MAX read INT32_MAX.  vacc (may be NULL)
 * receives the vertex accumulator [n_rho][n_theta]. */
int oracle_assoc_cluster(const or_grid* g, const float* r, const float* phi,
                         const uint8_t* layer, int32_t n_hits, const or_peak* peaks,
                         int32_t n_peaks, const or_cluster_cfg* cfg, int32_t* hit_owner,
                         or_track* tracks, int32_t track_cap, or_object* objects,
                         int32_t object_cap, int32_t* members, int32_t member_cap,
                         int32_t* vacc, int32_t* counts);

/* The duplicate cleaning step of oracle_assoc_cluster on its own (for the
 * pins): candidates p with n_in[p] >= 0 take part; hits is [n_cand][16], the
 * inlier hit of each layer (-1 none).  Each hit goes to the candidate with
 * the most inlier layers, then the smallest ss (float32), then the smallest
 * lin; owner[n_hits] receives that candidate (-1 none), n_owned[n_cand] the
 * inlier hits each candidate owns. */
int oracle_ownership(int32_t n_cand, const int32_t* n_in, const float* ss, const int32_t* lin,
                     const int32_t* hits, int32_t n_hits, int32_t* owner, int32_t* n_owned);

/* The vertex-peak rule of oracle_assoc_cluster on a given vertex accumulator
 * v[nm][nt] (theta periodic, rho clipped): cells in cell order into
 * out[capacity], full count in *n_found. */
int oracle_vertex_peaks(const int32_t* v, int32_t nm, int32_t nt, int32_t thr, int32_t* out,
                        int32_t capacity, int32_t* n_found);

/* OpenMP thread count for the calls above (determinism tests). */
void oracle_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
