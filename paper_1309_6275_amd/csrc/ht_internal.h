// Internal definitions of the gfx950 Hough trigger library: the plan and
// the launch helpers.  Device arithmetic lives in ht_device.h (included
// first, with its no-contraction pragma).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ht_device.h"
#include "houghtrig.h"

namespace ht {

// five groups of 64 counters, one 128-byte line each (the seed search's totals)
constexpr int kSpreadWords = 5 * 64 * 16;

// member lists by candidate: the distinct radii of an event's member-eligible
// hits go into a hash of kClsSlots; with at most kMaxClasses of them the hits
// are bucketed by (radius class, one of kBuckets azimuth buckets)
constexpr int kClsSlots = 64;
constexpr int kMaxClasses = 16;
constexpr int kBuckets = 1024;
constexpr int kBucketKeys = kMaxClasses * kBuckets;

// Hit slices for launches of one workgroup per 64-column tile: grids with
// fewer than 128 tiles also split the hits, so that about 256 workgroups run,
// with slices of at least 1024 hits of the bound the buffers were checked
// for (the kernels divide the hit count they read at run time).
inline int hit_slices(int tiles, int n_hits_bound) {
  if (tiles >= 128 || n_hits_bound < 2048) return 1;
  int n = (256 + tiles - 1) / tiles;
  const int by_hits = n_hits_bound / 1024;
  n = n < by_hits ? n : by_hits;
  return n > 1 ? n : 1;
}

// Per-plan state.  Tables are float32 bin-centre constants computed in
// float64 on the host and rounded once.
struct Plan {
  ht_grid grid;
  ht_limits lim;
  int device;
  int64_t dev_bytes;  // device bytes the plan allocated (each allocation rounded up to 4 KiB)
  int64_t n_cells;
  float phi_lo, invw;
  float* d_kap;  // [n_qpt]
  double* d_kapc;  // [n_qpt] curvature at the column centres (float64)
  double* d_d0c;   // [n_d0] d0 at the plane centres (float64)
  float* d_q;    // [n_d0][n_qpt]
  float* d_t;    // [n_d0][n_qpt]
  // band-vote corners: kappa at the smallest / largest edge [n_qpt], and Q,
  // T at (smallest kappa, lower d0 edge) and (largest kappa, upper d0 edge)
  float* d_ckl;
  float* d_ckh;
  float* d_cql;  // [n_d0][n_qpt]
  float* d_ctl;
  float* d_cqh;
  float* d_cth;
  // peak finder scratch
  uint32_t* d_bits;      // peak ballots, one bit per cell (tiles rounded up to 1024 cells)
  int32_t* d_tile_cnt;   // [n_tiles]
  int32_t* d_tile_off;   // [n_tiles]
  int32_t n_tiles;
  // refinement scratch
  uint32_t* d_pbits;     // [n_cells / 32 + 1] bitmap of the peaks handed to assoc_cluster
  int32_t* d_col_first;  // [n_qpt * n_d0] first peak index of each column
  double* d_hx;          // [max_hits] hit x, y, x^2+y^2
  double* d_hy;
  double* d_hq;
  float4* d_hitB;        // [max_hits] x, y (float32), the input radius and azimuth
  int32_t* d_mcount;     // [max_peaks] member counts
  uint2* d_mem;          // member pool: (hit, |x - cell centre| bits), member_cap slots per candidate
  int32_t* d_cstat;      // [max_peaks] candidate status / inlier count
  double* d_cgeo;        // [max_peaks * 5] seed ss, A, B, C, D
  int32_t* d_chit;       // [max_peaks * HT_MAX_LAYERS] inlier hit per layer
  int32_t* d_cnl;        // [max_peaks] member layer count
  unsigned long long* d_owner_key;  // [max_hits]
  int32_t* d_ctile_cnt;  // [candidate tiles]
  int32_t* d_ctile_off;
  int32_t* d_trk_peak;   // [max_tracks] peak index of each track
  int32_t* d_arc0;       // [max_tracks * max_n_rho] vertex arc start per row
  int32_t* d_arcn;       // [max_tracks * max_n_rho] vertex arc length per row
  int32_t* d_arci0;      // the same on the incoming branch (two-branch vote)
  int32_t* d_arcin;
  double2* d_tunit;      // [max_tracks] (-C, B) / |(B, C)| of each track's seed circle (isotropy)
  int32_t* d_vacc;       // [max_vertex_cells] vertex accumulator
  int32_t* d_obj_cnt;    // [max_vertex_cells] member count per object
  int32_t* d_vtile;      // [max_vertex_cells / 1024 + 1] vertex peaks per 1024-cell tile
  int32_t* d_scalars;    // [16] device counters
  unsigned long long* d_spread;  // [kSpreadWords] counters spread over 128-byte lines
  // member lists by candidate
  uint32_t* d_cls;      // [kClsSlots] hash of the hits' radii (float bits)
  int32_t* d_bkt;       // [kBucketKeys] hits per (class, bucket)
  int32_t* d_bkt_off;   // [kBucketKeys + 1] bucket starts; the bucketed hit count last
  int32_t* d_hkey;      // [max_hits] bucket key | slot << 14 of each hit, -1 if none
  int32_t* d_shit;      // [max_hits] hits in bucket order (hit | layer << 16)
  float* d_sphi;        // [max_hits] their azimuths
  // stage timing (ht_profile_*): HIP events recorded around the stages of
  // later calls; plan calls are ordered, so the counters need no locking
  mutable int32_t prof_depth;          // 0: off
  mutable hipEvent_t* prof_ev;         // [HT_STAGES][prof_depth][2]
  mutable int32_t prof_used[HT_STAGES];
  void prof_mark(int stage, int end, hipStream_t s) const {
    if (prof_depth == 0) return;
    const int u = prof_used[stage];
    if (u >= prof_depth) return;
    (void)hipEventRecord(prof_ev[((size_t)stage * prof_depth + u) * 2 + end], s);
    if (end) prof_used[stage] = u + 1;
  }
};

}  // namespace ht

struct ht_plan : ht::Plan {};

// Launch helpers implemented in the kernel files.
namespace ht {
// n_hits_dev (optional): device hit count of the event, at most n_hits,
// which then only bounds it (graph replays of events of any size)
int launch_vote(const Plan& p, const float* r, const float* phi, int32_t n_hits, int32_t* acc,
                unsigned long long* n_votes, hipStream_t s, const int32_t* n_hits_dev = nullptr);
// the vote of nb (<= 4) events in one launch on plan p's grid
int launch_vote_batch(const Plan& p, int nb, const float* const* r, const float* const* phi,
                      const int32_t* const* n_dev, int32_t n_hits_max, int32_t* const* acc,
                      hipStream_t s);
int launch_cell_vote(const Plan& p, const float* r, const float* phi, int32_t n_hits,
                     int32_t* acc, unsigned long long* n_votes, hipStream_t s);
int cell_vote_init(int n_phi);
int launch_peaks(const Plan& p, const int32_t* acc, int32_t min_votes, ht_peak* out,
                 int32_t capacity, int32_t* n_found, hipStream_t s);
// the peaks of nb (<= 4) events in one launch per kernel, each on its own
// plan's scratch (plans of one grid)
int launch_peaks_batch(int nb, const Plan* const* plans, const int32_t* const* acc,
                       int32_t min_votes, ht_peak* const* out, int32_t capacity,
                       int32_t* const* n_found, hipStream_t s);
// hough_peaks on the library's fixed device scratch array (no plan)
int launch_peaks_noalloc(const ht_grid& g, const int32_t* acc, int32_t min_votes, ht_peak* out,
                         int32_t capacity, int32_t* n_found, hipStream_t s);
int64_t noalloc_max_cells();
int launch_assoc(const Plan& p, const float* r, const float* phi, const uint8_t* layer,
                 int32_t n_hits, const ht_peak* peaks, const int32_t* n_peaks, int32_t peak_cap,
                 const int32_t* acc, const ht_cluster_cfg& cfg, const ht_cluster_out& out,
                 hipStream_t s, const int32_t* n_hits_dev = nullptr);
// assoc_cluster over nb events (<= 4) in one launch per kernel: event b has
// its own plan (scratch), hits, peaks and outputs; the plans share a grid and
// the events the configuration, hit bound and peak capacity
struct AssocEvent {
  const Plan* plan;
  const float* r;
  const float* phi;
  const uint8_t* layer;
  const int32_t* n_hits_dev;
  const ht_peak* peaks;
  const int32_t* n_peaks;
  const int32_t* acc;
  ht_cluster_out out;
};
int launch_assoc_batch(int nb, const AssocEvent* ev, int32_t n_hits_max, int32_t peak_cap,
                       const ht_cluster_cfg& cfg, hipStream_t s);
int launch_asin(const float* u, float* out, int64_t n, hipStream_t s);
int launch_sqrt(const double* x, double* out, int64_t n, hipStream_t s);
int launch_scan(const int32_t* cnt, int32_t* off, int n, int32_t* total, hipStream_t s);
// nb (<= 4) scans of n counts each in one launch
int launch_scan_batch(int nb, const int32_t* const* cnt, int32_t* const* off, int n,
                      int32_t* const* total, hipStream_t s);
int launch_compact(const float* r, const float* phi, const uint8_t* layer, const int32_t* owner,
                   int32_t n, float* out_r, float* out_phi, uint8_t* out_layer,
                   int32_t* out_index, int32_t* n_out, hipStream_t s);
int launch_remap(ht_track* tracks, int32_t track_cap, const int32_t* counts,
                 const int32_t* index, int32_t n_index, hipStream_t s);
// assoc_cluster's configuration checks (HT_OK, HT_EINVAL or HT_EUNSUPPORTED)
int check_cluster(const Plan& p, const ht_cluster_cfg& c, int32_t n_hits, int32_t peak_cap,
                  int32_t track_cap);
size_t cnn_workspace_bytes(int32_t max_windows, int training);
int launch_cnn_windows(const Plan& p, const int32_t* acc, const ht_peak* peaks, const int32_t* n_peaks,
                       int32_t cap, uint16_t* win, hipStream_t s);
int launch_cnn_forward(const float* params, const uint16_t* win, const int32_t* n_dev, int32_t n_max,
                       float* logits, void* ws, hipStream_t s);
int launch_cnn_score(const Plan& p, const float* params, const int32_t* acc, const ht_peak* peaks,
                     const int32_t* n_peaks, int32_t cap, float* logits, void* ws, hipStream_t s);
int launch_cnn_train(float* params, float* mom, const uint16_t* win, const float* labels, int32_t n,
                     float lr, float momentum, float pos_weight, float* loss, void* ws, hipStream_t s);
int launch_cnn_keep(const Plan& p, const float* logits, const ht_peak* peaks, const int32_t* n_peaks,
                    int32_t cap, float thr, ht_peak* out, int32_t out_cap, int32_t* n_out,
                    hipStream_t s);
int vote_init(int n_phi);
int peaks_init(int n_phi);
}  // namespace ht

#define HT_CHECK(x)                              \
  do {                                           \
    if ((x) != hipSuccess) return HT_EDEVICE;    \
  } while (0)
