// Candidate refinement, duplicate cleaning, refit and the second transform
// (paper, section "Jet and Black Hole Detection": candidates from the peak
// finder are refined, then a second Hough transform over the tracks finds
// the vertices they share, away from the interaction point).
//
// Launch sequence (all on the caller's stream, no host synchronisation; the
// device peak count bounds every per-candidate loop):
//   prep      per hit: float64 Cartesian coordinates (canonical sincos) and
//             a float32 record; ownership keys cleared; counters and the
//             vertex accumulator zeroed;
//   mark      peak bitmap and the first peak index of every column (and,
//             with an accumulator, the count of hits beyond the layer
//             range);
//   members   by candidate: the hits grouped by (radius class, azimuth
//             bucket) with a counting sort (the classes in the mark launch,
//             then bcount, scan, bscatter), then one wave per candidate
//             tests the hits of the buckets its member window reaches for
//             each class (mcand); events with
//             more distinct radii than the classes hold use a sweep shaped
//             like the vote instead (member_kernel);
//   refine    one wave per candidate: member layers, seed layers, the
//             seed_k nearest members of each seed layer by rank, then one
//             seed combination per lane (<= 64) scored against the members
//             in LDS, smallest non-seed layers first; the best lane wins by
//             (inliers, sum, index) and offers each inlier hit its 64-bit
//             ownership key (atomicMax); totals go to spread counters;
//   survive   ordered compaction of the candidates owning >= min_layers
//             hits into the track list (tile counts and their sums per 64
//             tiles, then each tile places its survivors);
//   fit+vvote one launch: float64 Gauss-Newton, one wave per track (lanes =
//             hits), beside one thread per (track, vertex row) voting its
//             crossing arcs into the vertex accumulator (the Kalman filter,
//             one thread per track, runs as a launch of its own first);
//   vpeaks    vertex local maxima in cell order: counts per 1024-cell tile,
//             then each tile places its own (vpcount, vpemit);
//   vcount,   member counts, one wave per (object, 64 tracks), then one
//   vmembers  wave per object: member tracks by ballot, written in order,
//             isotropy summed in track order;
//   counts    the output counts (the spread counters summed), by the wave
//             of the last object in the member pass.
// Every decision that selects an integer result uses float32 vote
// arithmetic or float64 arithmetic and square roots in a fixed order, so the
// results match the CPU reference bit for bit; the refit uses the device
// asin/atan2 and matches to rounding.
#include <type_traits>

#include "ht_internal.h"

namespace ht {
namespace {

constexpr int kSweepWaves = 16;
constexpr int kSweepThreads = kSweepWaves * kWave;
constexpr int kMaxMembers = 1024; // largest member_cap (LDS slots per wave in refine)
constexpr int kGridCap = 8192;    // grid-stride launches use at most this many blocks

// S_NBAD: valid hits whose layer is HT_MAX_LAYERS or more (they vote but are no members)
constexpr float kPiF = 3.14159265358979f;
constexpr float k2PiF = 6.28318530717959f;

// S_MODE: 1 when the member lists are built by candidate (see radius_classes);
// S_COVER: set when the hits have more distinct radii than the hash holds
enum { S_NP = 0, S_NBAD = 2, S_NTRK = 3, S_NOBJ = 4, S_NMEM = 5, S_MODE = 6, S_COVER = 7 };
// The seed search's totals (road tests, refined candidates, candidates over
// member_cap, (candidate, member) pairs within it) are summed per workgroup
// and added to kSpread counters in separate 128-byte lines, chosen by
// workgroup: tens of thousands of waves adding into one address serialise in
// one L2 channel (about a fifth of the kernel's time when measured, and most
// of it on events where every candidate overflows); write_counts sums the
// slots.
constexpr int kSpread = 64;
constexpr int kSpreadStride = 16;  // 64-bit words: one 128-byte line per slot
// group g of the counters starts at slot g * kSpread: 0 road tests,
// 1 refined candidates, 2 candidates over member_cap, 3 pairs within it,
// 4 float64 circle distances computed
enum { SP_TESTS = 0, SP_NCAND = kSpread, SP_NOVER = 2 * kSpread, SP_PAIRS = 3 * kSpread,
       SP_EXEC = 4 * kSpread };
static_assert(5 * kSpread * kSpreadStride == kSpreadWords, "spread counter layout");

__device__ __forceinline__ float bcastf(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ int bcasti(int v, int lane) {
  return __builtin_amdgcn_readlane(v, lane);
}

// ---- canonical float64 functions (arithmetic only) ------------------------
// Cody-Waite reduction by pi/2 (33-bit high part) and Taylor series of sin
// and cos on |r| <= pi/4; valid for |a| <= 4.
__device__ void csincos(double a, double* s_out, double* c_out) {
  const double PIO2_HI = 1.57079632673412561417e+00;
  const double PIO2_LO = 6.07710050650619224932e-11;
  double t = a * 0.63661977236758134308;
  double kf = floor(t + 0.5);
  double r = a - kf * PIO2_HI;
  r = r - kf * PIO2_LO;
  double z = r * r;
  double ps = -1.0 / 355687428096000.0;
  ps = ps * z + 1.0 / 1307674368000.0;
  ps = ps * z - 1.0 / 6227020800.0;
  ps = ps * z + 1.0 / 39916800.0;
  ps = ps * z - 1.0 / 362880.0;
  ps = ps * z + 1.0 / 5040.0;
  ps = ps * z - 1.0 / 120.0;
  ps = ps * z + 1.0 / 6.0;
  double sn = r - r * z * ps;
  double pc = 1.0 / 20922789888000.0;
  pc = pc * z - 1.0 / 87178291200.0;
  pc = pc * z + 1.0 / 479001600.0;
  pc = pc * z - 1.0 / 3628800.0;
  pc = pc * z + 1.0 / 40320.0;
  pc = pc * z - 1.0 / 720.0;
  pc = pc * z + 1.0 / 24.0;
  pc = pc * z - 0.5;
  double cs = 1.0 + z * pc;
  int q = ((int)kf) & 3;
  if (q == 0) { *s_out = sn; *c_out = cs; }
  else if (q == 1) { *s_out = cs; *c_out = -sn; }
  else if (q == 2) { *s_out = -sn; *c_out = -cs; }
  else { *s_out = -cs; *c_out = sn; }
}

// Octant reduction, atan z = pi/6 + atan((sqrt3 z - 1)/(z + sqrt3)) above
// tan(pi/12), Taylor series of atan to z^35.
__device__ double catan2(double y, double x) {
  double ax = fabs(x), ay = fabs(y);
  bool swap = ay > ax;
  double num = swap ? ax : ay, den = swap ? ay : ax;
  if (den == 0.0) return 0.0;
  double z = num / den;
  double base = 0.0;
  const double SQRT3 = 1.73205080756887729353;
  const double TAN_PI_12 = 0.26794919243112270647;
  if (z > TAN_PI_12) {
    z = (z * SQRT3 - 1.0) / (z + SQRT3);
    base = kPi / 6.0;
  }
  double w = z * z;
  double p = -1.0 / 35.0;
  p = p * w + 1.0 / 33.0;
  p = p * w - 1.0 / 31.0;
  p = p * w + 1.0 / 29.0;
  p = p * w - 1.0 / 27.0;
  p = p * w + 1.0 / 25.0;
  p = p * w - 1.0 / 23.0;
  p = p * w + 1.0 / 21.0;
  p = p * w - 1.0 / 19.0;
  p = p * w + 1.0 / 17.0;
  p = p * w - 1.0 / 15.0;
  p = p * w + 1.0 / 13.0;
  p = p * w - 1.0 / 11.0;
  p = p * w + 1.0 / 9.0;
  p = p * w - 1.0 / 7.0;
  p = p * w + 1.0 / 5.0;
  p = p * w - 1.0 / 3.0;
  double a = base + (z + z * w * p);
  if (swap) a = kPi / 2.0 - a;
  if (x < 0.0) a = kPi - a;
  if (y < 0.0) a = -a;
  return a;
}

// Circle A(x^2+y^2) + Bx + Cy + D = 0 through P1, P2, P3 (inner to outer),
// normalised to B^2 + C^2 - 4AD = 1 and oriented so that (-C, B), the
// direction of motion at the perigee, points from P1 towards P3.
__device__ bool circle3(double x1, double y1, double x2, double y2, double x3, double y3,
                        double* A, double* B, double* C, double* D) {
  double X2 = x2 - x1, Y2 = y2 - y1, X3 = x3 - x1, Y3 = y3 - y1;
  double q2 = X2 * X2 + Y2 * Y2;
  double q3 = X3 * X3 + Y3 * Y3;
  double a = X2 * Y3 - Y2 * X3;
  double b = Y2 * q3 - q2 * Y3;
  double c = q2 * X3 - X2 * q3;
  double nrm2 = b * b + c * c;
  if (!(nrm2 > 0.0)) return false;
  double nrm = sqrt_d(nrm2);
  double q1 = x1 * x1 + y1 * y1;
  double AA = a;
  double BB = b - 2.0 * a * x1;
  double CC = c - 2.0 * a * y1;
  double DD = a * q1 - b * x1 - c * y1;
  AA = AA / nrm;
  BB = BB / nrm;
  CC = CC / nrm;
  DD = DD / nrm;
  double dir = -CC * (x3 - x1) + BB * (y3 - y1);
  if (dir == 0.0) return false;
  if (dir < 0.0) { AA = -AA; BB = -BB; CC = -CC; DD = -DD; }
  *A = AA; *B = BB; *C = CC; *D = DD;
  return true;
}

// signed distance of a point from the normalised circle
__device__ __forceinline__ double circle_dist(double A, double B, double C, double D, double x,
                                              double y, double q) {
  double f = A * q + B * x + C * y + D;
  double s = 1.0 + 4.0 * A * f;
  if (s < 0.0) s = 0.0;
  return 2.0 * f / (1.0 + sqrt(s));
}

// float32 phi0 coordinate of a hit in a column (the vote formula); false
// when |u| > 1
__device__ __forceinline__ bool phi0_coord(float r2, float ir, float ph, float ck, float cq,
                                           float ct, float phi_lo, float invw, float* x,
                                           float* u_out) {
  const float a = ck * r2;
  const float b = a + cq;
  const float c = b * ir;
  const float u = c * ct;
  *u_out = u;
  if (!(fabsf(u) <= 1.0f)) return false;
  const float s = asin_f(u);
  const float phi0 = ph - s;
  const float d = phi0 - phi_lo;
  *x = d * invw;
  return true;
}

// |x - (i + 0.5)| on the periodic image of x nearest the cell
__device__ __forceinline__ float cell_adx(float x, int i, int n_phi) {
  const float xi = (float)i + 0.5f;
  const float half_n = 0.5f * (float)n_phi;
  float dx = x - xi;
  if (dx > half_n) dx = (x - (float)n_phi) - xi;
  else if (dx < -half_n) dx = (x + (float)n_phi) - xi;
  return fabsf(dx);
}

// member window half-width in bins: the column-width part depends on the
// hit only (e5), the arcsine slope 1 / sqrt(1 - u^2) on the column too
__device__ __forceinline__ float member_e5(float r, float ir, float hd0, float hk, float invw) {
  const float e1 = hd0 * ir;
  const float e2 = r * 0.5f;
  const float e3 = hk * e2;
  const float e4 = e1 + e3;
  return invw * e4;
}
__device__ __forceinline__ float member_window(float e5, float u, float wbase) {
  const float uu = u * u;
  const float gg = 1.0f - uu;  // 0 or >= 2^-24: the square root below is exact
  const float sg = sqrt_unit(gg);
  const float e6 = e5 * 1.5f;
  const float e7 = e6 / sg;
  return wbase + e7;
}

struct AssocArgs {
  // grid
  int n_phi, n_qpt, n_d0;
  int64_t n_cells;
  float phi_lo, invw;
  const float* kap;
  const float* qt;
  const float* tt;
  const double* kapc;  // column-centre curvature and plane-centre d0, float64
  const double* d0c;
  bool origin_seed;
  double kap_bin, d0_bin;
  float hk, hd0;
  double cb;  // 0.299792458e-2 B: curvature per unit q/pT
  // hits
  const float* r;
  const float* phi;
  const uint8_t* layer;
  int n_hits;                 // hits, or the bound of the device count below
  const int32_t* n_hits_dev;  // device hit count (optional)
  double* hx;
  double* hy;
  double* hq;
  float4* hitB;  // x, y (float32), the input radius and azimuth
  // the point-vote accumulator of these hits, or null (no member-count bound)
  const int32_t* acc;
  // peaks
  const ht_peak* peaks;
  const int32_t* n_peaks;
  int peak_cap;
  // cfg
  ht_cluster_cfg cfg;
  // scratch
  uint32_t* pbits;
  int32_t* col_first;
  int32_t* mcount;
  // member_cap slots per candidate: hit | layer << 16, |x - cell centre| bits
  uint2* pool;
  int32_t* cstat;
  int32_t* cnl;
  double* cgeo;
  int32_t* chit;
  unsigned long long* owner_key;
  int32_t* ctile_cnt;  // survivors per 256-candidate tile
  int32_t* ctile_off;  // their sums per group of 64 tiles
  int32_t* trk_peak;
  int32_t* arc0;   // vertex arc per (track, row), outgoing branch: first bin, length
  int32_t* arcn;
  int32_t* arci0;  // the same on the incoming branch (two-branch vote)
  int32_t* arcin;
  double2* tunit;  // per track: (-C, B) / |(B, C)| of its seed circle
  int32_t* vacc;
  int32_t* obj_cnt;
  int32_t* vtile;  // vertex peaks per 1024-cell tile
  int32_t* sc;  // device scalars
  unsigned long long* spread;  // [kSpreadWords] spread counters
  // member lists by candidate
  uint32_t* cls;       // hash of the radii
  int32_t* bkt;        // hits per (class, bucket)
  int32_t* bkt_off;    // bucket starts
  int32_t* hkey;       // each hit's bucket key | slot << 14, or -1
  int32_t* shit;       // hits in bucket order (hit | layer << 16)
  float* sphi;         // their azimuths
  // outputs
  ht_cluster_out out;
};

// Up to kMaxBatch events in one launch: each kernel takes the arguments of
// all of them (in the kernel argument segment) and blockIdx.z picks the
// event (the member sweep splits z into event and hit slice).  One event is
// the batch of one.
constexpr int kMaxBatch = 4;
template <int NB>
struct AssocBatch {
  AssocArgs a[NB];
};
static_assert(sizeof(AssocBatch<kMaxBatch>) <= 4096, "a batch's arguments fit the kernel argument segment");
template <int NB>
__device__ __forceinline__ const AssocArgs& event_args(const AssocBatch<NB>& B) {
  return B.a[NB == 1 ? 0 : blockIdx.z];
}

// first word of a member entry: the hit (< 65536) and its layer (< 16)
__device__ __forceinline__ unsigned member_word(const AssocArgs& A, int h) {
  return (unsigned)h | ((unsigned)A.layer[h] << 16);
}

__device__ __forceinline__ int n_cands(const AssocArgs& A) { return A.sc[S_NP]; }
__device__ __forceinline__ int hits_of(const AssocArgs& A) {
  return A.n_hits_dev ? min(max(*A.n_hits_dev, 0), A.n_hits) : A.n_hits;
}

// ---- prep ------------------------------------------------------------------
template <int NB>
__global__ void init_kernel(AssocBatch<NB> AB, int words, int surv_groups) {
  const AssocArgs& A = event_args(AB);
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (tid < 16) A.sc[tid] = 0;
  for (int64_t w = tid; w < kSpreadWords; w += stride) A.spread[w] = 0ull;
  if (tid == 0) {
    int np = *A.n_peaks;
    np = np < 0 ? 0 : (np > A.peak_cap ? A.peak_cap : np);
    A.sc[S_NP] = np;
  }
  for (int64_t w = tid; w < words; w += stride) A.pbits[w] = 0u;
  for (int64_t w = tid; w < kClsSlots; w += stride) A.cls[w] = kRadEmpty;
  for (int64_t w = tid; w < kBucketKeys; w += stride) A.bkt[w] = 0;
  for (int64_t w = tid; w < surv_groups; w += stride) A.ctile_off[w] = 0;
  const int n_hits = hits_of(A);
  for (int64_t h = tid; h < n_hits; h += stride) {
    const float r = A.r[h], ph = A.phi[h];
    const bool ok = hit_ok(r, ph);
    double s, c;
    csincos(ok ? (double)ph : 0.0, &s, &c);
    const double rr = (double)r;
    const double x = rr * c;
    const double y = rr * s;
    const double q = x * x + y * y;
    A.hx[h] = x;
    A.hy[h] = y;
    A.hq[h] = q;
    A.hitB[h] = make_float4((float)x, (float)y, r, ph);
    A.owner_key[h] = 0ull;
    A.out.hit_owner[h] = -1;
  }
  const int ncell_v = A.cfg.n_rho * A.cfg.n_theta;
  for (int64_t v = tid; v < ncell_v; v += stride) A.vacc[v] = 0;
}

__device__ void mark_peaks(const AssocArgs& A, int bid, int nblk) {
  if (A.acc) {
    const int n_hits = hits_of(A);
    for (int h = bid * blockDim.x + threadIdx.x; h < n_hits; h += nblk * blockDim.x)
      if (A.layer[h] >= HT_MAX_LAYERS && hit_ok(A.r[h], A.phi[h])) atomicAdd(&A.sc[S_NBAD], 1);
  }
  const int np = n_cands(A);
  for (int p = bid * blockDim.x + threadIdx.x; p < np; p += nblk * blockDim.x) {
    A.mcount[p] = 0;
    const int lin = A.peaks[p].lin;
    if (lin < 0 || lin >= A.n_cells) continue;
    atomicOr(&A.pbits[lin >> 5], 1u << (lin & 31));
    const int col = lin / A.n_phi;
    bool first = p == 0;
    if (!first) {
      const int pl = A.peaks[p - 1].lin;
      first = pl < 0 || pl >= A.n_cells || pl / A.n_phi != col;
    }
    if (first) A.col_first[col] = p;
  }
}

// ---- member lists by candidate -------------------------------------------------
// A hit of radius r is a member of the candidate at cell (i, j, k) when the
// float32 coordinate x = ((phi - s) - phi_lo) invw of the vote (s the arcsine
// of column (j, k) at radius r) lies within the member window w(r, j, k) of
// the cell centre, on the periodic image of x nearest the cell.  x is a
// monotone function of the azimuth, so a candidate's members of one radius
// are the hits of that radius in one interval of azimuth (periodic).  When
// the event's member-eligible hits (valid, layer below HT_MAX_LAYERS) have at
// most kMaxClasses distinct radii, they are bucketed by (radius class,
// azimuth bucket) and one wave per candidate tests, for each radius, only
// the hits of the buckets its interval reaches (one bucket of margin on each
// side, far above every rounding), with the very operations of the sweep
// below, and writes its member list contiguously.  Otherwise the sweep runs.

// inclusive prefix sum over the wave
__device__ __forceinline__ int wave_incl_scan_i32(int v, int lane) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// insert float bits k into a linear-probing hash of kClsSlots (LDS or
// global); false when the hash is full
__device__ __forceinline__ bool hash_insert(uint32_t* key, uint32_t k) {
  uint32_t slot = rad_hash(k);
  for (int p = 0; p < kClsSlots; ++p) {
    const uint32_t v = __hip_atomic_load(&key[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v == k) return true;
    if (v == kRadEmpty) {
      const uint32_t old = atomicCAS(&key[slot], kRadEmpty, k);
      if (old == kRadEmpty || old == k) return true;
    }
    slot = (slot + 1) & (kClsSlots - 1);
  }
  return false;
}

// azimuth in [-pi, pi) (up to rounding) and its bucket, the same function for
// hits and interval ends (monotone in the wrapped azimuth)
__device__ __forceinline__ float wrap_pi_f(float a) {
  return a - k2PiF * floorf((a + kPiF) * (1.0f / k2PiF));
}
__device__ __forceinline__ float bucket_coord(float aw) {
  return (aw + kPiF) * ((float)kBuckets / k2PiF);
}
__device__ __forceinline__ int bucket_of(float aw) {
  const float t = bucket_coord(aw);
  return t < 1.0f ? 0 : (t >= (float)(kBuckets - 1) ? kBuckets - 1 : (int)t);
}

// the event's distinct radii (each workgroup's, then merged into the event's hash)
__device__ void radius_classes(const AssocArgs& A, int bid, int nblk) {
  __shared__ uint32_t key[kClsSlots];
  __shared__ int over;
  if (threadIdx.x < kClsSlots) key[threadIdx.x] = kRadEmpty;
  if (threadIdx.x == 0) over = 0;
  __syncthreads();
  const int n = hits_of(A);
  uint32_t last = kRadEmpty;
  for (int h = bid * blockDim.x + threadIdx.x; h < n; h += nblk * blockDim.x) {
    const float rv = A.r[h];
    if (!hit_ok(rv, A.phi[h]) || A.layer[h] >= HT_MAX_LAYERS) continue;
    const uint32_t k = __float_as_uint(rv);
    if (k == last) continue;
    last = k;
    if (!hash_insert(key, k)) over = 1;
  }
  __syncthreads();
  if (threadIdx.x < kClsSlots) {
    const uint32_t k = key[threadIdx.x];
    if (k != kRadEmpty && !hash_insert(A.cls, k)) over = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0 && over) atomicOr(&A.sc[S_COVER], 1);
}

// the peak marks (workgroups below mark_blocks, 256 threads) and the radius
// classes (the rest) in one launch
template <int NB>
__global__ __launch_bounds__(256) void mark_kernel(AssocBatch<NB> AB, int mark_blocks) {
  const AssocArgs& A = event_args(AB);
  if ((int)blockIdx.x < mark_blocks)
    mark_peaks(A, blockIdx.x, mark_blocks);
  else
    radius_classes(A, blockIdx.x - mark_blocks, gridDim.x - mark_blocks);
}

// class index of each hash slot (rank among the filled slots, the same in
// every workgroup); returns the class count, or -1 when the lists are built
// by the sweep.  Whole workgroup; ends with a barrier.
__device__ __forceinline__ int class_table(const AssocArgs& A, int32_t* idx, float* cr) {
  __shared__ int ncls;
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    static_assert(kClsSlots == kWave, "one hash slot per lane");
    const uint32_t k = A.cls[lane];
    const bool full = k != kRadEmpty;
    const uint64_t m = __ballot(full);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    const int n = __popcll(m);
    const bool on = n <= kMaxClasses && A.sc[S_COVER] == 0;
    idx[lane] = full && on ? rank : -1;
    if (full && on) cr[rank] = __uint_as_float(k);
    if (lane == 0) ncls = on ? n : -1;
  }
  __syncthreads();
  return ncls;
}

__device__ __forceinline__ int class_of(const AssocArgs& A, const int32_t* idx, uint32_t k) {
  uint32_t slot = rad_hash(k);
  for (int p = 0; p < kClsSlots; ++p) {
    const uint32_t v = A.cls[slot];
    if (v == k) return idx[slot];
    if (v == kRadEmpty) return -1;
    slot = (slot + 1) & (kClsSlots - 1);
  }
  return -1;
}

// each member-eligible hit's bucket and slot in it
template <int NB>
__global__ __launch_bounds__(256) void bcount_kernel(AssocBatch<NB> AB) {
  const AssocArgs& A = event_args(AB);
  __shared__ int32_t idx[kClsSlots];
  __shared__ float cr[kMaxClasses];
  const int ncls = class_table(A, idx, cr);
  if (blockIdx.x == 0 && threadIdx.x == 0) A.sc[S_MODE] = ncls >= 0 ? 1 : 0;
  if (ncls < 0) return;
  const int n = hits_of(A);
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < n; h += gridDim.x * blockDim.x) {
    const float rv = A.r[h], ph = A.phi[h];
    int key = -1;
    if (hit_ok(rv, ph) && A.layer[h] < HT_MAX_LAYERS) {
      const int c = class_of(A, idx, __float_as_uint(rv));
      if (c >= 0) {
        const int b = c * kBuckets + bucket_of(wrap_pi_f(ph));
        key = b | (atomicAdd(&A.bkt[b], 1) << 14);
      }
    }
    A.hkey[h] = key;
  }
}

template <int NB>
__global__ __launch_bounds__(256) void bscatter_kernel(AssocBatch<NB> AB) {
  const AssocArgs& A = event_args(AB);
  if (A.sc[S_MODE] == 0) return;
  const int n = hits_of(A);
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < n; h += gridDim.x * blockDim.x) {
    const int key = A.hkey[h];
    if (key < 0) continue;
    const int e = A.bkt_off[key & (kBucketKeys - 1)] + (key >> 14);
    A.shit[e] = h | ((int)A.layer[h] << 16);  // a member entry's first word
    A.sphi[e] = A.phi[h];
  }
}

// One wave per candidate: lane c < the class count works out class c's
// arcsine, window and bucket ranges, then the wave tests the hits of each
// class's ranges, 64 at a time, and appends the members (ballot prefix).
template <int NB>
__global__ __launch_bounds__(256) void mcand_kernel(AssocBatch<NB> AB) {
  const AssocArgs& A = event_args(AB);
  __shared__ int32_t idx[kClsSlots];
  __shared__ float cr[kMaxClasses];
  __shared__ float cir[kMaxClasses], ce5[kMaxClasses];  // 1 / r and the window's hit part
  const int ncls = class_table(A, idx, cr);
  if (ncls < 0) return;
  if ((int)threadIdx.x < ncls) {
    const float ir = 1.0f / cr[threadIdx.x];
    cir[threadIdx.x] = ir;
    ce5[threadIdx.x] = member_e5(cr[threadIdx.x], ir, A.hd0, A.hk, A.invw);
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int waves = (int)(blockDim.x / kWave);
  const int np = n_cands(A);
  const int cap = A.cfg.member_cap;
  const int n_phi = A.n_phi;
  const float wbase = 0.5f + (float)A.cfg.win_bins;
  // bin width for the bucket ranges only (their margin is a whole bucket,
  // far above this product's rounding)
  const float binw = 1.0f / A.invw;
  for (int p = blockIdx.x * waves + (int)(threadIdx.x / kWave); p < np; p += gridDim.x * waves) {
    const int lin = A.peaks[p].lin;
    if (lin < 0 || lin >= A.n_cells) continue;  // no members (mark_kernel set the count to 0)
    const int col = lin / n_phi;
    const int i = lin - col * n_phi;
    const int j = col % A.n_qpt;
    const int k = col / A.n_qpt;
    float s = __builtin_nanf(""), w = 0.0f;
    int st0 = 0, en0 = 0, st1 = 0, en1 = 0;
    if (lane < ncls) {
      const float rv = cr[lane];
      const float ir = cir[lane];
      float x = 0.0f, u = 0.0f;
      const bool ok = phi0_coord(rv * rv, ir, 0.0f, A.kap[j], A.qt[(size_t)k * A.n_qpt + j],
                                 A.tt[(size_t)k * A.n_qpt + j], A.phi_lo, A.invw, &x, &u);
      if (ok) {
        s = asin_f(u);
        w = member_window(ce5[lane], u, wbase);
        // azimuths whose x lies within w of the cell centre, as bucket
        // coordinates: [lo, lo + len] (periodic), one bucket of margin
        const float xc = (float)i + 0.5f;
        const float a = ((xc - w) * binw + A.phi_lo) + s;
        const float lo = bucket_coord(wrap_pi_f(a)) - 1.0f;
        const float len = 2.0f * w * binw * ((float)kBuckets / k2PiF) + 2.0f;
        const int base = lane * kBuckets;
        if (!(len < (float)(kBuckets - 2)) || !(lo == lo)) {
          st0 = A.bkt_off[base];
          en0 = A.bkt_off[base + kBuckets];
        } else {
          const int b0 = (int)floorf(lo);
          const int b1 = (int)floorf(lo + len) + 1;  // one past the last bucket
          // b0 in [-2, kBuckets], b1 - b0 < kBuckets
          const int c0 = b0 < 0 ? b0 + kBuckets : (b0 >= kBuckets ? b0 - kBuckets : b0);
          const int c1 = c0 + (b1 - b0);
          if (c1 <= kBuckets) {
            st0 = A.bkt_off[base + c0];
            en0 = A.bkt_off[base + c1];
          } else {
            st0 = A.bkt_off[base + c0];
            en0 = A.bkt_off[base + kBuckets];
            st1 = A.bkt_off[base];
            en1 = A.bkt_off[base + c1 - kBuckets];
          }
        }
      }
    }
    // The classes' ranges, range q = 2 c + part held by lane q, laid end to
    // end: a sparse event's candidate (a few hits per class) reads them 64
    // hits at a time whatever their lengths.
    const int nr = 2 * ncls;
    const int qc = lane >> 1;
    const int rst0 = __shfl(st0, qc, kWave), ren0 = __shfl(en0, qc, kWave);
    const int rst1 = __shfl(st1, qc, kWave), ren1 = __shfl(en1, qc, kWave);
    const float rs = __shfl(s, qc, kWave);
    const int rst = (lane & 1) ? rst1 : rst0;
    const int rlen = lane < nr && rs == rs ? ((lane & 1) ? ren1 - rst1 : ren0 - rst0) : 0;
    const int rend = wave_incl_scan_i32(rlen, lane);  // end of range q in the laid-out order
    const int rbase = rst - (rend - rlen);  // position t of range q is hit rbase + t
    const int total = __builtin_amdgcn_readlane(rend, kWave - 1);
    int cnt = 0;
    uint2* pool = A.pool + (size_t)p * cap;
    auto test = [&](int e, bool in, float sc, float wc) {
      bool mem = false;
      int h = 0;
      float adx = 0.0f;
      if (in) {
        h = A.shit[e];
        const float x = ((A.sphi[e] - sc) - A.phi_lo) * A.invw;
        adx = cell_adx(x, i, n_phi);
        mem = adx <= wc;
      }
      const uint64_t m = __ballot(mem);
      if (mem) {
        const int slot = cnt + __popcll(m & ((1ull << lane) - 1ull));
        if (slot < cap) pool[slot] = make_uint2((unsigned)h, __float_as_uint(adx));
      }
      cnt += __popcll(m);
    };
    if (total > 3 * kWave) {
      // dense: class by class (the lookup of a hit's range costs more than
      // the partly filled last pass of each range)
      for (int c = 0; c < ncls; ++c) {
        const float sc = bcastf(s, c);
        if (!(sc == sc)) continue;
        const float wc = bcastf(w, c);
#pragma unroll
        for (int part = 0; part < 2; ++part) {
          const int st = bcasti(part ? st1 : st0, c);
          const int en = bcasti(part ? en1 : en0, c);
          for (int e0 = st; e0 < en; e0 += kWave) test(e0 + lane, e0 + lane < en, sc, wc);
        }
      }
    } else for (int t0 = 0; t0 < total; t0 += kWave) {
      const int t = t0 + lane;
      // range of t: the number of ranges that end at or before it, by a
      // binary search over the ends (non-decreasing in q, nr <= 32)
      int q = 0;
#pragma unroll
      for (int step = 32; step > 0; step >>= 1) {
        // every lane reads (a lane's value can only be read while it is active)
        const int end = __shfl(rend, min(q + step - 1, kWave - 1), kWave);
        if (q + step <= nr && end <= t) q += step;
      }
      const int qs = q < kWave ? q : kWave - 1;
      const int e = __shfl(rbase, qs, kWave) + t;
      test(e, t < total, __shfl(s, qs >> 1, kWave), __shfl(w, qs >> 1, kWave));
    }
    if (lane == 0) A.mcount[p] = cnt;
  }
}

// ---- member sweep -----------------------------------------------------------
// LDS per column: the column's peak bits (starting at bit i = 0) and the
// number of peaks before each 32-bit word.  The workgroup owns the peaks of
// its 64 columns, which are consecutive in the (cell-ordered) peak list, so
// it counts their members with LDS atomics and writes each member straight
// into its candidate's member_cap slots of the pool: one sweep, and the
// workgroup's member lists form one contiguous region of the pool.
constexpr int kMaxPhiWords = 32;  // n_phi <= 1024
constexpr int kMaxWgPeaks = 4096; // LDS counters; more peaks fall back to global counters
constexpr int kQueue = 2 * kWave; // per-wave queue of (hit, column) pairs with a peak in reach

struct SweepShared {
  uint32_t cbits[kWave][kMaxPhiWords + 1];  // every peak of the column (candidate indices)
  // the peaks still taking members: a candidate's bit is cleared once it
  // holds more than member_cap (it is dropped whatever else it would get)
  uint32_t lbits[kWave][kMaxPhiWords + 1];
  int32_t cpre[kWave][kMaxPhiWords + 1];
  int32_t ccnt[kWave];
  int32_t cfirst[kWave];      // first peak of each column, relative to p_lo
  int32_t cnt[kMaxWgPeaks];   // member counts = next free slot of each candidate
  // Pairs whose window range holds a peak bit wait here until a full wave of
  // them can be resolved at once: x, u, the window's hit part e5, the peak
  // bits in range, and hit | column lane << 16 | first cell of the range << 22.
  float qx[kSweepWaves][kQueue];
  float qu[kSweepWaves][kQueue];
  float qe[kSweepWaves][kQueue];
  uint32_t qbits[kSweepWaves][kQueue];
  uint32_t qmeta[kSweepWaves][kQueue];
  int32_t np_wg, p_lo;
  // per (distinct hit radius, column): arcsine (NaN when |u| > 1), u, and
  // the upper bound of the member window
  RadiusSet R;
  float s_tab[kMaxRadii][kWave];
  float u_tab[kMaxRadii][kWave];
  float whi_tab[kMaxRadii][kWave];
};

// One pass over the workgroup's (hit, column) pairs; for every member
// (candidate q = p - p_lo, hit h, |x - cell centre| adx) call fn(q, h, adx),
// which returns true when the candidate has just gone over member_cap; its
// live bit is then cleared and later hits skip it.  A lane (column) first
// bounds the window from above with cheap arithmetic and reads the peak bits
// it covers; the rare pairs with a peak bit in range are queued and resolved
// (exact window, candidate index, fn) a wave at a time, so the exact test
// does not run with most lanes idle.
// The live bits are cleared by other lanes during the sweep; a stale bit
// only means one more member test of a candidate that is dropped anyway.
__device__ __forceinline__ uint32_t live_bits(SweepShared& S, int cl, int w) {
  return __hip_atomic_load(&S.lbits[cl][w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <typename F>
__device__ __forceinline__ void sweep_members(const AssocArgs& A, SweepShared& S, int k, int j0,
                                              int h0, int h1, F fn) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6;
  const int n_phi = A.n_phi;
  const int j = j0 + lane;
  const bool col_ok = j < A.n_qpt;
  float ck = 0.0f, cq = 0.0f, ct = 0.0f;
  const bool has = col_ok && S.ccnt[lane] > 0;
  if (col_ok) {
    ck = A.kap[j];
    cq = A.qt[(size_t)k * A.n_qpt + j];
    ct = A.tt[(size_t)k * A.n_qpt + j];
  }
  const int cfirst = S.cfirst[lane];
  const float wbase = 0.5f + (float)A.cfg.win_bins;
  // the per-radius tables (whole workgroup); thread t fills entry (t / 64, lane)
  radius_set_build(S.R, A.r, A.phi, h0, h1);
  for (int t = threadIdx.x; t < S.R.n * kWave; t += kSweepThreads) {
    const float rv = S.R.r[t >> 6];
    const float ir = 1.0f / rv;
    float x = 0.0f, u = 0.0f;
    const bool ok = col_ok && phi0_coord(rv * rv, ir, 0.0f, ck, cq, ct, A.phi_lo, A.invw, &x, &u);
    const float e5 = member_e5(rv, ir, A.hd0, A.hk, A.invw);
    const float gg = 1.0f - u * u;
    S.s_tab[t >> 6][lane] = ok ? asin_f(u) : __builtin_nanf("");
    S.u_tab[t >> 6][lane] = u;
    S.whi_tab[t >> 6][lane] = wbase + e5 * 1.5f * __builtin_amdgcn_rsqf(gg) * 1.001f;
  }
  __syncthreads();
  const int np_wg = S.np_wg;
  const int nwords = (n_phi + 31) >> 5;
  const bool fast_bits = (n_phi & 31) == 0;
  int head = 0, tail = 0;  // queue positions, uniform over the wave
  auto drain = [&](int nproc) {
    if (lane < nproc) {
      const int slot = (head + lane) & (kQueue - 1);
      const float x = S.qx[wave][slot];
      const float u = S.qu[wave][slot];
      const float e5 = S.qe[wave][slot];
      uint32_t bits = S.qbits[wave][slot];
      const uint32_t meta = S.qmeta[wave][slot];
      const int hh = (int)(meta & 0xffffu);
      const int cl = (int)((meta >> 16) & 63u);
      const int iw0 = (int)(meta >> 22);
      const float w = member_window(e5, u, wbase);
      while (bits) {
        const int b = __builtin_ctz(bits);
        bits &= bits - 1u;
        int ic = iw0 + b;
        if (ic >= n_phi) ic -= n_phi;
        const float adx = cell_adx(x, ic, n_phi);
        if (!(adx <= w)) continue;
        const int wi = ic >> 5;
        const uint32_t below = S.cbits[cl][wi] & ((1u << (ic & 31)) - 1u);
        const int q = S.cfirst[cl] + S.cpre[cl][wi] + __popc(below);
        if (q < 0 || q >= np_wg) continue;  // only for peak lists not sorted by cell
        if (fn(q, hh, adx)) atomicAnd(&S.lbits[cl][wi], ~(1u << (ic & 31)));
      }
    }
    head += nproc;
  };
  for (int base = h0 + wave * kWave; base < h1; base += kSweepThreads) {
    const int h = base + lane;
    float hr = 1.0f, hp = 0.0f;
    bool hv = false;
    if (h < h1) {
      hr = A.r[h];
      hp = A.phi[h];
      hv = hit_ok(hr, hp) && A.layer[h] < HT_MAX_LAYERS;
    }
    const float hr2 = hr * hr;
    const float hir = 1.0f / hr;
    const float he5 = member_e5(hr, hir, A.hd0, A.hk, A.invw);
    const int hri = hv ? radius_index(S.R, hr) : -1;
    uint64_t todo = __ballot(hv);
    while (todo) {
      const int src = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int ri = __builtin_amdgcn_readlane(hri, src);
      const float ph = bcastf(hp, src);
      const float e5 = bcastf(he5, src);
      const int hh = base + src;
      float x = 0.0f, u = 0.0f;
      uint32_t bits = 0u;
      int iw0 = 0, ilo = 0, ihi = -1;
      bool slow = false;
      bool valid = false;
      float w_hi = 0.0f;
      if (has) {
        if (ri >= 0) {
          // the same operations as phi0_coord, the radius part from the table
          const float s = S.s_tab[ri][lane];
          valid = s == s;
          if (valid) {
            u = S.u_tab[ri][lane];
            x = ((ph - s) - A.phi_lo) * A.invw;
            w_hi = S.whi_tab[ri][lane];
          }
        } else {
          const float r2 = bcastf(hr2, src);
          const float ir = bcastf(hir, src);
          valid = phi0_coord(r2, ir, ph, ck, cq, ct, A.phi_lo, A.invw, &x, &u);
          // upper bound of the window with the hardware reciprocal square
          // root (1 ulp) and a 0.1% margin
          const float gg = 1.0f - u * u;
          w_hi = wbase + e5 * 1.5f * __builtin_amdgcn_rsqf(gg) * 1.001f;
        }
      }
      if (valid) {
        ilo = 0;
        ihi = n_phi - 1;
        if (w_hi < 0.5f * (float)n_phi) {
          const int lo = (int)floorf(x - w_hi - 0.5f) - 1;
          const int hi = (int)floorf(x + w_hi - 0.5f) + 1;
          if (hi - lo + 1 < n_phi) { ilo = lo; ihi = hi; }
        }
        const int len = ihi - ilo + 1;
        if (fast_bits && len <= 32) {
          // the range fits in 64 bits starting at ilo's word (n_phi is a
          // multiple of 32, so the column bits are cyclic by word)
          iw0 = ilo < 0 ? ilo + n_phi : (ilo >= n_phi ? ilo - n_phi : ilo);
          const int w0 = iw0 >> 5;
          const int w1 = w0 + 1 == nwords ? 0 : w0 + 1;
          const uint64_t two = (uint64_t)live_bits(S, lane, w0) |
                               ((uint64_t)live_bits(S, lane, w1) << 32);
          bits = (uint32_t)((two >> (iw0 & 31)) & ((1ull << len) - 1ull));
        } else {
          slow = true;
        }
      }
      const bool push = bits != 0u;
      const uint64_t pm = __ballot(push);
      if (pm) {
        if (push) {
          const uint64_t lower = lane ? (pm & ((1ull << lane) - 1ull)) : 0ull;
          const int slot = (tail + __popcll(lower)) & (kQueue - 1);
          S.qx[wave][slot] = x;
          S.qu[wave][slot] = u;
          S.qe[wave][slot] = e5;
          S.qbits[wave][slot] = bits;
          S.qmeta[wave][slot] = (uint32_t)hh | ((uint32_t)lane << 16) | ((uint32_t)iw0 << 22);
        }
        tail += __popcll(pm);
        if (tail - head >= kWave) drain(kWave);
      }
      if (slow) {
        // general range: word by word over the cyclic column
        float w = -1.0f;
        int i = ilo;
        while (i <= ihi) {
          // i lies in (-n_phi, 2 n_phi) for n_phi >= 14; smaller grids take the modulo
          int iw = i < 0 ? i + n_phi : (i >= n_phi ? i - n_phi : i);
          if (iw < 0 || iw >= n_phi) iw = ((i % n_phi) + n_phi) % n_phi;
          const int wi = iw >> 5, bit = iw & 31;
          int span = 32 - bit;
          span = min(span, ihi - i + 1);
          span = min(span, n_phi - iw);
          uint32_t wbits = live_bits(S, lane, wi) >> bit;
          if (span < 32) wbits &= (1u << span) - 1u;
          while (wbits) {
            const int b = __builtin_ctz(wbits);
            wbits &= wbits - 1u;
            if (w < 0.0f) w = member_window(e5, u, wbase);
            const int ic = iw + b;
            const float adx = cell_adx(x, ic, n_phi);
            if (!(adx <= w)) continue;
            const uint32_t below = S.cbits[lane][wi] & ((1u << (bit + b)) - 1u);
            const int q = cfirst + S.cpre[lane][wi] + __popc(below);
            if (q < 0 || q >= np_wg) continue;  // only for peak lists not sorted by cell
            if (fn(q, hh, adx)) atomicAnd(&S.lbits[lane][wi], ~(1u << (ic & 31)));
          }
          i += span;
        }
      }
    }
  }
  while (tail > head) drain(min(kWave, tail - head));
}

// Candidates that provably hold more than member_cap members are dropped
// before the sweep (their member count is set past the cap and their live
// bit cleared).  Every valid hit with a layer below HT_MAX_LAYERS that votes
// in one of the 2 win_bins + 1 cells around the candidate in its column is a
// member: its |x - cell centre| is at most win_bins + 0.5 (float rounding is
// monotone and the interval ends are exact), and the member window is never
// narrower (0.5 + win_bins plus a term that is positive on grids with a d0
// axis).  So those cells' votes, less the valid hits of higher layers, bound
// the member count from below.
__device__ void drop_overfull(const AssocArgs& A, SweepShared& S, int k, int j0, int32_t* cnt_lds,
                              int32_t* cnt_glob) {
  const int n_phi = A.n_phi;
  const int nwords = (n_phi + 31) >> 5;
  const int b = A.cfg.win_bins;
  const int cap = A.cfg.member_cap;
  const long long lim = (long long)cap + A.sc[S_NBAD];
  const int np_wg = S.np_wg;
  for (int e = threadIdx.x; e < kWave * nwords; e += kSweepThreads) {
    const int cl = e / nwords, w = e - cl * nwords;
    const int j = j0 + cl;
    const uint32_t bits = S.cbits[cl][w];
    if (j >= A.n_qpt || !bits) continue;
    const int32_t* row = A.acc + ((size_t)k * A.n_qpt + j) * n_phi;
    const int q0 = S.cfirst[cl] + S.cpre[cl][w];
    uint32_t rest = bits;
    int rank = 0;
    while (rest) {
      const int bit = __builtin_ctz(rest);
      rest &= rest - 1u;
      const int ic = w * 32 + bit;
      long long sum = 0;
      for (int d = -b; d <= b; ++d) {
        int ii = ic + d;  // |d| < n_phi / 4: one period of correction
        ii = ii < 0 ? ii + n_phi : (ii >= n_phi ? ii - n_phi : ii);
        sum += row[ii];
      }
      const int q = q0 + rank;
      ++rank;
      if (sum <= lim || q < 0 || q >= np_wg) continue;
      atomicAnd(&S.lbits[cl][w], ~(1u << bit));
      if (cnt_lds)
        cnt_lds[q] = cap + 1;
      else
        atomicMax(&cnt_glob[q], cap + 1);
    }
  }
}

template <int NB>
__global__ __launch_bounds__(kSweepThreads) void member_kernel(AssocBatch<NB> AB) {
  __shared__ SweepShared S;
  // blockIdx.z = event * slices + slice of the hits (see hit_slices)
  const int n_slices = gridDim.z / NB;
  const int slice = (int)blockIdx.z % n_slices;
  const AssocArgs& A = AB.a[NB == 1 ? 0 : (int)blockIdx.z / n_slices];
  if (A.sc[S_MODE] != 0) return;  // the lists are built by candidate
  const int j0 = blockIdx.x * kWave;
  const int k = blockIdx.y;
  const int n_all = hits_of(A);
  const int chunk = ((n_all + n_slices - 1) / n_slices + kWave - 1) / kWave * kWave;
  const int h0 = slice * chunk;
  const int h1 = min(n_all, h0 + chunk);
  if (h0 >= h1) return;
  const int n_phi = A.n_phi;
  const int nwords = (n_phi + 31) >> 5;
  const int cap = A.cfg.member_cap;
  // gather the column bitmaps (column bits are not word aligned in general)
  for (int e = threadIdx.x; e < kWave * nwords; e += kSweepThreads) {
    const int cl = e / nwords, w = e - cl * nwords;
    const int j = j0 + cl;
    uint32_t v = 0;
    if (j < A.n_qpt) {
      const int64_t bit0 = ((int64_t)k * A.n_qpt + j) * n_phi + (int64_t)w * 32;
      const int nb = min(32, n_phi - w * 32);
      const int64_t wi = bit0 >> 5;
      const int sh = (int)(bit0 & 31);
      uint64_t two = (uint64_t)A.pbits[wi];
      if (sh + nb > 32) two |= (uint64_t)A.pbits[wi + 1] << 32;
      v = (uint32_t)(two >> sh);
      if (nb < 32) v &= (1u << nb) - 1u;
    }
    S.cbits[cl][w] = v;
    S.lbits[cl][w] = v;
  }
  __syncthreads();
  if (threadIdx.x < kWave) {
    int s = 0;
    for (int w = 0; w < nwords; ++w) {
      S.cpre[threadIdx.x][w] = s;
      s += __popc(S.cbits[threadIdx.x][w]);
    }
    S.ccnt[threadIdx.x] = s;
    // the first column with peaks gives the workgroup's first peak index
    const uint64_t hasm = __ballot(s > 0);
    int tot = s;
    for (int d = 32; d > 0; d >>= 1) tot += __shfl_xor(tot, d);
    if (threadIdx.x == 0) {
      S.np_wg = tot;
      S.p_lo = 0;
      if (hasm) {
        const int c0 = __builtin_ctzll(hasm);
        S.p_lo = A.col_first[(size_t)k * A.n_qpt + j0 + c0];
      }
    }
  }
  __syncthreads();
  const int np_wg = S.np_wg;
  const int p_lo = S.p_lo;
  // a cell-ordered peak list gives p_lo + np_wg <= n_peaks; anything else is
  // a malformed list, whose candidates in these columns then get no members
  if (np_wg == 0 || p_lo < 0 || p_lo + np_wg > n_cands(A)) return;
  if (threadIdx.x < kWave) {
    const int j = j0 + threadIdx.x;
    S.cfirst[threadIdx.x] =
        (j < A.n_qpt && S.ccnt[threadIdx.x] > 0) ? A.col_first[(size_t)k * A.n_qpt + j] - p_lo : 0;
  }
  __syncthreads();
  uint2* pool = A.pool + (size_t)p_lo * cap;
  const bool lds_cnt = n_slices == 1 && np_wg <= kMaxWgPeaks;
  if (lds_cnt) {
    for (int q = threadIdx.x; q < np_wg; q += kSweepThreads) S.cnt[q] = 0;
    __syncthreads();
  }
  if (A.acc) {
    drop_overfull(A, S, k, j0, lds_cnt ? S.cnt : nullptr, A.mcount + p_lo);
    __syncthreads();
  }
  if (lds_cnt) {
    sweep_members(A, S, k, j0, h0, h1, [&](int q, int hh, float adx) {
      const int slot = atomicAdd(&S.cnt[q], 1);
      if (slot < cap)
        pool[(size_t)q * cap + slot] = make_uint2(member_word(A, hh), __float_as_uint(adx));
      return slot == cap;
    });
    __syncthreads();
    for (int q = threadIdx.x; q < np_wg; q += kSweepThreads) A.mcount[p_lo + q] = S.cnt[q];
  } else {
    // counters in global memory (zeroed by mark_kernel), shared by the hit
    // slices; each slice drops a candidate at its first member past the cap
    int32_t* cnt = A.mcount + p_lo;
    sweep_members(A, S, k, j0, h0, h1, [&](int q, int hh, float adx) {
      const int slot = atomicAdd(&cnt[q], 1);
      if (slot < cap)
        pool[(size_t)q * cap + slot] = make_uint2(member_word(A, hh), __float_as_uint(adx));
      return slot >= cap;
    });
  }
}

// ---- refine: one wave per candidate ------------------------------------------
// Ownership key of a refined candidate's inlier hits: most inlier layers,
// then the smallest float32 seed sum of squared distances, then the lowest
// candidate index; each hit keeps the largest key offered to it.
__device__ __forceinline__ unsigned long long own_key(int n_in, double ss, int p) {
  const uint32_t sb = __float_as_uint((float)ss);
  return ((unsigned long long)n_in << 58) | ((unsigned long long)(0xffffffffu - sb) << 26) |
         (unsigned long long)(0x3ffffff - p);
}

// Members are grouped by layer in LDS as (x, y, x^2+y^2) in float32 plus the
// hit index, one 16-byte record each, for a conservative float32 pre-filter;
// the float64 coordinates of the seeds and of the few members that pass are
// read from global memory (the hit arrays stay in L2).  Lanes are seed
// combinations.  They visit the layers that are not seed layers first, so a
// combination that can no longer reach min_layers inlier layers drops out
// early, and the wave leaves the candidate as soon as every lane has dropped
// out.  The seed sum of squares is a float64 sum over layers in increasing
// layer order; the lanes that tie for the most inlier layers recompute it in
// that order at the end.
// hit indices are < 65535 (at most 65535 hits), so 0xffff marks "no hit"
constexpr uint16_t kNoHit = 0xffff;

// a member: float32 x, y of the hit, its |x - cell centre| in the column
// (the seed ranking key) and the hit index; the float32 x^2 + y^2 of the
// pre-filter is recomputed from x and y
struct alignas(16) Mem4 {
  float x, y, adx;
  int32_t h;
};

__device__ __forceinline__ float mem_q(const Mem4& v) { return __builtin_fmaf(v.x, v.x, v.y * v.y); }

template <int CAP>
struct RawMembers {  // members in pool order, before grouping
  Mem4 mem[CAP];
  int16_t slot[CAP];
  int8_t L[CAP];
};

// Angle bins of a layer's members (caps above 128).  Within each layer the
// members are grouped by kNB bins of their azimuth (relative to the cell's
// phi0 centre), between the smallest and largest azimuth of the layer.  When
// every member of a layer has the same radius r, a seed circle's points at r
// within the road lie on two arcs that follow from the circle's equation, and
// a lane tests only the members of the bins those arcs reach.
constexpr int kNB = 32;
constexpr int kBinKeys = HT_MAX_LAYERS * kNB;
// padding of every computed angle (radians): far above the float32 rounding
// of the azimuths, of the circle's direction and of the arc half-widths
constexpr float kAngPad = 1e-5f;

template <bool ON>
struct LayerBins {};
template <>
struct LayerBins<true> {
  // group counts, then group starts (entry kBinKeys: the member count), as
  // 16-bit entries two to a word (counts and starts are at most 1024)
  uint32_t bpack[kBinKeys / 2 + 1];
  __device__ __forceinline__ int start(int key) const {
    return (int)((bpack[key >> 1] >> ((key & 1) * 16)) & 0xffffu);
  }
  float lr[HT_MAX_LAYERS];    // the layer's radius when all its members share it, else 0
  float lmn[HT_MAX_LAYERS], lmx[HT_MAX_LAYERS];  // azimuth range of the layer's members
  float linv[HT_MAX_LAYERS];  // bins per radian
};

// a layer's radius and azimuth ranges while the members are loaded
struct LayerStats {
  int32_t rlo[HT_MAX_LAYERS], rhi[HT_MAX_LAYERS];  // members' radius bits, smallest and largest
  int32_t alo[HT_MAX_LAYERS], ahi[HT_MAX_LAYERS];  // members' azimuth (ordered bits)
};

// float bits in an order that int comparisons follow
__device__ __forceinline__ int32_t ord_bits(float f) {
  const int32_t b = __float_as_int(f);
  return b >= 0 ? b : b ^ 0x7fffffff;
}
__device__ __forceinline__ float ord_float(int32_t b) {
  return __int_as_float(b >= 0 ? b : b ^ 0x7fffffff);
}

// azimuth relative to ref, in [-pi, pi) (azimuths of valid hits lie in [-4, 4])
__device__ __forceinline__ float rel_angle(float ph, float ref) {
  float d = ph - ref;
  if (d >= kPiF) d -= k2PiF;
  if (d >= kPiF) d -= k2PiF;
  if (d < -kPiF) d += k2PiF;
  if (d < -kPiF) d += k2PiF;
  return d;
}

// bin of a relative azimuth: monotone in rel, clamped to [0, kNB - 1]
__device__ __forceinline__ int angle_bin(float rel, float mn, float inv) {
  const float t = (rel - mn) * inv;
  return t < 1.0f ? 0 : (t >= (float)(kNB - 1) ? kNB - 1 : (int)t);
}

// the bins holding every member whose relative azimuth lies in [a, b]
__device__ __forceinline__ unsigned bin_span(float a, float b, float mn, float mx, float inv) {
  if (!(b >= mn) || !(a <= mx) || !(a <= b)) return 0u;
  const int ba = angle_bin(a, mn, inv), bb = angle_bin(b, mn, inv);
  return ((2u << bb) - 1u) & ~((1u << ba) - 1u);
}

// Bins of a layer of radius r that can hold a member within the road of the
// circle f = A q + B x + C y + D (float32 coefficients; R = |(B, C)|, phB the
// direction of (B, C)): a point (r, phi) has f = A r^2 + D + r R cos(phi - phB),
// so |f| <= thr needs cos(phi - phB) in [lo, hi], i.e. phi - phB within
// [acos(hi), acos(lo)] of 0 on either side.  The cosine interval is widened
// by far more than the float32 rounding of its terms, and the arcs by
// kAngPad, so no member that the float64 road test keeps is left out.
__device__ __forceinline__ unsigned road_bins(float r, float Af, float Df, float Rf, float phB,
                                              float thr, float ref, float mn, float mx,
                                              float inv) {
  constexpr unsigned kAll = kNB == 32 ? ~0u : (1u << (kNB & 31)) - 1u;
  const float r2 = r * r;
  const float den = r * Rf;
  if (!(den > 1e-30f) || !(thr < 1e30f)) return kAll;
  const float base = Af * r2 + Df;
  const float mag = fabsf(Af) * r2 + fabsf(Df) + thr;
  const float epsc = 1e-5f * (mag / den) + 1e-6f;
  const float hi = (thr - base) / den + epsc;
  const float lo = (-thr - base) / den - epsc;
  if (hi < -1.0f || lo > 1.0f) return 0u;  // no point of radius r comes within the road
  if (!(hi == hi) || !(lo == lo)) return kAll;
  const float a1 = hi >= 1.0f ? 0.0f : fmaxf(acosf(hi) - kAngPad, 0.0f);
  const float a2 = lo <= -1.0f ? kPiF + kAngPad : acosf(lo) + kAngPad;
  const float c = rel_angle(phB, ref);
  unsigned m = 0u;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const float u = side ? c + a1 - kAngPad : c - a2 - kAngPad;
    const float v = side ? c + a2 + kAngPad : c - a1 + kAngPad;
    m |= bin_span(u, v, mn, mx, inv);
    if (v > kPiF - kAngPad) m |= bin_span(u - k2PiF, v - k2PiF, mn, mx, inv);
    if (u < -kPiF + kAngPad) m |= bin_span(u + k2PiF, v + k2PiF, mn, mx, inv);
  }
  return m;
}

// each lane's inlier hit per layer: a row in LDS (caps up to 128), or eight
// registers of two 16-bit entries (larger caps, whose LDS limits residency)
template <bool REG>
struct InlierRow {
  uint16_t* row;
  __device__ __forceinline__ void init(uint16_t* r) {
    row = r;
    for (int L = 0; L < HT_MAX_LAYERS; ++L) row[L] = kNoHit;
  }
  __device__ __forceinline__ void set(int L, uint16_t v) { row[L] = v; }
  __device__ __forceinline__ int get(int L) const { return row[L]; }
};
template <>
struct InlierRow<true> {
  // eight words of two 16-bit entries, layer L in word L / 2 (named
  // registers selected by a switch on the wave-uniform layer: an indexed
  // array would be placed in scratch memory)
  uint32_t w0, w1, w2, w3, w4, w5, w6, w7;
  __device__ __forceinline__ void init(uint16_t*) {
    w0 = w1 = w2 = w3 = w4 = w5 = w6 = w7 = 0xffffffffu;
  }
  // L must be the same in every lane
  __device__ __forceinline__ void set(int L, uint16_t v) {
    const int Lu = __builtin_amdgcn_readfirstlane(L);
    const uint32_t sh = (uint32_t)(Lu & 1) * 16u;
    const uint32_t keep = ~(0xffffu << sh);
    const uint32_t val = (uint32_t)v << sh;
    switch (Lu >> 1) {
      case 0: w0 = (w0 & keep) | val; break;
      case 1: w1 = (w1 & keep) | val; break;
      case 2: w2 = (w2 & keep) | val; break;
      case 3: w3 = (w3 & keep) | val; break;
      case 4: w4 = (w4 & keep) | val; break;
      case 5: w5 = (w5 & keep) | val; break;
      case 6: w6 = (w6 & keep) | val; break;
      default: w7 = (w7 & keep) | val; break;
    }
  }
  // L must be the same in every lane
  __device__ __forceinline__ int get(int L) const {
    const int Lu = __builtin_amdgcn_readfirstlane(L);
    uint32_t x;
    switch (Lu >> 1) {
      case 0: x = w0; break;
      case 1: x = w1; break;
      case 2: x = w2; break;
      case 3: x = w3; break;
      case 4: x = w4; break;
      case 5: x = w5; break;
      case 6: x = w6; break;
      default: x = w7; break;
    }
    return (int)((x >> ((Lu & 1) * 16)) & 0xffffu);
  }
  // lane win's entry for layer L (L may differ between lanes; every lane calls it)
  __device__ __forceinline__ int of_lane(int win, int L) const {
    const int i = (L >> 1) & 7;
    uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)w0, win);
    x = i == 1 ? (uint32_t)__builtin_amdgcn_readlane((int)w1, win) : x;
    x = i == 2 ? (uint32_t)__builtin_amdgcn_readlane((int)w2, win) : x;
    x = i == 3 ? (uint32_t)__builtin_amdgcn_readlane((int)w3, win) : x;
    x = i == 4 ? (uint32_t)__builtin_amdgcn_readlane((int)w4, win) : x;
    x = i == 5 ? (uint32_t)__builtin_amdgcn_readlane((int)w5, win) : x;
    x = i == 6 ? (uint32_t)__builtin_amdgcn_readlane((int)w6, win) : x;
    x = i == 7 ? (uint32_t)__builtin_amdgcn_readlane((int)w7, win) : x;
    return (int)((x >> ((L & 1) * 16)) & 0xffffu);
  }
};


template <int CAP>
struct WaveMem {
  // grouped by layer (and by azimuth bin within a layer for caps above 128);
  // above cap 128, before the grouping, its first CAP floats hold each
  // member's relative azimuth in pool order
  Mem4 mem[CAP];
  union {
    // members in pool order before grouping, staged in LDS for CAP <= 128;
    // larger caps stage them in registers (LDS, not registers, limits their
    // occupancy)
    RawMembers<(CAP <= 128 ? CAP : 1)> raw;
    LayerStats st;  // caps above 128, until the bins are set
    // each lane's inlier per layer, kNoHit if none (caps up to 128; larger
    // caps keep them in registers)
    uint16_t hit[CAP <= 128 ? kWave : 1][HT_MAX_LAYERS + 2];
  } u;
  LayerBins<(CAP > 128)> lb;
  int32_t lstart[HT_MAX_LAYERS + 1];
  int32_t lcnt[HT_MAX_LAYERS + 1];
  int32_t seed[3][4];
};

// Waves of a refine workgroup work on different candidates and share
// nothing; each has its own LDS area, as many as the LDS of a CU allows at
// good occupancy.  Ordering of a wave's own LDS accesses needs only a
// wave-scope fence.
template <int CAP>
struct RefineShape {
  static constexpr int kWaves = CAP <= 128 ? 4 : (CAP <= 256 ? 2 : 1);
  // waves per SIMD the register budget is set for (the second launch bound
  // of HIP): seven for caps up to 128 (72 registers, a few spilled; the LDS
  // of seven four-wave workgroups fits; 4% faster than six waves without the
  // spill on the displaced-jet workload); four at cap 512 (128 registers, a few spilled; sixteen
  // one-wave workgroups of 10 KB fit the LDS; 4% faster than three waves
  // with no spill on the 55k-hit workload); two at cap 1024 (at most 256
  // registers, so that the eight one-wave workgroups the LDS allows can all
  // be resident); else left to the compiler
  static constexpr int kMinWavesPerSimd =
      CAP <= 128 ? 7 : (CAP >= 1024 ? 2 : (CAP == 512 ? 4 : 1));
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave reductions with DPP: within each row of 16 lanes, xor-1 and xor-2
// quad permutes, then the half-row and row mirrors leave the row's result in
// every lane; the four row results are read into scalars.  No LDS round
// trips.  Called with all 64 lanes active.
template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}
constexpr int kQuadXor1 = 0xb1;   // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4e;   // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;

template <typename Op>
__device__ __forceinline__ int wave_reduce_i32(int v, Op op) {
  v = op(v, dpp<kQuadXor1>(v));
  v = op(v, dpp<kQuadXor2>(v));
  v = op(v, dpp<kRowHalfMirror>(v));
  v = op(v, dpp<kRowMirror>(v));
  const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
  const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
  return op(op(r0, r1), op(r2, r3));
}

__device__ __forceinline__ int wave_max_i32(int v) {
  return wave_reduce_i32(v, [](int a, int b) { return a > b ? a : b; });
}
__device__ __forceinline__ unsigned wave_or(unsigned v) {
  return (unsigned)wave_reduce_i32((int)v, [](int a, int b) { return a | b; });
}
// maximum of non-negative floats (their bit patterns order like the values)
__device__ __forceinline__ float wave_max_nonneg(float v) {
  return __int_as_float(wave_max_i32(__float_as_int(v)));
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
  auto step = [](unsigned long long x, unsigned long long o) { return o < x ? o : x; };
  auto perm = [](unsigned long long x, auto tag) {
    constexpr int C = decltype(tag)::value;
    const unsigned lo = (unsigned)dpp<C>((int)(unsigned)x);
    const unsigned hi = (unsigned)dpp<C>((int)(unsigned)(x >> 32));
    return ((unsigned long long)hi << 32) | lo;
  };
  v = step(v, perm(v, std::integral_constant<int, kQuadXor1>{}));
  v = step(v, perm(v, std::integral_constant<int, kQuadXor2>{}));
  v = step(v, perm(v, std::integral_constant<int, kRowHalfMirror>{}));
  v = step(v, perm(v, std::integral_constant<int, kRowMirror>{}));
  unsigned long long r = ~0ull;
#pragma unroll
  for (int row = 0; row < 4; ++row) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, row * 16);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), row * 16);
    r = step(r, ((unsigned long long)hi << 32) | lo);
  }
  return r;
}

// inclusive prefix sum within each row of 16 lanes (row_shr with zero fill)
__device__ __forceinline__ int row_scan_incl(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  return v;
}

// index of the n-th (0-based) set bit of a 16-bit mask
__device__ __forceinline__ int nth_set_bit(unsigned mask, int n) {
  for (int L = 0; L < HT_MAX_LAYERS; ++L) {
    if ((mask >> L) & 1u) {
      if (n == 0) return L;
      --n;
    }
  }
  return HT_MAX_LAYERS - 1;
}

template <int CAP, int NB>
__global__ __launch_bounds__(RefineShape<CAP>::kWaves * kWave, RefineShape<CAP>::kMinWavesPerSimd) void
refine_kernel(AssocBatch<NB> AB, int n_lo, int n_hi) {
  const AssocArgs& A = event_args(AB);
  constexpr int W = RefineShape<CAP>::kWaves;
  // members per chunk of the road loop (registers: 4 per member); the
  // short member lists of caps up to 128 keep one member at a time, which
  // leaves the registers for a fifth wave per SIMD
  constexpr int kChunk = CAP <= 128 ? 1 : 8;
  // passing members per lane and layer whose float64 distances wait for the
  // end of the layer (chunked path)
  constexpr int kDefer = 4;
  __shared__ WaveMem<CAP> MW[W];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6;
  WaveMem<CAP>& M = MW[wave];
  const int np = n_cands(A);
  const ht_cluster_cfg& cfg = A.cfg;
  const int cap = cfg.member_cap;
  const double road = (double)cfg.road_sigmas * (double)cfg.sigma_rphi;
  // the wave's rarely changed totals (candidates over member_cap, member
  // pairs) stay in its LDS slot, kept by lane 0, rather than in registers
  // live across the whole search
  __shared__ unsigned long long tot[W][5];
  if (lane == 0) {
    tot[wave][2] = 0;
    tot[wave][3] = 0;
  }
  unsigned long long tests = 0, ncand = 0;
  uint32_t exec = 0;  // this lane's float64 circle distances
  // above cap 128 the next candidate's cell and member count are requested
  // while this one is worked on (two registers; at cap 128 they would cost
  // the kernel its occupancy)
  constexpr bool kAhead = CAP > 128;
  const int pstep = gridDim.x * W;
  int lin_a = -1, n_a = 0;
  if (kAhead && blockIdx.x * W + wave < np) {
    lin_a = A.peaks[blockIdx.x * W + wave].lin;
    n_a = A.mcount[blockIdx.x * W + wave];
  }
  for (int p = blockIdx.x * W + wave; p < np; p += pstep) {
    const int lin = kAhead ? lin_a : A.peaks[p].lin;
    const int n = kAhead ? n_a : A.mcount[p];
    if (kAhead && p + pstep < np) {
      lin_a = A.peaks[p + pstep].lin;
      n_a = A.mcount[p + pstep];
    }
    // a launch takes the candidates with n_lo <= n <= n_hi (the others are
    // another launch's)
    if (n < n_lo || n > n_hi) continue;
    if (lin < 0 || lin >= A.n_cells) {
      if (lane == 0) { A.cstat[p] = -1; A.cnl[p] = 0; }
      continue;
    }
    if (n > cap) {
      if (lane == 0) { A.cstat[p] = -2; A.cnl[p] = 0; tot[wave][2] += 1; }
      continue;
    }
    if (lane == 0) tot[wave][3] += (unsigned long long)n;
    const int col = lin / A.n_phi;
    const int j = col % A.n_qpt;
    const int k = col / A.n_qpt;
    const double kapc = A.kapc[j], d0c = A.d0c[k];  // issued early, used by the box check
    const size_t moff = (size_t)p * cap;
    // azimuth origin of the angle bins: the cell's phi0 centre
    const float ref = -kPiF + ((float)(lin - col * A.n_phi) + 0.5f) * (k2PiF / (float)A.n_phi);
    constexpr bool kRawLds = CAP <= 128;
    constexpr int RM = kRawLds ? 1 : CAP / kWave;
    Mem4 rec[RM];
    int rL[RM];
    unsigned lmask = 0;
    float qmax = 0.0f;
    if constexpr (kRawLds) {
      // load members in pool order
      for (int m = lane; m < n; m += kWave) {
        const uint2 pe = A.pool[moff + m];
        const int h = (int)(pe.x & 0xffffu);
        const int L = (int)(pe.x >> 16);
        const float4 hb = A.hitB[h];
        Mem4 r4;
        r4.x = hb.x;
        r4.y = hb.y;
        r4.adx = __uint_as_float(pe.y);
        r4.h = h;
        M.u.raw.mem[m] = r4;
        M.u.raw.L[m] = (int8_t)L;
        lmask |= 1u << L;
        qmax = fmaxf(qmax, mem_q(r4));
      }
    } else {
      // the layers' radius and azimuth ranges start empty; the group counts at 0
      if constexpr (!kRawLds) {
        if (lane < HT_MAX_LAYERS) {
          M.u.st.rlo[lane] = 0x7fffffff;
          M.u.st.rhi[lane] = 0;
          M.u.st.alo[lane] = 0x7fffffff;
          M.u.st.ahi[lane] = (int32_t)0x80000000;
        }
        for (int e = lane; e <= kBinKeys / 2; e += kWave) M.lb.bpack[e] = 0u;
      }
      wave_sync();
      // load members in pool order into registers: member lane + 64 t is
      // entry t of the lane (n <= cap <= CAP); each member's radius and
      // azimuth (the hit's inputs) widen its layer's ranges
#pragma unroll
      for (int t = 0; t < RM; ++t) {
        const int m = lane + t * kWave;
        rL[t] = -1;
        if (m < n) {
          const uint2 pe = A.pool[moff + m];
          const int h = (int)(pe.x & 0xffffu);
          const int L = (int)(pe.x >> 16);
          const float4 hb = A.hitB[h];
          rec[t].x = hb.x;
          rec[t].y = hb.y;
          rec[t].adx = __uint_as_float(pe.y);
          rec[t].h = h;
          rL[t] = L;
          lmask |= 1u << L;
          qmax = fmaxf(qmax, mem_q(rec[t]));
          const float rel = rel_angle(hb.w, ref);
          reinterpret_cast<float*>(M.mem)[m] = rel;
          atomicMin(&M.u.st.rlo[L], __float_as_int(hb.z));
          atomicMax(&M.u.st.rhi[L], __float_as_int(hb.z));
          atomicMin(&M.u.st.alo[L], ord_bits(rel));
          atomicMax(&M.u.st.ahi[L], ord_bits(rel));
        }
      }
    }
    lmask = wave_or(lmask);
    qmax = wave_max_nonneg(qmax);
    const float rmax = __builtin_sqrtf(qmax) * 1.0001f;
    const int nS = __popc(lmask);
    if (nS < cfg.min_layers || nS < 3) {
      if (lane == 0) { A.cstat[p] = -1; A.cnl[p] = nS; }
      wave_sync();
      continue;
    }
    // group members by layer (and, above cap 128, by azimuth bin within the
    // layer): counting sort with LDS atomics (order within a group does not
    // matter, every selection breaks ties on the hit index)
    int ls;  // lane L < 16: start of layer L; lane 16: the member count
    if constexpr (kRawLds) {
      if (lane <= HT_MAX_LAYERS) M.lcnt[lane] = 0;
      wave_sync();
      for (int m = lane; m < n; m += kWave)
        M.u.raw.slot[m] = (int16_t)atomicAdd(&M.lcnt[M.u.raw.L[m]], 1);
      wave_sync();
      // layer starts: exclusive scan of the 16 layer counts in the first row
      // of lanes; lane 16 holds the total
      {
        const int c = lane < HT_MAX_LAYERS ? M.lcnt[lane] : 0;
        const int incl = row_scan_incl(c);
        const int total = __builtin_amdgcn_readlane(incl, HT_MAX_LAYERS - 1);
        ls = lane < HT_MAX_LAYERS ? incl - c : total;
        if (lane <= HT_MAX_LAYERS) M.lstart[lane] = ls;
      }
      wave_sync();
      for (int m = lane; m < n; m += kWave) {
        const int e = M.lstart[M.u.raw.L[m]] + M.u.raw.slot[m];
        M.mem[e] = M.u.raw.mem[m];
      }
    } else {
      wave_sync();
      // the layers' bin parameters
      if (lane < HT_MAX_LAYERS) {
        const float mn = ord_float(M.u.st.alo[lane]), mx = ord_float(M.u.st.ahi[lane]);
        M.lb.lr[lane] = M.u.st.rlo[lane] == M.u.st.rhi[lane] ? __int_as_float(M.u.st.rlo[lane]) : 0.0f;
        M.lb.lmn[lane] = mn;
        M.lb.lmx[lane] = mx;
        const float span = mx - mn;
        M.lb.linv[lane] = span > 1e-30f ? (float)kNB / span : 0.0f;
      }
      wave_sync();
#pragma unroll
      for (int t = 0; t < RM; ++t) {
        if (rL[t] < 0) continue;
        const int L = rL[t];
        const int key = L * kNB + angle_bin(reinterpret_cast<const float*>(M.mem)[lane + t * kWave],
                                            M.lb.lmn[L], M.lb.linv[L]);
        // group and slot in one register (key < 512, slot < 1024)
        const int sh = (key & 1) * 16;
        const uint32_t old = atomicAdd(&M.lb.bpack[key >> 1], 1u << sh);
        rL[t] = key | ((int)((old >> sh) & 0xffffu) << 10);
      }
      wave_sync();
      // group starts: exclusive scan of the kBinKeys counts, lane l owning
      // groups G l .. G l + G - 1
      {
        constexpr int G = kBinKeys / kWave;  // groups per lane, G / 2 words
        static_assert(kBinKeys == G * kWave && G % 2 == 0, "whole words per lane");
        uint32_t c[G / 2];
        int sum = 0;
#pragma unroll
        for (int i = 0; i < G / 2; ++i) {
          c[i] = M.lb.bpack[(G / 2) * lane + i];
          sum += (int)(c[i] & 0xffffu) + (int)(c[i] >> 16);
        }
        const int incl = wave_incl_scan_i32(sum, lane);
        int run = incl - sum;
#pragma unroll
        for (int i = 0; i < G / 2; ++i) {
          const int lo = run;
          run += (int)(c[i] & 0xffffu);
          M.lb.bpack[(G / 2) * lane + i] = (uint32_t)lo | ((uint32_t)run << 16);
          run += (int)(c[i] >> 16);
        }
        if (lane == kWave - 1) M.lb.bpack[kBinKeys / 2] = (uint32_t)incl;
      }
      wave_sync();
      ls = M.lb.start(lane < HT_MAX_LAYERS ? lane * kNB : kBinKeys);
      if (lane <= HT_MAX_LAYERS) M.lstart[lane] = ls;
#pragma unroll
      for (int t = 0; t < RM; ++t) {
        if (rL[t] < 0) continue;
        const int e = M.lb.start(rL[t] & 0x3ff) + (rL[t] >> 10);
        M.mem[e] = rec[t];
      }
    }
    wave_sync();
    // seed layers: innermost, middle and outermost of the outer min(nS, min_layers)
    const int span = nS < cfg.min_layers ? nS : cfg.min_layers;
    const int Ls[3] = {nth_set_bit(lmask, nS - span),
                       nth_set_bit(lmask, nS - span + (span - 1) / 2), nth_set_bit(lmask, nS - 1)};
    // seed_k nearest members per seed layer, by rank of (adx, h)
    const int kk = cfg.seed_k;
    int ns[3], sst[3], sen[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      sst[s] = __builtin_amdgcn_readlane(ls, Ls[s]);
      sen[s] = __builtin_amdgcn_readlane(ls, Ls[s] + 1);
      ns[s] = sen[s] - sst[s] < kk ? sen[s] - sst[s] : kk;
    }
    const int n0 = sen[0] - sst[0], n1 = sen[1] - sst[1], n2 = sen[2] - sst[2];
    if (n0 + n1 + n2 <= kWave) {
      // the three seed layers side by side: lane -> (seed layer, member)
      int s = -1, st = 0, en = 0;
      if (lane < n0) { s = 0; st = sst[0]; en = sen[0]; }
      else if (lane < n0 + n1) { s = 1; st = sst[1]; en = sen[1]; }
      else if (lane < n0 + n1 + n2) { s = 2; st = sst[2]; en = sen[2]; }
      const int e = st + lane - (s == 1 ? n0 : (s == 2 ? n0 + n1 : 0));
      unsigned long long key = 0;
      if (s >= 0) key = ((unsigned long long)__float_as_uint(M.mem[e].adx) << 32) | (unsigned)M.mem[e].h;
      const int nmax = max(n0, max(n1, n2));
      int rank = 0;
      // every lane reads every round (the reads of four rounds in flight
      // together); rounds past the lane's own layer read a record inside the
      // member list and do not count
#pragma unroll 4
      for (int t = 0; t < nmax; ++t) {
        const int e2 = st + t;
        const Mem4 m2 = M.mem[e2 < n ? e2 : n - 1];
        const unsigned long long k2 =
            ((unsigned long long)__float_as_uint(m2.adx) << 32) | (unsigned)m2.h;
        rank += (s >= 0 && e2 < en && k2 < key) ? 1 : 0;
      }
      if (s >= 0 && rank < kk) M.seed[s][rank] = e;
    } else {
      // more members than lanes: the ns[s] smallest keys of each seed layer
      // by repeated wave minima; lane l holds members st + l + 64 t, and the
      // keys are distinct (a hit is a member once), so each minimum has one
      // owner, which records it and leaves it out of the next round
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const int st = sst[s], en = sen[s];
        if (en - st <= kWave) {
          // a layer of at most 64 members: each lane's key is read once
          const int e = st + lane;
          unsigned long long key = ~0ull;
          if (e < en) key = ((unsigned long long)__float_as_uint(M.mem[e].adx) << 32) | (unsigned)M.mem[e].h;
          for (int r = 0; r < ns[s]; ++r) {
            const unsigned long long best = wave_min_u64(key);
            if (e < en && key == best) {
              M.seed[s][r] = e;
              key = ~0ull;
            }
          }
          continue;
        }
        unsigned long long taken = 0;
        for (int r = 0; r < ns[s]; ++r) {
          unsigned long long mine = ~0ull;
          int arg = -1;
          for (int e = st + lane, t = 0; e < en; e += kWave, ++t) {
            if ((taken >> t) & 1ull) continue;
            const unsigned long long key =
                ((unsigned long long)__float_as_uint(M.mem[e].adx) << 32) | (unsigned)M.mem[e].h;
            if (key < mine) { mine = key; arg = t; }
          }
          const unsigned long long best = wave_min_u64(mine);
          if (arg >= 0 && mine == best) {
            M.seed[s][r] = st + lane + arg * kWave;
            taken |= 1ull << arg;
          }
        }
      }
    }
    // the grouped raw records are dead from here on; the union holds the
    // per-lane inlier rows (caps up to 128)
    InlierRow<(kChunk > 1)> hitL;
    hitL.init(M.u.hit[kChunk > 1 ? 0 : lane]);
    wave_sync();
    if (A.origin_seed) ns[0] = 1;
    // one combination per lane: lane = 16 a + 4 b + c (seed_k <= 4), which
    // orders the lanes like the combinations (a, b, c)
    const int a = lane >> 4, b = (lane >> 2) & 3, c = lane & 3;
    double cA = 0.0, cB = 0.0, cC = 0.0, cD = 0.0;
    bool ok = false;
    if (a < ns[0] && b < ns[1] && c < ns[2]) {
      const int ha = M.mem[M.seed[0][a]].h, hb = M.mem[M.seed[1][b]].h;
      const int hc = M.mem[M.seed[2][c]].h;
      double xa = 0.0, ya = 0.0;
      if (!A.origin_seed) { xa = A.hx[ha]; ya = A.hy[ha]; }
      ok = circle3(xa, ya, A.hx[hb], A.hy[hb], A.hx[hc], A.hy[hc], &cA, &cB, &cC, &cD);
      if (ok) {
        double ktol = (0.5 + (double)cfg.box_margin) * A.kap_bin;
        if (ktol < 1e-6) ktol = 1e-6;
        const double dtol = (0.5 + (double)cfg.box_margin) * A.d0_bin + road;
        const double kap = 2.0 * cA;
        const double sq = sqrt(cB * cB + cC * cC);
        const double d0 = 2.0 * cD / (1.0 + sq);
        ok = (fabs(kap - kapc) <= ktol) && (fabs(d0 - d0c) <= dtol);
      }
    }
    // |dist| >= |f| / (1 + |A||f|): a member with |f| > road / (1 - road |A|)
    // cannot be within the road, and road / (1 - x) <= road (1 + 2x) for
    // x <= 1/2, a bound without a division.  The float32 test allows a margin of 2e-6
    // of a bound on the magnitudes of the terms and partial sums over all
    // members (|x|, |y| <= rmax, q <= qmax), far above what the rounding of
    // the coefficients, of the coordinates, of q = x^2 + y^2 recomputed in
    // float32 and of three fused multiply-adds can move f (< 8e-7 of that
    // bound), so it never drops a member the float64 test keeps.
    float Af = 0.0f, Bf = 0.0f, Cf = 0.0f, Df = 0.0f, thr = -1.0f;
    float Rf = 0.0f, phB = 0.0f;  // |(B, C)| and its direction (angle bins)
    if (ok) {
      const double ra = road * fabs(cA);
      const float pre = ra <= 0.5 ? (float)(road * (1.0 + 2.0 * ra) * 1.000001) : __builtin_inff();
      Af = (float)cA;
      Bf = (float)cB;
      Cf = (float)cC;
      Df = (float)cD;
      const float mag = fabsf(Af) * qmax + (fabsf(Bf) + fabsf(Cf)) * rmax + fabsf(Df);
      thr = pre + mag * 2e-6f;
      if constexpr (kChunk > 1) {
        Rf = __builtin_sqrtf(Bf * Bf + Cf * Cf);
        phB = atan2f(Cf, Bf);
      }
    }
    // road tests the method defines for this candidate: every member
    // against every admissible seed circle
    tests += (unsigned long long)__popcll(__ballot(ok)) * (unsigned long long)n;
    int n_in = ok ? 0 : -1;
    bool active = ok;
    // visiting order: the layers that are not seed layers by increasing
    // member count (then index), so that lanes meet a layer without an
    // inlier early and drop out after few members; then the seed layers.
    // The per-lane outcome does not depend on the order.
    const unsigned smask = (1u << Ls[0]) | (1u << Ls[1]) | (1u << Ls[2]);
    const unsigned nsm = lmask & ~smask;
    const int n_ns = __popc(nsm);
    int orderv = 0;  // lane i: the i-th layer to visit
    {
      const int nxt = __shfl_down(ls, 1, kWave);  // start of the next layer
      const bool mine = lane < HT_MAX_LAYERS && ((nsm >> lane) & 1u);
      const int key = mine ? (((nxt - ls) << 4) | lane) : 0x7fffffff;
      int rank = 0;
      for (int t = 0; t < HT_MAX_LAYERS; ++t) rank += __shfl(key, t, kWave) < key ? 1 : 0;
      // lane rank receives the layer of that rank (a forward permute; the
      // other lanes send to lane 63, whose value is never read)
      orderv = __builtin_amdgcn_ds_permute((mine ? rank : kWave - 1) * 4, lane);
    }
    unsigned sseq = smask;
    int remaining = nS;
    for (int it = 0; it < nS; ++it) {
      int L;
      if (it < n_ns) {
        L = __builtin_amdgcn_readlane(orderv, it);
      } else {
        L = __builtin_ctz(sseq);
        sseq &= sseq - 1u;
      }
      --remaining;
      if (active && n_in + remaining + 1 < cfg.min_layers) {
        active = false;
        n_in = -2;
      }
      if (__ballot(active) == 0ull) break;
      const int st = __builtin_amdgcn_readlane(ls, L);
      const int en = __builtin_amdgcn_readlane(ls, L + 1);
      double bd = 0.0;
      int bh = -1;
      // members in chunks: the chunk's LDS reads (broadcasts, every lane
      // reads the same member) are issued together, then the float32
      // pre-filter of each lane's circle marks the members worth a float64
      // distance; the selection (smallest distance, then hit index) does not
      // depend on the visiting order
      if constexpr (kChunk == 1) {
        for (int e = st; e < en; ++e) {
          const Mem4 v = M.mem[e];
          const float f32 =
              __builtin_fmaf(Af, mem_q(v), __builtin_fmaf(Bf, v.x, __builtin_fmaf(Cf, v.y, Df)));
          if (!(active && fabsf(f32) <= thr)) continue;
          const int hh = v.h;
          ++exec;
          const double dist = fabs(circle_dist(cA, cB, cC, cD, A.hx[hh], A.hy[hh], A.hq[hh]));
          if (!(dist <= road)) continue;
          if (bh < 0 || dist < bd || (dist == bd && hh < bh)) { bh = hh; bd = dist; }
        }
      } else {
        // The float64 distances of the members that pass are deferred to the
        // end of the layer, where the loads of their float64 coordinates
        // (L2 gathers) are issued together: one round trip per layer instead
        // of one per chunk with a pass.  A lane with more than kDefer passes
        // in the layer takes the others at once.
        int q[kDefer];
#pragma unroll
        for (int t = 0; t < kDefer; ++t) q[t] = -1;
        int nq = 0;
        auto take = [&](int hh) {
          ++exec;
          if (nq < kDefer) {
#pragma unroll
            for (int t = 0; t < kDefer; ++t) q[t] = nq == t ? hh : q[t];
            ++nq;
            return;
          }
          const double dist = fabs(circle_dist(cA, cB, cC, cD, A.hx[hh], A.hy[hh], A.hq[hh]));
          if (!(dist <= road)) return;
          if (bh < 0 || dist < bd || (dist == bd && hh < bh)) { bh = hh; bd = dist; }
        };
        const float lr = M.lb.lr[L];
        if (lr > 0.0f) {
          // every member of the layer has radius lr: each lane reads only the
          // members of the azimuth bins its road reaches
          unsigned bm = active ? road_bins(lr, Af, Df, Rf, phB, thr, ref, M.lb.lmn[L],
                                           M.lb.lmx[L], M.lb.linv[L])
                               : 0u;
          const int kb = L * kNB;
          int e = 0, eend = 0;
          for (;;) {
            while (e >= eend && bm) {
              const int b0 = __builtin_ctz(bm);
              int b1 = b0;  // adjacent bins are one contiguous run
              while (b1 + 1 < kNB && ((bm >> (b1 + 1)) & 1u)) ++b1;
              bm &= ~(((2u << b1) - 1u) & ~((1u << b0) - 1u));
              e = M.lb.start(kb + b0);
              eend = M.lb.start(kb + b1 + 1);
            }
            const bool has = e < eend;
            if (__ballot(has) == 0ull) break;
            if (has) {
              // up to four members of the run at once (their reads in flight together)
              constexpr int kW = 4;
              Mem4 v[kW];
#pragma unroll
              for (int u = 0; u < kW; ++u) v[u] = M.mem[min(e + u, eend - 1)];
              const int cnt = min(kW, eend - e);
              e += cnt;
#pragma unroll
              for (int u = 0; u < kW; ++u) {
                const float f32 = __builtin_fmaf(
                    Af, mem_q(v[u]), __builtin_fmaf(Bf, v[u].x, __builtin_fmaf(Cf, v[u].y, Df)));
                if (u < cnt && fabsf(f32) <= thr) take(v[u].h);
              }
            }
          }
        } else {
          for (int e0 = st; e0 < en; e0 += kChunk) {
            Mem4 v[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) v[u] = M.mem[min(e0 + u, en - 1)];
            unsigned pass = 0;
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
              const float f32 = __builtin_fmaf(
                  Af, mem_q(v[u]), __builtin_fmaf(Bf, v[u].x, __builtin_fmaf(Cf, v[u].y, Df)));
              pass |= (fabsf(f32) <= thr ? 1u : 0u) << u;
            }
            const int left = en - e0;
            if (!active) pass = 0;
            if (left < kChunk) pass &= (1u << left) - 1u;
            while (pass) {
              const int u = __builtin_ctz(pass);
              pass &= pass - 1u;
              take(M.mem[e0 + u].h);
            }
          }
        }
        double qx[kDefer], qy[kDefer], qq[kDefer];
#pragma unroll
        for (int t = 0; t < kDefer; ++t) {
          qx[t] = qy[t] = qq[t] = 0.0;
          if (q[t] >= 0) {
            qx[t] = A.hx[q[t]];
            qy[t] = A.hy[q[t]];
            qq[t] = A.hq[q[t]];
          }
        }
#pragma unroll
        for (int t = 0; t < kDefer; ++t) {
          if (q[t] < 0) continue;
          const int hh = q[t];
          const double dist = fabs(circle_dist(cA, cB, cC, cD, qx[t], qy[t], qq[t]));
          if (!(dist <= road)) continue;
          if (bh < 0 || dist < bd || (dist == bd && hh < bh)) { bh = hh; bd = dist; }
        }
      }
      if (active) {
        hitL.set(L, bh < 0 ? kNoHit : (uint16_t)bh);
        if (bh >= 0) ++n_in;
      }
    }
    // best lane: most inliers, then smallest sum, then lowest combination index
    const int best_n = wave_max_i32(n_in);
    if (best_n < cfg.min_layers) {
      if (lane == 0) { A.cstat[p] = -1; A.cnl[p] = nS; }
      wave_sync();
      continue;
    }
    double ss = 0.0;
    if (kChunk == 1 && n_in == best_n) {
      for (unsigned lm = lmask; lm; lm &= lm - 1u) {
        const int hh = hitL.get(__builtin_ctz(lm));
        if (hh == kNoHit) continue;
        ++exec;
        const double d = fabs(circle_dist(cA, cB, cC, cD, A.hx[hh], A.hy[hh], A.hq[hh]));
        ss += d * d;
      }
    } else if (n_in == best_n) {
      // above cap 128: four layers at a time, their coordinate loads in
      // flight together, then the sum in layer order (at cap 128 the
      // registers would cost the kernel its occupancy)
      for (unsigned lm = lmask; lm;) {
        int hq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          hq[u] = kNoHit;
          if (lm) {
            hq[u] = hitL.get(__builtin_ctz(lm));
            lm &= lm - 1u;
          }
        }
        double X[4], Y[4], Q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int h = hq[u] == kNoHit ? 0 : hq[u];
          X[u] = A.hx[h];
          Y[u] = A.hy[h];
          Q[u] = A.hq[h];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (hq[u] == kNoHit) continue;
          ++exec;
          const double d = fabs(circle_dist(cA, cB, cC, cD, X[u], Y[u], Q[u]));
          ss += d * d;
        }
      }
    }
    unsigned long long key = ~0ull;
    if (n_in == best_n) key = (unsigned long long)__double_as_longlong(ss);
    const unsigned long long best_ss = wave_min_u64(key);
    const unsigned long long ballot = __ballot(n_in == best_n && key == best_ss);
    const int win = __builtin_ctzll(ballot);
    if (lane == win) {
      A.cstat[p] = best_n;
      A.cnl[p] = nS;
      double* g = A.cgeo + (size_t)p * 5;
      g[0] = ss; g[1] = cA; g[2] = cB; g[3] = cC; g[4] = cD;
    }
    ++ncand;
    wave_sync();
    int whh;
    if constexpr (kChunk > 1)
      whh = hitL.of_lane(win, lane);
    else
      whh = lane < HT_MAX_LAYERS ? (int)M.u.hit[win][lane] : 0;
    if (lane < HT_MAX_LAYERS) {
      A.chit[(size_t)p * HT_MAX_LAYERS + lane] = whh == kNoHit ? -1 : whh;
      if (whh != kNoHit)
        atomicMax(&A.owner_key[whh], own_key(best_n, __longlong_as_double((long long)best_ss), p));
    }
    wave_sync();
  }
  // the workgroup's totals, one atomic per counter from lanes 0-4 of wave 0
  unsigned long long ex = exec;
  for (int off = kWave / 2; off > 0; off >>= 1) ex += __shfl_xor(ex, off);
  if (lane == 0) {
    tot[wave][0] = tests;
    tot[wave][1] = ncand;
    tot[wave][4] = ex;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    unsigned long long v = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) v += tot[w][threadIdx.x];
    const int slot = blockIdx.x & (kSpread - 1);
    if (v) atomicAdd(&A.spread[(size_t)(threadIdx.x * kSpread + slot) * kSpreadStride], v);
  }
}

// ---- ownership -----------------------------------------------------------------
// (the seed search offers each inlier hit its candidate's key, own_key)
__device__ __forceinline__ int owned_count(const AssocArgs& A, int p) {
  int own = 0;
  for (int L = 0; L < HT_MAX_LAYERS; ++L) {
    const int h = A.chit[(size_t)p * HT_MAX_LAYERS + L];
    if (h >= 0 && (int)(0x3ffffff - (A.owner_key[h] & 0x3ffffffull)) == p) ++own;
  }
  return own;
}

__device__ __forceinline__ bool survives(const AssocArgs& A, int p, int* own) {
  if (A.cstat[p] < 0) return false;
  *own = owned_count(A, p);
  return *own >= A.cfg.min_layers;
}

// survivor counts per 256-candidate tile, and their sums per group of 64
// tiles (zeroed by init_kernel)
template <int NB>
__global__ __launch_bounds__(256) void surv_count_kernel(AssocBatch<NB> AB, int tiles) {
  const AssocArgs& A = event_args(AB);
  __shared__ int32_t wc[4];
  const int np = n_cands(A);
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int p = tile * 256 + threadIdx.x;
    int own = 0;
    const bool s = p < np && survives(A, p, &own);
    const uint64_t m = __ballot(s);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
      const int c = wc[0] + wc[1] + wc[2] + wc[3];
      A.ctile_cnt[tile] = c;
      if (c) atomicAdd(&A.ctile_off[tile >> 6], c);
    }
    __syncthreads();
  }
}

// The survivors as tracks, in candidate order: a tile's first track index is
// the sum of the group sums before its group and of the tile counts before
// it in its group (wave 0 reads both, 64 at a time); the last tile writes
// the track count.
template <int NB>
__global__ __launch_bounds__(256) void surv_emit_kernel(AssocBatch<NB> AB, int tiles) {
  const AssocArgs& A = event_args(AB);
  __shared__ int32_t wc[4];
  __shared__ int32_t base_s;
  const int np = n_cands(A);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    if (wave == 0) {
      const int g = tile >> 6;
      int b = 0;
      for (int q = lane; q < g; q += kWave) b += A.ctile_off[q];
      if (g * 64 + lane < tile) b += A.ctile_cnt[g * 64 + lane];
      for (int off = kWave / 2; off > 0; off >>= 1) b += __shfl_xor(b, off);
      if (lane == 0) base_s = b;
    }
    const int p = tile * 256 + threadIdx.x;
    int own = 0;
    const bool s = p < np && survives(A, p, &own);
    const uint64_t m = __ballot(s);
    if (lane == 0) wc[wave] = __popcll(m);
    __syncthreads();
    if (tile == tiles - 1 && threadIdx.x == 0) A.sc[S_NTRK] = base_s + wc[0] + wc[1] + wc[2] + wc[3];
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wc[w];
    if (s) {
      const uint64_t lower = lane ? (m & ((1ull << lane) - 1ull)) : 0ull;
      const int t = base_s + before + __popcll(lower);
      if (t < A.out.track_cap) {
        ht_track tr;
        tr.peak = p;
        tr.lin = A.peaks[p].lin;
        tr.votes = A.peaks[p].votes;
        tr.n_layers = A.cnl[p];
        tr.n_inliers = A.cstat[p];
        tr.n_owned = own;
        tr.status = 0;
        tr.seed_ss = (float)A.cgeo[(size_t)p * 5];
        tr.phi0 = tr.qpt = tr.d0 = tr.chi2 = 0.0f;
        float rf = __builtin_inff();
        for (int L = 0; L < HT_MAX_LAYERS; ++L) {
          int h = A.chit[(size_t)p * HT_MAX_LAYERS + L];
          if (h >= 0 && (int)(0x3ffffff - (A.owner_key[h] & 0x3ffffffull)) != p) h = -1;
          tr.hits[L] = h;
          if (h >= 0) {
            if (A.r[h] < rf) rf = A.r[h];
            A.out.hit_owner[h] = t;
          }
        }
        tr.r_first = rf;
        A.out.tracks[t] = tr;
        A.trk_peak[t] = p;
      }
    }
    __syncthreads();
  }
}

// ---- refit ----------------------------------------------------------------------
__device__ __forceinline__ double wrap_pi(double a) {
  return a - 2.0 * kPi * floor((a + kPi) / (2.0 * kPi));
}

// wave sum, then lane 0's value everywhere (the butterfly rounds differently
// on each lane; the solve below must see one value so control stays uniform)
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return __shfl(v, 0);
}

// One wave per track, lane = layer: each lane forms its hit's residual and
// Jacobian row, the normal equations are summed across the wave and every
// lane solves the same (at most 3x3) system by Cholesky.  Fixed parameters
// (one bin in q/pT or d0) get a zero Jacobian column and a unit diagonal, so
// their step is exactly zero.
__device__ void fit_tracks(const AssocArgs& A, int bid, int nblk) {
  const int lane = threadIdx.x & 63;
  const int ntrk = min(A.sc[S_NTRK], A.out.track_cap);
  const bool fk = A.n_qpt > 1, fd = A.n_d0 > 1;
  for (int t = bid * 4 + (threadIdx.x >> 6); t < ntrk; t += nblk * 4) {
    ht_track& tr = A.out.tracks[t];
    const int p = A.trk_peak[t];
    const double* g = A.cgeo + (size_t)p * 5;
    const double gA = g[1], gB = g[2], gC = g[3], gD = g[4];
    const int lin = tr.lin;
    const int i = lin % A.n_phi, col = lin / A.n_phi, j = col % A.n_qpt, k = col / A.n_qpt;
    const double kap_c = A.kapc[j];
    const double d0_c = A.d0c[k];
    const double sq0 = sqrt(gB * gB + gC * gC);
    double p0 = atan2(gB, -gC);
    double p1 = fk ? 2.0 * gA : kap_c;
    double p2 = fd ? 2.0 * gD / (1.0 + sq0) : d0_c;
    const int h = lane < HT_MAX_LAYERS ? tr.hits[lane] : -1;
    const double rr = h >= 0 ? (double)A.r[h] : 1.0;
    const double ph = h >= 0 ? (double)A.phi[h] : 0.0;
    int status = 0;
    for (int it = 0; it < A.cfg.fit_iters && status == 0; ++it) {
      double j0 = 0.0, j1 = 0.0, j2 = 0.0, res = 0.0, w = 0.0;
      int bad = 0;
      if (h >= 0) {
        const double den = 1.0 + p1 * p2;
        const double u = (p1 * (rr * rr + p2 * p2) + 2.0 * p2) / (2.0 * rr * den);
        if (!(fabs(u) < 1.0)) {
          bad = 1;
        } else {
          const double sq = sqrt(1.0 - u * u);
          res = wrap_pi(ph - (p0 + asin(u)));
          j0 = 1.0;
          j1 = fk ? (rr * rr - p2 * p2) / (2.0 * rr * den * den) / sq : 0.0;
          j2 = fd ? (den * den + 1.0 - p1 * p1 * rr * rr) / (2.0 * rr * den * den) / sq : 0.0;
          w = rr * rr;
        }
      }
      if (__ballot(bad)) { status = 1; break; }
      const double a00 = wave_sum_d(w * j0 * j0), a01 = wave_sum_d(w * j0 * j1);
      const double a02 = wave_sum_d(w * j0 * j2), a11 = wave_sum_d(w * j1 * j1);
      const double a12 = wave_sum_d(w * j1 * j2), a22 = wave_sum_d(w * j2 * j2);
      const double g0 = wave_sum_d(w * j0 * res), g1 = wave_sum_d(w * j1 * res);
      const double g2 = wave_sum_d(w * j2 * res);
      // Cholesky of the 3x3 system with unit diagonal for fixed parameters
      const double m11 = fk ? a11 : 1.0, m22 = fd ? a22 : 1.0;
      if (!(a00 > 0.0)) { status = 2; break; }
      const double l00 = sqrt(a00);
      const double l10 = a01 / l00, l20 = a02 / l00;
      const double d1 = m11 - l10 * l10;
      if (!(d1 > 0.0)) { status = 2; break; }
      const double l11 = sqrt(d1);
      const double l21 = (a12 - l20 * l10) / l11;
      const double d2 = m22 - l20 * l20 - l21 * l21;
      if (!(d2 > 0.0)) { status = 2; break; }
      const double l22 = sqrt(d2);
      const double y0 = g0 / l00, y1 = (g1 - l10 * y0) / l11, y2 = (g2 - l20 * y0 - l21 * y1) / l22;
      const double x2 = y2 / l22, x1 = (y1 - l21 * x2) / l11, x0 = (y0 - l10 * x1 - l20 * x2) / l00;
      p0 += x0;
      if (fk) p1 += x1;
      if (fd) p2 += x2;
    }
    double chi2 = 0.0;
    if (status == 0) {
      double z2 = 0.0;
      int bad = 0;
      if (h >= 0) {
        const double den = 1.0 + p1 * p2;
        const double u = (p1 * (rr * rr + p2 * p2) + 2.0 * p2) / (2.0 * rr * den);
        if (!(fabs(u) < 1.0)) {
          bad = 1;
        } else {
          const double res = wrap_pi(ph - (p0 + asin(u)));
          const double z = rr * res / (double)A.cfg.sigma_rphi;
          z2 = z * z;
        }
      }
      if (__ballot(bad)) status = 1;
      chi2 = wave_sum_d(z2);
    }
    if (status != 0) {
      p0 = -kPi + ((double)i + 0.5) * (2.0 * kPi / (double)A.n_phi);
      p1 = kap_c;
      p2 = d0_c;
      chi2 = -1.0;
    }
    if (lane == 0) {
      tr.status = status;
      tr.phi0 = (float)wrap_pi(p0);
      tr.qpt = (float)(-p1 / A.cb);
      tr.d0 = (float)p2;
      tr.chi2 = (float)chi2;
    }
  }
}

// Refit by a Kalman filter (the paper's Kalman filter that refines
// candidates, section "Jet and Black Hole Detection", run on the device as
// its outlook suggests).  State (phi0, kappa, d0) at the perigee from the
// seed circle.  Each pass filters the deviation dp from a reference state
// (the seed, then the previous pass's result) with the azimuth model
// phi0 + asin(u) linearised at the reference, as track fits do about a
// reference trajectory: prior dp = 0 with covariance diag(0.1^2, 0.01^2,
// 10^2); the owned hits in layer order, each of variance (sigma / r)^2 with
// innovation res - H dp; no process noise; the pass ends with p += dp.
// A fixed parameter (one-column grid axis) keeps a zero row and column in
// the covariance, so its gain is zero and it never moves.  Status 1 when a
// hit has |u| >= 1, 2 when an innovation variance is not positive.  The
// filter is sequential in the hits, so one thread owns one track.
template <int NB>
__global__ __launch_bounds__(64) void kf_kernel(AssocBatch<NB> AB) {
  const AssocArgs& A = event_args(AB);
  const int ntrk = min(A.sc[S_NTRK], A.out.track_cap);
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= ntrk) return;
  const bool fk = A.n_qpt > 1, fd = A.n_d0 > 1;
  ht_track& tr = A.out.tracks[t];
  const int p = A.trk_peak[t];
  const double* g = A.cgeo + (size_t)p * 5;
  const double gA = g[1], gB = g[2], gC = g[3], gD = g[4];
  const int lin = tr.lin;
  const int i = lin % A.n_phi, col = lin / A.n_phi, j = col % A.n_qpt, k = col / A.n_qpt;
  const double kap_c = A.kapc[j];
  const double d0_c = A.d0c[k];
  const double sq0 = sqrt(gB * gB + gC * gC);
  double x[3];
  x[0] = atan2(gB, -gC);
  x[1] = fk ? 2.0 * gA : kap_c;
  x[2] = fd ? 2.0 * gD / (1.0 + sq0) : d0_c;
  const double prior[3] = {0.01, fk ? 1e-4 : 0.0, fd ? 100.0 : 0.0};
  const double s2 = (double)A.cfg.sigma_rphi * (double)A.cfg.sigma_rphi;
  int hit[HT_MAX_LAYERS];
  for (int L = 0; L < HT_MAX_LAYERS; ++L) hit[L] = tr.hits[L];
  int status = 0;
  for (int it = 0; it < A.cfg.fit_iters && status == 0; ++it) {
    double P[3][3];
    double dp[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) P[a][b] = a == b ? prior[a] : 0.0;
    for (int L = 0; L < HT_MAX_LAYERS; ++L) {
      const int h = hit[L];
      if (h < 0) continue;
      const double rr = (double)A.r[h], ph = (double)A.phi[h];
      const double kap = x[1], d0 = x[2];
      const double den = 1.0 + kap * d0;
      const double u = (kap * (rr * rr + d0 * d0) + 2.0 * d0) / (2.0 * rr * den);
      if (!(fabs(u) < 1.0)) { status = 1; break; }
      const double sq = sqrt(1.0 - u * u);
      const double res = wrap_pi(ph - (x[0] + asin(u)));
      double H[3];
      H[0] = 1.0;
      H[1] = fk ? (rr * rr - d0 * d0) / (2.0 * rr * den * den) / sq : 0.0;
      H[2] = fd ? (den * den + 1.0 - kap * kap * rr * rr) / (2.0 * rr * den * den) / sq : 0.0;
      double PH[3];
      for (int a = 0; a < 3; ++a) PH[a] = P[a][0] * H[0] + P[a][1] * H[1] + P[a][2] * H[2];
      const double S = s2 / (rr * rr) + H[0] * PH[0] + H[1] * PH[1] + H[2] * PH[2];
      if (!(S > 0.0)) { status = 2; break; }
      const double innov = res - H[0] * dp[0] - H[1] * dp[1] - H[2] * dp[2];
      double K[3];
      for (int a = 0; a < 3; ++a) K[a] = PH[a] / S;
      for (int a = 0; a < 3; ++a) dp[a] += K[a] * innov;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) P[a][b] -= K[a] * PH[b];
    }
    if (status != 0) break;
    for (int a = 0; a < 3; ++a) x[a] += dp[a];
  }
  double chi2 = 0.0;
  if (status == 0) {
    for (int L = 0; L < HT_MAX_LAYERS; ++L) {
      const int h = hit[L];
      if (h < 0) continue;
      const double rr = (double)A.r[h], ph = (double)A.phi[h];
      const double den = 1.0 + x[1] * x[2];
      const double u = (x[1] * (rr * rr + x[2] * x[2]) + 2.0 * x[2]) / (2.0 * rr * den);
      if (!(fabs(u) < 1.0)) { status = 1; break; }
      const double z = rr * wrap_pi(ph - (x[0] + asin(u))) / (double)A.cfg.sigma_rphi;
      chi2 += z * z;
    }
  }
  if (status != 0) {
    x[0] = -kPi + ((double)i + 0.5) * (2.0 * kPi / (double)A.n_phi);
    x[1] = kap_c;
    x[2] = d0_c;
    chi2 = -1.0;
  }
  tr.status = status;
  tr.phi0 = (float)wrap_pi(x[0]);
  tr.qpt = (float)(-x[1] / A.cb);
  tr.d0 = (float)x[2];
  tr.chi2 = (float)chi2;
}

// ---- second transform --------------------------------------------------------------
// branch > 0: the crossing at radius rho ahead of the perigee along the
// direction of motion (outgoing branch); branch < 0: the one before it
__device__ __forceinline__ double crossing_theta(double cA, double cB, double cC, double cD,
                                                 double sn, double rho, int branch) {
  const double c0 = -(cA * rho * rho + cD);
  const double dl = c0 / sn;
  const double hh = (rho - dl) * (rho + dl);
  double h = hh > 0.0 ? sqrt(hh) : 0.0;
  if (branch < 0) h = -h;
  const double px = (dl / sn) * cB + (h / sn) * (-cC);
  const double py = (dl / sn) * cC + (h / sn) * cB;
  return catan2(py, px);
}

__device__ __forceinline__ int theta_bin(double th, int nt) {
  int t = (int)floor((th + kPi) / (2.0 * kPi / (double)nt));
  t %= nt;
  return t < 0 ? t + nt : t;
}

// the arc of theta bins between the crossings of one branch at radii ra < rb
// (the shorter way round)
__device__ __forceinline__ void branch_arc(double cA, double cB, double cC, double cD,
                                           double sn, double ra, double rb, int branch, int nt,
                                           int* start, int* len) {
  const int ta = theta_bin(crossing_theta(cA, cB, cC, cD, sn, ra, branch), nt);
  const int tb = theta_bin(crossing_theta(cA, cB, cC, cD, sn, rb, branch), nt);
  int d = (tb - ta) % nt;
  if (d < 0) d += nt;
  if (d <= nt / 2) { *start = ta; *len = d + 1; }
  else { *start = tb; *len = nt - d + 1; }
}

// One thread per (track, vertex row): the row's arcs and their votes, one
// per cell of the union of the outgoing arc (perigee to first hit) and, with
// the two-branch vote, the incoming arc (perigee radius to the row's top).
// (A thread per track walked its rows in sequence, a chain of float64
// square roots and arctangents per row on only as many threads as tracks.)
__device__ void vote_rows(const AssocArgs& A, int bid, int nblk) {
  const int ntrk = min(A.sc[S_NTRK], A.out.track_cap);
  const int nm = A.cfg.n_rho, nt = A.cfg.n_theta;
  const double rw = ((double)A.cfg.rho_hi - (double)A.cfg.rho_lo) / (double)nm;
  const int64_t work = (int64_t)ntrk * nm;
  for (int64_t e = (int64_t)bid * blockDim.x + threadIdx.x; e < work;
       e += (int64_t)nblk * blockDim.x) {
    const int t = (int)(e / nm), m = (int)(e - (int64_t)t * nm);
    const int p = A.trk_peak[t];
    const double* g = A.cgeo + (size_t)p * 5;
    const double cA = g[1], cB = g[2], cC = g[3], cD = g[4];
    const double sn = sqrt(cB * cB + cC * cC);
    const double pca = fabs(2.0 * cD / (1.0 + sn));
    const double rf = (double)A.out.tracks[t].r_first;
    // a track passing within vtx_min_d0 of the beam line is an IP feature
    const bool votes = !(pca < (double)A.cfg.vtx_min_d0);
    int start = 0, len = 0, istart = 0, ilen = 0;
    const double e0 = (double)A.cfg.rho_lo + (double)m * rw;
    const double e1 = (double)A.cfg.rho_lo + (double)(m + 1) * rw;
    const double ra = e0 > pca ? e0 : pca;
    if (votes) {
      const double rb = e1 < rf ? e1 : rf;
      if (ra < rb) branch_arc(cA, cB, cC, cD, sn, ra, rb, +1, nt, &start, &len);
      if (A.cfg.vtx_two_branch && ra < e1)
        branch_arc(cA, cB, cC, cD, sn, ra, e1, -1, nt, &istart, &ilen);
      for (int q = 0; q < len; ++q) {
        int c = start + q;
        if (c >= nt) c -= nt;
        atomicAdd(&A.vacc[m * nt + c], 1);
      }
      for (int q = 0; q < ilen; ++q) {
        int c = istart + q;
        if (c >= nt) c -= nt;
        int off = (c - start) % nt;
        if (off < 0) off += nt;
        if (off >= len) atomicAdd(&A.vacc[m * nt + c], 1);
      }
    }
    if (m == 0) A.tunit[t] = make_double2(-cC / sn, cB / sn);
    A.arc0[(size_t)t * nm + m] = start;
    A.arcn[(size_t)t * nm + m] = len;
    A.arci0[(size_t)t * nm + m] = istart;
    A.arcin[(size_t)t * nm + m] = ilen;
  }
}

// the vertex votes after the Kalman filter (kf_kernel)
template <int NB>
__global__ __launch_bounds__(256) void vvote_kernel(AssocBatch<NB> AB) {
  vote_rows(event_args(AB), blockIdx.x, gridDim.x);
}

// the refit (workgroups below fit_blocks) and the vertex votes (the rest) in
// one launch: the votes read the tracks' seed circles and first radii, which
// the refit does not change
template <int NB>
__global__ __launch_bounds__(256) void fit_vote_kernel(AssocBatch<NB> AB, int fit_blocks) {
  const AssocArgs& A = event_args(AB);
  if ((int)blockIdx.x < fit_blocks)
    fit_tracks(A, blockIdx.x, fit_blocks);
  else
    vote_rows(A, blockIdx.x - fit_blocks, gridDim.x - fit_blocks);
}

// Vertex peaks in cell order, in two launches over 1024-cell tiles (thread t
// of a tile tests cells 4t .. 4t + 3): vpcount counts each tile's peaks (and
// clears the first n_zero object member counts, the input of vcount), then
// vpemit places each tile's peaks after those of the tiles before it (it sums
// their counts) and writes them in cell order; the last tile writes the count.
constexpr int kVTile = 1024;
__device__ __forceinline__ bool vertex_peak(const int32_t* vv, int nm, int nt, int c, int thr) {
  const int m = c / nt, ti = c - m * nt;
  const int v = vv[c];
  if (v < thr) return false;
  for (int dm = -1; dm <= 1; ++dm) {
    const int mm = m + dm;
    if (mm < 0 || mm >= nm) continue;
    for (int dt = -1; dt <= 1; ++dt) {
      if (dm == 0 && dt == 0) continue;
      int tt = ti + dt;
      tt = tt < 0 ? tt + nt : (tt >= nt ? tt - nt : tt);
      const int w = vv[mm * nt + tt];
      const bool neg = dm < 0 || (dm == 0 && dt < 0);
      if (neg ? !(v > w) : !(v >= w)) return false;
    }
  }
  return true;
}

// the tile's peak flags of this thread's four cells, as bits
__device__ __forceinline__ unsigned vertex_flags(const AssocArgs& A, int tile) {
  const int nm = A.cfg.n_rho, nt = A.cfg.n_theta, ncell = nm * nt;
  const int c0 = tile * kVTile + (int)threadIdx.x * 4;
  unsigned f = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (c0 + u < ncell && vertex_peak(A.vacc, nm, nt, c0 + u, A.cfg.vtx_min_votes)) f |= 1u << u;
  return f;
}

template <int NB>
__global__ __launch_bounds__(256) void vpcount_kernel(AssocBatch<NB> AB, int n_zero) {
  const AssocArgs& A = event_args(AB);
  __shared__ int32_t wc[4];
  for (int c = blockIdx.x * 256 + threadIdx.x; c < n_zero; c += gridDim.x * 256) A.obj_cnt[c] = 0;
  const int cnt = __popc(vertex_flags(A, blockIdx.x));
  int x = cnt;
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) A.vtile[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

template <int NB>
__global__ __launch_bounds__(256) void vpemit_kernel(AssocBatch<NB> AB) {
  const AssocArgs& A = event_args(AB);
  __shared__ int32_t wsum[4];
  __shared__ int32_t base_s;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nm = A.cfg.n_rho, nt = A.cfg.n_theta;
  const double rw = ((double)A.cfg.rho_hi - (double)A.cfg.rho_lo) / (double)nm;
  if (wave == 0) {  // peaks of the tiles before this one
    int b = 0;
    for (int q = lane; q < (int)blockIdx.x; q += kWave) b += A.vtile[q];
    for (int off = kWave / 2; off > 0; off >>= 1) b += __shfl_xor(b, off);
    if (lane == 0) base_s = b;
  }
  const unsigned f = vertex_flags(A, blockIdx.x);
  const int cnt = __popc(f);
  int x = cnt;  // inclusive scan over the wave, then over the four wave totals
  for (int d = 1; d < kWave; d <<= 1) {
    const int y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) wsum[wave] = x;
  __syncthreads();
  int o = base_s + x - cnt;
  for (int w = 0; w < wave; ++w) o += wsum[w];
  const int c0 = (int)blockIdx.x * kVTile + (int)threadIdx.x * 4;
  for (unsigned b = f; b; b &= b - 1) {
    const int c = c0 + __builtin_ctz(b);
    if (o < A.out.object_cap) {
      const int m = c / nt, ti = c - m * nt;
      ht_object ob;
      ob.lin = c;
      ob.votes = A.vacc[c];
      ob.n_tracks = 0;
      ob.kind = 0;
      ob.rho = (float)((double)A.cfg.rho_lo + ((double)m + 0.5) * rw);
      ob.theta = (float)(-kPi + ((double)ti + 0.5) * (2.0 * kPi / (double)nt));
      ob.isotropy = 0.0f;
      ob.member_begin = 0;
      A.out.objects[o] = ob;
    }
    ++o;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 255)
    A.sc[S_NOBJ] = base_s + wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// a track is a member of the object at (m, ti) when one of its arcs (either
// branch) in rows m - 1 .. m + 1, widened by one bin each side, holds ti.
// t < the track count; the twelve loads do not depend on each other.
__device__ __forceinline__ bool is_member(const AssocArgs& A, int t, int m, int ti) {
  const int nm = A.cfg.n_rho, nt = A.cfg.n_theta;
  bool in = false;
#pragma unroll
  for (int dm = -1; dm <= 1; ++dm) {
    const int mm = m + dm;
    const bool row = mm >= 0 && mm < nm;
    const size_t a = (size_t)t * nm + (row ? mm : m);
    const int len = A.arcn[a], st = A.arc0[a], ilen = A.arcin[a], ist = A.arci0[a];
    int off = (ti - st + 1) % nt;
    if (off < 0) off += nt;
    int ioff = (ti - ist + 1) % nt;
    if (ioff < 0) ioff += nt;
    in = in || (row && ((len > 0 && off < len + 2) || (ilen > 0 && ioff < ilen + 2)));
  }
  return in;
}

// pass 1: member count per object, one wave per (object, 64 tracks)
template <int NB>
__global__ __launch_bounds__(256) void vcount_kernel(AssocBatch<NB> AB) {
  const AssocArgs& A = event_args(AB);
  const int nobj = min(A.sc[S_NOBJ], A.out.object_cap);
  const int ntrk = min(A.sc[S_NTRK], A.out.track_cap);
  const int nch = (ntrk + kWave - 1) / kWave;
  const int64_t pairs = (int64_t)nobj * nch;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t q = (int64_t)blockIdx.x * 4 + wave; q < pairs; q += (int64_t)gridDim.x * 4) {
    const int o = (int)(q / nch), ch = (int)(q - (int64_t)o * nch);
    const int c = A.out.objects[o].lin;
    const int m = c / A.cfg.n_theta, ti = c % A.cfg.n_theta;
    const int t = ch * kWave + lane;
    const int cnt = __popcll(__ballot(is_member(A, min(t, ntrk - 1), m, ti) && t < ntrk));
    if (lane == 0 && cnt) atomicAdd(&A.obj_cnt[o], cnt);
  }
}

// the event's counts, by one wave (uniform control): lane i reads spread
// slot i of each counter; n_mem is the object members' total
__device__ void write_counts(const AssocArgs& A, int n_mem) {
  static_assert(kSpread == kWave, "one spread slot per lane");
  int32_t* c = A.out.counts;
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long ncand = A.spread[(size_t)(SP_NCAND + lane) * kSpreadStride];
  unsigned long long tests = A.spread[(size_t)(SP_TESTS + lane) * kSpreadStride];
  unsigned long long nover = A.spread[(size_t)(SP_NOVER + lane) * kSpreadStride];
  unsigned long long pairs = A.spread[(size_t)(SP_PAIRS + lane) * kSpreadStride];
  unsigned long long exec = A.spread[(size_t)(SP_EXEC + lane) * kSpreadStride];
  for (int off = kWave / 2; off > 0; off >>= 1) {
    ncand += __shfl_xor(ncand, off);
    tests += __shfl_xor(tests, off);
    nover += __shfl_xor(nover, off);
    pairs += __shfl_xor(pairs, off);
    exec += __shfl_xor(exec, off);
  }
  if (lane != 0) return;
  if (A.out.work) {
    A.out.work[0] = tests;
    A.out.work[1] = exec;
  }
  c[0] = (int32_t)ncand;
  c[1] = A.sc[S_NTRK];
  c[2] = A.sc[S_NOBJ];
  c[3] = n_mem;
  c[4] = (int32_t)nover;
  c[5] = pairs > 0x7fffffffull ? 0x7fffffff : (int32_t)pairs;
  c[6] = tests > 0x7fffffffull ? 0x7fffffff : (int32_t)tests;
  c[7] = 0;
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// pass 2: members in track order and the isotropy, one wave per object.  An
// object's members start after those of the objects before it (the wave sums
// their counts).  The tracks are tested kVGroup chunks of 64 at a time (their
// loads in flight together); the direction sums then take the members one by
// one in track order from the lanes' registers, the order that defines them.
constexpr int kVGroup = 4;
template <int NB>
__global__ __launch_bounds__(256) void vmembers_kernel(AssocBatch<NB> AB) {
  const AssocArgs& A = event_args(AB);
  const int nobj = min(A.sc[S_NOBJ], A.out.object_cap);
  const int ntrk = min(A.sc[S_NTRK], A.out.track_cap);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = lane ? ((1ull << lane) - 1ull) : 0ull;
  for (int o = blockIdx.x * 4 + wave; o < nobj; o += gridDim.x * 4) {
    ht_object& ob = A.out.objects[o];
    const int c = ob.lin;
    const int m = c / A.cfg.n_theta, ti = c % A.cfg.n_theta;
    int begin = 0;
    for (int q = lane; q < o; q += kWave) begin += A.obj_cnt[q];
    for (int off = kWave / 2; off > 0; off >>= 1) begin += __shfl_xor(begin, off);
    int cnt = 0;
    double sx = 0.0, sy = 0.0;
    for (int t0 = 0; t0 < ntrk; t0 += kVGroup * kWave) {
      bool mem[kVGroup];
      double2 u[kVGroup];
#pragma unroll
      for (int g = 0; g < kVGroup; ++g) {
        const int t = t0 + g * kWave + lane;
        const int tl = min(t, ntrk - 1);
        mem[g] = is_member(A, tl, m, ti) && t < ntrk;
        u[g] = A.tunit[tl];
      }
#pragma unroll
      for (int g = 0; g < kVGroup; ++g) {
        const uint64_t msk = __ballot(mem[g]);
        if (mem[g]) {
          const int idx = begin + cnt + __popcll(msk & below);
          if (idx < A.out.member_cap) A.out.members[idx] = t0 + g * kWave + lane;
        }
        for (uint64_t b = msk; b; b &= b - 1) {
          const int l = __builtin_ctzll(b);
          sx += readlane_d(u[g].x, l);
          sy += readlane_d(u[g].y, l);
        }
        cnt += __popcll(msk);
      }
    }
    if (lane == 0) {
      const double R = cnt > 0 ? sqrt(sx * sx + sy * sy) / (double)cnt : 0.0;
      ob.n_tracks = cnt;
      ob.member_begin = begin;
      ob.isotropy = (float)R;
      ob.kind = (cnt >= A.cfg.bh_min_tracks && R <= (double)A.cfg.bh_max_isotropy) ? 1 : 0;
      if (o == nobj - 1) A.sc[S_NMEM] = begin + cnt;
    }
    if (o == nobj - 1) write_counts(A, begin + cnt);
  }
  if (nobj == 0 && blockIdx.x == 0 && wave == 0) write_counts(A, 0);
}




int blocks_for(int64_t n, int per) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > kGridCap) b = kGridCap;
  return (int)b;
}

template <int CAP, int NB>
void launch_refine(const AssocBatch<NB>& AB, int peak_cap, hipStream_t s, int n_lo = 0,
                   int n_hi = 0x7fffffff) {
  constexpr int W = RefineShape<CAP>::kWaves;
  refine_kernel<CAP, NB><<<dim3(blocks_for(peak_cap, W), 1, NB), W * kWave, 0, s>>>(AB, n_lo, n_hi);
}

// The arguments of one event's assoc_cluster.
AssocArgs make_args(const Plan& P, const float* r, const float* phi, const uint8_t* layer,
                    int32_t n_hits, const ht_peak* peaks, const int32_t* n_peaks,
                    int32_t peak_cap, const int32_t* acc, const ht_cluster_cfg& cfg,
                    const ht_cluster_out& out, const int32_t* n_hits_dev) {
  const ht_grid& g = P.grid;
  AssocArgs A;
  A.n_phi = g.n_phi;
  A.n_qpt = g.n_qpt;
  A.n_d0 = g.n_d0;
  A.n_cells = P.n_cells;
  A.phi_lo = P.phi_lo;
  A.invw = P.invw;
  A.kap = P.d_kap;
  A.kapc = P.d_kapc;
  A.d0c = P.d_d0c;
  A.qt = P.d_q;
  A.tt = P.d_t;
  A.origin_seed = (g.n_d0 == 1 && g.d0_lo == 0.0f && g.d0_hi == 0.0f);
  const double cb = kCLight * (double)g.bfield;
  A.kap_bin = cb * ((double)g.qpt_hi - (double)g.qpt_lo) / (double)g.n_qpt;
  A.d0_bin = ((double)g.d0_hi - (double)g.d0_lo) / (double)g.n_d0;
  A.hk = (float)(0.5 * A.kap_bin);
  A.hd0 = (float)(0.5 * A.d0_bin);
  A.cb = cb;
  A.r = r;
  A.phi = phi;
  A.layer = layer;
  A.n_hits = n_hits;
  A.n_hits_dev = n_hits_dev;
  A.hx = P.d_hx;
  A.hy = P.d_hy;
  A.hq = P.d_hq;
  A.hitB = P.d_hitB;
  // the member-count bound needs a window of at least 0.5 + win_bins bins
  // (a d0 axis keeps its extra term positive) and distinct neighbour cells
  A.acc = (acc && A.hd0 >= 1e-20f && (int64_t)g.n_phi >= 4 * ((int64_t)cfg.win_bins + 1)) ? acc
                                                                                        : nullptr;
  A.peaks = peaks;
  A.n_peaks = n_peaks;
  A.peak_cap = peak_cap;
  A.cfg = cfg;
  A.pbits = P.d_pbits;
  A.col_first = P.d_col_first;
  A.mcount = P.d_mcount;
  A.pool = P.d_mem;
  A.cstat = P.d_cstat;
  A.cnl = P.d_cnl;
  A.cgeo = P.d_cgeo;
  A.chit = P.d_chit;
  A.owner_key = P.d_owner_key;
  A.ctile_cnt = P.d_ctile_cnt;
  A.ctile_off = P.d_ctile_off;
  A.trk_peak = P.d_trk_peak;
  A.arc0 = P.d_arc0;
  A.arcn = P.d_arcn;
  A.arci0 = P.d_arci0;
  A.arcin = P.d_arcin;
  A.tunit = P.d_tunit;
  A.vacc = out.vacc ? out.vacc : P.d_vacc;
  A.obj_cnt = P.d_obj_cnt;
  A.vtile = P.d_vtile;
  A.sc = P.d_scalars;
  A.spread = P.d_spread;
  A.cls = P.d_cls;
  A.bkt = P.d_bkt;
  A.bkt_off = P.d_bkt_off;
  A.hkey = P.d_hkey;
  A.shit = P.d_shit;
  A.sphi = P.d_sphi;
  A.out = out;
  return A;
}

// The kernels of assoc_cluster for the NB events of AB, each launch covering
// all of them (blockIdx.z); P are their plans (the first one's stage timers
// are marked).  Sizes that set grids (hit bound, peak capacity, output
// capacities, grid) are the first event's, the same for all.
template <int NB>
int assoc_sequence(const AssocBatch<NB>& AB, const Plan* const* P, int32_t n_hits,
                   int32_t peak_cap, hipStream_t s) {
  const Plan& P0 = *P[0];
  const ht_grid& g = P0.grid;
  const ht_cluster_cfg& cfg = AB.a[0].cfg;
  const ht_cluster_out& out = AB.a[0].out;
  if (cfg.member_cap > kMaxMembers) return HT_EUNSUPPORTED;
  const int words = P0.n_tiles * 8 + 2;
  const int64_t init_n = words > n_hits ? words : n_hits;
  P0.prof_mark(HT_STAGE_ASSOC, 0, s);
  const int surv_tiles = (peak_cap + 255) / 256 > 0 ? (peak_cap + 255) / 256 : 1;
  init_kernel<NB><<<dim3(blocks_for(init_n, 256), 1, NB), 256, 0, s>>>(AB, words,
                                                                      (surv_tiles + 63) / 64);
  HT_CHECK(hipGetLastError());
  const int hblocks = blocks_for(n_hits, 256) < 256 ? blocks_for(n_hits, 256) : 256;
  {
    const int mblocks = blocks_for(peak_cap, 256);
    mark_kernel<NB><<<dim3(mblocks + hblocks, 1, NB), 256, 0, s>>>(AB, mblocks);
    HT_CHECK(hipGetLastError());
  }
  const int col_tiles = (g.n_qpt + kWave - 1) / kWave;
  dim3 sweep(col_tiles, g.n_d0, hit_slices(col_tiles * g.n_d0, n_hits) * NB);
  P0.prof_mark(HT_STAGE_MEMBERS, 0, s);
  {
    const dim3 hgrid(hblocks, 1, NB);
    bcount_kernel<NB><<<hgrid, 256, 0, s>>>(AB);
    HT_CHECK(hipGetLastError());
    const int32_t* bc[NB];
    int32_t* bo[NB];
    int32_t* bt[NB];
    for (int b = 0; b < NB; ++b) {
      bc[b] = P[b]->d_bkt;
      bo[b] = P[b]->d_bkt_off;
      bt[b] = P[b]->d_bkt_off + kBucketKeys;
    }
    const int brc = NB == 1 ? launch_scan(bc[0], bo[0], kBucketKeys, bt[0], s)
                            : launch_scan_batch(NB, bc, bo, kBucketKeys, bt, s);
    if (brc != HT_OK) return brc;
    bscatter_kernel<NB><<<hgrid, 256, 0, s>>>(AB);
    HT_CHECK(hipGetLastError());
    mcand_kernel<NB><<<dim3(blocks_for(peak_cap, 4), 1, NB), 256, 0, s>>>(AB);
    HT_CHECK(hipGetLastError());
  }
  member_kernel<NB><<<sweep, kSweepThreads, 0, s>>>(AB);
  HT_CHECK(hipGetLastError());
  P0.prof_mark(HT_STAGE_MEMBERS, 1, s);
  P0.prof_mark(HT_STAGE_REFINE, 0, s);
  if (cfg.member_cap <= 128)
    launch_refine<128, NB>(AB, peak_cap, s);
  else if (cfg.member_cap <= 256)
    launch_refine<256, NB>(AB, peak_cap, s);
  else if (cfg.member_cap <= 512)
    launch_refine<512, NB>(AB, peak_cap, s);
  else {
    // caps above 512: the candidates with at most 512 members take the
    // cap-512 kernel (fewer registers and LDS per wave: four waves per SIMD
    // instead of two), the others the cap-1024 kernel
    launch_refine<512, NB>(AB, peak_cap, s, 0, 512);
    HT_CHECK(hipGetLastError());
    launch_refine<kMaxMembers, NB>(AB, peak_cap, s, 513);
  }
  HT_CHECK(hipGetLastError());
  P0.prof_mark(HT_STAGE_REFINE, 1, s);
  const int tiles = surv_tiles;
  surv_count_kernel<NB><<<dim3(blocks_for(tiles, 1), 1, NB), 256, 0, s>>>(AB, tiles);
  HT_CHECK(hipGetLastError());
  surv_emit_kernel<NB><<<dim3(blocks_for(tiles, 1), 1, NB), 256, 0, s>>>(AB, tiles);
  HT_CHECK(hipGetLastError());
  const int tcap = out.track_cap > 0 ? out.track_cap : 1;
  if (out.track_cap > 0) {
    const int vblocks = blocks_for((int64_t)tcap * cfg.n_rho, 256);
    if (cfg.fit_kind == 1) {
      kf_kernel<NB><<<dim3(blocks_for(tcap, 64), 1, NB), 64, 0, s>>>(AB);
      HT_CHECK(hipGetLastError());
      vvote_kernel<NB><<<dim3(vblocks, 1, NB), 256, 0, s>>>(AB);
    } else {
      const int fblocks = blocks_for(tcap, 4);
      fit_vote_kernel<NB><<<dim3(fblocks + vblocks, 1, NB), 256, 0, s>>>(AB, fblocks);
    }
    HT_CHECK(hipGetLastError());
  }
  const int ocap = out.object_cap > 0 ? out.object_cap : 1;
  const int ozero = ocap < P0.lim.max_vertex_cells ? ocap : P0.lim.max_vertex_cells;
  {
    const int vt = (cfg.n_rho * cfg.n_theta + kVTile - 1) / kVTile;
    vpcount_kernel<NB><<<dim3(vt, 1, NB), 256, 0, s>>>(AB, ozero);
    HT_CHECK(hipGetLastError());
    vpemit_kernel<NB><<<dim3(vt, 1, NB), 256, 0, s>>>(AB);
    HT_CHECK(hipGetLastError());
  }
  if (out.object_cap > 0) {
    vcount_kernel<NB><<<dim3(blocks_for((int64_t)ocap * ((tcap + kWave - 1) / kWave), 4), 1, NB),
                        256, 0, s>>>(AB);
    HT_CHECK(hipGetLastError());
  }
  // members and isotropy; the wave of the last object (block 0 when there
  // are none) writes the counts, whose other inputs are final by now
  vmembers_kernel<NB><<<dim3(blocks_for(ocap, 4), 1, NB), 256, 0, s>>>(AB);
  HT_CHECK(hipGetLastError());
  P0.prof_mark(HT_STAGE_ASSOC, 1, s);
  return HT_OK;
}

}  // namespace

int launch_assoc(const Plan& P, const float* r, const float* phi, const uint8_t* layer,
                 int32_t n_hits, const ht_peak* peaks, const int32_t* n_peaks, int32_t peak_cap,
                 const int32_t* acc, const ht_cluster_cfg& cfg, const ht_cluster_out& out,
                 hipStream_t s, const int32_t* n_hits_dev) {
  AssocBatch<1> AB;
  AB.a[0] = make_args(P, r, phi, layer, n_hits, peaks, n_peaks, peak_cap, acc, cfg, out,
                      n_hits_dev);
  const Plan* plans[1] = {&P};
  return assoc_sequence<1>(AB, plans, n_hits, peak_cap, s);
}

namespace {
template <int NB>
int assoc_batch_nb(const AssocEvent* ev, int32_t n_hits_max, int32_t peak_cap,
                   const ht_cluster_cfg& cfg, hipStream_t s) {
  AssocBatch<NB> AB;
  const Plan* plans[NB];
  for (int b = 0; b < NB; ++b) {
    AB.a[b] = make_args(*ev[b].plan, ev[b].r, ev[b].phi, ev[b].layer, n_hits_max, ev[b].peaks,
                        ev[b].n_peaks, peak_cap, ev[b].acc, cfg, ev[b].out, ev[b].n_hits_dev);
    plans[b] = ev[b].plan;
  }
  return assoc_sequence<NB>(AB, plans, n_hits_max, peak_cap, s);
}
}  // namespace

int launch_assoc_batch(int nb, const AssocEvent* ev, int32_t n_hits_max, int32_t peak_cap,
                       const ht_cluster_cfg& cfg, hipStream_t s) {
  switch (nb) {
    case 1: return assoc_batch_nb<1>(ev, n_hits_max, peak_cap, cfg, s);
    case 2: return assoc_batch_nb<2>(ev, n_hits_max, peak_cap, cfg, s);
    case 3: return assoc_batch_nb<3>(ev, n_hits_max, peak_cap, cfg, s);
    case 4: return assoc_batch_nb<4>(ev, n_hits_max, peak_cap, cfg, s);
    default: return HT_EUNSUPPORTED;
  }
}

}  // namespace ht
