// Internal definitions of the gfx950 Hough trigger library (device code and
// the plan).  Every floating-point expression here is evaluated one IEEE
// operation at a time: the library is compiled with -ffp-contract=off and
// the pragma below, so no multiply-add is fused.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "houghtrig.h"

#pragma clang fp contract(off)

namespace ht {

constexpr double kPi = 3.14159265358979323846;
constexpr double kCLight = 0.299792458e-2;  // cm^-1 per (T GeV^-1)
constexpr int kWave = 64;

// Hit validity: r in (0, 1e4) cm, |phi| <= 4 rad, no NaN.
__device__ __forceinline__ bool hit_ok(float r, float phi) {
  return r > 0.0f && r < 1.0e4f && fabsf(phi) <= 4.0f;
}

// Correctly rounded square root for x = 0 or 2^-24 <= x <= 1 (the arguments
// 1 - |u| of the arcsine and 1 - u*u of the member window never lie below
// 2^-24 unless they are 0).  The
// hardware v_sqrt_f32 is within one ulp; the neighbours s -/+ 1 ulp are
// tested by the exact residuals x - s_dn*s and x - s_up*s (one fused
// rounding each), which decide round-to-nearest because no float x lies
// strictly between s_dn*s and the squared midpoint.  At x = 0 both tests
// fail and 0 is returned.  (Inputs here are never denormal, so the general
// expansion's rescaling and class checks are not needed.)
__device__ __forceinline__ float sqrt_unit(float x) {
  const float s = __builtin_amdgcn_sqrtf(x);
  const float s_dn = __int_as_float(__float_as_int(s) - 1);
  const float s_up = __int_as_float(__float_as_int(s) + 1);
  const float r_dn = __builtin_fmaf(-s_dn, s, x);
  const float r_up = __builtin_fmaf(-s_up, s, x);
  float t = r_dn <= 0.0f ? s_dn : s;
  t = r_up > 0.0f ? s_up : t;
  return t;
}

// Canonical arcsine: Abramowitz & Stegun 4.4.46,
//   asin a = pi/2 - sqrt(1 - a) (a0 + a1 a + ... + a7 a^7),  0 <= a <= 1,
// Horner with separate multiply and add, correctly rounded square root,
// sign restored with copysign.
__device__ __forceinline__ float asin_f(float u) {
  const float a = fabsf(u);
  float p = -0.0012624911f;
  p = p * a; p = p + 0.0066700901f;
  p = p * a; p = p + -0.0170881256f;
  p = p * a; p = p + 0.0308918810f;
  p = p * a; p = p + -0.0501743046f;
  p = p * a; p = p + 0.0889789874f;
  p = p * a; p = p + -0.2145988016f;
  p = p * a; p = p + 1.5707963050f;
  const float s = sqrt_unit(1.0f - a);
  const float r = 1.57079632679489661923f - s * p;
  return copysignf(r, u);
}

// Per-plan state.  Tables are float32 bin-centre constants computed in
// float64 on the host and rounded once.
struct Plan {
  ht_grid grid;
  ht_limits lim;
  int device;
  int64_t n_cells;
  float phi_lo, invw;
  float* d_kap;  // [n_qpt]
  float* d_q;    // [n_d0][n_qpt]
  float* d_t;    // [n_d0][n_qpt]
  // peak finder scratch
  uint32_t* d_bits;      // [n_cells / 32 + 1] peak bitmap
  int32_t* d_tile_cnt;   // [n_tiles]
  int32_t* d_tile_off;   // [n_tiles]
  int32_t n_tiles;
  // refinement scratch
  uint32_t* d_pbits;     // [n_cells / 32 + 1] bitmap of the peaks handed to assoc_cluster
  int32_t* d_col_first;  // [n_qpt * n_d0] first peak index of each column
  double* d_hx;          // [max_hits] hit x, y, x^2+y^2
  double* d_hy;
  double* d_hq;
  float4* d_hitA;        // [max_hits] r, phi, r*r, 1/r
  float4* d_hitB;        // [max_hits] x, y, x^2+y^2 (float32), layer
  int32_t* d_mcount;     // [max_peaks] member counts
  int32_t* d_mem;        // member pool: uint16 hit indices, member_cap slots per candidate
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
  int32_t* d_vacc;       // [max_vertex_cells] vertex accumulator
  int32_t* d_obj_cnt;    // [max_vertex_cells] member count per object
  int32_t* d_obj_off;    // [max_vertex_cells] member offset per object
  int32_t* d_scalars;    // [16] device counters
};

}  // namespace ht

struct ht_plan : ht::Plan {};

// Launch helpers implemented in the kernel files.
namespace ht {
int launch_vote(const Plan& p, const float* r, const float* phi, int32_t n_hits, int32_t* acc,
                unsigned long long* n_votes, hipStream_t s);
int launch_peaks(const Plan& p, const int32_t* acc, int32_t min_votes, ht_peak* out,
                 int32_t capacity, int32_t* n_found, hipStream_t s);
int launch_assoc(const Plan& p, const float* r, const float* phi, const uint8_t* layer,
                 int32_t n_hits, const ht_peak* peaks, const int32_t* n_peaks, int32_t peak_cap,
                 const ht_cluster_cfg& cfg, const ht_cluster_out& out, hipStream_t s);
int launch_asin(const float* u, float* out, int64_t n, hipStream_t s);
int launch_scan(const int32_t* cnt, int32_t* off, int n, int32_t* total, hipStream_t s);
int vote_init(int n_phi);
int peaks_init(int n_phi);
}  // namespace ht

#define HT_CHECK(x)                              \
  do {                                           \
    if ((x) != hipSuccess) return HT_EDEVICE;    \
  } while (0)
