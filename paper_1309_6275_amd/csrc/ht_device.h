// Device arithmetic shared by the kernels of the gfx950 Hough trigger
// library: hit validity, the correctly rounded square root and the canonical
// float32 arcsine of the vote.  Every floating-point expression here is
// evaluated one IEEE operation at a time: the library is compiled with
// -ffp-contract=off and the pragma below, so no multiply-add is fused.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Correctly rounded float64 square root for 2^-120 <= x <= 2^120 (other
// arguments take the hardware path), without the float64 reciprocal square
// root instruction, whose use in long dependent chains proved slow here:
// float32 seed of 1/sqrt(x) (relative error < 2^-21), two Newton steps in
// float64, s = x y, one residual correction, then the exact residual test of
// s and its neighbours that sqrt_unit uses in float32 (Tuckerman's test: no
// double x lies strictly between s_dn * s and the squared midpoint, because
// s_dn * s is a multiple of the square of s's ulp and x a multiple of it).
__device__ __forceinline__ double sqrt_d(double x) {
  if (!(x >= 0x1p-120 && x <= 0x1p120)) return __builtin_sqrt(x);
  double y = (double)__builtin_amdgcn_rsqf((float)x);
  const double hx = 0.5 * x;
  y = y * __builtin_fma(-hx * y, y, 1.5);
  y = y * __builtin_fma(-hx * y, y, 1.5);
  double s = x * y;
  s = __builtin_fma(__builtin_fma(-s, s, x), 0.5 * y, s);
  const double s_dn = __longlong_as_double(__double_as_longlong(s) - 1);
  const double s_up = __longlong_as_double(__double_as_longlong(s) + 1);
  const double r_dn = __builtin_fma(-s_dn, s, x);
  const double r_up = __builtin_fma(-s_up, s, x);
  double t = r_dn <= 0.0 ? s_dn : s;
  t = r_up > 0.0 ? s_up : t;
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

// ---- distinct hit radii -------------------------------------------------------
// The hits of a barrel layer share one radius, so u = ((kappa r^2 + Q) / r) T,
// its arcsine and everything else that depends only on (r, column) can be
// computed once per distinct radius and column instead of once per hit.  A
// workgroup collects the distinct radii of its valid hits in an LDS hash set
// (kRadSlots slots, linear probing, insertion by compare-and-swap); the first
// kMaxRadii of them in slot order get an index.  Hits whose radius has no
// index take the per-hit path.  The values computed per radius come from the
// same operations on the same operands as the per-hit ones, so both paths
// give identical bits.
constexpr int kRadSlots = 64;  // one slot per lane of a wave
constexpr int kMaxRadii = 16;
constexpr uint32_t kRadEmpty = 0xffffffffu;  // a NaN pattern, never a valid radius

struct RadiusSet {
  uint32_t key[kRadSlots];  // float bits of a radius, or kRadEmpty
  int32_t idx[kRadSlots];   // its index, or -1
  float r[kMaxRadii];
  int32_t n;
};

__device__ __forceinline__ uint32_t rad_hash(uint32_t k) { return (k * 2654435761u) >> 26; }

// Whole workgroup, over the hits [h0, h1); starts and ends with a barrier.
__device__ inline void radius_set_build(RadiusSet& R, const float* __restrict__ r,
                                        const float* __restrict__ phi, int h0, int h1) {
  static_assert(kRadSlots == kWave, "one hash slot per lane");
  __syncthreads();
  for (int t = threadIdx.x; t < kRadSlots; t += blockDim.x) R.key[t] = kRadEmpty;
  __syncthreads();
  uint32_t last = kRadEmpty;
  for (int h = h0 + (int)threadIdx.x; h < h1; h += blockDim.x) {
    const float rv = r[h];
    if (!hit_ok(rv, phi[h])) continue;
    const uint32_t k = __float_as_uint(rv);
    if (k == last) continue;
    last = k;
    uint32_t slot = rad_hash(k);
    for (int p = 0; p < kRadSlots; ++p) {
      const uint32_t v =
          __hip_atomic_load(&R.key[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (v == k) break;
      if (v == kRadEmpty) {
        const uint32_t old = atomicCAS(&R.key[slot], kRadEmpty, k);
        if (old == kRadEmpty || old == k) break;
      }
      slot = (slot + 1) & (kRadSlots - 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    const bool full = R.key[lane] != kRadEmpty;
    const uint64_t m = __ballot(full);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    const int id = (full && rank < kMaxRadii) ? rank : -1;
    R.idx[lane] = id;
    if (id >= 0) R.r[id] = __uint_as_float(R.key[lane]);
    if (lane == 0) R.n = __popcll(m) < kMaxRadii ? __popcll(m) : kMaxRadii;
  }
  __syncthreads();
}

// index of radius rv in the set, or -1
__device__ __forceinline__ int radius_index(const RadiusSet& R, float rv) {
  const uint32_t k = __float_as_uint(rv);
  uint32_t slot = rad_hash(k);
  for (int p = 0; p < kRadSlots; ++p) {
    const uint32_t v = R.key[slot];
    if (v == k) return R.idx[slot];
    if (v == kRadEmpty) return -1;
    slot = (slot + 1) & (kRadSlots - 1);
  }
  return -1;
}

}  // namespace ht
