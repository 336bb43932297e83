// Band (cell) vote, a variant of the first transform: each valid hit votes
// for every phi0 bin its curve reaches while (kappa, d0) range over a
// column's cell, instead of the point at the column centre (the paper's
// instances are cells of the parameter space, section "Hough Transform
// Algorithm").  u = sin(phi - phi0) is increasing in kappa and d0 over the
// cell, so the band runs between the phi0 of two corners: (smallest kappa,
// lower d0 edge) and (largest kappa, upper d0 edge), each from the float32
// vote formula with that corner's tables; u is clipped to [-1, 1], and no
// vote is cast when the whole cell lies beyond |u| = 1.
//
// Same gfx950 mapping as the point vote: a workgroup owns 64 q/pT columns of
// one d0 plane in LDS (lane = column), waves split the hits and broadcast
// them through SGPRs.  A hit adds one LDS atomic per bin of its band, about
// four per column on the displaced-jet grid.  Grids with few tiles also split
// the hits into slices that add their tiles into a cleared accumulator, as
// the point vote does.
#include "ht_internal.h"

namespace ht {
namespace {

constexpr int kCellWaves = 16;
constexpr int kCellThreads = kCellWaves * kWave;
constexpr int kLdsBytes = 160 * 1024;

__device__ __forceinline__ float bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

bool cell_wide(int n_phi) { return (size_t)kWave * (size_t)(n_phi | 1) * 4 <= (size_t)kLdsBytes; }
int cell_stride(int n_phi) {
  const int words = cell_wide(n_phi) ? n_phi : (n_phi + 1) / 2;
  return words | 1;  // odd dword stride
}

template <bool WIDE>
__device__ __forceinline__ void add_vote(uint32_t* col, int i) {
  if (WIDE)
    atomicAdd(&col[i], 1u);
  else
    atomicAdd(&col[i >> 1], (i & 1) ? 65536u : 1u);
}

template <bool WIDE>
__global__ __launch_bounds__(kCellThreads) void cell_vote_kernel(
    const float* __restrict__ r, const float* __restrict__ phi, int n_all,
    const float* __restrict__ kl, const float* __restrict__ kh, const float* __restrict__ ql,
    const float* __restrict__ tl, const float* __restrict__ qh, const float* __restrict__ th,
    int n_phi, int n_qpt, float phi_lo, float invw, int stride, int32_t* __restrict__ acc,
    unsigned long long* __restrict__ n_votes) {
  extern __shared__ uint32_t lds[];
  const int n_slices = gridDim.z;
  const int chunk = ((n_all + n_slices - 1) / n_slices + kWave - 1) / kWave * kWave;
  const int h0 = (int)blockIdx.z * chunk;
  const int n_hits = min(n_all, h0 + chunk);
  if (n_slices > 1 && h0 >= n_hits) return;  // an empty slice adds nothing
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6;
  const int j0 = blockIdx.x * kWave;
  const int k = blockIdx.y;
  const int j = j0 + lane;
  const bool col_ok = j < n_qpt;

  for (int w = threadIdx.x; w < kWave * stride; w += kCellThreads) lds[w] = 0u;
  float ckl = 0.0f, ckh = 0.0f, cql = 0.0f, ctl = 0.0f, cqh = 0.0f, cth = 0.0f;
  if (col_ok) {
    const size_t c = (size_t)k * n_qpt + j;
    ckl = kl[j];
    ckh = kh[j];
    cql = ql[c];
    ctl = tl[c];
    cqh = qh[c];
    cth = th[c];
  }
  __syncthreads();

  uint32_t* col = lds + lane * stride;
  unsigned long long votes = 0;
  for (int base = h0 + wave * kWave; base < n_hits; base += kCellThreads) {
    const int h = base + lane;
    float hr = 1.0f, hp = 0.0f;
    bool hv = false;
    if (h < n_hits) {
      hr = r[h];
      hp = phi[h];
      hv = hit_ok(hr, hp);
    }
    const float hr2 = hr * hr;
    const float hir = 1.0f / hr;
    uint64_t todo = __ballot(hv);
    while (todo) {
      const int src = __builtin_ctzll(todo);
      todo &= todo - 1;
      const float r2 = bcast(hr2, src);
      const float ir = bcast(hir, src);
      const float ph = bcast(hp, src);
      float ulo = ((ckl * r2 + cql) * ir) * ctl;
      float uhi = ((ckh * r2 + cqh) * ir) * cth;
      const bool ok = col_ok && !(ulo > 1.0f) && !(uhi < -1.0f);
      ulo = fmaxf(ulo, -1.0f);
      uhi = fminf(uhi, 1.0f);
      const float xa = ((ph - asin_f(uhi)) - phi_lo) * invw;
      const float xb = ((ph - asin_f(ulo)) - phi_lo) * invw;
      const float lo = fminf(xa, xb), hi = fmaxf(xa, xb);
      // both lie in [-n_phi - 1, 2 n_phi + 1): one period of correction
      int ia = (int)floorf(lo);
      const int ib = (int)floorf(hi);
      int m = ib - ia + 1;
      if (m >= n_phi) {
        m = n_phi;
        ia = 0;
      }
      ia = ia < 0 ? ia + n_phi : ia;
      ia = ia >= n_phi ? ia - n_phi : ia;
      if (ok) {
        int i = ia;
        for (int q = 0; q < m; ++q) {
          add_vote<WIDE>(col, i);
          i = i + 1 == n_phi ? 0 : i + 1;
        }
        votes += (unsigned long long)m;
      }
    }
  }
  __syncthreads();

  const int ncol = min(kWave, n_qpt - j0);
  int32_t* out = acc + ((size_t)k * n_qpt + j0) * n_phi;
  const int total = ncol * n_phi;
  auto tile = [&](int e) {
    const int cj = e / n_phi;
    const int i = e - cj * n_phi;
    if (WIDE) return (int32_t)lds[cj * stride + i];
    const uint32_t w = lds[cj * stride + (i >> 1)];
    return (int32_t)((i & 1) ? (w >> 16) : (w & 0xFFFFu));
  };
  if (n_slices == 1) {
    for (int e = threadIdx.x; e < total; e += kCellThreads) out[e] = tile(e);
  } else {
    for (int e = threadIdx.x; e < total; e += kCellThreads) {
      const int32_t v = tile(e);
      if (v) atomicAdd(&out[e], v);
    }
  }

  if (n_votes) {
    unsigned long long v = votes;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0 && v) atomicAdd(n_votes, v);
  }
}

__global__ void zero_u64(unsigned long long* p) { *p = 0ull; }

__global__ void zero_i32(int32_t* __restrict__ p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = 0;
}

}  // namespace

int cell_vote_init(int n_phi) {
  const int bytes = kWave * cell_stride(n_phi) * 4;
  const hipFuncAttribute at = hipFuncAttributeMaxDynamicSharedMemorySize;
  HT_CHECK(hipFuncSetAttribute((const void*)cell_vote_kernel<true>, at, bytes));
  HT_CHECK(hipFuncSetAttribute((const void*)cell_vote_kernel<false>, at, bytes));
  return HT_OK;
}

int launch_cell_vote(const Plan& p, const float* r, const float* phi, int32_t n_hits,
                     int32_t* acc, unsigned long long* n_votes, hipStream_t s) {
  const ht_grid& g = p.grid;
  const int stride = cell_stride(g.n_phi);
  const size_t lds_bytes = (size_t)kWave * stride * 4;
  if (n_votes) {
    zero_u64<<<1, 1, 0, s>>>(n_votes);
    HT_CHECK(hipGetLastError());
  }
  const int tiles = (g.n_qpt + kWave - 1) / kWave * g.n_d0;
  const int slices = hit_slices(tiles, n_hits);
  dim3 grid((g.n_qpt + kWave - 1) / kWave, g.n_d0, slices);
  if (slices > 1) {
    const int64_t cells = p.n_cells;
    const int64_t blocks = (cells + 1023) / 1024 < 1024 ? (cells + 1023) / 1024 : 1024;
    zero_i32<<<(unsigned)blocks, 256, 0, s>>>(acc, cells);
    HT_CHECK(hipGetLastError());
  }
  auto kern = cell_wide(g.n_phi) ? cell_vote_kernel<true> : cell_vote_kernel<false>;
  p.prof_mark(HT_STAGE_VOTE, 0, s);
  kern<<<grid, kCellThreads, lds_bytes, s>>>(r, phi, n_hits, p.d_ckl, p.d_ckh, p.d_cql, p.d_ctl,
                                             p.d_cqh, p.d_cth, g.n_phi, g.n_qpt, p.phi_lo,
                                             p.invw, stride, acc, n_votes);
  HT_CHECK(hipGetLastError());
  p.prof_mark(HT_STAGE_VOTE, 1, s);
  return HT_OK;
}

}  // namespace ht
