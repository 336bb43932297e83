// First Hough transform: every valid hit votes once in every (q/pT, d0)
// column, for the phi0 bin of the outgoing circle branch through it (paper,
// section "Hough Transform Algorithm").
//
// gfx950 mapping.  One workgroup owns a tile of 64 consecutive q/pT columns
// at one d0 (lane = column), so a tile's accumulator rows are one contiguous
// block of the output.  The tile's counters live in LDS: 32-bit counters
// when 64 rows fit in the 160 KiB of a gfx950 CU (n_phi <= 639), otherwise
// 16-bit halves of 32 rows, column c in the low half of row c and column
// c + 32 in the high half (a column holds at most n_hits <= 65535 votes per
// bin, so a ds_add_u32 of 1 or 1 << 16 never carries across the halves; a
// lane's row and increment are fixed, so a vote costs the same instructions
// as with 32-bit counters).  The row stride is odd in dwords so neighbouring
// columns fall in different banks.  Waves of
// the workgroup split the hits: each wave loads 64 hits with one coalesced
// load, keeps them in VGPRs and broadcasts them one at a time through SGPRs
// (v_readlane), so the per-evaluation work is pure VALU with scalar hit
// operands plus one LDS atomic.  The arcsine and the |u| <= 1 test depend on
// the hit only through its radius: the workgroup first collects the distinct
// radii of its hits (the layers of a barrel tracker) and computes them once
// per radius and column into an LDS table, so a hit on a known radius costs
// one table read, three operations, the wrap and the atomic.  The tile is written to HBM once, by
// contiguous stores, so no clearing pass is needed.  No MFMA: the vote is a
// scatter, not a contraction.
//
// Grids with few tiles (the 2D grid has four) would leave most CUs idle, so
// there the hits are also split into slices (gridDim.z): each workgroup votes
// one slice of the hits into its LDS tile and adds the non-zero counters into
// the accumulator, cleared beforehand, with integer atomics (exact in any
// order).  The slices divide the hit count read at run time, so an event of
// any size spreads over the whole chip.  Dense events (16384 hits or more) on
// grids of at most one tile per CU take two slices with 16-bit counters: two
// workgroups then share each CU, which doubles the waves that hide the
// latency of the read, compute and LDS-atomic chain.
#include "ht_internal.h"

namespace ht {
namespace {

constexpr int kVoteWaves = 16;
constexpr int kVoteThreads = kVoteWaves * kWave;

__device__ __forceinline__ float bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// The events of one launch (a batch of NB events; one event is the batch of
// one): hits, device hit count (optional), accumulator and vote total
// (optional) of each.
template <int NB>
struct VoteBatch {
  const float* r[NB];
  const float* phi[NB];
  const int32_t* n_dev[NB];
  int32_t* acc[NB];
  unsigned long long* n_votes[NB];
};

template <bool POW2, bool WIDE, int NB>
__global__ __launch_bounds__(kVoteThreads) void vote_kernel(
    VoteBatch<NB> V, int n_hits_max, const float* __restrict__ kap,
    const float* __restrict__ qt, const float* __restrict__ tt, int n_phi, int n_qpt,
    float phi_lo, float invw, int stride) {
  extern __shared__ uint32_t lds[];
  __shared__ RadiusSet R;
  __shared__ float s_tab[kMaxRadii][kWave];  // arcsine per (radius, column), NaN: no vote
  // blockIdx.z = event * slices + slice of the event's hits
  const int n_slices = gridDim.z / NB;
  const int ev = NB == 1 ? 0 : (int)blockIdx.z / n_slices;
  const int slice = (int)blockIdx.z % n_slices;
  const float* __restrict__ r = V.r[ev];
  const float* __restrict__ phi = V.phi[ev];
  const int32_t* __restrict__ n_hits_dev = V.n_dev[ev];
  int32_t* __restrict__ acc = V.acc[ev];
  unsigned long long* __restrict__ n_votes = V.n_votes[ev];
  // hits of this event: the device count when given (clamped to the bound the
  // buffers were checked for), else the host count
  const int n_all = n_hits_dev ? min(max(*n_hits_dev, 0), n_hits_max) : n_hits_max;
  const int chunk = ((n_all + n_slices - 1) / n_slices + kWave - 1) / kWave * kWave;
  const int h0 = slice * chunk;
  const int n_hits = min(n_all, h0 + chunk);
  if (n_slices > 1 && h0 >= n_hits) return;  // an empty slice adds nothing
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6;
  const int j0 = blockIdx.x * kWave;
  const int k = blockIdx.y;
  const int j = j0 + lane;
  const bool col_ok = j < n_qpt;

  constexpr int kRows = WIDE ? kWave : kWave / 2;
  for (int w = threadIdx.x; w < kRows * stride; w += kVoteThreads) lds[w] = 0u;
  float ck = 0.0f, cq = 0.0f, ct = 0.0f;
  if (col_ok) {
    ck = kap[j];
    cq = qt[(size_t)k * n_qpt + j];
    ct = tt[(size_t)k * n_qpt + j];
  }
  radius_set_build(R, r, phi, h0, n_hits);
  // thread t fills entry (t / 64, lane): its own column
  for (int t = threadIdx.x; t < R.n * kWave; t += kVoteThreads) {
    const float rv = R.r[t >> 6];
    const float r2 = rv * rv;
    const float ir = 1.0f / rv;
    const float a = ck * r2;
    const float b = a + cq;
    const float c = b * ir;
    const float u = c * ct;
    const bool ok = col_ok && (fabsf(u) <= 1.0f);
    s_tab[t >> 6][lane] = ok ? asin_f(u) : __builtin_nanf("");
  }
  __syncthreads();
  // the lane's column of the table in registers, indexed by the
  // wave-uniform radius index (no LDS round trip per hit)
  float sreg[kMaxRadii];
#pragma unroll
  for (int a = 0; a < kMaxRadii; ++a) sreg[a] = a < R.n ? s_tab[a][lane] : __builtin_nanf("");

  uint32_t* col = lds + (lane % kRows) * stride;
  const uint32_t inc = WIDE || lane < kRows ? 1u : 65536u;
  for (int base = h0 + wave * kWave; base < n_hits; base += kVoteThreads) {
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
    const int hri = hv ? radius_index(R, hr) : -1;
    uint64_t todo = __ballot(hv);
    while (todo) {
      const int src = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int ri = __builtin_amdgcn_readlane(hri, src);
      const float ph = bcast(hp, src);
      bool ok;
      float s;
      if (ri >= 0) {
        s = sreg[ri];
        ok = s == s;
      } else {
        const float r2 = bcast(hr2, src);
        const float ir = bcast(hir, src);
        const float a = ck * r2;
        const float b = a + cq;
        const float c = b * ir;
        const float u = c * ct;
        ok = col_ok && (fabsf(u) <= 1.0f);
        s = asin_f(u);
      }
      const float phi0 = ph - s;
      const float d = phi0 - phi_lo;
      const float x = d * invw;
      // x lies in [-n_phi, 2 n_phi) (|phi| <= 4, |asin| <= pi/2): one
      // period of correction is enough; a power of two wraps with a mask
      // floor and conversion in one instruction (x is finite and in range
      // whenever the vote counts)
      int i;
      asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(i) : "v"(x));
      if (POW2) {
        i &= n_phi - 1;
      } else {
        i = i < 0 ? i + n_phi : i;
        i = i >= n_phi ? i - n_phi : i;
      }
      if (ok) {
        atomicAdd(&col[i], inc);
      }
    }
  }
  __syncthreads();

  // write the tile: rows j0 .. j0+ncol-1 of plane k are contiguous
  const int ncol = min(kWave, n_qpt - j0);
  int32_t* out = acc + ((size_t)k * n_qpt + j0) * n_phi;
  const int total = ncol * n_phi;
  auto tile = [&](int e) {
    const int cj = e / n_phi;
    const int i = e - cj * n_phi;
    if (WIDE) return (int32_t)lds[cj * stride + i];
    const uint32_t w = lds[(cj % kRows) * stride + i];
    return (int32_t)(cj >= kRows ? (w >> 16) : (w & 0xFFFFu));
  };
  // the vote count, when asked for, is the sum of the tile's counters (the
  // loop above keeps no count of its own)
  uint32_t votes = 0;
  if (n_slices == 1) {
    for (int e = threadIdx.x; e < total; e += kVoteThreads) {
      const int32_t v = tile(e);
      out[e] = v;
      votes += (uint32_t)v;
    }
  } else {
    for (int e = threadIdx.x; e < total; e += kVoteThreads) {
      const int32_t v = tile(e);
      if (v) atomicAdd(&out[e], v);
      votes += (uint32_t)v;
    }
  }

  if (n_votes) {
    unsigned long long v = votes;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0 && v) atomicAdd(n_votes, v);
  }
}

__global__ void asin_kernel(const float* __restrict__ u, float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = asin_f(u[i]);
}

__global__ void sqrt_kernel(const double* __restrict__ x, double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = sqrt_d(x[i]);
}

__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

__global__ void zero_i32_kernel(int32_t* __restrict__ p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = 0;
}

// LDS of a CU less the kernel's static arrays (radius set and table)
constexpr int kLdsBytes = 160 * 1024 - (int)sizeof(RadiusSet) - kMaxRadii * kWave * 4;
bool vote_wide(int n_phi) { return (size_t)kWave * (size_t)(n_phi | 1) * 4 <= (size_t)kLdsBytes; }
int vote_stride(int n_phi) { return n_phi | 1; }  // odd dword stride
// LDS bytes of a tile: 64 rows of 32-bit counters, or 32 rows of 16-bit pairs
size_t vote_lds_bytes(int n_phi, bool wide) {
  return (size_t)(wide ? kWave : kWave / 2) * vote_stride(n_phi) * 4;
}

}  // namespace

namespace {
template <int NB>
int vote_init_nb(int bytes) {
  const hipFuncAttribute at = hipFuncAttributeMaxDynamicSharedMemorySize;
  HT_CHECK(hipFuncSetAttribute((const void*)vote_kernel<true, true, NB>, at, bytes));
  HT_CHECK(hipFuncSetAttribute((const void*)vote_kernel<false, true, NB>, at, bytes));
  HT_CHECK(hipFuncSetAttribute((const void*)vote_kernel<true, false, NB>, at, bytes));
  HT_CHECK(hipFuncSetAttribute((const void*)vote_kernel<false, false, NB>, at, bytes));
  return HT_OK;
}

// The vote of NB events on one plan's grid (the plan gives the tables).
template <int NB>
int vote_launch(const Plan& p, const VoteBatch<NB>& V, int32_t n_hits, hipStream_t s) {
  const ht_grid& g = p.grid;
  for (int b = 0; b < NB; ++b) {
    if (V.n_votes[b]) {
      zero_u64_kernel<<<1, 1, 0, s>>>(V.n_votes[b]);
      HT_CHECK(hipGetLastError());
    }
  }
  const int tiles = (g.n_qpt + kWave - 1) / kWave * g.n_d0;
  int slices = hit_slices(tiles, n_hits);
  bool wide = vote_wide(g.n_phi);
  // Dense events on grids of at most one tile per CU: 16-bit counters, so
  // that two workgroups fit a CU's LDS, and two hit slices, so that two run
  // on each CU (8 waves per SIMD instead of 4).  55k-hit events on the
  // 512x256x64 grid: 0.62 -> 0.53 ms.
  if (slices == 1 && tiles <= 256 && n_hits >= 16384) {
    slices = 2;
    wide = false;
  }
  const int stride = vote_stride(g.n_phi);
  const size_t lds_bytes = vote_lds_bytes(g.n_phi, wide);
  dim3 grid((g.n_qpt + kWave - 1) / kWave, g.n_d0, slices * NB);
  if (slices > 1) {
    // the slices add into the accumulator: clear it first (a kernel, so the
    // sequence can be captured in a graph)
    const int64_t cells = p.n_cells;
    const int64_t blocks = (cells + 1023) / 1024 < 1024 ? (cells + 1023) / 1024 : 1024;
    for (int b = 0; b < NB; ++b) {
      zero_i32_kernel<<<(unsigned)blocks, 256, 0, s>>>(V.acc[b], cells);
      HT_CHECK(hipGetLastError());
    }
  }
  const bool pow2 = (g.n_phi & (g.n_phi - 1)) == 0;
  auto kern = pow2 ? (wide ? vote_kernel<true, true, NB> : vote_kernel<true, false, NB>)
                   : (wide ? vote_kernel<false, true, NB> : vote_kernel<false, false, NB>);
  p.prof_mark(HT_STAGE_VOTE, 0, s);
  kern<<<grid, kVoteThreads, lds_bytes, s>>>(V, n_hits, p.d_kap, p.d_q, p.d_t, g.n_phi, g.n_qpt,
                                             p.phi_lo, p.invw, stride);
  HT_CHECK(hipGetLastError());
  p.prof_mark(HT_STAGE_VOTE, 1, s);
  return HT_OK;
}

template <int NB>
int vote_batch_nb(const Plan& p, const float* const* r, const float* const* phi,
                  const int32_t* const* n_dev, int32_t n_hits_max, int32_t* const* acc,
                  hipStream_t s) {
  VoteBatch<NB> V;
  for (int b = 0; b < NB; ++b) {
    V.r[b] = r[b];
    V.phi[b] = phi[b];
    V.n_dev[b] = n_dev[b];
    V.acc[b] = acc[b];
    V.n_votes[b] = nullptr;
  }
  return vote_launch<NB>(p, V, n_hits_max, s);
}
}  // namespace

int vote_init(int n_phi) {
  const int bytes = (int)vote_lds_bytes(n_phi, vote_wide(n_phi));
  int rc = vote_init_nb<1>(bytes);
  if (rc == HT_OK) rc = vote_init_nb<2>(bytes);
  if (rc == HT_OK) rc = vote_init_nb<3>(bytes);
  if (rc == HT_OK) rc = vote_init_nb<4>(bytes);
  return rc;
}

int launch_vote_batch(const Plan& p, int nb, const float* const* r, const float* const* phi,
                      const int32_t* const* n_dev, int32_t n_hits_max, int32_t* const* acc,
                      hipStream_t s) {
  switch (nb) {
    case 1: return vote_batch_nb<1>(p, r, phi, n_dev, n_hits_max, acc, s);
    case 2: return vote_batch_nb<2>(p, r, phi, n_dev, n_hits_max, acc, s);
    case 3: return vote_batch_nb<3>(p, r, phi, n_dev, n_hits_max, acc, s);
    case 4: return vote_batch_nb<4>(p, r, phi, n_dev, n_hits_max, acc, s);
    default: return HT_EUNSUPPORTED;
  }
}

int launch_vote(const Plan& p, const float* r, const float* phi, int32_t n_hits, int32_t* acc,
                unsigned long long* n_votes, hipStream_t s, const int32_t* n_hits_dev) {
  VoteBatch<1> V;
  V.r[0] = r;
  V.phi[0] = phi;
  V.n_dev[0] = n_hits_dev;
  V.acc[0] = acc;
  V.n_votes[0] = n_votes;
  return vote_launch<1>(p, V, n_hits, s);
}

int launch_sqrt(const double* x, double* out, int64_t n, hipStream_t s) {
  if (n == 0) return HT_OK;
  const int threads = 256;
  const int64_t blocks = (n + threads - 1) / threads;
  sqrt_kernel<<<(unsigned)blocks, threads, 0, s>>>(x, out, n);
  HT_CHECK(hipGetLastError());
  return HT_OK;
}

int launch_asin(const float* u, float* out, int64_t n, hipStream_t s) {
  if (n == 0) return HT_OK;
  const int threads = 256;
  const int64_t blocks = (n + threads - 1) / threads;
  asin_kernel<<<(unsigned)blocks, threads, 0, s>>>(u, out, n);
  HT_CHECK(hipGetLastError());
  return HT_OK;
}

}  // namespace ht
