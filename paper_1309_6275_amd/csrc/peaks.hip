// Local maxima of the accumulator (paper, section "Hough Transform
// Algorithm"), written in cell order.
//
// Three launches, each a sweep over the cell range:
//   1. flag: the 26-neighbour rule; a wave's flags become ballot words and
//      each tile writes its peak count;
//   2. scan: one workgroup turns tile counts into tile offsets and the
//      total count;
//   3. emit: one workgroup per tile reads its ballot words and writes its
//      peaks at offset + rank, the rank coming from popcount prefix sums, so
//      the list is sorted by cell index with no sort.
// When n_phi is a multiple of 4 (and the accumulator 16-byte aligned) a lane
// takes 4 consecutive cells of one row and a tile is 1024 cells.  If n_phi
// divides the tile (and n_qpt is a multiple of the tile's rows), the tile's
// 3 x (rows + 2) neighbour rows are staged in LDS once; otherwise each of the
// 9 neighbour rows is one 16-byte load plus the two cells beside it, from
// L2.  Other n_phi: a lane takes one cell and a tile is 256 cells.
#include <mutex>

#include "ht_internal.h"

namespace ht {
namespace {

constexpr int kTile = 256;

// The events of one launch (NB of them; blockIdx.y picks one): accumulator,
// peak ballots, tile counts and offsets, output list and count of each.
template <int NB>
struct PeakBatch {
  const int32_t* acc[NB];
  void* bits[NB];
  int32_t* cnt[NB];
  int32_t* off[NB];
  ht_peak* out[NB];
};
#define HT_PEAK_EVENT(PB)                                                     \
  const int ev_ = NB == 1 ? 0 : (int)blockIdx.y;                              \
  const int32_t* __restrict__ acc = (PB).acc[ev_];                            \
  (void)acc;

__device__ __forceinline__ bool is_peak(const int32_t* __restrict__ acc, int n_phi, int n_qpt,
                                        int n_d0, int k, int j, int i, int32_t thr) {
  const int32_t v = acc[((size_t)k * n_qpt + j) * n_phi + i];
  if (v < thr) return false;
  const int im = i == 0 ? n_phi - 1 : i - 1;
  const int ip = i == n_phi - 1 ? 0 : i + 1;
#pragma unroll
  for (int dk = -1; dk <= 1; ++dk) {
    const int kk = k + dk;
    if (kk < 0 || kk >= n_d0) continue;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      const int jj = j + dj;
      if (jj < 0 || jj >= n_qpt) continue;
      const int32_t* row = acc + ((size_t)kk * n_qpt + jj) * n_phi;
      const int32_t wm = row[im], w0 = row[i], wp = row[ip];
      if (dk < 0 || (dk == 0 && dj < 0)) {
        if (!(v > wm && v > w0 && v > wp)) return false;
      } else if (dk == 0 && dj == 0) {
        if (!(v > wm && v >= wp)) return false;
      } else {
        if (!(v >= wm && v >= w0 && v >= wp)) return false;
      }
    }
  }
  return true;
}

template <int NB>
__global__ __launch_bounds__(kTile) void flag_kernel(PeakBatch<NB> PB, int n_phi, int n_qpt,
                                                     int n_d0, int64_t n_cells, int32_t thr) {
  HT_PEAK_EVENT(PB)
  uint32_t* __restrict__ bits = static_cast<uint32_t*>(PB.bits[ev_]);
  int32_t* __restrict__ tile_cnt = PB.cnt[ev_];
  __shared__ int32_t wcnt[kTile / kWave];
  const int64_t lin = (int64_t)blockIdx.x * kTile + threadIdx.x;
  bool pk = false;
  if (lin < n_cells) {
    const int i = (int)(lin % n_phi);
    const int64_t col = lin / n_phi;
    const int j = (int)(col % n_qpt);
    const int k = (int)(col / n_qpt);
    pk = is_peak(acc, n_phi, n_qpt, n_d0, k, j, i, thr);
  }
  const uint64_t m = __ballot(pk);
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6;
  if (lane == 0) {
    const int64_t w = ((int64_t)blockIdx.x * kTile + wave * kWave) >> 5;
    bits[w] = (uint32_t)m;
    bits[w + 1] = (uint32_t)(m >> 32);
    wcnt[wave] = __popcll(m);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int w = 0; w < kTile / kWave; ++w) s += wcnt[w];
    tile_cnt[blockIdx.x] = s;
  }
}

template <int NB>
__global__ __launch_bounds__(kTile) void emit_kernel(PeakBatch<NB> PB, int64_t n_cells,
                                                     int32_t capacity) {
  HT_PEAK_EVENT(PB)
  const uint32_t* __restrict__ bits = static_cast<const uint32_t*>(PB.bits[ev_]);
  const int32_t* __restrict__ tile_off = PB.off[ev_];
  ht_peak* __restrict__ out = PB.out[ev_];
  __shared__ int32_t wpre[kTile / kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6;
  const int64_t lin = (int64_t)blockIdx.x * kTile + threadIdx.x;
  const int64_t wbase = ((int64_t)blockIdx.x * kTile + wave * kWave) >> 5;
  const uint64_t m = (uint64_t)bits[wbase] | ((uint64_t)bits[wbase + 1] << 32);
  if (lane == 0) wpre[wave] = __popcll(m);
  __syncthreads();
  int32_t before = 0;
  for (int w = 0; w < wave; ++w) before += wpre[w];
  const bool pk = (m >> lane) & 1ull;
  if (pk && lin < n_cells) {
    const uint64_t lower = lane ? (m & ((1ull << lane) - 1ull)) : 0ull;
    const int64_t idx = (int64_t)tile_off[blockIdx.x] + before + __popcll(lower);
    if (idx < capacity) {
      ht_peak p;
      p.lin = (int32_t)lin;
      p.votes = acc[lin];
      out[idx] = p;
    }
  }
}

// ---- four cells per lane ------------------------------------------------------
constexpr int kTile4 = 1024;  // 4 waves x 64 lanes x 4 cells
constexpr int kXcds = 8;      // MI355X: workgroup b runs on XCD b mod 8

// Tile of workgroup b: each XCD takes one contiguous range of tiles, so the
// neighbour rows that consecutive tiles share stay in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int n_tiles) {
  const int per = n_tiles / kXcds, rem = n_tiles % kXcds;
  const int x = b % kXcds, i = b / kXcds;
  return x * per + min(x, rem) + i;
}

// cells i0-1 .. i0+4 of a row (phi0 periodic); i0 is a multiple of 4
__device__ __forceinline__ void load_row6(const int32_t* __restrict__ row, int i0, int n_phi,
                                          int32_t w[6]) {
  const int4 m = *reinterpret_cast<const int4*>(row + i0);
  w[0] = row[i0 == 0 ? n_phi - 1 : i0 - 1];
  w[1] = m.x;
  w[2] = m.y;
  w[3] = m.z;
  w[4] = m.w;
  w[5] = row[i0 + 4 == n_phi ? 0 : i0 + 4];
}

// Ballot words: wave w of tile b writes 4 words at (b * 4 + w) * 4; bit l of
// word t flags cell b * 1024 + w * 256 + 4 l + t.
template <int NB>
__global__ __launch_bounds__(256) void flag4_kernel(PeakBatch<NB> PB, int n_phi, int n_qpt,
                                                    int n_d0, int64_t n_cells, int32_t thr) {
  HT_PEAK_EVENT(PB)
  uint64_t* __restrict__ bits = static_cast<uint64_t*>(PB.bits[ev_]);
  int32_t* __restrict__ tile_cnt = PB.cnt[ev_];
  __shared__ int32_t wcnt[4];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  // n_cells < 2^31, so cell indices of a tile fit in 32 bits unsigned
  const uint32_t lin0 = (uint32_t)tile * kTile4 + threadIdx.x * 4u;
  bool f[4] = {false, false, false, false};
  if (lin0 < (uint64_t)n_cells) {  // n_cells is a multiple of 4: all four cells exist
    const uint32_t col = lin0 / (uint32_t)n_phi;
    const int i0 = (int)(lin0 - col * (uint32_t)n_phi);
    const int k = (int)(col / (uint32_t)n_qpt);
    const int j = (int)col - k * n_qpt;
    const int4 c4 = *reinterpret_cast<const int4*>(acc + lin0);
    const int32_t v[4] = {c4.x, c4.y, c4.z, c4.w};
    bool any = false;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f[t] = v[t] >= thr;
      any = any || f[t];
    }
    if (any) {
      // The rule in maxima: a cell must exceed the largest of its neighbours
      // in the rows before it (dk < 0, or dk = 0 and dj < 0) and of its left
      // neighbour, and reach the largest in the rows after it and its right
      // neighbour.  Per row the 3-cell maxima of the four cells share their
      // pairwise maxima.
      int32_t neg[4], pos[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) neg[t] = pos[t] = INT32_MIN;
#pragma unroll
      for (int dk = -1; dk <= 1; ++dk) {
        const int kk = k + dk;
        if (kk < 0 || kk >= n_d0) continue;
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
          const int jj = j + dj;
          if (jj < 0 || jj >= n_qpt) continue;
          int32_t w[6];
          load_row6(acc + ((size_t)kk * n_qpt + jj) * n_phi, i0, n_phi, w);
          if (dk == 0 && dj == 0) {
#pragma unroll
            for (int t = 0; t < 4; ++t) f[t] = f[t] && v[t] > w[t] && v[t] >= w[t + 2];
            continue;
          }
          int32_t pm[5];
#pragma unroll
          for (int t = 0; t < 5; ++t) pm[t] = max(w[t], w[t + 1]);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int32_t m3 = max(pm[t], w[t + 2]);  // cells i-1, i, i+1
            if (dk < 0 || (dk == 0 && dj < 0))
              neg[t] = max(neg[t], m3);
            else
              pos[t] = max(pos[t], m3);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) f[t] = f[t] && v[t] > neg[t] && v[t] >= pos[t];
    }
  }
  uint64_t m[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) m[t] = __ballot(f[t]);
  if (lane == 0) {
    uint64_t* wb = bits + ((size_t)tile * 4 + wave) * 4;
    int c = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      wb[t] = m[t];
      c += __popcll(m[t]);
    }
    wcnt[wave] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) tile_cnt[tile] = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
}

// The same flags with the tile's neighbourhood staged in LDS, for grids
// whose phi axis divides the 1024-cell tile (n_phi = 1024 / R) and whose
// q/pT axis is a multiple of R, so a tile is R whole rows of one d0 plane.
// The 3 x (R + 2) rows around it are read once, coalesced, instead of nine
// overlapping row reads per lane from L2.
template <int R, int NB>
__global__ __launch_bounds__(256) void flag4s_kernel(PeakBatch<NB> PB, int n_qpt, int n_d0,
                                                     int32_t thr) {
  HT_PEAK_EVENT(PB)
  uint64_t* __restrict__ bits = static_cast<uint64_t*>(PB.bits[ev_]);
  int32_t* __restrict__ tile_cnt = PB.cnt[ev_];
  constexpr int NP = kTile4 / R;  // n_phi
  constexpr int ROWS = R + 2;
  __shared__ int32_t sm[3][ROWS][NP];
  __shared__ int32_t wcnt[4];
  __shared__ int32_t rok[3][ROWS];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int c0 = tile * R;          // first row (q/pT, d0 column) of the tile
  const int k = c0 / n_qpt;
  const int j0 = c0 - k * n_qpt;
  if (threadIdx.x < 3 * ROWS) {
    const int dk = threadIdx.x / ROWS - 1, jr = threadIdx.x % ROWS - 1;
    const int kk = k + dk, jj = j0 + jr;
    rok[dk + 1][jr + 1] = (kk >= 0 && kk < n_d0 && jj >= 0 && jj < n_qpt) ? 1 : 0;
  }
  __syncthreads();
  constexpr int Q = NP / 4;  // int4 per row
  for (int e = threadIdx.x; e < 3 * ROWS * Q; e += 256) {
    const int row = e / Q, q4 = e - row * Q;
    const int dk = row / ROWS, jr = row - dk * ROWS;
    if (!rok[dk][jr]) continue;
    const int kk = k + dk - 1, jj = j0 + jr - 1;
    const int4 v4 = *reinterpret_cast<const int4*>(acc + ((size_t)kk * n_qpt + jj) * NP + q4 * 4);
    *reinterpret_cast<int4*>(&sm[dk][jr][q4 * 4]) = v4;
  }
  __syncthreads();
  const int r = (threadIdx.x * 4) / NP;       // row of the tile
  const int i0 = (threadIdx.x * 4) % NP;
  const int im = i0 == 0 ? NP - 1 : i0 - 1;   // phi0 periodic
  const int ip = i0 + 4 == NP ? 0 : i0 + 4;
  int32_t v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) v[t] = sm[1][r + 1][i0 + t];
  bool f[4];
  bool any = false;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f[t] = v[t] >= thr;
    any = any || f[t];
  }
  if (any) {
    int32_t neg[4], pos[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) neg[t] = pos[t] = INT32_MIN;
#pragma unroll
    for (int dk = 0; dk < 3; ++dk) {
#pragma unroll
      for (int dj = 0; dj < 3; ++dj) {
        if (!rok[dk][r + dj]) continue;
        const int32_t* row = sm[dk][r + dj];
        int32_t w[6];
        w[0] = row[im];
#pragma unroll
        for (int t = 0; t < 4; ++t) w[t + 1] = row[i0 + t];
        w[5] = row[ip];
        if (dk == 1 && dj == 1) {
#pragma unroll
          for (int t = 0; t < 4; ++t) f[t] = f[t] && v[t] > w[t] && v[t] >= w[t + 2];
          continue;
        }
        int32_t pm[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) pm[t] = max(w[t], w[t + 1]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int32_t m3 = max(pm[t], w[t + 2]);
          if (dk < 1 || (dk == 1 && dj < 1))
            neg[t] = max(neg[t], m3);
          else
            pos[t] = max(pos[t], m3);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) f[t] = f[t] && v[t] > neg[t] && v[t] >= pos[t];
  }
  uint64_t m[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) m[t] = __ballot(f[t]);
  if (lane == 0) {
    uint64_t* wb = bits + ((size_t)tile * 4 + wave) * 4;
    int c = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      wb[t] = m[t];
      c += __popcll(m[t]);
    }
    wcnt[wave] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) tile_cnt[tile] = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
}

template <int NB>
__global__ __launch_bounds__(256) void emit4_kernel(PeakBatch<NB> PB, int64_t n_cells,
                                                    int32_t capacity) {
  HT_PEAK_EVENT(PB)
  const uint64_t* __restrict__ bits = static_cast<const uint64_t*>(PB.bits[ev_]);
  const int32_t* __restrict__ tile_off = PB.off[ev_];
  ht_peak* __restrict__ out = PB.out[ev_];
  __shared__ int32_t wpre[4];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint64_t* wb = bits + ((size_t)tile * 4 + wave) * 4;
  uint64_t m[4];
  int c = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    m[t] = wb[t];
    c += __popcll(m[t]);
  }
  if (lane == 0) wpre[wave] = c;
  __syncthreads();
  int64_t idx = tile_off[tile];
  for (int w = 0; w < wave; ++w) idx += wpre[w];
  const uint64_t below = lane ? ((1ull << lane) - 1ull) : 0ull;
#pragma unroll
  for (int t = 0; t < 4; ++t) idx += __popcll(m[t] & below);
  const int64_t lin0 = (int64_t)tile * kTile4 + (int64_t)threadIdx.x * 4;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if ((m[t] >> lane) & 1ull) {
      const int64_t lin = lin0 + t;
      if (idx < capacity && lin < n_cells) {
        ht_peak p;
        p.lin = (int32_t)lin;
        p.votes = acc[lin];
        out[idx] = p;
      }
      ++idx;
    }
  }
}

}  // namespace

int peaks_init(int) { return HT_OK; }

template <int NB>
int peaks_batch_core(const ht_grid& g, int64_t n_cells, const PeakBatch<NB>& PB, int32_t min_votes,
                     int32_t capacity, int32_t* const* n_found, hipStream_t s) {
  bool four = (g.n_phi & 3) == 0;
  for (int b = 0; b < NB; ++b) four = four && ((uintptr_t)PB.acc[b] & 15) == 0;
  const int tiles = (int)(four ? (n_cells + kTile4 - 1) / kTile4 : (n_cells + kTile - 1) / kTile);
  const int R = four && kTile4 % g.n_phi == 0 ? kTile4 / g.n_phi : 0;
  const dim3 grid(tiles, NB);
  if (R == 1)
    flag4s_kernel<1, NB><<<grid, 256, 0, s>>>(PB, g.n_qpt, g.n_d0, min_votes);
  else if (R == 2 && g.n_qpt % 2 == 0)
    flag4s_kernel<2, NB><<<grid, 256, 0, s>>>(PB, g.n_qpt, g.n_d0, min_votes);
  else if (R == 4 && g.n_qpt % 4 == 0)
    flag4s_kernel<4, NB><<<grid, 256, 0, s>>>(PB, g.n_qpt, g.n_d0, min_votes);
  else if (four)
    flag4_kernel<NB><<<grid, 256, 0, s>>>(PB, g.n_phi, g.n_qpt, g.n_d0, n_cells, min_votes);
  else
    flag_kernel<NB><<<grid, kTile, 0, s>>>(PB, g.n_phi, g.n_qpt, g.n_d0, n_cells, min_votes);
  HT_CHECK(hipGetLastError());
  const int rc = NB == 1 ? launch_scan(PB.cnt[0], PB.off[0], tiles, n_found[0], s)
                         : launch_scan_batch(NB, PB.cnt, PB.off, tiles, n_found, s);
  if (rc != HT_OK) return rc;
  if (capacity > 0) {
    if (four)
      emit4_kernel<NB><<<grid, 256, 0, s>>>(PB, n_cells, capacity);
    else
      emit_kernel<NB><<<grid, kTile, 0, s>>>(PB, n_cells, capacity);
    HT_CHECK(hipGetLastError());
  }
  return HT_OK;
}

int launch_peaks_core(const ht_grid& g, int64_t n_cells, const int32_t* acc, int32_t min_votes,
                      ht_peak* out, int32_t capacity, int32_t* n_found, void* bits_v,
                      int32_t* tile_cnt, int32_t* tile_off, hipStream_t s) {
  PeakBatch<1> PB;
  PB.acc[0] = acc;
  PB.bits[0] = bits_v;
  PB.cnt[0] = tile_cnt;
  PB.off[0] = tile_off;
  PB.out[0] = out;
  int32_t* nf[1] = {n_found};
  return peaks_batch_core<1>(g, n_cells, PB, min_votes, capacity, nf, s);
}

template <int NB>
int peaks_batch_nb(const Plan* const* plans, const int32_t* const* acc, int32_t min_votes,
                   ht_peak* const* out, int32_t capacity, int32_t* const* n_found, hipStream_t s) {
  PeakBatch<NB> PB;
  for (int b = 0; b < NB; ++b) {
    PB.acc[b] = acc[b];
    PB.bits[b] = plans[b]->d_bits;
    PB.cnt[b] = plans[b]->d_tile_cnt;
    PB.off[b] = plans[b]->d_tile_off;
    PB.out[b] = out[b];
  }
  const Plan& p0 = *plans[0];
  p0.prof_mark(HT_STAGE_PEAKS, 0, s);
  const int rc = peaks_batch_core<NB>(p0.grid, p0.n_cells, PB, min_votes, capacity, n_found, s);
  if (rc != HT_OK) return rc;
  p0.prof_mark(HT_STAGE_PEAKS, 1, s);
  return HT_OK;
}

int launch_peaks(const Plan& p, const int32_t* acc, int32_t min_votes, ht_peak* out,
                 int32_t capacity, int32_t* n_found, hipStream_t s) {
  p.prof_mark(HT_STAGE_PEAKS, 0, s);
  const int rc = launch_peaks_core(p.grid, p.n_cells, acc, min_votes, out, capacity, n_found,
                                   p.d_bits, p.d_tile_cnt, p.d_tile_off, s);
  if (rc != HT_OK) return rc;
  p.prof_mark(HT_STAGE_PEAKS, 1, s);
  return HT_OK;
}

int launch_peaks_batch(int nb, const Plan* const* plans, const int32_t* const* acc,
                       int32_t min_votes, ht_peak* const* out, int32_t capacity,
                       int32_t* const* n_found, hipStream_t s) {
  switch (nb) {
    case 1: return peaks_batch_nb<1>(plans, acc, min_votes, out, capacity, n_found, s);
    case 2: return peaks_batch_nb<2>(plans, acc, min_votes, out, capacity, n_found, s);
    case 3: return peaks_batch_nb<3>(plans, acc, min_votes, out, capacity, n_found, s);
    case 4: return peaks_batch_nb<4>(plans, acc, min_votes, out, capacity, n_found, s);
    default: return HT_EUNSUPPORTED;
  }
}

// Largest accumulator hough_peaks_noalloc takes, and its scratch: the ballot
// words (one bit per cell, tiles rounded up), the tile counts and the tile
// offsets (256-cell tiles at most).
constexpr int64_t kNoAllocMaxCells = (int64_t)1 << 24;
constexpr size_t kNoAllocBitsBytes = (size_t)(kNoAllocMaxCells / 8) + 256;
constexpr size_t kNoAllocTileBytes = (size_t)(kNoAllocMaxCells / 256) * 4;
constexpr size_t kNoAllocScratchBytes = kNoAllocBitsBytes + 2 * kNoAllocTileBytes;

}  // namespace ht

// ---- hough_peaks_noalloc: the same kernels on a fixed device array ------------
//
// The scratch lives in this array, one copy per GPU, held until the process
// ends.  In host code its name is only a host-side stand-in; the device
// address of the current GPU's copy comes from hipGetSymbolAddress, taken
// once per device on the first call there and kept.  Every call on a GPU
// uses that GPU's copy, so calls that overlap on one GPU (two streams) race.
// Nothing needs clearing between calls: the flag kernel writes every ballot
// word and tile count that the scan and emit kernels read, and the scan
// writes every offset.
static __device__ __align__(256) unsigned char scratch[ht::kNoAllocScratchBytes];

namespace ht {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

int scratch_address(void** out) {
  int dev = 0;
  HT_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return HT_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HT_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HT_OK;
}
}  // namespace

int64_t noalloc_max_cells() { return kNoAllocMaxCells; }

int launch_peaks_noalloc(const ht_grid& g, const int32_t* acc, int32_t min_votes, ht_peak* out,
                         int32_t capacity, int32_t* n_found, hipStream_t s) {
  const int64_t n_cells = (int64_t)g.n_phi * g.n_qpt * g.n_d0;
  if (n_cells > kNoAllocMaxCells) return HT_EUNSUPPORTED;
  void* base = nullptr;
  const int rc = scratch_address(&base);
  if (rc != HT_OK) return rc;
  unsigned char* b = static_cast<unsigned char*>(base);
  int32_t* cnt = reinterpret_cast<int32_t*>(b + kNoAllocBitsBytes);
  return launch_peaks_core(g, n_cells, acc, min_votes, out, capacity, n_found, b, cnt,
                           cnt + kNoAllocTileBytes / 4, s);
}

}  // namespace ht
