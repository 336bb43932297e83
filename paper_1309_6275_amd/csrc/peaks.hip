// Local maxima of the accumulator (paper, section "Hough Transform
// Algorithm"), written in cell order.
//
// Three launches, each a sweep over the cell range:
//   1. flag: one thread per cell evaluates the 26-neighbour rule, a wave's
//      flags become two bitmap words through one ballot, and each
//      256-cell tile writes its peak count;
//   2. scan: one workgroup turns tile counts into tile offsets and the
//      total count;
//   3. emit: one workgroup per tile reads its 8 bitmap words and writes its
//      peaks at offset + rank, the rank coming from ballot/popcount prefix
//      sums, so the list is sorted by cell index with no sort.
// Neighbour reads of pass 1 hit L2 (the accumulator rows of a tile are read
// by neighbouring tiles at the same time).
#include "ht_internal.h"

namespace ht {
namespace {

constexpr int kTile = 256;

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

__global__ __launch_bounds__(kTile) void flag_kernel(const int32_t* __restrict__ acc, int n_phi,
                                                     int n_qpt, int n_d0, int64_t n_cells,
                                                     int32_t thr, uint32_t* __restrict__ bits,
                                                     int32_t* __restrict__ tile_cnt) {
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

__global__ __launch_bounds__(kTile) void emit_kernel(const int32_t* __restrict__ acc,
                                                     const uint32_t* __restrict__ bits,
                                                     const int32_t* __restrict__ tile_off,
                                                     int64_t n_cells, ht_peak* __restrict__ out,
                                                     int32_t capacity) {
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

}  // namespace

int peaks_init(int) { return HT_OK; }

int launch_peaks(const Plan& p, const int32_t* acc, int32_t min_votes, ht_peak* out,
                 int32_t capacity, int32_t* n_found, hipStream_t s) {
  const ht_grid& g = p.grid;
  const int tiles = p.n_tiles;
  flag_kernel<<<tiles, kTile, 0, s>>>(acc, g.n_phi, g.n_qpt, g.n_d0, p.n_cells, min_votes,
                                      p.d_bits, p.d_tile_cnt);
  HT_CHECK(hipGetLastError());
  const int rc = launch_scan(p.d_tile_cnt, p.d_tile_off, tiles, n_found, s);
  if (rc != HT_OK) return rc;
  if (capacity > 0) {
    emit_kernel<<<tiles, kTile, 0, s>>>(acc, p.d_bits, p.d_tile_off, p.n_cells, out, capacity);
    HT_CHECK(hipGetLastError());
  }
  return HT_OK;
}

}  // namespace ht
