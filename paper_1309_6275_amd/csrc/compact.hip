// Iterative hit removal: keeping the hits that no track of an earlier pass
// owns, and mapping the hit indices of a later pass back to the event.
// The paper's tracker (section "Current Tracker and Tracking Algorithm")
// finds the easy, prompt tracks first and removes their hits, so that later
// passes search for displaced tracks among far fewer combinations.
//
// Events hold at most 65535 hits, so one 1024-thread workgroup compacts a
// whole event: thread t takes a run of ceil(n / 1024) consecutive hits,
// counts its kept hits, a wave scan plus a scan over the 16 wave totals
// gives each run its output offset, and the run is written in order.  The
// kernel reads under 1 MB; its cost is launch latency.
#include "ht_internal.h"

namespace ht {
namespace {

constexpr int kCompactThreads = 1024;

__global__ __launch_bounds__(kCompactThreads) void compact_kernel(
    const float* __restrict__ r, const float* __restrict__ phi,
    const uint8_t* __restrict__ layer, const int32_t* __restrict__ owner, int32_t n,
    float* __restrict__ out_r, float* __restrict__ out_phi, uint8_t* __restrict__ out_layer,
    int32_t* __restrict__ out_index, int32_t* __restrict__ n_out) {
  __shared__ int32_t wsum[kCompactThreads / kWave];
  const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
  const int run = (n + kCompactThreads - 1) / kCompactThreads;
  const int b = min(t * run, n), e = min(b + run, n);
  int c = 0;
  for (int h = b; h < e; ++h) c += owner[h] < 0 ? 1 : 0;
  int x = c;  // inclusive scan over the wave
  for (int d = 1; d < kWave; d <<= 1) {
    const int y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) wsum[w] = x;
  __syncthreads();
  int base = 0;
  for (int k = 0; k < w; ++k) base += wsum[k];
  int o = base + x - c;
  for (int h = b; h < e; ++h) {
    if (owner[h] >= 0) continue;
    out_r[o] = r[h];
    out_phi[o] = phi[h];
    out_layer[o] = layer[h];
    out_index[o] = h;
    ++o;
  }
  if (t == kCompactThreads - 1) n_out[0] = base + x;
}

__global__ __launch_bounds__(256) void remap_kernel(ht_track* __restrict__ tracks,
                                                    int32_t track_cap,
                                                    const int32_t* __restrict__ counts,
                                                    const int32_t* __restrict__ index,
                                                    int32_t n_index) {
  const int n = min(counts[1], track_cap);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n * HT_MAX_LAYERS) return;
  int32_t* hits = tracks[i / HT_MAX_LAYERS].hits;
  const int h = hits[i % HT_MAX_LAYERS];
  if (h >= 0 && h < n_index) hits[i % HT_MAX_LAYERS] = index[h];
}

}  // namespace

int launch_compact(const float* r, const float* phi, const uint8_t* layer, const int32_t* owner,
                   int32_t n, float* out_r, float* out_phi, uint8_t* out_layer,
                   int32_t* out_index, int32_t* n_out, hipStream_t s) {
  compact_kernel<<<1, kCompactThreads, 0, s>>>(r, phi, layer, owner, n, out_r, out_phi,
                                               out_layer, out_index, n_out);
  HT_CHECK(hipGetLastError());
  return HT_OK;
}

int launch_remap(ht_track* tracks, int32_t track_cap, const int32_t* counts,
                 const int32_t* index, int32_t n_index, hipStream_t s) {
  const int64_t work = (int64_t)track_cap * HT_MAX_LAYERS;
  const int blocks = (int)((work + 255) / 256);
  remap_kernel<<<blocks, 256, 0, s>>>(tracks, track_cap, counts, index, n_index);
  HT_CHECK(hipGetLastError());
  return HT_OK;
}

}  // namespace ht
