// Exclusive prefix sum of int32 counts (tile counts -> tile offsets), one
// workgroup of 16 waves: each wave owns a contiguous chunk read 64 elements
// at a time (coalesced); pass 1 sums the chunks, pass 2 scans each chunk
// from its wave's offset with shuffle prefix sums.  Offsets and the total
// are clamped to INT32_MAX.
#include "ht_internal.h"

namespace ht {
namespace {

constexpr int kScanWaves = 16;

__device__ __forceinline__ long long wave_incl_scan(long long v, int lane) {
  for (int d = 1; d < kWave; d <<= 1) {
    const long long o = __shfl_up(v, d);
    if (lane >= d) v += o;
  }
  return v;
}

__global__ __launch_bounds__(kScanWaves* kWave) void scan_kernel(const int32_t* __restrict__ cnt,
                                                                 int32_t* __restrict__ off, int n,
                                                                 int32_t* __restrict__ total) {
  __shared__ long long wsum[kScanWaves];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6;
  const int chunk = ((n + kScanWaves - 1) / kScanWaves + kWave - 1) / kWave * kWave;
  const int b = wave * chunk;
  const int e = min(n, b + chunk);
  long long s = 0;
  for (int x = b + lane; x < e; x += kWave) s += cnt[x];
  for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d);
  if (lane == 0) wsum[wave] = s;
  __syncthreads();
  long long run = 0;
  for (int w = 0; w < wave; ++w) run += wsum[w];
  for (int base = b; base < e; base += kWave) {
    const int x = base + lane;
    const long long v = x < e ? cnt[x] : 0;
    const long long incl = wave_incl_scan(v, lane);
    const long long ex = run + incl - v;
    if (x < e) off[x] = ex > 0x7fffffffLL ? 0x7fffffff : (int32_t)ex;
    run += __shfl(incl, kWave - 1);
  }
  if (threadIdx.x == 0 && total) {
    long long t = 0;
    for (int w = 0; w < kScanWaves; ++w) t += wsum[w];
    *total = t > 0x7fffffffLL ? 0x7fffffff : (int32_t)t;
  }
}

}  // namespace

int launch_scan(const int32_t* cnt, int32_t* off, int n, int32_t* total, hipStream_t s) {
  scan_kernel<<<1, kScanWaves * kWave, 0, s>>>(cnt, off, n, total);
  HT_CHECK(hipGetLastError());
  return HT_OK;
}

}  // namespace ht
