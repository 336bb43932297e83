// Exclusive prefix sum of int32 counts (tile counts -> tile offsets) in one
// workgroup of 1024 threads.  Thread t owns the contiguous run
// [t * per, (t + 1) * per) of the n counts: it sums its run, the workgroup
// scans the 1024 run sums (one wave scan and 16 wave totals), and the thread
// walks its run again writing offsets.  Each thread's loads stay in its own
// cache lines, and the only cross-lane steps are one scan per wave, not one
// per 64 counts.  Offsets and the total are clamped to INT32_MAX.
#include "ht_internal.h"

namespace ht {
namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanWaves = kScanThreads / kWave;

__device__ __forceinline__ long long wave_incl_scan(long long v, int lane) {
  for (int d = 1; d < kWave; d <<= 1) {
    const long long o = __shfl_up(v, d);
    if (lane >= d) v += o;
  }
  return v;
}

__device__ __forceinline__ int32_t clamp_i32(long long v) {
  return v > 0x7fffffffLL ? 0x7fffffff : (int32_t)v;
}

// pointers of up to kScanBatch scans run by one launch (one workgroup each)
constexpr int kScanBatch = 4;
struct ScanBatch {
  const int32_t* cnt[kScanBatch];
  int32_t* off[kScanBatch];
  int32_t* total[kScanBatch];
};

__device__ void scan_one(const int32_t* __restrict__ cnt, int32_t* __restrict__ off, int n,
                         int32_t* __restrict__ total);

__global__ __launch_bounds__(kScanThreads) void scan_kernel(const int32_t* __restrict__ cnt,
                                                            int32_t* __restrict__ off, int n,
                                                            int32_t* __restrict__ total) {
  scan_one(cnt, off, n, total);
}

__global__ __launch_bounds__(kScanThreads) void scan_batch_kernel(ScanBatch B, int n) {
  scan_one(B.cnt[blockIdx.x], B.off[blockIdx.x], n, B.total[blockIdx.x]);
}

__device__ void scan_one(const int32_t* __restrict__ cnt, int32_t* __restrict__ off, int n,
                         int32_t* __restrict__ total) {
  __shared__ long long wsum[kScanWaves];
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1);
  const int wave = t >> 6;
  const int per = (n + kScanThreads - 1) / kScanThreads;
  const int b = (int)min((long long)n, (long long)t * per);
  const int e = min(n, b + per);
  // whole 16-byte vectors per thread when the runs and the arrays allow
  const bool vec = (per & 3) == 0 && (n & 3) == 0 && ((uintptr_t)cnt & 15) == 0 &&
                   ((uintptr_t)off & 15) == 0;
  long long s = 0;
  if (vec) {
    for (int x = b; x < e; x += 4) {
      const int4 c = *reinterpret_cast<const int4*>(cnt + x);
      s += (long long)c.x + c.y + c.z + c.w;
    }
  } else {
    for (int x = b; x < e; ++x) s += cnt[x];
  }
  const long long incl = wave_incl_scan(s, lane);
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  long long base = 0;
  for (int w = 0; w < wave; ++w) base += wsum[w];
  long long run = base + incl - s;
  if (vec) {
    for (int x = b; x < e; x += 4) {
      const int4 c = *reinterpret_cast<const int4*>(cnt + x);
      int4 o;
      o.x = clamp_i32(run);
      run += c.x;
      o.y = clamp_i32(run);
      run += c.y;
      o.z = clamp_i32(run);
      run += c.z;
      o.w = clamp_i32(run);
      run += c.w;
      *reinterpret_cast<int4*>(off + x) = o;
    }
  } else {
    for (int x = b; x < e; ++x) {
      off[x] = clamp_i32(run);
      run += cnt[x];
    }
  }
  if (t == kScanThreads - 1 && total) *total = clamp_i32(base + incl);
}

}  // namespace

int launch_scan(const int32_t* cnt, int32_t* off, int n, int32_t* total, hipStream_t s) {
  scan_kernel<<<1, kScanThreads, 0, s>>>(cnt, off, n, total);
  HT_CHECK(hipGetLastError());
  return HT_OK;
}

int launch_scan_batch(int nb, const int32_t* const* cnt, int32_t* const* off, int n,
                      int32_t* const* total, hipStream_t s) {
  if (nb < 1 || nb > kScanBatch) return HT_EUNSUPPORTED;
  ScanBatch B = {};
  for (int b = 0; b < nb; ++b) {
    B.cnt[b] = cnt[b];
    B.off[b] = off[b];
    B.total[b] = total[b];
  }
  scan_batch_kernel<<<nb, kScanThreads, 0, s>>>(B, n);
  HT_CHECK(hipGetLastError());
  return HT_OK;
}

}  // namespace ht
