// Learned peak filter: a 3D CNN that scores each threshold peak from the
// 5 x 5 x 5 votes around it (the paper's call for efficiency and purity
// improvements of the peak finding, section "Summary").
//
// Precision contract (identical in the oracle): bfloat16 inputs, weights and
// activations, float32 accumulation; bias after the sum; ReLU; activations
// rounded to bfloat16 (round to nearest even) before the next layer.
//
// Inference (the per-event hot part) runs on the matrix cores: one wave
// scores 16 windows with v_mfma_f32_16x16x16_bf16 (A: 16 x 16 bf16 with row
// m = lane % 16 and k = 4 (lane / 16) + i in element i; B likewise with
// column n = lane % 16; D: row 4 (lane / 16) + i, column lane % 16):
//   conv1  27 output positions x 2 k-steps (27 taps padded to 32): M = the
//          16 windows, N = 16 channels;
//   conv2  27 k-steps (one per position, 16 input channels each);
//   fc1    4 n-tiles of 16 features; fc2 a dot product on the VALU.
// The weights are packed once per call into B-operand order (8 bytes per
// lane per k-step).  Training (offline, milliseconds per step) runs the same
// forward, keeps the activations, and computes the gradients on the VALU with
// float32 sums in LDS, then one atomic add per parameter and workgroup.
#include "ht_internal.h"

namespace ht {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWin = HT_CNN_WINDOW;  // bf16 per window (125 used)

__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// parameter offsets in the flat float32 vector
constexpr int oW1 = 0, ob1 = oW1 + 16 * 27, oW2 = ob1 + 16, ob2 = oW2 + 16 * 16 * 27,
              oW3 = ob2 + 16, ob3 = oW3 + 64 * 16, oW4 = ob3 + 64, ob4 = oW4 + 64;
static_assert(ob4 + 1 == HT_CNN_PARAMS, "parameter layout");

struct alignas(16) Packed {
  uint16_t w1[2 * 64 * 4];    // conv1 B operand per k-step and lane
  uint16_t w2[27 * 64 * 4];   // conv2 B operand per position and lane
  uint16_t w3[4 * 64 * 4];    // fc1 B operand per n-tile and lane
  float b1[16], b2[16], b3[64], w4[64], b4[4];
};

// input cell of output position p and tap t (t >= 27: padding, -1)
__device__ __forceinline__ int tap_cell(int p, int t) {
  if (t >= 27) return -1;
  const int a = p / 9, b = (p / 3) % 3, c = p % 3;
  const int dk = t / 9, dj = (t / 3) % 3, di = t % 3;
  return (a + dk) * 25 + (b + dj) * 5 + (c + di);
}

__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ P, Packed* __restrict__ W) {
  for (int e = threadIdx.x; e < 2 * 64 * 4; e += blockDim.x) {
    const int s = e / 256, l = (e / 4) % 64, i = e % 4;
    const int t = 16 * s + 4 * (l / 16) + i, c = l % 16;
    W->w1[e] = t < 27 ? to_bf16(P[oW1 + c * 27 + t]) : (uint16_t)0;
  }
  for (int e = threadIdx.x; e < 27 * 64 * 4; e += blockDim.x) {
    const int p = e / 256, l = (e / 4) % 64, i = e % 4;
    const int cin = 4 * (l / 16) + i, c = l % 16;
    W->w2[e] = to_bf16(P[oW2 + (c * 16 + cin) * 27 + p]);
  }
  for (int e = threadIdx.x; e < 4 * 64 * 4; e += blockDim.x) {
    const int nt = e / 256, l = (e / 4) % 64, i = e % 4;
    const int c = 4 * (l / 16) + i, f = 16 * nt + l % 16;
    W->w3[e] = to_bf16(P[oW3 + f * 16 + c]);
  }
  const int t = threadIdx.x;
  if (t < 16) { W->b1[t] = P[ob1 + t]; W->b2[t] = P[ob2 + t]; }
  if (t < 64) { W->b3[t] = P[ob3 + t]; W->w4[t] = from_bf16(to_bf16(P[oW4 + t])); }
  if (t == 0) W->b4[0] = P[ob4];
}

// windows around peaks: votes * 1/16 as bfloat16, phi0 periodic, q/pT and d0
// outside the grid read 0; entries 125..127 are 0
__global__ __launch_bounds__(256) void windows_kernel(const int32_t* __restrict__ acc, int n_phi,
                                                      int n_qpt, int n_d0,
                                                      const ht_peak* __restrict__ peaks,
                                                      const int32_t* __restrict__ n_peaks, int cap,
                                                      uint16_t* __restrict__ win) {
  const int np = min(max(*n_peaks, 0), cap);
  const int64_t n_cells = (int64_t)n_phi * n_qpt * n_d0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)np * kWin;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int w = (int)(e / kWin), c = (int)(e % kWin);
    float v = 0.0f;
    const int lin = peaks[w].lin;
    if (c < 125 && lin >= 0 && lin < n_cells) {
      const int i = lin % n_phi, col = lin / n_phi, j = col % n_qpt, k = col / n_qpt;
      const int kk = k + c / 25 - 2, jj = j + (c / 5) % 5 - 2;
      int ii = i + c % 5 - 2;
      ii = ii < 0 ? ii + n_phi : (ii >= n_phi ? ii - n_phi : ii);
      if (kk >= 0 && kk < n_d0 && jj >= 0 && jj < n_qpt)
        v = (float)acc[((size_t)kk * n_qpt + jj) * n_phi + ii] * 0.0625f;
    }
    win[e] = to_bf16(v);
  }
}

constexpr int kFwdWaves = 4;

// Forward of 16 windows per wave.  ACT keeps the activations for training.
template <bool ACT>
__global__ __launch_bounds__(kFwdWaves * 64) void forward_kernel(
    const Packed* __restrict__ W, const uint16_t* __restrict__ win, const int32_t* __restrict__ n_dev,
    int n_max, float* __restrict__ logits, uint16_t* __restrict__ h1o, uint16_t* __restrict__ h2o,
    uint16_t* __restrict__ h3o) {
  __shared__ uint16_t xs[kFwdWaves][16][kWin];
  __shared__ uint16_t h1s[kFwdWaves][16][27][16];
  __shared__ uint16_t h2s[kFwdWaves][16][16];
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int n = n_dev ? min(max(*n_dev, 0), n_max) : n_max;
  const int tiles = (n + 15) / 16;
  for (int tile = blockIdx.x * kFwdWaves + wave; tile < tiles; tile += gridDim.x * kFwdWaves) {
    const int w0 = tile * 16;
    // 16 windows x 256 bytes, 16-byte chunks
    for (int ch = l; ch < 16 * 16; ch += 64) {
      const int w = ch / 16, o = (ch % 16) * 8;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (w0 + w < n) v = *reinterpret_cast<const uint4*>(win + (size_t)(w0 + w) * kWin + o);
      *reinterpret_cast<uint4*>(&xs[wave][w][o]) = v;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const int row = l % 16, kq = 4 * (l / 16);
    // conv1
    for (int p = 0; p < 27; ++p) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        bf16x4 a;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int cell = tap_cell(p, 16 * s + kq + i);
          a[i] = cell >= 0 ? (short)xs[wave][row][cell] : (short)0;
        }
        const bf16x4 b = *reinterpret_cast<const bf16x4*>(&W->w1[(s * 64 + l) * 4]);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
      }
      const int c = l % 16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float h = fmaxf(acc[i] + W->b1[c], 0.0f);
        h1s[wave][kq + i][p][c] = to_bf16(h);
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // conv2
    f32x4 acc2 = {0.f, 0.f, 0.f, 0.f};
    for (int p = 0; p < 27; ++p) {
      const bf16x4 a = *reinterpret_cast<const bf16x4*>(&h1s[wave][row][p][kq]);
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(&W->w2[(p * 64 + l) * 4]);
      acc2 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc2, 0, 0, 0);
    }
    {
      const int c = l % 16;
#pragma unroll
      for (int i = 0; i < 4; ++i) h2s[wave][kq + i][c] = to_bf16(fmaxf(acc2[i] + W->b2[c], 0.0f));
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // fc1 and fc2
    const bf16x4 a3 = *reinterpret_cast<const bf16x4*>(&h2s[wave][row][kq]);
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(&W->w3[(nt * 64 + l) * 4]);
      f32x4 z = {0.f, 0.f, 0.f, 0.f};
      z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a3, b, z, 0, 0, 0);
      const int f = 16 * nt + l % 16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint16_t hb = to_bf16(fmaxf(z[i] + W->b3[f], 0.0f));
        part[i] += W->w4[f] * from_bf16(hb);
        if (ACT && w0 + kq + i < n) h3o[(size_t)(w0 + kq + i) * 64 + f] = hb;
      }
    }
    // sum over the 16 lanes of a row (the 64 features of one window)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v = part[i];
      for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
      if (l % 16 == 0 && w0 + kq + i < n) logits[w0 + kq + i] = v + W->b4[0];
    }
    if (ACT) {
      for (int e = l; e < 16 * 27 * 16; e += 64) {
        const int w = e / 432;
        if (w0 + w < n) h1o[(size_t)(w0 + w) * 432 + e % 432] = (&h1s[wave][0][0][0])[e];
      }
      for (int e = l; e < 16 * 16; e += 64) {
        const int w = e / 16;
        if (w0 + w < n) h2o[(size_t)(w0 + w) * 16 + e % 16] = (&h2s[wave][0][0])[e];
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

// Backward of 64 windows per workgroup (one wave): dz, dh3, dh2, dh1 per
// window in LDS, then every parameter's gradient summed over the 64 windows
// by one lane and added to the global gradient.
constexpr int kBwdWin = 8;

__global__ __launch_bounds__(64) void backward_kernel(
    const float* __restrict__ P, const uint16_t* __restrict__ win, const float* __restrict__ labels,
    int n, float pos_weight, const float* __restrict__ logits, const uint16_t* __restrict__ h1g,
    const uint16_t* __restrict__ h2g, const uint16_t* __restrict__ h3g, float* __restrict__ grad,
    float* __restrict__ loss) {
  __shared__ float dzs[kBwdWin];
  __shared__ float dh3s[kBwdWin][64];
  __shared__ float dh2s[kBwdWin][16];
  __shared__ float dh1s[kBwdWin][27][16];
  __shared__ float h3s[kBwdWin][64];
  __shared__ float h2s[kBwdWin][16];
  __shared__ float h1s[kBwdWin][27][16];
  __shared__ float xs[kBwdWin][125];
  const int l = threadIdx.x;
  const int w0 = blockIdx.x * kBwdWin;
  const int nw = min(kBwdWin, n - w0);
  if (nw <= 0) return;
  // stage activations and inputs as float
  for (int e = l; e < nw * 125; e += 64) xs[e / 125][e % 125] = from_bf16(win[(size_t)(w0 + e / 125) * kWin + e % 125]);
  for (int e = l; e < nw * 432; e += 64) (&h1s[0][0][0])[e] = from_bf16(h1g[(size_t)w0 * 432 + e]);
  for (int e = l; e < nw * 16; e += 64) (&h2s[0][0])[e] = from_bf16(h2g[(size_t)w0 * 16 + e]);
  for (int e = l; e < nw * 64; e += 64) (&h3s[0][0])[e] = from_bf16(h3g[(size_t)w0 * 64 + e]);
  __syncthreads();
  float lsum = 0.0f;
  if (l < nw) {
    const float z = logits[w0 + l], y = labels[w0 + l];
    const float wgt = y > 0.5f ? pos_weight : 1.0f;
    const float sp = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
    lsum = wgt * (sp - y * z) / (float)n;
    dzs[l] = wgt * (1.0f / (1.0f + expf(-z)) - y) / (float)n;
  }
  __syncthreads();
  // dh3 = dz W4 [h3 > 0]
  for (int e = l; e < nw * 64; e += 64) {
    const int w = e / 64, f = e % 64;
    dh3s[w][f] = h3s[w][f] > 0.0f ? dzs[w] * from_bf16(to_bf16(P[oW4 + f])) : 0.0f;
  }
  __syncthreads();
  // dh2 = dh3 W3 [h2 > 0]
  for (int e = l; e < nw * 16; e += 64) {
    const int w = e / 16, c = e % 16;
    float s = 0.0f;
    for (int f = 0; f < 64; ++f) s += dh3s[w][f] * from_bf16(to_bf16(P[oW3 + f * 16 + c]));
    dh2s[w][c] = h2s[w][c] > 0.0f ? s : 0.0f;
  }
  __syncthreads();
  // dh1[p][c'] = sum_c dh2[c] W2[c][c'][p] [h1 > 0]
  for (int e = l; e < nw * 432; e += 64) {
    const int w = e / 432, p = (e % 432) / 16, ci = e % 16;
    float s = 0.0f;
    for (int c = 0; c < 16; ++c) s += dh2s[w][c] * from_bf16(to_bf16(P[oW2 + (c * 16 + ci) * 27 + p]));
    dh1s[w][p][ci] = h1s[w][p][ci] > 0.0f ? s : 0.0f;
  }
  __syncthreads();
  // parameter gradients
  for (int q = l; q < HT_CNN_PARAMS; q += 64) {
    float s = 0.0f;
    if (q < ob1) {                       // W1[c][t]
      const int c = q / 27, t = q % 27;
      for (int w = 0; w < nw; ++w)
        for (int p = 0; p < 27; ++p) s += dh1s[w][p][c] * xs[w][tap_cell(p, t)];
    } else if (q < oW2) {                // b1
      const int c = q - ob1;
      for (int w = 0; w < nw; ++w)
        for (int p = 0; p < 27; ++p) s += dh1s[w][p][c];
    } else if (q < ob2) {                // W2[c][c'][p]
      const int r = q - oW2, c = r / 432, ci = (r / 27) % 16, p = r % 27;
      for (int w = 0; w < nw; ++w) s += dh2s[w][c] * h1s[w][p][ci];
    } else if (q < oW3) {                // b2
      const int c = q - ob2;
      for (int w = 0; w < nw; ++w) s += dh2s[w][c];
    } else if (q < ob3) {                // W3[f][c]
      const int r = q - oW3, f = r / 16, c = r % 16;
      for (int w = 0; w < nw; ++w) s += dh3s[w][f] * h2s[w][c];
    } else if (q < oW4) {                // b3
      const int f = q - ob3;
      for (int w = 0; w < nw; ++w) s += dh3s[w][f];
    } else if (q < ob4) {                // W4
      const int f = q - oW4;
      for (int w = 0; w < nw; ++w) s += dzs[w] * h3s[w][f];
    } else {                             // b4
      for (int w = 0; w < nw; ++w) s += dzs[w];
    }
    atomicAdd(&grad[q], s);
  }
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
  if (l == 0) atomicAdd(loss, lsum);
}

__global__ void zero_f32_kernel(float* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0f;
}

__global__ void sgd_kernel(float* __restrict__ P, float* __restrict__ mom, float* __restrict__ grad,
                           float lr, float momentum) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < HT_CNN_PARAMS) {
    const float m = momentum * mom[q] + grad[q];
    mom[q] = m;
    P[q] = P[q] - lr * m;
    grad[q] = 0.0f;
  }
}

// ordered compaction of the peaks whose logit reaches the threshold
__global__ __launch_bounds__(256) void keep_count_kernel(const float* __restrict__ logits,
                                                         const int32_t* __restrict__ n_peaks, int cap,
                                                         float thr, int32_t* __restrict__ tile_cnt) {
  __shared__ int32_t wc[4];
  const int np = min(max(*n_peaks, 0), cap);
  const int p = blockIdx.x * 256 + threadIdx.x;
  const uint64_t m = __ballot(p < np && logits[p] >= thr);
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) tile_cnt[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

__global__ __launch_bounds__(256) void keep_emit_kernel(const float* __restrict__ logits,
                                                        const ht_peak* __restrict__ peaks,
                                                        const int32_t* __restrict__ n_peaks, int cap,
                                                        float thr, const int32_t* __restrict__ tile_off,
                                                        ht_peak* __restrict__ out, int out_cap) {
  __shared__ int32_t wc[4];
  const int np = min(max(*n_peaks, 0), cap);
  const int p = blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool k = p < np && logits[p] >= thr;
  const uint64_t m = __ballot(k);
  if (lane == 0) wc[wave] = __popcll(m);
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += wc[w];
  if (k) {
    const uint64_t lower = lane ? (m & ((1ull << lane) - 1ull)) : 0ull;
    const int idx = tile_off[blockIdx.x] + before + __popcll(lower);
    if (idx < out_cap) out[idx] = peaks[p];
  }
}

int blocks(int64_t n, int per, int cap = 8192) {
  int64_t b = (n + per - 1) / per;
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

size_t cnn_workspace_bytes(int32_t max_windows, int training) {
  size_t b = (sizeof(Packed) + 255) / 256 * 256;
  if (training) {
    const size_t n = (size_t)(max_windows > 0 ? max_windows : 1);
    b += (n * 4 + 255) / 256 * 256;                 // logits
    b += (n * 432 * 2 + 255) / 256 * 256;           // h1
    b += (n * 16 * 2 + 255) / 256 * 256;           // h2
    b += (n * 64 * 2 + 255) / 256 * 256;           // h3
    b += ((size_t)HT_CNN_PARAMS * 4 + 255) / 256 * 256;  // gradient
  }
  return b;
}

int launch_cnn_windows(const Plan& p, const int32_t* acc, const ht_peak* peaks, const int32_t* n_peaks,
                       int32_t cap, uint16_t* win, hipStream_t s) {
  const ht_grid& g = p.grid;
  windows_kernel<<<blocks((int64_t)cap * kWin, 256), 256, 0, s>>>(acc, g.n_phi, g.n_qpt, g.n_d0,
                                                                  peaks, n_peaks, cap, win);
  HT_CHECK(hipGetLastError());
  return HT_OK;
}

int launch_cnn_forward(const float* params, const uint16_t* win, const int32_t* n_dev, int32_t n_max,
                       float* logits, void* ws, hipStream_t s) {
  Packed* W = reinterpret_cast<Packed*>(ws);
  pack_kernel<<<1, 256, 0, s>>>(params, W);
  HT_CHECK(hipGetLastError());
  const int tiles = (n_max + 15) / 16;
  forward_kernel<false><<<blocks(tiles, kFwdWaves, 4096), kFwdWaves * 64, 0, s>>>(
      W, win, n_dev, n_max, logits, nullptr, nullptr, nullptr);
  HT_CHECK(hipGetLastError());
  return HT_OK;
}

int launch_cnn_train(float* params, float* mom, const uint16_t* win, const float* labels, int32_t n,
                     float lr, float momentum, float pos_weight, float* loss, void* ws, hipStream_t s) {
  char* base = reinterpret_cast<char*>(ws);
  Packed* W = reinterpret_cast<Packed*>(base);
  size_t o = (sizeof(Packed) + 255) / 256 * 256;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  float* logits = reinterpret_cast<float*>(base + o);
  o += (nn * 4 + 255) / 256 * 256;
  uint16_t* h1 = reinterpret_cast<uint16_t*>(base + o);
  o += (nn * 432 * 2 + 255) / 256 * 256;
  uint16_t* h2 = reinterpret_cast<uint16_t*>(base + o);
  o += (nn * 16 * 2 + 255) / 256 * 256;
  uint16_t* h3 = reinterpret_cast<uint16_t*>(base + o);
  o += (nn * 64 * 2 + 255) / 256 * 256;
  float* grad = reinterpret_cast<float*>(base + o);
  zero_f32_kernel<<<34, 256, 0, s>>>(grad, HT_CNN_PARAMS);
  zero_f32_kernel<<<1, 64, 0, s>>>(loss, 1);
  pack_kernel<<<1, 256, 0, s>>>(params, W);
  HT_CHECK(hipGetLastError());
  const int tiles = (n + 15) / 16;
  forward_kernel<true><<<blocks(tiles, kFwdWaves, 4096), kFwdWaves * 64, 0, s>>>(
      W, win, nullptr, n, logits, h1, h2, h3);
  HT_CHECK(hipGetLastError());
  backward_kernel<<<(n + kBwdWin - 1) / kBwdWin, 64, 0, s>>>(params, win, labels, n, pos_weight,
                                                             logits, h1, h2, h3, grad, loss);
  HT_CHECK(hipGetLastError());
  sgd_kernel<<<(HT_CNN_PARAMS + 255) / 256, 256, 0, s>>>(params, mom, grad, lr, momentum);
  HT_CHECK(hipGetLastError());
  return HT_OK;
}

int launch_cnn_keep(const Plan& p, const float* logits, const ht_peak* peaks, const int32_t* n_peaks,
                    int32_t cap, float thr, ht_peak* out, int32_t out_cap, int32_t* n_out,
                    hipStream_t s) {
  const int tiles = (cap + 255) / 256 > 0 ? (cap + 255) / 256 : 1;
  keep_count_kernel<<<tiles, 256, 0, s>>>(logits, n_peaks, cap, thr, p.d_ctile_cnt);
  HT_CHECK(hipGetLastError());
  const int rc = launch_scan(p.d_ctile_cnt, p.d_ctile_off, tiles, n_out, s);
  if (rc != HT_OK) return rc;
  keep_emit_kernel<<<tiles, 256, 0, s>>>(logits, peaks, n_peaks, cap, thr, p.d_ctile_off, out,
                                         out_cap);
  HT_CHECK(hipGetLastError());
  return HT_OK;
}

}  // namespace ht
