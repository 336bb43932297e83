// Learned peak filter: a 3D CNN that scores each threshold peak from the
// 5 x 5 x 5 votes around it (the paper's call for efficiency and purity
// improvements of the peak finding, section "Summary").
//
// Precision contract (identical in the oracle): bfloat16 inputs, weights and
// activations, float32 accumulation; bias after the sum; ReLU; activations
// rounded to bfloat16 (round to nearest even) before the next layer.
//
// Inference runs on the matrix cores with gfx950's v_mfma_f32_16x16x32_bf16
// (A: 16 x 32 bf16 with row m = lane % 16 and k = 8 (lane / 16) + i in
// element i; B likewise with column n = lane % 16; D: row 4 (lane / 16) + i,
// column lane % 16; checked on the device against a host product).  One
// wave scores 16 windows:
//   conv1  one k-step per output position (27 taps padded to 32): M = the 16
//          windows, N = 16 channels; the A operand gathers the window's
//          cells at per-lane tap offsets;
//   conv2  14 k-steps of two positions x 16 input channels each, each step
//          right after the conv1 of its two positions (their activations
//          pass through a 1 KB LDS buffer, not a 27-position one);
//   fc1    4 n-tiles of 16 features with the K = 16 instruction; fc2 a dot
//          product on the VALU.
// The packed weights (B-operand order) are copied into LDS once per
// workgroup.  ht_cnn_score builds each wave's 16 windows in LDS straight
// from the accumulator (no window buffer in HBM).  Training (offline) runs
// the same forward, keeps the activations, and computes the gradients with
// the matrix cores as well (see backward_kernel).
#include "ht_internal.h"

namespace ht {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) {
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

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

constexpr int kC2Steps = 14;  // conv2 k-steps: two positions x 16 channels (position 27 zero)

struct alignas(16) Packed {
  uint16_t w1[64 * 8];             // conv1 B operand per lane (K = 32: taps, padded)
  uint16_t w2[kC2Steps * 64 * 8];  // conv2 B operand per k-step and lane (K = 32)
  uint16_t w3[4 * 64 * 4];         // fc1 B operand per n-tile and lane (K = 16)
  float b1[16], b2[16], b3[64], w4[64], b4[4];
};
static_assert(sizeof(Packed) % 16 == 0, "packed weights are copied in 16-byte chunks");

__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ P, Packed* __restrict__ W) {
  for (int e = threadIdx.x; e < 64 * 8; e += blockDim.x) {
    const int l = e / 8, i = e % 8;
    const int t = 8 * (l / 16) + i, c = l % 16;
    W->w1[e] = t < 27 ? to_bf16(P[oW1 + c * 27 + t]) : (uint16_t)0;
  }
  for (int e = threadIdx.x; e < kC2Steps * 64 * 8; e += blockDim.x) {
    const int st = e / 512, l = (e / 8) % 64, i = e % 8;
    const int k = 8 * (l / 16) + i;
    const int p = 2 * st + k / 16, cin = k % 16, c = l % 16;
    W->w2[e] = p < 27 ? to_bf16(P[oW2 + (c * 16 + cin) * 27 + p]) : (uint16_t)0;
  }
  for (int e = threadIdx.x; e < 4 * 64 * 4; e += blockDim.x) {
    const int nt = e / 256, l = (e / 4) % 64, i = e % 4;
    const int c = 4 * (l / 16) + i, f = 16 * nt + l % 16;
    W->w3[e] = to_bf16(P[oW3 + f * 16 + c]);
  }
  const int t = threadIdx.x;
  if (t < 16) { W->b1[t] = P[ob1 + t]; W->b2[t] = P[ob2 + t]; }
  if (t < 64) { W->b3[t] = P[ob3 + t]; W->w4[t] = from_bf16(to_bf16(P[oW4 + t])); }
  if (t < 4) W->b4[t] = t == 0 ? P[ob4] : 0.0f;
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
// LDS row stride of a window (bf16): 130 = 65 dwords, odd, so the 16 rows a
// conv1 gather reads at one column fall in different banks
constexpr int kXs = 130;

// One window into LDS: votes * 1/16 as bfloat16 around a peak cell, phi0
// periodic, q/pT and d0 outside the grid 0, entries 125..127 0.  The wave
// fills 16 windows, a lane per (window, dk, dj) row of 5 cells at a time.
__device__ __forceinline__ void build_windows(const int32_t* __restrict__ acc, int n_phi, int n_qpt,
                                              int n_d0, const ht_peak* __restrict__ peaks, int w0,
                                              int n, int l, uint16_t (*xs)[kXs]) {
  const int64_t n_cells = (int64_t)n_phi * n_qpt * n_d0;
  for (int e = l; e < 16 * 25; e += 64) {
    const int w = e / 25, r = e % 25;
    const int dk = r / 5 - 2, dj = r % 5 - 2;
    uint16_t v[5] = {0, 0, 0, 0, 0};
    const int lin = w0 + w < n ? peaks[w0 + w].lin : -1;
    if (lin >= 0 && lin < n_cells) {
      const int i = lin % n_phi, col = lin / n_phi, j = col % n_qpt, k = col / n_qpt;
      const int kk = k + dk, jj = j + dj;
      if (kk >= 0 && kk < n_d0 && jj >= 0 && jj < n_qpt) {
        const int32_t* row = acc + ((size_t)kk * n_qpt + jj) * n_phi;
#pragma unroll
        for (int d = 0; d < 5; ++d) {
          int ii = i + d - 2;
          ii = ii < 0 ? ii + n_phi : (ii >= n_phi ? ii - n_phi : ii);
          v[d] = to_bf16((float)row[ii] * 0.0625f);
        }
      }
    }
#pragma unroll
    for (int d = 0; d < 5; ++d) xs[w][r * 5 + d] = v[d];
  }
  if (l < 16 * 3) xs[l / 3][125 + l % 3] = 0;
}

// Forward of 16 windows per wave.  FUSED: the windows come from the
// accumulator and peak list (ht_cnn_score), else from a window buffer.
// ACT keeps the activations for training.
template <bool FUSED, bool ACT>
__global__ __launch_bounds__(kFwdWaves * 64) void forward_kernel(
    const Packed* __restrict__ Wg, const uint16_t* __restrict__ win,
    const int32_t* __restrict__ acc, int n_phi, int n_qpt, int n_d0,
    const ht_peak* __restrict__ peaks, const int32_t* __restrict__ n_dev, int n_max,
    float* __restrict__ logits, uint16_t* __restrict__ h1o, uint16_t* __restrict__ h2o,
    uint16_t* __restrict__ h3o) {
  __shared__ Packed W;
  __shared__ uint16_t xs[kFwdWaves][16][kXs];
  __shared__ uint16_t hb[kFwdWaves][2][2][16][16];  // [step parity][position of the pair][window][channel]
  __shared__ uint16_t h2s[kFwdWaves][16][16];
  {
    const uint4* src = reinterpret_cast<const uint4*>(Wg);
    uint4* dst = reinterpret_cast<uint4*>(&W);
    for (int e = threadIdx.x; e < (int)(sizeof(Packed) / 16); e += blockDim.x) dst[e] = src[e];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int n = n_dev ? min(max(*n_dev, 0), n_max) : n_max;
  const int tiles = (n + 15) / 16;
  const int row = l % 16, g = l / 16;
  // this lane's conv1 taps: t = 8 g + i, cell offset (dk, dj, di) in the window
  int off[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int t = 8 * g + i;
    off[i] = t < 27 ? (t / 9) * 25 + ((t / 3) % 3) * 5 + t % 3 : -1;
  }
  const bf16x8 b1v = as_bf16x8(*reinterpret_cast<const uint4*>(&W.w1[l * 8]));
  const int c = l % 16;
  for (int tile = blockIdx.x * kFwdWaves + wave; tile < tiles; tile += gridDim.x * kFwdWaves) {
    const int w0 = tile * 16;
    if constexpr (FUSED) {
      build_windows(acc, n_phi, n_qpt, n_d0, peaks, w0, n, l, xs[wave]);
    } else {
      // 16 windows x 256 bytes, 16-byte global reads, 4-byte LDS writes (odd row stride)
      for (int ch = l; ch < 16 * 16; ch += 64) {
        const int w = ch / 16, o = (ch % 16) * 8;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (w0 + w < n) v = *reinterpret_cast<const uint4*>(win + (size_t)(w0 + w) * kWin + o);
        uint32_t* d = reinterpret_cast<uint32_t*>(&xs[wave][w][o]);
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    f32x4 acc2 = {0.f, 0.f, 0.f, 0.f};
    for (int st = 0; st < kC2Steps; ++st) {
      const int par = st & 1;
      // conv1 at positions 2 st and 2 st + 1 (27: zero)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int p = 2 * st + h;
        uint16_t outv[4] = {0, 0, 0, 0};
        if (p < 27) {
          const int base = (p / 9) * 25 + ((p / 3) % 3) * 5 + p % 3;
          bf16x8 a;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const uint16_t x = off[i] >= 0 ? xs[wave][row][base + off[i]] : (uint16_t)0;
            a[i] = __builtin_bit_cast(__bf16, x);
          }
          f32x4 z = {0.f, 0.f, 0.f, 0.f};
          z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1v, z, 0, 0, 0);
#pragma unroll
          for (int i = 0; i < 4; ++i) outv[i] = to_bf16(fmaxf(z[i] + W.b1[c], 0.0f));
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          hb[wave][par][h][4 * g + i][c] = outv[i];
          if (ACT && p < 27 && w0 + 4 * g + i < n)
            h1o[(size_t)(w0 + 4 * g + i) * 432 + p * 16 + c] = outv[i];
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      // conv2 k-step: lane (row, g) takes position 2 st + g / 2, channels 8 (g % 2) .. + 7
      const bf16x8 a2 = as_bf16x8(*reinterpret_cast<const uint4*>(&hb[wave][par][g >> 1][row][8 * (g & 1)]));
      const bf16x8 b2 = as_bf16x8(*reinterpret_cast<const uint4*>(&W.w2[(st * 64 + l) * 8]));
      acc2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b2, acc2, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) h2s[wave][4 * g + i][c] = to_bf16(fmaxf(acc2[i] + W.b2[c], 0.0f));
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // fc1 (K = 16) and fc2
    const int kq = 4 * g;
    const bf16x4 a3 = *reinterpret_cast<const bf16x4*>(&h2s[wave][row][kq]);
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(&W.w3[(nt * 64 + l) * 4]);
      f32x4 z = {0.f, 0.f, 0.f, 0.f};
      z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a3, b, z, 0, 0, 0);
      const int f = 16 * nt + c;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint16_t hv = to_bf16(fmaxf(z[i] + W.b3[f], 0.0f));
        part[i] += W.w4[f] * from_bf16(hv);
        if (ACT && w0 + kq + i < n) h3o[(size_t)(w0 + kq + i) * 64 + f] = hv;
      }
    }
    // sum over the 16 lanes of a row (the 64 features of one window)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v = part[i];
      for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
      if (c == 0 && w0 + kq + i < n) logits[w0 + kq + i] = v + W.b4[0];
    }
    if (ACT) {
      for (int e = l; e < 16 * 16; e += 64) {
        const int w = e / 16;
        if (w0 + w < n) h2o[(size_t)(w0 + w) * 16 + e % 16] = (&h2s[wave][0][0])[e];
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

// Backward on the matrix cores (v_mfma_f32_16x16x16_bf16, K = 16; same
// lane layout as above with k = 4 (lane / 16) + i).  One wave per tile of 16
// windows, tiles grid-strided; the wave keeps its parameter gradients in
// MFMA accumulators and adds them to the global gradient once.  Precision
// contract (the oracle's too): the backward signals dh3, dh2, dh1 are
// rounded to bfloat16 after their ReLU masks, like the activations, and every
// contraction accumulates in float32; dz and the last layer stay float32.
//   dh2 = dh3 W3           M = 16 windows, N = 16 channels, K = 64 features
//   dh1[p] = dh2 W2[.][.][p]   per position p: M = 16 windows, N = 16, K = 16
//   dW1 += dh1[p]^T x_p    per position: M = 16 channels, N = 32 taps, K = 16 windows
//   dW2[p] += dh2^T h1[p]  per position: M = 16, N = 16, K = 16 windows
//   dW3 += dh3^T h2        M = 64 features, N = 16 channels, K = 16 windows
constexpr int kBwdWaves = 4;

__device__ __forceinline__ bf16x4 pack4(uint16_t a, uint16_t b, uint16_t c, uint16_t d) {
  bf16x4 v;
  v[0] = (short)a; v[1] = (short)b; v[2] = (short)c; v[3] = (short)d;
  return v;
}

__global__ __launch_bounds__(kBwdWaves * 64) void backward_kernel(
    const float* __restrict__ P, const uint16_t* __restrict__ win, const float* __restrict__ labels,
    int n, float pos_weight, const float* __restrict__ logits, const uint16_t* __restrict__ h1g,
    const uint16_t* __restrict__ h2g, const uint16_t* __restrict__ h3g, float* __restrict__ grad,
    float* __restrict__ loss) {
  __shared__ uint16_t xs[kBwdWaves][16][kWin];
  __shared__ uint16_t h1s[kBwdWaves][16][27][16];
  __shared__ uint16_t h2s[kBwdWaves][16][16];
  __shared__ uint16_t h3s[kBwdWaves][16][64];
  __shared__ uint16_t d3s[kBwdWaves][16][64];   // dh3 (bf16)
  __shared__ uint16_t d2s[kBwdWaves][16][16];   // dh2 (bf16)
  __shared__ uint16_t d1s[kBwdWaves][16][16];   // dh1 at one position (bf16)
  __shared__ float dzs[kBwdWaves][16];
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int row = l % 16, g = l / 16;
  const int tiles = (n + 15) / 16;
  f32x4 aw1[2], aw2[27], aw3[4];
#pragma unroll
  for (int q = 0; q < 2; ++q) aw1[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < 27; ++q) aw2[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < 4; ++q) aw3[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, gw4 = 0.f, gb4 = 0.f, lsum = 0.f;
  const float w4b = from_bf16(to_bf16(P[oW4 + l]));
  for (int tile = blockIdx.x * kBwdWaves + wave; tile < tiles; tile += gridDim.x * kBwdWaves) {
    const int w0 = tile * 16;
    const int nw = min(16, n - w0);
    // stage the tile's inputs and activations (zeros past the last window)
    for (int e = l; e < 16 * kWin; e += 64) {
      const int w = e / kWin;
      (&xs[wave][0][0])[e] = w < nw ? win[(size_t)w0 * kWin + e] : (uint16_t)0;
    }
    for (int e = l; e < 16 * 432; e += 64)
      (&h1s[wave][0][0][0])[e] = e / 432 < nw ? h1g[(size_t)w0 * 432 + e] : (uint16_t)0;
    for (int e = l; e < 16 * 16; e += 64)
      (&h2s[wave][0][0])[e] = e / 16 < nw ? h2g[(size_t)w0 * 16 + e] : (uint16_t)0;
    for (int e = l; e < 16 * 64; e += 64)
      (&h3s[wave][0][0])[e] = e / 64 < nw ? h3g[(size_t)w0 * 64 + e] : (uint16_t)0;
    if (l < 16) {
      float dz = 0.f;
      if (l < nw) {
        const float z = logits[w0 + l], y = labels[w0 + l];
        const float wgt = y > 0.5f ? pos_weight : 1.0f;
        const float sp = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
        lsum += wgt * (sp - y * z) / (float)n;
        dz = wgt * (1.0f / (1.0f + expf(-z)) - y) / (float)n;
      }
      dzs[wave][l] = dz;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // dh3 = dz W4 [h3 > 0] (lane = feature), and the last layer's gradients
#pragma unroll 4
    for (int w = 0; w < 16; ++w) {
      const float dz = dzs[wave][w];
      const float h3 = from_bf16(h3s[wave][w][l]);
      const uint16_t d3 = h3 > 0.0f ? to_bf16(dz * w4b) : (uint16_t)0;
      d3s[wave][w][l] = d3;
      gb3 += from_bf16(d3);
      gw4 += dz * h3;
      if (l == 0) gb4 += dz;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // dh2 = dh3 W3 [h2 > 0]
    {
      f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int f = 16 * st + 4 * g;
        const bf16x4 a = *reinterpret_cast<const bf16x4*>(&d3s[wave][row][f]);
        const bf16x4 b = pack4(to_bf16(P[oW3 + (f + 0) * 16 + row]), to_bf16(P[oW3 + (f + 1) * 16 + row]),
                               to_bf16(P[oW3 + (f + 2) * 16 + row]), to_bf16(P[oW3 + (f + 3) * 16 + row]));
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, d, 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int w = 4 * g + i;
        const uint16_t v = h2s[wave][w][row] != 0 ? to_bf16(d[i]) : (uint16_t)0;
        d2s[wave][w][row] = v;
        gb2 += from_bf16(v);
      }
    }
    // dW3 += dh3^T h2
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    {
      const bf16x4 b = pack4(h2s[wave][4 * g][row], h2s[wave][4 * g + 1][row], h2s[wave][4 * g + 2][row],
                             h2s[wave][4 * g + 3][row]);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const int f = 16 * mt + row;
        const bf16x4 a = pack4(d3s[wave][4 * g][f], d3s[wave][4 * g + 1][f], d3s[wave][4 * g + 2][f],
                               d3s[wave][4 * g + 3][f]);
        aw3[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, aw3[mt], 0, 0, 0);
      }
    }
    // per position: dh1[p], then dW1 and dW2 at p
    const bf16x4 a_dh2_t = pack4(d2s[wave][4 * g][row], d2s[wave][4 * g + 1][row],
                                 d2s[wave][4 * g + 2][row], d2s[wave][4 * g + 3][row]);  // [c][w]
    const bf16x4 a_dh2 = *reinterpret_cast<const bf16x4*>(&d2s[wave][row][4 * g]);      // [w][c]
#pragma unroll 1
    for (int p = 0; p < 27; ++p) {
      const int base = (p / 9) * 25 + ((p / 3) % 3) * 5 + p % 3;
      {
        const int c0 = 4 * g;
        const bf16x4 b = pack4(to_bf16(P[oW2 + ((c0 + 0) * 16 + row) * 27 + p]),
                               to_bf16(P[oW2 + ((c0 + 1) * 16 + row) * 27 + p]),
                               to_bf16(P[oW2 + ((c0 + 2) * 16 + row) * 27 + p]),
                               to_bf16(P[oW2 + ((c0 + 3) * 16 + row) * 27 + p]));
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
        d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_dh2, b, d, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int w = 4 * g + i;
          const uint16_t v = h1s[wave][w][p][row] != 0 ? to_bf16(d[i]) : (uint16_t)0;
          d1s[wave][w][row] = v;
          gb1 += from_bf16(v);
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      // dW1[c][t] += sum_w dh1[w][p][c] x[w][cell(p, t)]
      const bf16x4 a1 = pack4(d1s[wave][4 * g][row], d1s[wave][4 * g + 1][row],
                              d1s[wave][4 * g + 2][row], d1s[wave][4 * g + 3][row]);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const int t = 16 * nt + row;
        const int cell = t < 27 ? base + (t / 9) * 25 + ((t / 3) % 3) * 5 + t % 3 : -1;
        const bf16x4 b = cell >= 0 ? pack4(xs[wave][4 * g][cell], xs[wave][4 * g + 1][cell],
                                           xs[wave][4 * g + 2][cell], xs[wave][4 * g + 3][cell])
                                   : pack4(0, 0, 0, 0);
        aw1[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b, aw1[nt], 0, 0, 0);
      }
      // dW2[c][c'][p] += sum_w dh2[w][c] h1[w][p][c']
      const bf16x4 b2 = pack4(h1s[wave][4 * g][p][row], h1s[wave][4 * g + 1][p][row],
                              h1s[wave][4 * g + 2][p][row], h1s[wave][4 * g + 3][p][row]);
#pragma unroll
      for (int q = 0; q < 27; ++q)
        if (q == p) aw2[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_dh2_t, b2, aw2[q], 0, 0, 0);
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
  }
  // the wave's gradients into the global sum
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = 4 * g + i, t = 16 * nt + row;
      if (t < 27) atomicAdd(&grad[oW1 + c * 27 + t], aw1[nt][i]);
    }
#pragma unroll
  for (int q = 0; q < 27; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) atomicAdd(&grad[oW2 + ((4 * g + i) * 16 + row) * 27 + q], aw2[q][i]);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) atomicAdd(&grad[oW3 + (16 * mt + 4 * g + i) * 16 + row], aw3[mt][i]);
  atomicAdd(&grad[ob1 + row], gb1);
  atomicAdd(&grad[ob2 + row], gb2);
  atomicAdd(&grad[ob3 + l], gb3);
  atomicAdd(&grad[oW4 + l], gw4);
  for (int o = 32; o > 0; o >>= 1) {
    lsum += __shfl_xor(lsum, o);
    gb4 += __shfl_xor(gb4, o);
  }
  if (l == 0) {
    atomicAdd(&grad[ob4], gb4);
    atomicAdd(loss, lsum);
  }
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

// inference grid: the workgroups that fit the chip at once (3 per CU by LDS),
// each wave looping over tiles, so the weights are copied into LDS once per
// resident workgroup
constexpr int kFwdGrid = 768;

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
  forward_kernel<false, false><<<blocks(tiles, kFwdWaves, kFwdGrid), kFwdWaves * 64, 0, s>>>(
      W, win, nullptr, 0, 0, 0, nullptr, n_dev, n_max, logits, nullptr, nullptr, nullptr);
  HT_CHECK(hipGetLastError());
  return HT_OK;
}

int launch_cnn_score(const Plan& p, const float* params, const int32_t* acc, const ht_peak* peaks,
                     const int32_t* n_peaks, int32_t cap, float* logits, void* ws, hipStream_t s) {
  Packed* W = reinterpret_cast<Packed*>(ws);
  pack_kernel<<<1, 256, 0, s>>>(params, W);
  HT_CHECK(hipGetLastError());
  const ht_grid& g = p.grid;
  const int tiles = (cap + 15) / 16;
  forward_kernel<true, false><<<blocks(tiles, kFwdWaves, kFwdGrid), kFwdWaves * 64, 0, s>>>(
      W, nullptr, acc, g.n_phi, g.n_qpt, g.n_d0, peaks, n_peaks, cap, logits, nullptr, nullptr,
      nullptr);
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
  forward_kernel<false, true><<<blocks(tiles, kFwdWaves, 4096), kFwdWaves * 64, 0, s>>>(
      W, win, nullptr, 0, 0, 0, nullptr, nullptr, n, logits, h1, h2, h3);
  HT_CHECK(hipGetLastError());
  backward_kernel<<<blocks(tiles, kBwdWaves, 64), kBwdWaves * 64, 0, s>>>(
      params, win, labels, n, pos_weight, logits, h1, h2, h3, grad, loss);
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
