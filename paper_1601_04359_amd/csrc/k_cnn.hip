// Swap-proposal CNN: forward, backward and Adam, hand-written for gfx950 MFMA.
//
// The network ranks pixel interchanges for the annealer (the paper leaves the modification
// operator open, Sec. 4); the exact lineal-path change still judges every move.
//   X0 = (pixel, interface flag)   -> conv3x3 16 -> relu -> conv3x3 16 -> relu -> conv3x3 16
//   -> relu -> 1x1 head = per-pixel score S.   Periodic 'same' padding on the cell.
// Activations and weights are bfloat16, accumulation fp32.  Tensors are channels-last:
// X0 [B][H][W][4] (2 used), A_l [B][H][W][16]; forward weights Wf[tap][co][ci], backward-data
// weights Wt[tap][ci][co] (tap = 3 dy + dx, input offset (dy-1, dx-1)).
//
// A convolution is an implicit GEMM: a wave computes 16 pixels x 16 output channels with one
// v_mfma_f32_16x16x16_bf16 per tap (K = 16 input channels).  MFMA 16x16x16 operand layout on a
// 64-lane wave: lane l holds A[l%16][4(l/16)+j], B[4(l/16)+j][l%16] and D[4(l/16)+j][l%16],
// j = 0..3.  Pixel rows of A come from the (periodically) shifted neighbours, so the 8-byte
// operand of a lane is 4 consecutive channels of one pixel.
#include <math.h>

#include <algorithm>

#include "lpf_internal.h"

namespace lpf {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct PixelRef {
  int64_t base;  // b * H * W
  int y, x;
};

__device__ __forceinline__ PixelRef pixel_of(int64_t p, int W, int H) {
  const int64_t hw = (int64_t)W * H;
  const int64_t b = p / hw;
  const int r = (int)(p - b * hw);
  const int y = r / W;
  return PixelRef{b * hw, y, r - y * W};
}

__device__ __forceinline__ int64_t shifted(const PixelRef &q, int dy, int dx, int W, int H) {
  int y = q.y + dy, x = q.x + dx;
  y += y < 0 ? H : 0;
  y -= y >= H ? H : 0;
  x += x < 0 ? W : 0;
  x -= x >= W ? W : 0;
  return q.base + (int64_t)y * W + x;
}

// ------------------------------------------------------------------------------- features
__global__ void k_cnn_features(const uint64_t *__restrict__ bits, int W, int H, int64_t npix,
                               uint16_t *__restrict__ X0) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const PixelRef q = pixel_of(p, W, H);
  const int wpr = (W + 63) >> 6;
  const uint64_t *img = bits + (q.base / W) * wpr;  // image b starts at row b*H
  auto at = [&](int y, int x) -> int {
    return (int)((img[(size_t)y * wpr + (x >> 6)] >> (x & 63)) & 1ull);
  };
  const int v = at(q.y, q.x);
  const int xl = q.x ? q.x - 1 : W - 1, xr = q.x + 1 == W ? 0 : q.x + 1;
  const int yu = q.y ? q.y - 1 : H - 1, yd = q.y + 1 == H ? 0 : q.y + 1;
  const int itf = at(q.y, xl) != v || at(q.y, xr) != v || at(yu, q.x) != v || at(yd, q.x) != v;
  uint2 o;
  o.x = (uint32_t)(v ? 0x3f80u : 0u) | ((uint32_t)(itf ? 0x3f80u : 0u) << 16);
  o.y = 0;
  *reinterpret_cast<uint2 *>(X0 + 4 * p) = o;
}

// -------------------------------------------------------------------------------- forward
// A_out = bf16(relu(conv3x3(X) + bias)); X has `cin` (4 or 16) channels, of which the first
// 16 (or 4) enter the 16-wide K of the MFMA.
__global__ void __launch_bounds__(256)
k_cnn_conv_fwd(const uint16_t *__restrict__ X, int cin, const uint16_t *__restrict__ Wf,
               const float *__restrict__ bias, uint16_t *__restrict__ A_out, int W, int H,
               int64_t npix) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, m = lane & 15;
  s4v Bw[9];
#pragma unroll
  for (int t = 0; t < 9; ++t)
    Bw[t] = *reinterpret_cast<const s4v *>(Wf + (t * 16 + m) * 16 + 4 * g);
  const float bco = bias[m];
  const int64_t ntiles = (npix + 15) >> 4;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t tile = wave0; tile < ntiles; tile += nwaves) {
    const int64_t p = tile * 16 + m;
    const bool pin = p < npix;
    const PixelRef q = pixel_of(pin ? p : 0, W, H);
    f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int64_t src = shifted(q, t / 3 - 1, t % 3 - 1, W, H);
      s4v a = {0, 0, 0, 0};
      if (pin && 4 * g < cin) a = *reinterpret_cast<const s4v *>(X + src * cin + 4 * g);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, Bw[t], acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t po = tile * 16 + 4 * g + j;
      if (po < npix) A_out[po * 16 + m] = f2bf(fmaxf(acc[j] + bco, 0.f));
    }
  }
}

// Score of one pixel from its 16 layer-3 activations: sum_c A3[c] W4[c] + b4 (W4 rounded to
// bf16), summed in channel order.
__device__ __forceinline__ float head_score(const uint16_t *a3, const float *__restrict__ W4bf,
                                            const float *__restrict__ b4) {
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < 16; ++c) s += bf2f(a3[c]) * W4bf[c];
  return s + b4[0];
}

// S[p] = sum_c A3[p][c] W4[c] + b4.
__global__ void k_cnn_head_fwd(const uint16_t *__restrict__ A3, const float *__restrict__ W4bf,
                               const float *__restrict__ b4, int64_t npix, float *__restrict__ S) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  S[p] = head_score(A3 + p * 16, W4bf, b4);
}

// ---------------------------------------------------------------- single-image scores, fused
// The annealer's re-scoring of its cell in one launch.  A workgroup computes a 16 x 16 tile of
// scores: the features of the tile and a 3-pixel periodic halo (22 x 22), then each layer's
// activations on a halo one pixel narrower (20 x 20, 18 x 18, 16 x 16), all in LDS.  Halo pixels
// are real pixels of the periodic cell, so their activations are the ones the layered kernels
// compute; each output uses the same MFMA taps in the same order, the same bias, ReLU and bf16
// rounding and the same head, so the scores equal cnn_forward's bit for bit.
constexpr int kScoreTile = 16;

// One 3x3 layer on LDS regions: `in` is a (wout + 2)^2 region with cin (4 or 16) channels per
// pixel, `out` the wout^2 region inside it with 16; the workgroup's waves take 16-pixel tiles in
// turn.
__device__ __forceinline__ void conv_region(const uint16_t *in, int cin, uint16_t *out, int wout,
                                            const uint16_t *__restrict__ Wf,
                                            const float *__restrict__ bias) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, m = lane & 15;
  const int win = wout + 2, nout = wout * wout;
  s4v Bw[9];
#pragma unroll
  for (int t = 0; t < 9; ++t)
    Bw[t] = *reinterpret_cast<const s4v *>(Wf + (t * 16 + m) * 16 + 4 * g);
  const float bco = bias[m];
  const int nwaves = (int)(blockDim.x >> 6);
  for (int tile = wave; tile * 16 < nout; tile += nwaves) {
    const int i = tile * 16 + m;
    const bool pin = i < nout;
    const int ry = pin ? i / wout : 0, rx = pin ? i - ry * wout : 0;
    f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int src = (ry + t / 3) * win + rx + t % 3;  // input offset (t / 3 - 1, t % 3 - 1)
      s4v a = {0, 0, 0, 0};
      if (pin && 4 * g < cin) a = *reinterpret_cast<const s4v *>(in + src * cin + 4 * g);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, Bw[t], acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int po = tile * 16 + 4 * g + j;
      if (po < nout) out[po * 16 + m] = f2bf(fmaxf(acc[j] + bco, 0.f));
    }
  }
}

// 1024 threads: each layer's tiles spread over 16 waves (four per SIMD), so that the chains of
// MFMA and LDS latency of one wave overlap those of the others.
__global__ void __launch_bounds__(1024)
k_cnn_score(const uint64_t *__restrict__ bits, int W, int H, const uint16_t *__restrict__ Wf,
            const float *__restrict__ prm, const float *__restrict__ W4bf,
            float *__restrict__ S) {
  constexpr int T = kScoreTile;
  __shared__ __attribute__((aligned(16))) uint16_t X0[(T + 6) * (T + 6) * 4];
  __shared__ __attribute__((aligned(16))) uint16_t A1[(T + 4) * (T + 4) * 16];
  __shared__ __attribute__((aligned(16))) uint16_t A2[(T + 2) * (T + 2) * 16];
  __shared__ __attribute__((aligned(16))) uint16_t A3[T * T * 16];
  const int tx0 = blockIdx.x * T, ty0 = blockIdx.y * T;
  const int wpr = (W + 63) >> 6;
  auto at = [&](int y, int x) -> int {
    return (int)((bits[(size_t)y * wpr + (x >> 6)] >> (x & 63)) & 1ull);
  };
  for (int i = threadIdx.x; i < (T + 6) * (T + 6); i += blockDim.x) {
    const int ry = i / (T + 6), rx = i - ry * (T + 6);
    const int y = (((ty0 - 3 + ry) % H) + H) % H, x = (((tx0 - 3 + rx) % W) + W) % W;
    const int v = at(y, x);
    const int xl = x ? x - 1 : W - 1, xr = x + 1 == W ? 0 : x + 1;
    const int yu = y ? y - 1 : H - 1, yd = y + 1 == H ? 0 : y + 1;
    const int itf = at(y, xl) != v || at(y, xr) != v || at(yu, x) != v || at(yd, x) != v;
    uint2 o;
    o.x = (uint32_t)(v ? 0x3f80u : 0u) | ((uint32_t)(itf ? 0x3f80u : 0u) << 16);
    o.y = 0;
    *reinterpret_cast<uint2 *>(X0 + 4 * i) = o;
  }
  __syncthreads();
  conv_region(X0, 4, A1, T + 4, Wf, prm + 288);
  __syncthreads();
  conv_region(A1, 16, A2, T + 2, Wf + 2304, prm + 2608);
  __syncthreads();
  conv_region(A2, 16, A3, T, Wf + 4608, prm + 4928);
  __syncthreads();
  const int ry = threadIdx.x / T, rx = threadIdx.x - ry * T;
  const int y = ty0 + ry, x = tx0 + rx;
  if (threadIdx.x < T * T && y < H && x < W)
    S[(size_t)y * W + x] = head_score(A3 + threadIdx.x * 16, W4bf, prm + 4960);
}

// ------------------------------------------------------------------------------ loss / head
constexpr double kFx = 1099511627776.0;  // 2^40: fixed-point scale of the score gradient

__global__ void k_cnn_zero64(int64_t *__restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// r_i = S[img][a] + S[img][b] - y; dS[img][a], dS[img][b] += 2 r_i / n in 2^-40 fixed point
// (integer atomics: the sum does not depend on their order).
__global__ void k_cnn_loss(const float *__restrict__ S, const CnnSample *__restrict__ smp, int n,
                           int64_t hw, int batch, long long *__restrict__ dS_fx,
                           float *__restrict__ r_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const CnnSample s = smp[i];
  const bool ok = s.img >= 0 && s.img < batch && s.a >= 0 && s.a < hw && s.b >= 0 && s.b < hw;
  float r = 0.f;
  if (ok) {
    const int64_t o = (int64_t)s.img * hw;
    r = S[o + s.a] + S[o + s.b] - s.y;
    const long long g = llrint((2.0 * (double)r / (double)n) * kFx);
    atomicAdd((unsigned long long *)&dS_fx[o + s.a], (unsigned long long)g);
    atomicAdd((unsigned long long *)&dS_fx[o + s.b], (unsigned long long)g);
  }
  r_out[i] = r;
}

// loss = sum r^2 / n in a fixed order (one workgroup).
__global__ void __launch_bounds__(1024)
k_cnn_loss_sum(const float *__restrict__ r, int n, float *__restrict__ loss) {
  __shared__ double part[1024];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += (double)r[i] * (double)r[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) part[threadIdx.x] += part[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(part[0] / (double)n);
}

// dZ3 = bf16(dS * W4 * [A3 > 0]); per-block partials of dW4 (16) and db4 (1), fixed order.
__global__ void __launch_bounds__(256)
k_cnn_head_bwd(const long long *__restrict__ dS_fx, const uint16_t *__restrict__ A3,
               const float *__restrict__ W4bf, int64_t npix, uint16_t *__restrict__ dZ3,
               float *__restrict__ part /* [blocks][17] */) {
  __shared__ float red[256][17];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float loc[17];
#pragma unroll
  for (int c = 0; c < 17; ++c) loc[c] = 0.f;
  if (p < npix) {
    const float d = (float)((double)dS_fx[p] / kFx);
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const float a = bf2f(A3[p * 16 + c]);
      dZ3[p * 16 + c] = f2bf(a > 0.f ? d * W4bf[c] : 0.f);
      loc[c] = d * a;
    }
    loc[16] = d;
  }
#pragma unroll
  for (int c = 0; c < 17; ++c) red[threadIdx.x][c] = loc[c];
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k)
      for (int c = 0; c < 17; ++c) red[threadIdx.x][c] += red[threadIdx.x + k][c];
    __syncthreads();
  }
  if (threadIdx.x < 17) part[(size_t)blockIdx.x * 17 + threadIdx.x] = red[0][threadIdx.x];
}

// ------------------------------------------------------------------------- backward (data)
// dZ_prev = bf16(conv3x3^T(dZ; W) * [A_prev > 0]) with dX[p] = sum_t W[t]^T dZ[p - off(t)].
__global__ void __launch_bounds__(256)
k_cnn_conv_bwd_data(const uint16_t *__restrict__ dZ, const uint16_t *__restrict__ Wt,
                    const uint16_t *__restrict__ A_prev, uint16_t *__restrict__ dZ_prev, int W,
                    int H, int64_t npix) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, m = lane & 15;
  s4v Bw[9];
#pragma unroll
  for (int t = 0; t < 9; ++t)
    Bw[t] = *reinterpret_cast<const s4v *>(Wt + (t * 16 + m) * 16 + 4 * g);
  const int64_t ntiles = (npix + 15) >> 4;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t tile = wave0; tile < ntiles; tile += nwaves) {
    const int64_t p = tile * 16 + m;
    const bool pin = p < npix;
    const PixelRef q = pixel_of(pin ? p : 0, W, H);
    f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int64_t src = shifted(q, 1 - t / 3, 1 - t % 3, W, H);
      s4v a = {0, 0, 0, 0};
      if (pin) a = *reinterpret_cast<const s4v *>(dZ + src * 16 + 4 * g);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, Bw[t], acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t po = tile * 16 + 4 * g + j;
      if (po < npix) {
        const float a = bf2f(A_prev[po * 16 + m]);
        dZ_prev[po * 16 + m] = f2bf(a > 0.f ? acc[j] : 0.f);
      }
    }
  }
}

// ----------------------------------------------------------------------- backward (weights)
// Per-block partials of dW[t][co][ci] = sum_p dZ[p][co] X[p + off(t)][ci] and db[co] = sum_p
// dZ[p][co]; MFMA with M = co, N = ci, K = 16 pixels.
__global__ void __launch_bounds__(256)
k_cnn_conv_bwd_weight(const uint16_t *__restrict__ dZ, const uint16_t *__restrict__ X, int cin,
                      int W, int H, int64_t npix, float *__restrict__ part /* [blocks][9*256+16] */) {
  __shared__ float red[4][9 * 256 + 16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, m = lane & 15;
  f4v acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
  float dbl = 0.f;
  const int64_t nchunks = (npix + 15) >> 4;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t ch = wave0; ch < nchunks; ch += nwaves) {
    s4v a;
    int64_t pj[4];
    bool okj[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      pj[j] = ch * 16 + 4 * g + j;
      okj[j] = pj[j] < npix;
      const uint16_t v = okj[j] ? dZ[pj[j] * 16 + m] : (uint16_t)0;
      a[j] = (short)v;
      dbl += bf2f(v);
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      s4v bvec;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint16_t v = 0;
        if (okj[j] && m < cin) {
          const PixelRef q = pixel_of(pj[j], W, H);
          v = X[shifted(q, t / 3 - 1, t % 3 - 1, W, H) * cin + m];
        }
        bvec[j] = (short)v;
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bvec, acc[t], 0, 0, 0);
    }
  }
  // lane holds D[co = 4g + j][ci = m] for each tap, and a partial db for co = m
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wave][t * 256 + (4 * g + j) * 16 + m] = acc[t][j];
  // db[co]: lanes m, m+16, m+32, m+48 hold partials of channel m
  dbl += __shfl_xor(dbl, 16, 64);
  dbl += __shfl_xor(dbl, 32, 64);
  if (g == 0) red[wave][9 * 256 + m] = dbl;
  __syncthreads();
  for (int i = threadIdx.x; i < 9 * 256 + 16; i += blockDim.x)
    part[(size_t)blockIdx.x * (9 * 256 + 16) + i] =
        ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

// --------------------------------------------------------------------- gradient assembly
// The packed gradient (W1 [9][16][2], b1, W2 [9][16][16], b2, W3 [9][16][16], b3, W4 [16], b4)
// from the per-block partials, in a fixed order: slice s of kGradSlices sums its contiguous range
// of blocks in block order (k_cnn_grad_part), then the slices are added in slice order
// (k_cnn_grad_sum).
constexpr int kGradSlices = 64;

__device__ __forceinline__ float grad_partial(const float *__restrict__ p1,
                                              const float *__restrict__ p2,
                                              const float *__restrict__ p3,
                                              const float *__restrict__ ph, int i, int b) {
  const int stride = 9 * 256 + 16;
  if (i < 288) {  // W1[t][co][ci<2]
    const int t = i / 32, co = (i / 2) % 16, ci = i % 2;
    return p1[(size_t)b * stride + t * 256 + co * 16 + ci];
  }
  if (i < 304) return p1[(size_t)b * stride + 9 * 256 + (i - 288)];
  if (i < 2608) return p2[(size_t)b * stride + (i - 304)];
  if (i < 2624) return p2[(size_t)b * stride + 9 * 256 + (i - 2608)];
  if (i < 4928) return p3[(size_t)b * stride + (i - 2624)];
  if (i < 4944) return p3[(size_t)b * stride + 9 * 256 + (i - 4928)];
  return ph[(size_t)b * 17 + (i - 4944)];  // 0..15: W4, 16: b4
}

__global__ void k_cnn_grad_part(const float *__restrict__ p1, const float *__restrict__ p2,
                                const float *__restrict__ p3, int nb_conv,
                                const float *__restrict__ ph, int nb_head,
                                float *__restrict__ slices) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kCnnParams) return;
  const int sl = blockIdx.y;
  const int nb = i < 4944 ? nb_conv : nb_head;
  const int per = (nb + kGradSlices - 1) / kGradSlices;
  const int b0 = min(nb, sl * per), b1 = min(nb, b0 + per);
  float s = 0.f;
  for (int b = b0; b < b1; ++b) s += grad_partial(p1, p2, p3, ph, i, b);
  slices[(size_t)sl * kCnnParams + i] = s;
}

__global__ void k_cnn_grad_sum(const float *__restrict__ slices, float *__restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kCnnParams) return;
  float s = 0.f;
  for (int sl = 0; sl < kGradSlices; ++sl) s += slices[(size_t)sl * kCnnParams + i];
  grad[i] = s;
}

// ------------------------------------------------------------------------------ parameters
// bf16 weight layouts from the fp32 parameters.
__global__ void k_cnn_pack_weights(const float *__restrict__ prm, uint16_t *__restrict__ Wf,
                                   uint16_t *__restrict__ Wt, float *__restrict__ W4bf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // over 3 layers x 9 taps x 256
  if (i < 3 * 2304) {
    const int l = i / 2304, r = i % 2304, t = r / 256, co = (r / 16) % 16, ci = r % 16;
    float w;
    if (l == 0) w = ci < 2 ? prm[t * 32 + co * 2 + ci] : 0.f;
    else w = prm[(l == 1 ? 304 : 2624) + r];
    const uint16_t h = f2bf(w);
    Wf[l * 2304 + r] = h;                          // [t][co][ci]
    Wt[l * 2304 + t * 256 + ci * 16 + co] = h;     // [t][ci][co]
  }
  if (i < 16) W4bf[i] = bf2f(f2bf(prm[4944 + i]));
}

// One Adam step on the fp32 parameters (Kingma & Ba, 2015); c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void k_cnn_adam(float *__restrict__ prm, const float *__restrict__ grad,
                           float *__restrict__ mom, float *__restrict__ vel, float lr, float b1,
                           float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kCnnParams) return;
  const float g = grad[i];
  const float m = b1 * mom[i] + (1.f - b1) * g;
  const float v = b2 * vel[i] + (1.f - b2) * g * g;
  mom[i] = m;
  vel[i] = v;
  const float mh = m / c1, vh = v / c2;
  prm[i] = prm[i] - lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------------- launchers
static int conv_blocks(int64_t npix) {
  const int64_t tiles = (npix + 15) / 16;
  return (int)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, 4096));
}

hipError_t cnn_forward(const CnnBufs &B, const uint64_t *bits, int W, int H, int batch,
                       float *S, hipStream_t s) {
  const int64_t np = (int64_t)W * H * batch;
  const int nb = (int)((np + 255) / 256);
  const int cb = conv_blocks(np);
  hipLaunchKernelGGL(k_cnn_features, dim3(nb), dim3(256), 0, s, bits, W, H, np, B.X0);
  hipLaunchKernelGGL(k_cnn_conv_fwd, dim3(cb), dim3(256), 0, s, B.X0, 4, B.Wf, B.prm + 288, B.A1,
                     W, H, np);
  hipLaunchKernelGGL(k_cnn_conv_fwd, dim3(cb), dim3(256), 0, s, B.A1, 16, B.Wf + 2304,
                     B.prm + 2608, B.A2, W, H, np);
  hipLaunchKernelGGL(k_cnn_conv_fwd, dim3(cb), dim3(256), 0, s, B.A2, 16, B.Wf + 4608,
                     B.prm + 4928, B.A3, W, H, np);
  hipLaunchKernelGGL(k_cnn_head_fwd, dim3(nb), dim3(256), 0, s, B.A3, B.W4bf, B.prm + 4960, np, S);
  return hipGetLastError();
}

hipError_t cnn_score(const CnnBufs &B, const uint64_t *bits, int W, int H, float *S,
                     hipStream_t s) {
  const dim3 grid((unsigned)((W + kScoreTile - 1) / kScoreTile),
                  (unsigned)((H + kScoreTile - 1) / kScoreTile));
  hipLaunchKernelGGL(k_cnn_score, grid, dim3(1024), 0, s, bits, W, H, B.Wf, B.prm, B.W4bf, S);
  return hipGetLastError();
}

hipError_t cnn_grad(const CnnBufs &B, const uint64_t *bits, int W, int H, int batch,
                    const CnnSample *smp, int n, float *grad, float *loss, hipStream_t s) {
  const int64_t np = (int64_t)W * H * batch;
  const int nb = (int)((np + 255) / 256);
  const int cb = conv_blocks(np);
  hipError_t e = cnn_forward(B, bits, W, H, batch, B.S, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cnn_zero64, dim3(nb), dim3(256), 0, s, B.dS, np);
  hipLaunchKernelGGL(k_cnn_loss, dim3((n + 255) / 256), dim3(256), 0, s, B.S, smp, n,
                     (int64_t)W * H, batch, (long long *)B.dS, B.r);
  hipLaunchKernelGGL(k_cnn_loss_sum, dim3(1), dim3(1024), 0, s, B.r, n, loss);
  hipLaunchKernelGGL(k_cnn_head_bwd, dim3(nb), dim3(256), 0, s, (const long long *)B.dS, B.A3,
                     B.W4bf, np, B.dZ3, B.part_h);
  hipLaunchKernelGGL(k_cnn_conv_bwd_weight, dim3(cb), dim3(256), 0, s, B.dZ3, B.A2, 16, W, H, np,
                     B.part3);
  hipLaunchKernelGGL(k_cnn_conv_bwd_data, dim3(cb), dim3(256), 0, s, B.dZ3, B.Wt + 4608, B.A2,
                     B.dZ2, W, H, np);
  hipLaunchKernelGGL(k_cnn_conv_bwd_weight, dim3(cb), dim3(256), 0, s, B.dZ2, B.A1, 16, W, H, np,
                     B.part2);
  hipLaunchKernelGGL(k_cnn_conv_bwd_data, dim3(cb), dim3(256), 0, s, B.dZ2, B.Wt + 2304, B.A1,
                     B.dZ1, W, H, np);
  hipLaunchKernelGGL(k_cnn_conv_bwd_weight, dim3(cb), dim3(256), 0, s, B.dZ1, B.X0, 4, W, H, np,
                     B.part1);
  hipLaunchKernelGGL(k_cnn_grad_part, dim3((kCnnParams + 255) / 256, kGradSlices), dim3(256), 0, s,
                     B.part1, B.part2, B.part3, cb, B.part_h, nb, B.slices);
  hipLaunchKernelGGL(k_cnn_grad_sum, dim3((kCnnParams + 255) / 256), dim3(256), 0, s, B.slices,
                     grad);
  return hipGetLastError();
}

hipError_t cnn_pack(const CnnBufs &B, hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_pack_weights, dim3((3 * 2304 + 255) / 256), dim3(256), 0, s, B.prm,
                     B.Wf, B.Wt, B.W4bf);
  return hipGetLastError();
}

hipError_t cnn_adam(const CnnBufs &B, const float *grad, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_cnn_adam, dim3((kCnnParams + 255) / 256), dim3(256), 0, s, B.prm, grad,
                     B.mom, B.vel, lr, b1, b2, eps, c1, c2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return cnn_pack(B, s);
}

int cnn_conv_blocks(int64_t npix) { return conv_blocks(npix); }

}  // namespace lpf
