// Full evaluation of the lineal path function on gfx950.
//
// The paper's Alg. "L2_eval" tests, for every segment and every translation, the segment's
// pixels one by one.  Here 32 translations (start pixels) share one 32-bit word: for a segment
// with pixels p_k = (px_k, py_k) (translated so that every offset is >= 0, which leaves the
// count unchanged on a periodic image), a lane owning start word w of row y forms
//     t_k = bits [32w + px_k, 32w + px_k + 32) of row y + py_k      (one v_alignbit_b32)
//     A   = AND_k t_k    -> bit b set   <=> every pixel of the segment is phase 1
//     O   = OR_k  t_k    -> bit b clear <=> every pixel of the segment is phase 0
// and popcounts A and ~O.  Both phases share the aligned word.  The segment's pixels are
// generated on the scalar unit (the vector is wave-uniform), so px_k and py_k live in SGPRs.
//
// Periodicity (Sec. 2.1) is handled by an extended image E: row y of E holds row y of the image
// followed by wrapped copies, so bit j of E row y is pixel (j mod W, y).  Rows wrap when they are
// staged into LDS.  This replaces the paper's 2x2-tiled image A and translation table C.
#include "lpf_internal.h"

namespace lpf {

// ------------------------------------------------------------------------------------ pack
__global__ void k_pack(const uint8_t *__restrict__ img, int W, int H, int wpr,
                       uint64_t *__restrict__ bits) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y;
  if (j >= wpr || y >= H) return;
  const uint8_t *row = img + (size_t)y * W;
  uint64_t w = 0;
  int x0 = j * 64;
  int nb = min(64, W - x0);
  for (int b = 0; b < nb; ++b) w |= (uint64_t)(row[x0 + b] != 0) << b;
  bits[(size_t)y * wpr + j] = w;
}

hipError_t launch_pack(const uint8_t *img, int W, int H, uint64_t *bits, hipStream_t stream) {
  int wpr = (W + 63) / 64;
  dim3 grid((wpr + 63) / 64, H);
  hipLaunchKernelGGL(k_pack, grid, dim3(64), 0, stream, img, W, H, wpr, bits);
  return hipGetLastError();
}

// ------------------------------------------------------------------------- extended image
// E[y][e], e < we: bit b = pixel ((32e + b) mod W, y).
__global__ void k_ext(const uint32_t *__restrict__ src, int W, int H, int src_stride, int we,
                      uint32_t *__restrict__ E) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y;
  if (e >= we || y >= H) return;
  const uint32_t *row = src + (size_t)y * src_stride;
  int s = (int)(((int64_t)32 * e) % W);
  uint32_t v;
  if (s + 32 <= W) {
    int q = s >> 5, sh = s & 31;
    uint32_t lo = row[q];
    uint32_t hi = sh ? row[q + 1] : 0u;  // q + 1 < ceil(W/32) whenever sh != 0 here
    v = __builtin_amdgcn_alignbit(hi, lo, sh);
  } else {
    v = 0;
    int x = s;
    for (int b = 0; b < 32; ++b) {
      v |= ((row[x >> 5] >> (x & 31)) & 1u) << b;
      x = (x + 1 == W) ? 0 : x + 1;
    }
  }
  E[(size_t)y * we + e] = v;
}

hipError_t launch_ext(const uint64_t *bits, int W, int H, int we, uint32_t *ext,
                      hipStream_t stream) {
  int src_stride = 2 * ((W + 63) / 64);
  dim3 grid((we + 63) / 64, H);
  hipLaunchKernelGGL(k_ext, grid, dim3(64), 0, stream, reinterpret_cast<const uint32_t *>(bits),
                     W, H, src_stride, we, ext);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------ full kernel

// Path product of one segment for the lane's R words: A &= t, O |= t over all pixels.
// XM: x is the major axis.  Q2: the vector has dx < 0 (mirrored in x, shifted by |dx|).
template <int R, bool XM, bool Q2>
__device__ __forceinline__ void path_product(const uint32_t *__restrict__ base, int rst, int adx,
                                             int n, int m, uint32_t (&A)[R], uint32_t (&O)[R]) {
  int err = n, q = 0;
  for (int k = 0; k <= n; ++k) {
    if (k) {
      err += 2 * m;
      if (err >= 2 * n) {
        err -= 2 * n;
        ++q;
      }
    }
    const int X = XM ? k : q;
    const int Y = XM ? q : k;
    const int px = Q2 ? adx - X : X;
    const uint32_t *p = base + Y * rst + (px >> 5);
    const int sh = px & 31;
    uint32_t d[R + 1];
#pragma unroll
    for (int c = 0; c <= R; ++c) d[c] = p[c];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const uint32_t t = __builtin_amdgcn_alignbit(d[i + 1], d[i], sh);
      A[i] &= t;
      O[i] |= t;
    }
  }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int R>
__global__ void __launch_bounds__(512)
k_lpf_full(const uint32_t *__restrict__ E, int W, int H, int we, int S, int tile, int lds_rows,
           int rst, const VecDesc *__restrict__ vecs, const int32_t *__restrict__ bin_off,
           int wpg, unsigned phase_mask, uint32_t *__restrict__ out, int nv) {
  extern __shared__ uint32_t lds[];
  const int t_id = blockIdx.y;
  const int Y0 = t_id * tile;
  const int rows_here = min(tile, H - Y0);

  // Stage rows Y0 .. Y0 + lds_rows - 1 (mod H) of E.
  for (int i = threadIdx.x; i < lds_rows * we; i += blockDim.x) {
    const int r = i / we;
    const int e = i - r * we;
    const int y = (Y0 + r) % H;
    lds[r * rst + e] = E[(size_t)y * we + e];
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rpw = 64 / S;
  const int strip = lane / rpw;
  const int r_in = lane - strip * rpw;
  const int swd = (W + 31) >> 5;
  const uint32_t lastmask = (W & 31) ? ((1u << (W & 31)) - 1u) : 0xffffffffu;
  const int nbands = (rows_here + rpw - 1) / rpw;
  const int nph = (phase_mask & 1) + ((phase_mask >> 1) & 1);

  const int bin = blockIdx.x * wpg + wave;
  const int vb = bin_off[bin], ve = bin_off[bin + 1];
  for (int j = vb; j < ve; ++j) {
    const VecDesc v = vecs[j];
    const int dx = v.dx, dy = v.dy;
    const int adx = dx < 0 ? -dx : dx;
    const int n = adx > dy ? adx : dy;
    const bool xm = adx >= dy;
    const int m = xm ? dy : adx;
    uint32_t c0 = 0, c1 = 0;
    for (int band = 0; band < nbands; ++band) {
      const int row = band * rpw + r_in;
      const uint32_t *base = lds + row * rst + strip * R;
      uint32_t A[R], O[R];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        A[i] = 0xffffffffu;
        O[i] = 0u;
      }
      if (xm) {
        if (dx < 0) path_product<R, true, true>(base, rst, adx, n, m, A, O);
        else path_product<R, true, false>(base, rst, adx, n, m, A, O);
      } else {
        if (dx < 0) path_product<R, false, true>(base, rst, adx, n, m, A, O);
        else path_product<R, false, false>(base, rst, adx, n, m, A, O);
      }
      const bool row_ok = row < rows_here;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int w = strip * R + i;
        uint32_t mk = (w < swd - 1) ? 0xffffffffu : (w == swd - 1 ? lastmask : 0u);
        mk = row_ok ? mk : 0u;
        c1 += __popc(A[i] & mk);
        c0 += __popc(~O[i] & mk);
      }
    }
    c0 = wave_sum(c0);
    c1 = wave_sum(c1);
    if (lane == 0) {
      int p = 0;
      uint32_t *o = out + (size_t)t_id * nph * nv;
      if (phase_mask & 1) o[(size_t)(p++) * nv + v.idx] = c0;
      if (phase_mask & 2) o[(size_t)p * nv + v.idx] = c1;
    }
  }
}

template <int R>
static hipError_t launch_full_r(const FullShape &sh, const uint32_t *ext, int W, int H,
                                const VecDesc *vecs, const int32_t *bin_off, unsigned phase_mask,
                                uint32_t *out, int nv, hipStream_t stream) {
  const int nwg = (sh.nbins + sh.wpg - 1) / sh.wpg;
  dim3 grid(nwg, sh.ntiles);
  size_t lds = (size_t)sh.lds_rows * sh.rst * sizeof(uint32_t);
  hipLaunchKernelGGL(k_lpf_full<R>, grid, dim3(64 * sh.wpg), lds, stream, ext, W, H, sh.we, sh.S,
                     sh.tile, sh.lds_rows, sh.rst, vecs, bin_off, sh.wpg, phase_mask, out, nv);
  return hipGetLastError();
}

hipError_t launch_full(const FullShape &sh, const uint32_t *ext, int W, int H, int /*cy*/,
                       const VecDesc *vecs, const int32_t *bin_off, unsigned phase_mask,
                       uint32_t *out, int nv, hipStream_t stream) {
  switch (sh.R) {
    case 1: return launch_full_r<1>(sh, ext, W, H, vecs, bin_off, phase_mask, out, nv, stream);
    case 2: return launch_full_r<2>(sh, ext, W, H, vecs, bin_off, phase_mask, out, nv, stream);
    case 4: return launch_full_r<4>(sh, ext, W, H, vecs, bin_off, phase_mask, out, nv, stream);
    case 8: return launch_full_r<8>(sh, ext, W, H, vecs, bin_off, phase_mask, out, nv, stream);
    case 16: return launch_full_r<16>(sh, ext, W, H, vecs, bin_off, phase_mask, out, nv, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t prepare_full_kernels(int max_lds_bytes) {
  hipError_t e = hipSuccess;
  const void *fns[] = {(const void *)k_lpf_full<1>, (const void *)k_lpf_full<2>,
                       (const void *)k_lpf_full<4>, (const void *)k_lpf_full<8>,
                       (const void *)k_lpf_full<16>};
  for (const void *f : fns) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
    if (r != hipSuccess) e = r;
  }
  return e;
}

// ---------------------------------------------------------------------------- tile sum / layout
__global__ void k_finish(const uint32_t *__restrict__ part, int ntiles, int nph, int nv,
                         const int16_t *__restrict__ dxdy, int cx, int cy, int layout,
                         uint32_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nph * nv) return;
  const int p = (int)(i / nv);
  const int v = (int)(i - (int64_t)p * nv);
  uint32_t s = 0;
  for (int t = 0; t < ntiles; ++t) s += part[((size_t)t * nph + p) * nv + v];
  if (layout == 0) {
    out[(size_t)p * nv + v] = s;
  } else {
    const int gw = 2 * cx + 1;
    const size_t g = (size_t)gw * (2 * cy + 1);
    const int dx = dxdy[2 * v], dy = dxdy[2 * v + 1];
    out[(size_t)p * g + (size_t)(dy + cy) * gw + (dx + cx)] = s;
    out[(size_t)p * g + (size_t)(cy - dy) * gw + (cx - dx)] = s;
  }
}

hipError_t launch_finish(const uint32_t *part, int ntiles, int nph, int nv, const int16_t *dxdy,
                         int cx, int cy, int layout, uint32_t *out, hipStream_t stream) {
  const int64_t n = (int64_t)nph * nv;
  dim3 grid((unsigned)((n + 255) / 256));
  hipLaunchKernelGGL(k_finish, grid, dim3(256), 0, stream, part, ntiles, nph, nv, dxdy, cx, cy,
                     layout, out);
  return hipGetLastError();
}

}  // namespace lpf
