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
// Pixels are taken in pairs: two funnel shifts, one 3-input AND (v_bitop3_b32) and one 3-input
// OR (v_or3_b32) per word; when both pixels of a pair read the same dwords (same row, same
// word column) the dwords are loaded once.
//
// SKIP (the paper's "enhanced" evaluation, Sec. 3.2, done per wave): every 16 pixels the wave
// stops when no start pixel of its rows can still count for a requested phase (phase 1 needs a
// set bit of A, phase 0 a clear bit of O, both under the lane's valid-bit mask mk).  Further
// pixels only clear bits of A and set bits of O, so the counts are those of the full product.
template <int R, bool XM, bool Q2, bool SKIP>
__device__ __forceinline__ void path_product(const uint32_t *__restrict__ base, int rst, int adx,
                                             int n, int m, uint32_t (&A)[R], uint32_t (&O)[R],
                                             const uint32_t (&mk)[R], unsigned phase_mask) {
  int err = n, q = 0;
  auto advance = [&]() {
    err += 2 * m;
    if (err >= 2 * n) {
      err -= 2 * n;
      ++q;
    }
  };
  auto pixel = [&](int k, int &off, int &sh) {
    const int X = XM ? k : q;
    const int Y = XM ? q : k;
    const int px = Q2 ? adx - X : X;
    off = Y * rst + (px >> 5);
    sh = px & 31;
  };
  int k = 0;
  for (; k + 1 <= n; k += 2) {
    int off0, sh0, off1, sh1;
    pixel(k, off0, sh0);
    advance();
    pixel(k + 1, off1, sh1);
    advance();
    const uint32_t *p0 = base + off0;
    uint32_t t0[R], t1[R];
    if (off0 == off1) {
      uint32_t d[R + 1];
#pragma unroll
      for (int c = 0; c <= R; ++c) d[c] = p0[c];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        t0[i] = __builtin_amdgcn_alignbit(d[i + 1], d[i], sh0);
        t1[i] = __builtin_amdgcn_alignbit(d[i + 1], d[i], sh1);
      }
    } else {
      const uint32_t *p1 = base + off1;
      uint32_t d0[R + 1], d1[R + 1];
#pragma unroll
      for (int c = 0; c <= R; ++c) {
        d0[c] = p0[c];
        d1[c] = p1[c];
      }
#pragma unroll
      for (int i = 0; i < R; ++i) {
        t0[i] = __builtin_amdgcn_alignbit(d0[i + 1], d0[i], sh0);
        t1[i] = __builtin_amdgcn_alignbit(d1[i + 1], d1[i], sh1);
      }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      A[i] = __builtin_amdgcn_bitop3_b32(A[i], t0[i], t1[i], 0x80);
      O[i] = O[i] | t0[i] | t1[i];
    }
    if constexpr (SKIP) {
      if ((k & 15) == 14) {
        uint32_t live = 0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          if (phase_mask & 2u) live |= A[i] & mk[i];
          if (phase_mask & 1u) live |= ~O[i] & mk[i];
        }
        if (!__any(live != 0u)) return;
      }
    }
  }
  if (k == n) {  // odd pixel count: the last pixel alone
    int off, sh;
    pixel(k, off, sh);
    const uint32_t *p = base + off;
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

// Count of vector `idx` = (dx, dy) for phase slot p, in the image's output layout (the GRID
// layout also fills -v, eq. (symmetry)).
__device__ __forceinline__ void put_count(const FullImg &I, int p, int idx, int dx, int dy,
                                          uint32_t c) {
  if (I.layout == 0) {
    I.out[(size_t)p * I.nv + idx] = c;
  } else {
    const int gw = 2 * I.cx + 1;
    const size_t g = (size_t)gw * (2 * I.cy + 1);
    I.out[(size_t)p * g + (size_t)(dy + I.cy) * gw + (dx + I.cx)] = c;
    I.out[(size_t)p * g + (size_t)(I.cy - dy) * gw + (I.cx - dx)] = c;
  }
}

// Vector i of the canonical half domain: [0,cx] x [0,cy] row by row, then [-cx,-1] x [1,cy].
__device__ __forceinline__ VecDesc canonical_vec(int i, int cx, int cy) {
  const int n1 = (cx + 1) * (cy + 1);
  VecDesc v;
  v.idx = i;
  if (i < n1) {
    const int dy = i / (cx + 1);
    v.dy = (int16_t)dy;
    v.dx = (int16_t)(i - dy * (cx + 1));
  } else {
    const int r = i - n1;
    const int dy = r / cx;
    v.dy = (int16_t)(1 + dy);
    v.dx = (int16_t)(-cx + (r - dy * cx));
  }
  return v;
}

// One work item: waves w = 0..wpg-1 of the workgroup take bins bin0 + w of image I and count
// their vectors over every row tile of the image.  lds: staged rows; cnt: per-wave count slots
// (used only when the image has several row tiles).  Each count is written once, by lane 0 of
// the wave owning the vector.
// CANON: no vector table; the wave with global index g of the I.nbins waves takes the canonical
// vectors g, g + nbins, g + 2 nbins, ... (interleaving spreads long and short vectors evenly).
template <int R, bool SKIP, bool CANON = false>
__device__ __forceinline__ void process_item(const FullImg &I, int bin0, int wpg,
                                             unsigned phase_mask, uint32_t *__restrict__ lds,
                                             uint32_t *__restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rpw = 64 / I.S;
  const int strip = lane / rpw;
  const int r_in = lane - strip * rpw;
  const int swd = (I.W + 31) >> 5;
  const uint32_t lastmask = (I.W & 31) ? ((1u << (I.W & 31)) - 1u) : 0xffffffffu;
  const int bin = bin0 + wave;
  int vb, ve;
  if constexpr (CANON) {
    vb = 0;
    ve = bin < I.nbins && bin < I.nv ? (I.nv - 1 - bin) / I.nbins + 1 : 0;
  } else {
    vb = bin < I.nbins ? I.bin_off[bin] : 0;
    ve = bin < I.nbins ? I.bin_off[bin + 1] : 0;
  }
  auto vec_at = [&](int j) -> VecDesc {
    if constexpr (CANON) return canonical_vec(bin + j * I.nbins, I.cx, I.cy);
    else return I.vecs[j];
  };
  const bool tiled = I.ntiles > 1;
  for (int t_id = 0; t_id < I.ntiles; ++t_id) {
    const int Y0 = t_id * I.tile;
    const int rows_here = min(I.tile, I.H - Y0);
    if (t_id) __syncthreads();  // every wave is done with the previous tile
    // Stage rows Y0 .. Y0 + lds_rows - 1 (mod H) of E.
    for (int i = threadIdx.x; i < I.lds_rows * I.we; i += blockDim.x) {
      const int r = i / I.we;
      const int e = i - r * I.we;
      const int y = (Y0 + r) % I.H;
      lds[r * I.rst + e] = I.E[(size_t)y * I.we + e];
    }
    __syncthreads();
    const int nbands = (rows_here + rpw - 1) / rpw;
    for (int j = vb; j < ve; ++j) {
      const VecDesc v = vec_at(j);
      const int dx = v.dx, dy = v.dy;
      const int adx = dx < 0 ? -dx : dx;
      const int n = adx > dy ? adx : dy;
      const bool xm = adx >= dy;
      const int m = xm ? dy : adx;
      uint32_t c0 = 0, c1 = 0;
      for (int band = 0; band < nbands; ++band) {
        const int row = band * rpw + r_in;
        const uint32_t *base = lds + row * I.rst + strip * R;
        const bool row_ok = row < rows_here;
        uint32_t A[R], O[R], mk[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
          A[i] = 0xffffffffu;
          O[i] = 0u;
          const int w = strip * R + i;
          const uint32_t mw = (w < swd - 1) ? 0xffffffffu : (w == swd - 1 ? lastmask : 0u);
          mk[i] = row_ok ? mw : 0u;
        }
        if (I.sample && row_ok) {
          // Monte-Carlo approximation: only start pixels of the position set count.  Lane bit b
          // of word w stands for the placement whose first pixel is 32w + b (+ |dx| for a
          // mirrored vector), so the set's extended row is read at that shift.
          const uint32_t *srow = I.sample + (size_t)(Y0 + row) * I.sample_stride + strip * R;
          const int so = dx < 0 ? (adx >> 5) : 0, ssh = dx < 0 ? (adx & 31) : 0;
#pragma unroll
          for (int i = 0; i < R; ++i)
            mk[i] &= __builtin_amdgcn_alignbit(srow[so + i + 1], srow[so + i], ssh);
        }
        if (xm) {
          if (dx < 0) path_product<R, true, true, SKIP>(base, I.rst, adx, n, m, A, O, mk, phase_mask);
          else path_product<R, true, false, SKIP>(base, I.rst, adx, n, m, A, O, mk, phase_mask);
        } else {
          if (dx < 0) path_product<R, false, true, SKIP>(base, I.rst, adx, n, m, A, O, mk, phase_mask);
          else path_product<R, false, false, SKIP>(base, I.rst, adx, n, m, A, O, mk, phase_mask);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
          c1 += __popc(A[i] & mk[i]);
          c0 += __popc(~O[i] & mk[i]);
        }
      }
      c0 = wave_sum(c0);
      c1 = wave_sum(c1);
      if (lane == 0) {
        if (!tiled) {
          int p = 0;
          if (phase_mask & 1) put_count(I, p++, v.idx, dx, dy, c0);
          if (phase_mask & 2) put_count(I, p, v.idx, dx, dy, c1);
        } else {
          uint32_t *slot = cnt + 2 * (wave * kMaxBin + (j - vb));
          slot[0] = t_id ? slot[0] + c0 : c0;
          slot[1] = t_id ? slot[1] + c1 : c1;
        }
      }
    }
  }
  if (tiled && lane == 0) {
    for (int j = vb; j < ve; ++j) {
      const VecDesc v = vec_at(j);
      const uint32_t *slot = cnt + 2 * (wave * kMaxBin + (j - vb));
      int p = 0;
      if (phase_mask & 1) put_count(I, p++, v.idx, v.dx, v.dy, slot[0]);
      if (phase_mask & 2) put_count(I, p, v.idx, v.dx, v.dy, slot[1]);
    }
  }
}

// One image, one workgroup per work item (item = blockIdx.x).
template <int R, bool SKIP>
__global__ void __launch_bounds__(1024)
k_lpf_full(FullImg I, int wpg, unsigned phase_mask, int cnt_off) {
  extern __shared__ uint32_t lds[];
  process_item<R, SKIP>(I, blockIdx.x * wpg, wpg, phase_mask, lds, lds + cnt_off);
}

// One image without a vector table (canonical vectors interleaved over the waves).
template <int R>
__global__ void __launch_bounds__(1024)
k_lpf_full_canon(FullImg I, int wpg, unsigned phase_mask, int cnt_off) {
  extern __shared__ uint32_t lds[];
  process_item<R, false, true>(I, blockIdx.x * wpg, wpg, phase_mask, lds, lds + cnt_off);
}

// Many images, persistent workgroups drawing work items from a device counter in descending
// cost order until the list is exhausted (every wave reaches the exit test).
__global__ void __launch_bounds__(1024)
k_lpf_batch(const FullImg *__restrict__ imgs, const int2 *__restrict__ items, int n_items,
            int *__restrict__ counter, int wpg, unsigned phase_mask, int cnt_off) {
  extern __shared__ uint32_t lds[];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= n_items) break;
    const int2 w = items[it];
    const FullImg I = imgs[w.x];
    switch (I.R) {
      case 1: process_item<1, false>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
      case 2: process_item<2, false>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
      case 4: process_item<4, false>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
      case 8: process_item<8, false>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
      default: process_item<16, false>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
    }
    __syncthreads();  // the item's last tile is no longer read before the next staging
  }
}

__global__ void k_reset_counter(int *counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = 0;
}

size_t full_lds_bytes(const FullShape &sh, int wpg) {
  size_t b = (size_t)sh.lds_rows * sh.rst * sizeof(uint32_t);
  if (sh.ntiles > 1) b += (size_t)wpg * kMaxBin * 2 * sizeof(uint32_t);
  return b;
}

template <int R, bool SKIP>
static hipError_t launch_full_r(const FullImg &I, const FullShape &sh, unsigned phase_mask,
                                hipStream_t stream) {
  const int nwg = sh.nbins / sh.wpg;
  const size_t lds = full_lds_bytes(sh, sh.wpg);
  const int cnt_off = sh.lds_rows * sh.rst;
  hipLaunchKernelGGL((k_lpf_full<R, SKIP>), dim3(nwg), dim3(64 * sh.wpg), lds, stream, I, sh.wpg,
                     phase_mask, cnt_off);
  return hipGetLastError();
}

template <bool SKIP>
static hipError_t launch_full_s(const FullImg &I, const FullShape &sh, unsigned phase_mask,
                                hipStream_t stream) {
  switch (sh.R) {
    case 1: return launch_full_r<1, SKIP>(I, sh, phase_mask, stream);
    case 2: return launch_full_r<2, SKIP>(I, sh, phase_mask, stream);
    case 4: return launch_full_r<4, SKIP>(I, sh, phase_mask, stream);
    case 8: return launch_full_r<8, SKIP>(I, sh, phase_mask, stream);
    case 16: return launch_full_r<16, SKIP>(I, sh, phase_mask, stream);
    default: return hipErrorInvalidValue;
  }
}

template <int R>
static hipError_t launch_canon_r(const FullImg &I, const FullShape &sh, unsigned phase_mask,
                                 hipStream_t stream) {
  const int nwg = sh.nbins / sh.wpg;
  const size_t lds = full_lds_bytes(sh, sh.wpg);
  const int cnt_off = sh.lds_rows * sh.rst;
  hipLaunchKernelGGL((k_lpf_full_canon<R>), dim3(nwg), dim3(64 * sh.wpg), lds, stream, I,
                     sh.wpg, phase_mask, cnt_off);
  return hipGetLastError();
}

hipError_t launch_full_canon(const FullImg &I, const FullShape &sh, unsigned phase_mask,
                             hipStream_t stream) {
  switch (sh.R) {
    case 1: return launch_canon_r<1>(I, sh, phase_mask, stream);
    case 2: return launch_canon_r<2>(I, sh, phase_mask, stream);
    case 4: return launch_canon_r<4>(I, sh, phase_mask, stream);
    case 8: return launch_canon_r<8>(I, sh, phase_mask, stream);
    case 16: return launch_canon_r<16>(I, sh, phase_mask, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_full(const FullImg &I, const FullShape &sh, unsigned phase_mask, bool skip,
                       hipStream_t stream) {
  return skip ? launch_full_s<true>(I, sh, phase_mask, stream)
              : launch_full_s<false>(I, sh, phase_mask, stream);
}

hipError_t launch_batch(const FullImg *imgs, const int2 *items, int n_items, int *counter,
                        int wpg, unsigned phase_mask, size_t lds_bytes, int cnt_off, int n_wg,
                        hipStream_t stream) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, stream, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lpf_batch, dim3(n_wg), dim3(64 * wpg), lds_bytes, stream, imgs, items,
                     n_items, counter, wpg, phase_mask, cnt_off);
  return hipGetLastError();
}

// E for many images in one launch: image b's rows at ext_off[b], we[b] dwords per row.
__global__ void k_ext_batch(const FullImg *__restrict__ imgs, const uint64_t *__restrict__ pool,
                            const int64_t *__restrict__ bits_off, uint32_t *__restrict__ ext,
                            const int64_t *__restrict__ ext_off) {
  const int b = blockIdx.z;
  const FullImg I = imgs[b];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (e >= I.we || y >= I.H) return;
  const uint32_t *row = reinterpret_cast<const uint32_t *>(pool + bits_off[b]) +
                        (size_t)y * 2 * ((I.W + 63) / 64);
  const int W = I.W;
  const int s = (int)(((int64_t)32 * e) % W);
  uint32_t v;
  if (s + 32 <= W) {
    const int q = s >> 5, sh = s & 31;
    v = __builtin_amdgcn_alignbit(sh ? row[q + 1] : 0u, row[q], sh);
  } else {
    v = 0;
    int x = s;
    for (int t = 0; t < 32; ++t) {
      v |= ((row[x >> 5] >> (x & 31)) & 1u) << t;
      x = (x + 1 == W) ? 0 : x + 1;
    }
  }
  ext[ext_off[b] + (size_t)y * I.we + e] = v;
}

hipError_t launch_ext_batch(const FullImg *imgs, int n_images, int max_we, int max_h,
                            const uint64_t *pool, const int64_t *bits_off, uint32_t *ext,
                            const int64_t *ext_off, hipStream_t stream) {
  dim3 grid((max_we + 63) / 64, max_h, n_images);
  hipLaunchKernelGGL(k_ext_batch, grid, dim3(64), 0, stream, imgs, pool, bits_off, ext, ext_off);
  return hipGetLastError();
}

hipError_t prepare_full_kernels(int max_lds_bytes) {
  hipError_t e = hipSuccess;
  const void *fns[] = {(const void *)k_lpf_full<1, false>, (const void *)k_lpf_full<2, false>,
                       (const void *)k_lpf_full<4, false>, (const void *)k_lpf_full<8, false>,
                       (const void *)k_lpf_full<16, false>, (const void *)k_lpf_full<1, true>,
                       (const void *)k_lpf_full<2, true>, (const void *)k_lpf_full<4, true>,
                       (const void *)k_lpf_full<8, true>, (const void *)k_lpf_full<16, true>,
                       (const void *)k_lpf_full_canon<1>, (const void *)k_lpf_full_canon<2>,
                       (const void *)k_lpf_full_canon<4>, (const void *)k_lpf_full_canon<8>,
                       (const void *)k_lpf_full_canon<16>};
  for (const void *f : fns) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
    if (r != hipSuccess) e = r;
  }
  // the batch kernel also holds one static LDS word
  hipError_t r = hipFuncSetAttribute((const void *)k_lpf_batch,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     max_lds_bytes - kBatchStaticLds);
  if (r != hipSuccess) e = r;
  return e;
}

}  // namespace lpf
