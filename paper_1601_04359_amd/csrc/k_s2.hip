// Two-point probability (Sec. 2.1, eq. (S2dis)) on gfx950: full evaluation over the canonical
// half domain, its change under a pixel interchange, and the annealing rounds that use it as the
// descriptor (the comparison of Secs. 5 and 6.1).
//
// Counts, not probabilities: C_p(v) = W H S2^p(v) = #{x : I(x) = p and I(x + v) = p} on the
// periodic image.  The paper evaluates S2 with the FFT over all W x H shifts; over a cutoff
// domain the direct count is exact in integers and costs one AND and one popcount per 32 start
// pixels and vector, so it is done that way here:
//   - a lane owns a family of up to J vectors (dx0 + 32 j, dy) and walks its wave's share of the
//     workgroup's row block (the four waves of a workgroup share 64 families); for start word w of row y it forms t = bits [32w + s, 32w + s + 32)
//     of row y + dy of the extended image (s = dx0 + W, one v_alignbit_b32), which is also member
//     j's shifted word at w - j, and adds popcount(row_y[w] & t) into the members' counters;
//   - row_y[w] is the same for every lane (an LDS broadcast), the shifted words are gathers from
//     LDS; families are sorted by dy so that one workgroup needs few distinct rows;
//   - phase 0 follows from eq. (S2add) in counts, C_0(v) = N - 2 N_1 + C_1(v), with
//     N_1 = C_1(0) (v = 0 is the first vector of the canonical order).
//
// Under the interchange of a (phase 1 -> 0) and b (phase 0 -> 1), with I the image before it,
//   dC_1(v) = -I(a + v) - I(a - v) + I(b + v) + I(b - v) + 2 [v = 0] - [v = b - a] - [v = a - b]
// (indices mod (W, H)): the pairs (x, x + v) that contain a or b, with the last three terms for
// the pairs that contain both.  N_1 does not change, so dC_0 = dC_1.
#include <limits.h>

#include "step_dev.h"

namespace lpf {

// ------------------------------------------------------------------------ full evaluation

// Phase-1 counts over start rows [y0, y0 + rb), y0 = blockIdx.y * rb, for the vector families of
// group blockIdx.x (at most 64: one per lane), added into acc (integer atomics: the sum does not
// depend on the order).  The workgroup's waves share the families and split the rows (wave w
// takes rows w, w + waves, ...); their counts are summed in LDS before one atomic per member.
// A family {dx0, dy, nj} is the vectors (dx0 + 32 j, dy), j < nj <= J, of one lane: with
// s = dx0 + W (the same pairs as dx0 on the periodic image) member j's shifted word at start word
// w is the family's shifted word at w + j, so one v_alignbit_b32 per word serves all J members.
// group = {first family, end, dy of the first, dy of the last}, families sorted by dy.
// LDS: A = the block's rows (swdp dwords each, zero past W), B = rows y0 + dy_lo ..
// y0 + dy_hi + rb - 1 (mod H) extended periodically to we dwords (ext_word, from the packed
// image P, src_stride dwords per row), rstB dwords apart, then the reduction.
// Word e of the periodic extension of a packed row (row32: the row as 32-bit words): bits
// [32 e, 32 e + 32) taken modulo W.
__device__ __forceinline__ uint32_t ext_word(const uint32_t *__restrict__ row32, int W, int e) {
  const int s = (32 * e) % W;
  if (s + 32 <= W) {
    const int q = s >> 5, sh = s & 31;
    return __builtin_amdgcn_alignbit(sh ? row32[q + 1] : 0u, row32[q], (uint32_t)sh);
  }
  uint32_t v = 0;
  int x = s;
  for (int b = 0; b < 32; ++b) {
    v |= ((row32[x >> 5] >> (x & 31)) & 1u) << b;
    x = x + 1 == W ? 0 : x + 1;
  }
  return v;
}

template <int J>
__global__ void __launch_bounds__(256)
k_s2_full(const uint32_t *__restrict__ P, int src_stride, int W, int H, int we, int swd, int swdp,
          int rb,
          int rstB, int cx, int q1, const int4 *__restrict__ fams,
          const int4 *__restrict__ groups, uint32_t *__restrict__ acc) {
  constexpr int CW = 8;  // start words per chunk (swdp is a multiple of CW)
  extern __shared__ uint32_t lds[];
  const int4 g = groups[blockIdx.x];
  const int y0 = blockIdx.y * rb;
  const int rows = min(rb, H - y0);
  const int nB = rows + g.w - g.z;
  const int span = g.w - g.z;
  uint32_t *A = lds;
  uint32_t *B = lds + rb * swdp;
  const uint32_t lastmask = (W & 31) ? ((1u << (W & 31)) - 1u) : 0xffffffffu;
  for (int i = threadIdx.x; i < rows * swdp; i += blockDim.x) {
    const int r = i / swdp, w = i - r * swdp;
    uint32_t v = w < swd ? P[(size_t)(y0 + r) * src_stride + w] : 0u;
    if (w == swd - 1) v &= lastmask;
    A[i] = v;
  }
  for (int i = threadIdx.x; i < nB * we; i += blockDim.x) {
    const int r = i / we, e = i - r * we;
    const int y = (y0 + g.z + r) % H;
    B[r * rstB + e] = ext_word(P + (size_t)y * src_stride, W, e);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  const int f = g.x + lane;
  const bool live = f < g.y;
  const int4 fm = live ? fams[f] : make_int4(0, g.z, 0, 0);
  uint32_t c[J];
#pragma unroll
  for (int jj = 0; jj < J; ++jj) c[jj] = 0;
  if (live) {
    const int s0 = fm.x + W;
    const int sh = s0 & 31;
    const uint32_t *b = B + (fm.y - g.z) * rstB + (s0 >> 5);
    for (int r = wave; r < rows; r += waves) {
      const uint32_t *a = A + r * swdp;
      const uint32_t *bb = b + r * rstB;
      for (int w0 = 0; w0 < swdp; w0 += CW) {
        uint32_t av[CW], d[CW + J], t[CW + J - 1];
#pragma unroll
        for (int i = 0; i < CW; ++i) av[i] = a[w0 + i];
#pragma unroll
        for (int k = 0; k < CW + J; ++k) d[k] = bb[w0 + k];
#pragma unroll
        for (int k = 0; k < CW + J - 1; ++k) t[k] = __builtin_amdgcn_alignbit(d[k + 1], d[k], sh);
#pragma unroll
        for (int jj = 0; jj < J; ++jj)
#pragma unroll
          for (int i = 0; i < CW; ++i) c[jj] += __popc(av[i] & t[i + jj]);
      }
    }
  }
  // sum the waves' counts of each family member in LDS (after the staged rows)
  uint32_t *red = B + (rb + span) * rstB;
#pragma unroll
  for (int jj = 0; jj < J; ++jj) red[(wave * J + jj) * 64 + lane] = c[jj];
  __syncthreads();
  if (wave == 0 && live) {
#pragma unroll
    for (int jj = 0; jj < J; ++jj) {
      uint32_t sum = 0;
      for (int w = 0; w < waves; ++w) sum += red[(w * J + jj) * 64 + lane];
      if (jj < fm.z && sum) {
        const int dx = fm.x + 32 * jj, dy = fm.y;
        const int idx = dx >= 0 ? dy * (cx + 1) + dx : q1 + (dy - 1) * cx + (dx + cx);
        atomicAdd(&acc[idx], sum);
      }
    }
  }
}

// Canonical vector i of the half domain with cutoff (cx, cy): the rectangle [0,cx] x [0,cy] row
// by row, then [-cx,-1] x [1,cy] row by row.
__device__ __forceinline__ void canonical_vector(int64_t i, int cx, int cy, int &dx, int &dy) {
  const int64_t q1 = (int64_t)(cx + 1) * (cy + 1);
  if (i < q1) {
    dy = (int)(i / (cx + 1));
    dx = (int)(i - (int64_t)dy * (cx + 1));
  } else {
    const int64_t j = i - q1;
    const int r = (int)(j / cx);
    dy = 1 + r;
    dx = -cx + (int)(j - (int64_t)r * cx);
  }
}

// Output layout from the phase-1 sums: HALF counts[p][i]; GRID counts[p][dy+cy][dx+cx] with the
// entry of -v equal to that of v (C(-v) = C(v) on a periodic image).  Also clears the other
// accumulator (ncap entries) for the next call, so that no launch zeroes acc before the counts.
__global__ void k_s2_finish(const uint32_t *__restrict__ acc, int64_t nv, int cx, int cy,
                            int64_t N, unsigned phase_mask, int layout,
                            uint32_t *__restrict__ out, uint32_t *__restrict__ clear,
                            int64_t ncap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncap) clear[i] = 0;
  if (i >= nv) return;
  const uint32_t c1 = acc[i];
  const uint32_t c0 = (uint32_t)(N - 2 * (int64_t)acc[0] + (int64_t)c1);
  int p = 0;
  uint32_t val[2];
  if (phase_mask & 1u) val[p++] = c0;
  if (phase_mask & 2u) val[p++] = c1;
  if (layout == 0) {
    for (int q = 0; q < p; ++q) out[(size_t)q * nv + i] = val[q];
  } else {
    int dx, dy;
    canonical_vector(i, cx, cy, dx, dy);
    const int gw = 2 * cx + 1;
    const size_t gs = (size_t)gw * (2 * cy + 1);
    for (int q = 0; q < p; ++q) {
      out[q * gs + (size_t)(dy + cy) * gw + (dx + cx)] = val[q];
      out[q * gs + (size_t)(cy - dy) * gw + (cx - dx)] = val[q];
    }
  }
}

hipError_t launch_s2_full(const S2Launch &L, hipStream_t stream) {
  hipError_t e;
  const dim3 grid((unsigned)L.ngroups, (unsigned)L.nrb);
  const int q1 = (L.cx + 1) * (L.cy + 1);
#define LPF_S2_FULL(JJ)                                                                        \
  hipLaunchKernelGGL((k_s2_full<JJ>), grid, dim3(256), L.lds_bytes, stream, L.E,                \
                     2 * ((L.W + 63) / 64), L.W, L.H, L.we,                                     \
                     L.swd, L.swdp, L.rb, L.rstB, L.cx, q1, L.fams, L.groups, L.acc)
  switch (L.J) {
    case 1: LPF_S2_FULL(1); break;
    case 2: LPF_S2_FULL(2); break;
    case 4: LPF_S2_FULL(4); break;
    case 8: LPF_S2_FULL(8); break;
    default: return hipErrorInvalidValue;
  }
#undef LPF_S2_FULL
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t nf = std::max(L.nv, L.ncap);
  hipLaunchKernelGGL(k_s2_finish, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, stream,
                     L.acc, L.nv, L.cx, L.cy, (int64_t)L.W * L.H, L.phase_mask, L.layout, L.out,
                     L.clear, L.ncap);
  return hipGetLastError();
}

// ------------------------------------------------------------------ interchange update

// Pixel (x, y) of the packed image (64-bit words, wpr per row) read as 32-bit words.
__device__ __forceinline__ int s2_pixel(const uint32_t *__restrict__ img, int wpr32, int x, int y) {
  return (int)((img[y * wpr32 + (x >> 5)] >> (x & 31)) & 1u);
}

__device__ __forceinline__ int wrap1(int v, int n) {  // v in (-n, 2n)
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

__device__ __forceinline__ bool same_mod(int u, int n) {  // u in (-2n, 2n): u = 0 mod n
  return u == 0 || u == n || u == -n;
}

// dC_1(v) (= dC_0(v)) for the interchange (a, b), a in phase 1, b in phase 0, given as
// coordinates with r = b - a.
__device__ __forceinline__ int s2_vector_delta(const uint32_t *__restrict__ img, int wpr32, int W,
                                               int H, int ax, int ay, int bx, int by, int dx,
                                               int dy) {
  int d = -s2_pixel(img, wpr32, wrap1(ax + dx, W), wrap1(ay + dy, H)) -
          s2_pixel(img, wpr32, wrap1(ax - dx, W), wrap1(ay - dy, H)) +
          s2_pixel(img, wpr32, wrap1(bx + dx, W), wrap1(by + dy, H)) +
          s2_pixel(img, wpr32, wrap1(bx - dx, W), wrap1(by - dy, H));
  const int rx = bx - ax, ry = by - ay;
  if (dx == 0 && dy == 0) d += 2;
  if (same_mod(dx - rx, W) && same_mod(dy - ry, H)) d -= 1;
  if (same_mod(dx + rx, W) && same_mod(dy + ry, H)) d -= 1;
  return d;
}

// Checks interchange (a, b) (both inside the image, distinct, of different phases) and returns
// it as coordinates with a the phase-1 pixel; false (and zero coordinates) otherwise.
__device__ __forceinline__ bool s2_candidate(const uint32_t *__restrict__ img, int wpr32, int W,
                                             int H, int a, int b, int &ax, int &ay, int &bx,
                                             int &by) {
  ax = ay = bx = by = 0;
  const int64_t N = (int64_t)W * H;
  if (a < 0 || b < 0 || a >= N || b >= N || a == b) return false;
  int y0 = a / W, x0 = a - y0 * W, y1 = b / W, x1 = b - y1 * W;
  const int va = s2_pixel(img, wpr32, x0, y0), vb = s2_pixel(img, wpr32, x1, y1);
  if (va == vb) return false;
  if (va == 0) {  // b is the phase-1 pixel
    ax = x1; ay = y1; bx = x0; by = y0;
  } else {
    ax = x0; ay = y0; bx = x1; by = y1;
  }
  return true;
}

// delta[s][p][i] for n interchanges (one thread per interchange and vector chunk).
__global__ void __launch_bounds__(256)
k_s2_delta(const uint64_t *__restrict__ bits, int W, int H, const int2 *__restrict__ swaps, int n,
           const int32_t *__restrict__ vec, int64_t nv, int nchunks, unsigned phase_mask,
           int32_t *__restrict__ delta) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int wpr32 = 2 * ((W + 63) >> 6);
  const uint32_t *img = reinterpret_cast<const uint32_t *>(bits);
  const int2 ab = swaps[s];
  const int nph = (int)(phase_mask & 1u) + (int)((phase_mask >> 1) & 1u);
  const int64_t v0 = nv * blockIdx.y / nchunks, v1 = nv * (blockIdx.y + 1) / nchunks;
  int32_t *out = delta + (size_t)s * nph * nv;
  int ax, ay, bx, by;
  const bool swap_ok = s2_candidate(img, wpr32, W, H, ab.x, ab.y, ax, ay, bx, by);
  for (int64_t i = v0; i < v1; ++i) {
    const int pk = vec[i];
    const int dx = (int)(int16_t)(pk & 0xffff), dy = (int)((uint32_t)pk >> 16);
    const int d = swap_ok ? s2_vector_delta(img, wpr32, W, H, ax, ay, bx, by, dx, dy) : 0;
    for (int p = 0; p < nph; ++p) out[(size_t)p * nv + i] = d;
  }
}

hipError_t launch_s2_delta(const uint64_t *bits, int W, int H, const int2 *swaps, int n,
                           const int32_t *vec, int64_t nv, unsigned phase_mask, int32_t *delta,
                           hipStream_t stream) {
  const int nchunks = (int)std::min<int64_t>(std::max<int64_t>(1, nv / 64), 64);
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)nchunks);
  hipLaunchKernelGGL(k_s2_delta, grid, dim3(256), 0, stream, bits, W, H, swaps, n, vec, nv,
                     nchunks, phase_mask, delta);
  return hipGetLastError();
}

// ------------------------------------------------------------------ annealing rounds

// One round of an annealing step with S2 as the descriptor: candidate = thread, vectors of chunk
// blockIdx.y; the image is staged in LDS when LDS is set.  Same protocol as the lineal path
// rounds: exact int64 energy sums into S_acc, dC per (term, candidate) into dl.
template <bool LDS>
__global__ void __launch_bounds__(256)
k_s2_round(const uint64_t *__restrict__ bits, int W, int H, const int2 *__restrict__ cand, int K,
           int k0, int C, const int32_t *__restrict__ vec, int nv, int nchunks,
           unsigned phase_mask, const uint32_t *__restrict__ counts,
           const uint32_t *__restrict__ target, int64_t N, int64_t Nt, int64_t *__restrict__ S_acc,
           int16_t *__restrict__ dl, StepCtl *__restrict__ ctl, const int32_t *__restrict__ order,
           const double *__restrict__ U, const double *__restrict__ Tp, int pi0, int pC) {
  extern __shared__ uint32_t lds[];
  __shared__ int s_prev;
  if (prev_round_accepted(S_acc, nullptr, cand, U, order, pi0, pC, Tp,
                          (double)N * (double)N * (double)Nt, ctl, &s_prev))
    return;
  const int wpr32 = 2 * ((W + 63) >> 6);
  const uint32_t *img = reinterpret_cast<const uint32_t *>(bits);
  if constexpr (LDS) {
    for (int i = threadIdx.x; i < H * wpr32; i += blockDim.x) lds[i] = img[i];
    __syncthreads();
    img = lds;
  }
  const int kr = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = k0 + kr;
  const bool ok = kr < C && i < K;
  const int k = ok && order ? order[i] : i;
  int a = -1, b = -1;
  if (ok) {
    const int2 ab = cand[k];
    a = ab.x;
    b = ab.y;
  }
  int ax = 0, ay = 0, bx = 0, by = 0;
  const bool live = ok && s2_candidate(img, wpr32, W, H, a, b, ax, ay, bx, by);
  const int v0 = (int)((int64_t)nv * blockIdx.y / nchunks);
  const int v1 = (int)((int64_t)nv * (blockIdx.y + 1) / nchunks);
  int64_t S = 0;
  for (int j = v0; j < v1; ++j) {
    const int pk = vec[j];
    const int dx = (int)(int16_t)(pk & 0xffff), dy = (int)((uint32_t)pk >> 16);
    const int d = live ? s2_vector_delta(img, wpr32, W, H, ax, ay, bx, by, dx, dy) : 0;
    int p = 0;
    if (phase_mask & 1u) {
      const size_t t = (size_t)p * nv + j;
      S += energy_term(d, counts[t], target[t], N, Nt);
      if (ok && dl) dl[t * K + k] = (int16_t)d;
      ++p;
    }
    if (phase_mask & 2u) {
      const size_t t = (size_t)p * nv + j;
      S += energy_term(d, counts[t], target[t], N, Nt);
      if (ok && dl) dl[t * K + k] = (int16_t)d;
    }
  }
  if (ok) add_acc(&S_acc[k], S);
}

hipError_t launch_s2_round(const StepLaunch &L, const RoundPlan &r, bool decide,
                           hipStream_t stream) {
  dim3 grid((unsigned)((r.C + r.block - 1) / r.block), (unsigned)r.nchunks);
  int16_t *dl = decide ? L.dl : nullptr;
  const int pi0 = decide ? r.pi0 : 0, pC = decide ? r.pC : 0;
  const size_t img_bytes = (size_t)L.H * ((L.W + 63) >> 6) * sizeof(uint64_t);
  if (L.use_lds)
    hipLaunchKernelGGL(k_s2_round<true>, grid, dim3(r.block), img_bytes, stream, L.bits, L.W, L.H,
                       L.cand, L.K, r.k0, r.C, L.s2vec, L.nv, r.nchunks, L.phase_mask, L.counts,
                       L.target, L.N, L.Nt, L.S_acc, dl, L.ctl, L.order, L.U, L.T, pi0, pC);
  else
    hipLaunchKernelGGL(k_s2_round<false>, grid, dim3(r.block), 0, stream, L.bits, L.W, L.H,
                       L.cand, L.K, r.k0, r.C, L.s2vec, L.nv, r.nchunks, L.phase_mask, L.counts,
                       L.target, L.N, L.Nt, L.S_acc, dl, L.ctl, L.order, L.U, L.T, pi0, pC);
  return hipGetLastError();
}

// The round kernel stages at most a 64 KiB cell (it also holds a static LDS word); the full
// evaluation may stage up to max_lds_bytes.
hipError_t prepare_s2_kernels(int max_lds_bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)k_s2_round<true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
  const void *full[] = {(const void *)k_s2_full<1>, (const void *)k_s2_full<2>,
                        (const void *)k_s2_full<4>, (const void *)k_s2_full<8>};
  for (const void *fn : full) {
    hipError_t r = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       max_lds_bytes);
    if (e == hipSuccess) e = r;
  }
  return e;
}

}  // namespace lpf
