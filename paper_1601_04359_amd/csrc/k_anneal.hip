// Device-resident simulated annealing on the lineal path function (Sec. 4, Alg. "annealing",
// objective eq. (LSE)).  One step: K candidate pixel interchanges are drawn (here), their exact
// energy changes are evaluated against the current state in evaluation order (draw order, or the
// learned ranking of k_propose / k_rank_merge) and the first candidate that passes the Metropolis test is applied
// (k_step.hip).  Rejected candidates leave the state unchanged, so this is the sequential chain
// of the algorithm over those draws with the step's later candidates unused.  Nothing returns to
// the host inside a step.
//
// Energy: e = sum_{i,v} (T_i(v)/Nt - L_i(v)/N)^2 over the phases of the mask and the canonical
// half domain, T = target counts over Nt pixels, L = current counts over N = W*H pixels.  The
// change of one interchange is exact in integers,
//     S = sum dL * (Nt * (dL + 2 L) - 2 N T),   de = S / (N^2 Nt),
// and converted to double once, so it does not depend on summation order.
#include <limits.h>
#include <math.h>

#include "draw_dev.h"
#include "rank_dev.h"
#include "lpf_internal.h"

namespace lpf {

// Draws of a step (draw_dev.h), plus the learned ranking's keys and workgroup lists when
// p.rank_score is given (the condition is workgroup-uniform).
__global__ void __launch_bounds__(256) k_propose(ProposeArgs p) {
  __shared__ uint64_t sl[2][64];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  int a = -1, b = -1;
  propose_draw(p, k, a, b);
  if (p.rank_score && (int)(blockIdx.x * blockDim.x) < min(p.K, kRankMax)) {
    const bool ranked = k < min(p.K, kRankMax);
    const uint64_t key = ranked ? rank_key(a, b, k, p.rank_score) : 0ull;
    if (ranked) p.rank_keys[k] = key;
    block_top64(key, sl, p.rank_lists + (size_t)blockIdx.x * kRankTop);
  }
}

// Inclusive prefix sums of w(p) = exp(clamp(beta * score[p], -60, 60)) over the pixel lists
// pos1 (into cw1) and pos0 (into cw0), in a fixed order: scans of 1024-entry blocks
// (k_learn_block), a scan of the block totals (k_learn_scan), block offsets added (k_learn_add).
// Blocks (b, list) past the list's length exit at once.
__device__ __forceinline__ double block_scan_1024(double x, double *wtot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wtot[wave] = x;
  __syncthreads();
  if (wave == 0) {
    double t = lane < 16 ? wtot[lane] : 0.0;
    for (int o = 1; o < 16; o <<= 1) {
      const double y = __shfl_up(t, o);
      if (lane >= o) t += y;
    }
    if (lane < 16) wtot[lane] = t;
  }
  __syncthreads();
  return x + (wave ? wtot[wave - 1] : 0.0);
}

__global__ void __launch_bounds__(1024)
k_learn_block(const AnnealDev *__restrict__ st, const float *__restrict__ score, double beta,
              double *__restrict__ cw1, double *__restrict__ cw0, double *__restrict__ bsum,
              int nb) {
  __shared__ double wtot[16];
  const int list = blockIdx.y;
  const int n = list == 0 ? st->n1 : st->n0;
  const int64_t i0 = (int64_t)blockIdx.x * 1024;
  if (i0 >= n) return;
  const int32_t *pos = list == 0 ? st->pos1 : st->pos0;
  double *cw = list == 0 ? cw1 : cw0;
  const int64_t i = i0 + threadIdx.x;
  double w = 0.0;
  if (i < n) w = exp(fmin(60.0, fmax(-60.0, beta * (double)score[pos[i]])));
  const double incl = block_scan_1024(w, wtot);
  if (i < n) cw[i] = incl;
  if (threadIdx.x == 1023) bsum[(size_t)list * nb + blockIdx.x] = incl;
}

// Exclusive scan of the block totals of one list (one wave per list): contiguous ranges per
// lane, then a scan of the lane totals.
__global__ void __launch_bounds__(64)
k_learn_scan(const AnnealDev *__restrict__ st, const double *__restrict__ bsum,
             double *__restrict__ boff, int nb) {
  const int list = blockIdx.x;
  const int n = list == 0 ? st->n1 : st->n0;
  const int m = (n + 1023) / 1024;
  const int lane = threadIdx.x;
  const int per = (m + 63) / 64;
  const int lo = min(m, per * lane), hi = min(m, lo + per);
  const double *bs = bsum + (size_t)list * nb;
  double *bo = boff + (size_t)list * nb;
  double s = 0.0;
  for (int b = lo; b < hi; ++b) s += bs[b];
  double x = s;
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  double run = x - s;
  for (int b = lo; b < hi; ++b) {
    bo[b] = run;
    run += bs[b];
  }
}

__global__ void __launch_bounds__(1024)
k_learn_add(const AnnealDev *__restrict__ st, double *__restrict__ cw1, double *__restrict__ cw0,
            const double *__restrict__ boff, int nb) {
  const int list = blockIdx.y;
  const int n = list == 0 ? st->n1 : st->n0;
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (blockIdx.x == 0 || i >= n) return;
  double *cw = list == 0 ? cw1 : cw0;
  cw[i] += boff[(size_t)list * nb + blockIdx.x];
}

// Pixel lists in ascending index order (one workgroup; each thread scans a contiguous range).
__global__ void __launch_bounds__(1024)
k_init_lists(AnnealDev *__restrict__ st, const uint64_t *__restrict__ bits, int W, int H) {
  __shared__ int ones[1024];
  const int64_t N = (int64_t)W * H;
  const int wpr = (W + 63) >> 6;
  const int64_t per = (N + blockDim.x - 1) / blockDim.x;
  const int64_t lo = min<int64_t>(N, per * threadIdx.x), hi = min<int64_t>(N, lo + per);
  int c = 0;
  for (int64_t q = lo; q < hi; ++q) {
    const int y = (int)(q / W), x = (int)(q - (int64_t)y * W);
    c += bit_at(bits, wpr, x, y);
  }
  ones[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      const int v = ones[t];
      ones[t] = run;
      run += v;
    }
    st->n1 = run;
    st->n0 = (int)(N - run);
  }
  __syncthreads();
  int o1 = ones[threadIdx.x];
  int o0 = (int)lo - o1;
  for (int64_t q = lo; q < hi; ++q) {
    const int y = (int)(q / W), x = (int)(q - (int64_t)y * W);
    if (bit_at(bits, wpr, x, y)) st->pos1[o1++] = (int)q;
    else st->pos0[o0++] = (int)q;
  }
}

// eq. (LSE) in canonical order (one thread, fixed order).
__global__ void k_lse(const uint32_t *__restrict__ counts, const uint32_t *__restrict__ target,
                      int64_t nterms, int64_t N, int64_t Nt, double *__restrict__ e) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int64_t j = 0; j < nterms; ++j) {
    const double d = (double)(N * (int64_t)target[j] - Nt * (int64_t)counts[j]);
    s += d * d;
  }
  *e = s / ((double)N * (double)N * (double)Nt * (double)Nt);
}

hipError_t launch_propose(const ProposeArgs &p, hipStream_t stream) {
  hipLaunchKernelGGL(k_propose, dim3((p.K + 255) / 256), dim3(256), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_learn_weights(const AnnealDev *st, const float *score, double beta, double *cw1,
                                double *cw0, int64_t N, double *scratch, hipStream_t stream) {
  const int nb = (int)((N + 1023) / 1024);
  double *bsum = scratch, *boff = scratch + 2 * (size_t)nb;
  hipLaunchKernelGGL(k_learn_block, dim3((unsigned)nb, 2), dim3(1024), 0, stream, st, score, beta,
                     cw1, cw0, bsum, nb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_learn_scan, dim3(2), dim3(64), 0, stream, st, bsum, boff, nb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_learn_add, dim3((unsigned)nb, 2), dim3(1024), 0, stream, st, cw1, cw0, boff,
                     nb);
  return hipGetLastError();
}

// Keys and workgroup lists of the first min(K, kRankMax) candidates (k_propose does the same when
// it draws them).
__global__ void __launch_bounds__(256)
k_rank_blocks(const int2 *__restrict__ cand, const float *__restrict__ score, int K,
              uint64_t *__restrict__ keys, uint64_t *__restrict__ lists) {
  __shared__ uint64_t sl[2][64];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool ranked = i < min(K, kRankMax);
  uint64_t key = 0ull;
  if (ranked) {
    const int2 ab = cand[i];
    key = rank_key(ab.x, ab.y, i, score);
    keys[i] = key;
  }
  block_top64(key, sl, lists + (size_t)blockIdx.x * kRankTop);
}

// Evaluation order from the workgroup lists and keys: the lists are merged pairwise (waves
// [h, n) hand theirs to waves [0, h) through LDS; two buffers alternate so that one barrier per
// level suffices), then every other draw of [0, R) follows in draw order, then draws R..K-1.
__global__ void __launch_bounds__(1024)
k_rank_merge(const uint64_t *__restrict__ lists, const uint64_t *__restrict__ keys, int K,
             int32_t *__restrict__ order) {
  static_assert(kRankMax == 4 * 1024 && kRankTop == 64, "k_rank_merge: 16 lists, 4 keys per thread");
  __shared__ uint64_t list[2][8][64];
  __shared__ int cnt[4][16];
  __shared__ uint64_t thr_s;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int R = min(K, kRankMax), nl = (R + 255) >> 8;
  uint64_t m = w < nl ? lists[w * kRankTop + lane] : 0ull;
  int buf = 0;
#pragma unroll
  for (int n = 16; n > 1; n >>= 1) {
    const int h = n >> 1;
    if (w >= h && w < n) list[buf][w - h][lane] = m;
    __syncthreads();
    if (w < h) m = merge_top64(m, list[buf][w][63 - lane], lane);
    buf ^= 1;
  }
  const int T = min(R, kRankTop);
  if (w == 0) {
    if (lane < T) order[lane] = (int32_t)~(uint32_t)m;
    if (lane == T - 1) thr_s = m;
  }
  __syncthreads();
  // every other draw of [0, R) in draw order (draw j * 1024 + t), after the best T
  const uint64_t thr = thr_s;
  uint64_t bal[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = j * 1024 + t;
    const uint64_t own = i < R ? keys[i] : 0ull;
    bal[j] = __ballot(i < R && own < thr);
    if (lane == 0) cnt[j][w] = __popcll(bal[j]);
  }
  __syncthreads();
  int base = T;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int before = 0, total = 0;
    for (int v = 0; v < 16; ++v) {
      before += v < w ? cnt[j][v] : 0;
      total += cnt[j][v];
    }
    if ((bal[j] >> lane) & 1ull) {
      const int below = __builtin_amdgcn_mbcnt_hi(
          (uint32_t)(bal[j] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal[j], 0u));
      order[base + before + below] = j * 1024 + t;
    }
    base += total;
  }
  for (int i = R + t; i < K; i += 1024) order[i] = i;
}

hipError_t launch_rank_merge(const uint64_t *lists, const uint64_t *keys, int K, int32_t *order,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_rank_merge, dim3(1), dim3(1024), 0, stream, lists, keys, K, order);
  return hipGetLastError();
}

hipError_t launch_rank(const int2 *cand, const float *score, int K, int32_t *order,
                       uint64_t *keys, uint64_t *lists, hipStream_t stream) {
  const int R = std::min(K, kRankMax);
  hipLaunchKernelGGL(k_rank_blocks, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, stream, cand,
                     score, K, keys, lists);
  const hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch_rank_merge(lists, keys, K, order, stream);
}

// Copy of the step's candidates as (a, b) pairs.
__global__ void k_copy_cand(const int2 *__restrict__ cand, int K, int32_t *__restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) {
    out[2 * k] = cand[k].x;
    out[2 * k + 1] = cand[k].y;
  }
}

hipError_t launch_copy_cand(const int2 *cand, int K, int32_t *out, hipStream_t stream) {
  hipLaunchKernelGGL(k_copy_cand, dim3((K + 255) / 256), dim3(256), 0, stream, cand, K, out);
  return hipGetLastError();
}

hipError_t launch_init_lists(AnnealDev *st, const uint64_t *bits, int W, int H,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_init_lists, dim3(1), dim3(1024), 0, stream, st, bits, W, H);
  return hipGetLastError();
}

hipError_t launch_lse(const uint32_t *counts, const uint32_t *target, int64_t nterms, int64_t N,
                      int64_t Nt, double *e, hipStream_t stream) {
  hipLaunchKernelGGL(k_lse, dim3(1), dim3(64), 0, stream, counts, target, nterms, N, Nt, e);
  return hipGetLastError();
}

}  // namespace lpf
