// Device-resident simulated annealing on the lineal path function (Sec. 4, Alg. "annealing",
// objective eq. (LSE)).  One step: K candidate pixel interchanges are drawn (here), their exact
// energy changes are evaluated against the current state in evaluation order (draw order, or the
// learned ranking of k_rank_chunks / k_rank_merge) and the first candidate that passes the Metropolis test is applied
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

#include "lpf_internal.h"

namespace lpf {

// Philox-4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

__device__ __forceinline__ int bit_at(const uint64_t *__restrict__ bits, int wpr, int x, int y) {
  return (int)((bits[(size_t)y * wpr + (x >> 6)] >> (x & 63)) & 1ull);
}

// A pixel with a periodic 4-neighbour of the other phase.
__device__ __forceinline__ bool interfacial(const uint64_t *__restrict__ bits, int W, int H, int q) {
  const int wpr = (W + 63) >> 6;
  const int y = q / W, x = q - y * W;
  const int v = bit_at(bits, wpr, x, y);
  const int xl = x ? x - 1 : W - 1, xr = x + 1 == W ? 0 : x + 1;
  const int yu = y ? y - 1 : H - 1, yd = y + 1 == H ? 0 : y + 1;
  return bit_at(bits, wpr, xl, y) != v || bit_at(bits, wpr, xr, y) != v ||
         bit_at(bits, wpr, x, yu) != v || bit_at(bits, wpr, x, yd) != v;
}

// Candidate k of the current step: ctr = {step, k, 0, 0}, key = {seed, 0x6c7066}.
// proposal 0: a, b uniform in the phase-1 / phase-0 lists; 1: as 0, void unless both pixels are
// interfacial; 2 (learned): with probability eps (r3) as 0, otherwise a drawn with probability
// proportional to the weights whose inclusive prefix sums are cw1 (over pos1) and b likewise
// with cw0 (over pos0), by inversion of r0, r1.
__device__ __forceinline__ int upper_index(const double *__restrict__ cw, int n, double u) {
  int lo = 0, hi = n - 1;  // first i with cw[i] > u
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cw[mid] > u) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

__global__ void k_propose(const AnnealDev *__restrict__ st, const uint64_t *__restrict__ bits,
                          int W, int H, uint64_t seed, int K, int proposal,
                          const double *__restrict__ cw1, const double *__restrict__ cw0,
                          double eps, int2 *__restrict__ cand, double *__restrict__ U,
                          int2 *__restrict__ slot, int64_t *__restrict__ S_acc,
                          StepCtl *__restrict__ ctl, const double *__restrict__ T_sched,
                          int64_t T_base, double T, double *__restrict__ T_cur) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (ctl && k == 0) {  // the step's control block and energy sums start at zero
    ctl->done = 0;
    ctl->ks = -1;
    ctl->S = 0;
  }
  if (T_cur && k == 0) *T_cur = T_sched ? T_sched[(int64_t)st->step - T_base] : T;
  if (k >= K) return;
  if (S_acc) S_acc[k] = 0;
  uint64_t c[4] = {st->step, (uint64_t)k, 0ull, 0ull};
  philox4x64_10(c, seed, 0x6c7066ull);
  const int n1 = st->n1, n0 = st->n0;
  int ia, ib;
  const double u3 = (double)(c[3] >> 11) * (1.0 / 9007199254740992.0);
  if (proposal == 2 && !(u3 < eps)) {
    const double ua = (double)(c[0] >> 11) * (1.0 / 9007199254740992.0) * cw1[n1 - 1];
    const double ub = (double)(c[1] >> 11) * (1.0 / 9007199254740992.0) * cw0[n0 - 1];
    ia = upper_index(cw1, n1, ua);
    ib = upper_index(cw0, n0, ub);
  } else {
    ia = (int)(((c[0] >> 32) * (uint64_t)n1) >> 32);
    ib = (int)(((c[1] >> 32) * (uint64_t)n0) >> 32);
  }
  int a = st->pos1[ia], b = st->pos0[ib];
  if (proposal == 1 && !(interfacial(bits, W, H, a) && interfacial(bits, W, H, b))) {
    a = -1;
    b = -1;
  }
  cand[k] = make_int2(a, b);
  slot[k] = make_int2(ia, ib);
  U[k] = (double)(c[2] >> 11) * (1.0 / 9007199254740992.0);
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

hipError_t launch_propose(const AnnealDev *st, const uint64_t *bits, int W, int H, uint64_t seed,
                          int K, int proposal, const double *cw1, const double *cw0, double eps,
                          int2 *cand, double *U, int2 *slot, int64_t *S_acc, StepCtl *ctl,
                          const double *T_sched, int64_t T_base, double T, double *T_cur,
                          hipStream_t stream) {
  hipLaunchKernelGGL(k_propose, dim3((K + 255) / 256), dim3(256), 0, stream, st, bits, W, H, seed,
                     K, proposal, cw1, cw0, eps, cand, U, slot, S_acc, ctl, T_sched, T_base, T,
                     T_cur);
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

// Evaluation order of a step's candidates: the kRankTop draws with the highest predicted gain
// score[a] + score[b] (fp32; void draws and NaN lowest; ties by draw index) among the first
// R = min(K, kRankMax), best first, then every other draw in draw order.  k_rank_chunks sorts
// chunks of 512 draws (one workgroup each) and keeps each chunk's best kRankTop; k_rank_merge
// sorts those (the overall best kRankTop are among them) and writes the order.
__device__ __forceinline__ bool rank_before(float ka, int ia, float kb, int ib) {
  return ka > kb || (ka == kb && ia < ib);
}

// Bitonic sort of 512 (key, index) pairs, one per thread of a 512-thread workgroup, best first;
// partners under 64 apart exchange through wave shuffles, the others through LDS.
__device__ __forceinline__ void bitonic512(float &key, int &id, float *sk, int *si) {
  const int e = threadIdx.x;
  for (int size = 2; size <= 512; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      float pk;
      int pi;
      if (stride >= 64) {
        sk[e] = key;
        si[e] = id;
        __syncthreads();
        pk = sk[e ^ stride];
        pi = si[e ^ stride];
        __syncthreads();
      } else {
        pk = __shfl_xor(key, stride);
        pi = __shfl_xor(id, stride);
      }
      const bool keep_first = ((e & stride) == 0) == ((e & size) == 0);
      const bool p_first = rank_before(pk, pi, key, id);
      if (keep_first ? p_first : !p_first) {
        key = pk;
        id = pi;
      }
    }
  }
}

__global__ void __launch_bounds__(512)
k_rank_chunks(const int2 *__restrict__ cand, const float *__restrict__ score, int K,
              float *__restrict__ top_key, int *__restrict__ top_id) {
  __shared__ float sk[512];
  __shared__ int si[512];
  const int R = min(K, kRankMax);
  const int i = blockIdx.x * 512 + threadIdx.x;
  float key = -INFINITY;
  int id = INT_MAX;
  if (i < R) {
    id = i;
    const int2 ab = cand[i];
    if (ab.x >= 0 && ab.y >= 0) {
      const float sc = score[ab.x] + score[ab.y];
      key = sc == sc ? sc : -INFINITY;
    }
  }
  bitonic512(key, id, sk, si);
  if (threadIdx.x < kRankTop) {
    top_key[blockIdx.x * kRankTop + threadIdx.x] = key;
    top_id[blockIdx.x * kRankTop + threadIdx.x] = id;
  }
}

__global__ void __launch_bounds__(512)
k_rank_merge(const float *__restrict__ top_key, const int *__restrict__ top_id, int K,
             int32_t *__restrict__ order) {
  __shared__ float sk[512];
  __shared__ int si[512];
  __shared__ uint32_t sel[kRankMax / 32];
  __shared__ int part[8];
  const int R = min(K, kRankMax);
  const int nchunks = (R + 511) / 512;
  const int t = threadIdx.x;
  float key = -INFINITY;
  int id = INT_MAX;
  if (t < nchunks * kRankTop) {
    key = top_key[t];
    id = top_id[t];
  }
  for (int w = t; w < kRankMax / 32; w += 512) sel[w] = 0u;
  bitonic512(key, id, sk, si);
  const int T = min(R, kRankTop);
  if (t < T) {
    order[t] = id;
    atomicOr(&sel[id >> 5], 1u << (id & 31));
  }
  __syncthreads();
  // the other draws of [0, R) in draw order: consecutive draws per thread, exclusive scan
  constexpr int per = kRankMax / 512;
  const int i0 = t * per;
  int cnt = 0;
  for (int j = 0; j < per; ++j) {
    const int i = i0 + j;
    cnt += (i < R && !((sel[i >> 5] >> (i & 31)) & 1u)) ? 1 : 0;
  }
  // inclusive scan of the counts: within the wave by shuffles, then over the 8 wave totals
  int x = cnt;
  const int lane = t & 63, wave = t >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) part[wave] = x;
  __syncthreads();
  int off = 0;
  for (int w = 0; w < wave; ++w) off += part[w];
  int pos = T + off + x - cnt;
  for (int j = 0; j < per; ++j) {
    const int i = i0 + j;
    if (i < R && !((sel[i >> 5] >> (i & 31)) & 1u)) order[pos++] = i;
  }
  for (int i = R + t; i < K; i += 512) order[i] = i;
}

hipError_t launch_rank(const int2 *cand, const float *score, int K, int32_t *order,
                       float *top_key, int *top_id, hipStream_t stream) {
  const int R = std::min(K, kRankMax);
  hipLaunchKernelGGL(k_rank_chunks, dim3((unsigned)((R + 511) / 512)), dim3(512), 0, stream, cand,
                     score, K, top_key, top_id);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rank_merge, dim3(1), dim3(512), 0, stream, top_key, top_id, K, order);
  return hipGetLastError();
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
