// Device-resident simulated annealing on the lineal path function (Sec. 4, Alg. "annealing",
// objective eq. (LSE)).  One step: K candidate pixel interchanges are drawn (here), their exact
// energy changes are evaluated against the current state in draw order and the first candidate
// that passes the Metropolis test is applied (k_step.hip).  Rejected candidates leave the state
// unchanged, so this is the sequential chain of the algorithm with the step's later candidates
// unused.  Nothing returns to the host inside a step.
//
// Energy: e = sum_{i,v} (T_i(v)/Nt - L_i(v)/N)^2 over the phases of the mask and the canonical
// half domain, T = target counts over Nt pixels, L = current counts over N = W*H pixels.  The
// change of one interchange is exact in integers,
//     S = sum dL * (Nt * (dL + 2 L) - 2 N T),   de = S / (N^2 Nt),
// and converted to double once, so it does not depend on summation order.
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
__global__ void k_propose(const AnnealDev *__restrict__ st, const uint64_t *__restrict__ bits,
                          int W, int H, uint64_t seed, int K, int proposal,
                          int2 *__restrict__ cand, double *__restrict__ U,
                          int2 *__restrict__ slot) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  uint64_t c[4] = {st->step, (uint64_t)k, 0ull, 0ull};
  philox4x64_10(c, seed, 0x6c7066ull);
  const uint64_t n1 = (uint64_t)st->n1, n0 = (uint64_t)st->n0;
  const int ia = (int)(((c[0] >> 32) * n1) >> 32);
  const int ib = (int)(((c[1] >> 32) * n0) >> 32);
  int a = st->pos1[ia], b = st->pos0[ib];
  if (proposal == 1 && !(interfacial(bits, W, H, a) && interfacial(bits, W, H, b))) {
    a = -1;
    b = -1;
  }
  cand[k] = make_int2(a, b);
  slot[k] = make_int2(ia, ib);
  U[k] = (double)(c[2] >> 11) * (1.0 / 9007199254740992.0);
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
                          int K, int proposal, int2 *cand, double *U, int2 *slot,
                          hipStream_t stream) {
  hipLaunchKernelGGL(k_propose, dim3((K + 255) / 256), dim3(256), 0, stream, st, bits, W, H, seed,
                     K, proposal, cand, U, slot);
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
