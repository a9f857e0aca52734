// Device side of the candidate rounds of an annealing step (shared by k_step.hip and
// k_rec.hip): every workgroup of a round adds its candidates' exact int64 energy sums into S_acc
// (integer addition, so the result does not depend on the order); a decision kernel per round
// then applies the Metropolis test in draw order.
#pragma once

#include <math.h>

#include "lpf_internal.h"

namespace lpf {

__device__ __forceinline__ void add_acc(int64_t *p, int64_t v) {
  if (v != 0) atomicAdd((unsigned long long *)p, (unsigned long long)v);
}

// First accepted evaluation position among i0 .. i0 + C - 1 (C <= 64), tested by the calling
// wave, one candidate per lane (accept iff de <= 0 or U < exp(-de / T)); every lane gets the
// answer, -1 when none.
__device__ __forceinline__ int wave_first_accepted(const int64_t *__restrict__ S_acc,
                                                   const int2 *__restrict__ cand,
                                                   const double *__restrict__ U,
                                                   const int32_t *__restrict__ order, int i0, int C,
                                                   double T, double scale) {
  const int lane = threadIdx.x & 63;
  bool acc = false;
  if (lane < C) {
    const int k = order ? order[i0 + lane] : i0 + lane;
    if (cand[k].x >= 0) {
      const double de = (double)S_acc[k] / scale;
      acc = de <= 0.0 || U[k] < exp(-de / T);
    }
  }
  const unsigned long long m = __ballot(acc);
  return m ? i0 + (__ffsll(m) - 1) : -1;
}

// Start of a round that also decides the previous round (pC > 0 candidates at positions pi0..):
// every workgroup evaluates that decision; when it accepted, workgroup (0, 0) records it and all
// workgroups return true (skip the round).
__device__ __forceinline__ bool prev_round_accepted(const int64_t *__restrict__ S_acc,
                                                   const int2 *__restrict__ cand,
                                                   const double *__restrict__ U,
                                                   const int32_t *__restrict__ order, int pi0,
                                                   int pC, const double *__restrict__ Tp,
                                                   double scale, StepCtl *__restrict__ ctl,
                                                   int *s_prev) {
  if (pC <= 0) return false;
  if (threadIdx.x < 64) {
    const int f = wave_first_accepted(S_acc, cand, U, order, pi0, pC, *Tp, scale);
    if (threadIdx.x == 0) *s_prev = f;
  }
  __syncthreads();
  const int f = *s_prev;
  if (f < 0) return false;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    const int ks = order ? order[f] : f;
    ctl->ks = ks;
    ctl->S = S_acc[ks];
    ctl->done = 1;
  }
  return true;
}

// Energy sum of one term: dL (Nt (dL + 2L) - 2 N T); every partial sum of a candidate stays in
// int64 under the bound lpf_anneal_create checks.
__device__ __forceinline__ int64_t energy_term(int d, int64_t L, int64_t T, int64_t N,
                                               int64_t Nt) {
  return (int64_t)d * (Nt * ((int64_t)d + 2 * L) - 2 * N * T);
}

}  // namespace lpf
