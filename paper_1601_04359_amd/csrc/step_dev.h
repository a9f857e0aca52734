// Device side of the candidate rounds of an annealing step (shared by k_step.hip and
// k_rec.hip): every workgroup of a round adds its candidates' exact int64 energy sums into S_acc
// (integer addition, so the result does not depend on the order); a decision kernel per round
// then applies the Metropolis test in draw order.
#pragma once

#include "lpf_internal.h"

namespace lpf {

__device__ __forceinline__ void add_acc(int64_t *p, int64_t v) {
  if (v != 0) atomicAdd((unsigned long long *)p, (unsigned long long)v);
}

// Energy sum of one term: dL (Nt (dL + 2L) - 2 N T); every partial sum of a candidate stays in
// int64 under the bound lpf_anneal_create checks.
__device__ __forceinline__ int64_t energy_term(int d, int64_t L, int64_t T, int64_t N,
                                               int64_t Nt) {
  return (int64_t)d * (Nt * ((int64_t)d + 2 * L) - 2 * N * T);
}

}  // namespace lpf
