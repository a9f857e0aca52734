// Device side of the candidate rounds of an annealing step (shared by k_step.hip and
// k_rec.hip): every workgroup of a round adds its candidates' exact int64 energy sums into S_acc
// (integer addition, so the result does not depend on the order); a decision kernel per round
// then applies the Metropolis test in draw order.
#pragma once

#include <limits.h>
#include <math.h>

#include "lpf_internal.h"

namespace lpf {

// v plus the value of the lane that DPP control CTRL selects (0 where ROW_MASK leaves a row out),
// on both 32-bit halves with the carry.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int64_t dpp_add64(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xF, false);
  return (int64_t)(u + (((uint64_t)hi << 32) | lo));
}

// Sum over the wave of a 64-bit value, valid in lane 63: DPP within quads, half rows and rows,
// then row broadcasts 15 and 31.  Every lane must be active.
__device__ __forceinline__ int64_t wave_sum63_i64(int64_t v) {
  v = dpp_add64<0xB1, 0xF>(v);   // quad_perm 1,0,3,2
  v = dpp_add64<0x4E, 0xF>(v);   // quad_perm 2,3,0,1
  v = dpp_add64<0x141, 0xF>(v);  // row_half_mirror
  v = dpp_add64<0x140, 0xF>(v);  // row_mirror
  v = dpp_add64<0x142, 0xA>(v);  // row_bcast:15
  v = dpp_add64<0x143, 0xC>(v);  // row_bcast:31
  return v;
}

__device__ __forceinline__ void add_acc(int64_t *p, int64_t v) {
  if (v != 0) atomicAdd((unsigned long long *)p, (unsigned long long)v);
}

// Energy sum of the candidate at round slot kr: S_acc[k], or S0[kr] for a round 0 that was
// evaluated in the launch of the draws (which zero S_acc meanwhile).
__device__ __forceinline__ int64_t round_sum(const int64_t *__restrict__ S_acc,
                                             const int64_t *__restrict__ S0, int kr, int k) {
  return S0 ? S0[kr] : S_acc[k];
}

// First accepted evaluation position among i0 .. i0 + C - 1 (C <= 64), tested by the calling
// wave, one candidate per lane (accept iff de <= 0 or U < exp(-de / T)); every lane gets the
// answer, -1 when none, and in ab the accepted candidate's pixels.
__device__ __forceinline__ int wave_first_accepted(const int64_t *__restrict__ S_acc,
                                                   const int64_t *__restrict__ S0,
                                                   const int2 *__restrict__ cand,
                                                   const double *__restrict__ U,
                                                   const int32_t *__restrict__ order, int i0, int C,
                                                   const double *__restrict__ Tp, double scale,
                                                   int2 &ab) {
  const int lane = threadIdx.x & 63;
  bool acc = false;
  int2 c = make_int2(-1, -1);
  if (lane < C) {
    const int k = order ? order[i0 + lane] : i0 + lane;
    c = cand[k];
    if (c.x >= 0) {
      const double de = (double)round_sum(S_acc, S0, lane, k) / scale;
      acc = de <= 0.0 || U[k] < exp(-de / *Tp);
    }
  }
  const unsigned long long m = __ballot(acc);
  if (!m) return -1;
  const int f = __ffsll(m) - 1;
  ab = make_int2(__shfl(c.x, f), __shfl(c.y, f));
  return i0 + f;
}

// Start of a round: true (skip the round) when an earlier round accepted (ctl->done) or when the
// previous round (pC > 0 candidates at positions pi0.., decided here by every workgroup)
// accepted; then workgroup (0, 0) records that decision (and copies its energy sum from S0 to
// S_acc when given).  The control block and the previous round's operands are loaded together,
// so the test costs one memory latency.
__device__ __forceinline__ bool prev_round_accepted(int64_t *__restrict__ S_acc,
                                                   const int64_t *__restrict__ S0,
                                                   const int2 *__restrict__ cand,
                                                   const double *__restrict__ U,
                                                   const int32_t *__restrict__ order, int pi0,
                                                   int pC, const double *__restrict__ Tp,
                                                   double scale, StepCtl *__restrict__ ctl,
                                                   int *s_prev) {
  if (pC <= 0) return ctl->done != 0;
  int2 ab = make_int2(-1, -1);
  if (threadIdx.x < 64) {
    const int done = ctl->done;
    const int f = wave_first_accepted(S_acc, S0, cand, U, order, pi0, pC, Tp, scale, ab);
    if (threadIdx.x == 0) *s_prev = done ? -2 : f;
  }
  __syncthreads();
  const int f = *s_prev;
  if (f == -1) return false;
  if (f >= 0 && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    const int ks = order ? order[f] : f;
    const int64_t S = round_sum(S_acc, S0, f - pi0, ks);
    if (S0) S_acc[ks] = S;
    ctl->ks = ks;
    ctl->a = ab.x;
    ctl->b = ab.y;
    ctl->S = S;
    ctl->done = 1;
  }
  return true;
}

// The step's accepted candidate when no earlier round accepted (ks0 < 0): the first candidate of
// the last round, in evaluation order, that passes the Metropolis test, -1 when none.  Called by
// every thread of a workgroup of any size; all get the same value.
__device__ __forceinline__ int step_choice(const FinalArgs &f, int ks0, int *s_first) {
  if (ks0 >= 0 || f.lC <= 0) return ks0;
  if (threadIdx.x == 0) *s_first = INT_MAX;
  __syncthreads();
  const double T = *f.Tp;
  const double scale = (double)f.N * (double)f.N * (double)f.Nt;
  for (int base = 0; base < f.lC; base += blockDim.x) {
    const int kr = base + threadIdx.x;
    if (kr < f.lC) {
      const int k = f.order ? f.order[f.li0 + kr] : f.li0 + kr;
      if (f.cand[k].x >= 0) {
        const double de = (double)f.S_acc[k] / scale;
        if (de <= 0.0 || f.U[k] < exp(-de / T)) atomicMin(s_first, kr);
      }
    }
    __syncthreads();
    const int fst = *s_first;
    __syncthreads();
    if (fst != INT_MAX) break;
  }
  const int fst = *s_first;
  return fst == INT_MAX ? -1 : (f.order ? f.order[f.li0 + fst] : f.li0 + fst);
}

// counts += dL of the accepted candidate ks for terms part, part + parts, ... (called by `parts`
// workgroups, part = 0 .. parts - 1, each over its threads).
__device__ __forceinline__ void step_counts(const FinalArgs &f, int ks, int part, int parts) {
  if (ks < 0) return;
  for (int t = part * (int)blockDim.x + (int)threadIdx.x; t < f.nterms; t += parts * (int)blockDim.x)
    f.counts[t] = (uint32_t)((int32_t)f.counts[t] + (int32_t)f.dl[t * f.dl_t + ks * f.dl_k]);
}

// The step's upkeep by one workgroup, given its accepted candidate ks (or -1): the control block
// when this step's decision was taken here (decided), counts += dL (unless with_counts is false:
// then the caller's workgroups share it through step_counts), image bits, pixel lists, energy,
// the step's record and the step counter; S0 (when given) is cleared.
__device__ __forceinline__ void step_apply(const FinalArgs &f, int ks, bool decided,
                                           bool with_counts = true) {
  if (f.S0 && threadIdx.x < 64) f.S0[threadIdx.x] = 0;  // clear for the next step's round 0
  if (with_counts) step_counts(f, ks, 0, 1);
  if (threadIdx.x != 0) return;
  AnnealDev *st = f.st;
  StepResult *out = f.out_base >= 0 ? f.out + ((int64_t)st->step - f.out_base) : f.out;
  StepResult r;
  r.step = st->step;
  r.pad = 0;
  if (ks >= 0) {
    const int a = f.cand[ks].x, b = f.cand[ks].y;  // a: phase 1 -> 0, b: phase 0 -> 1
    if (decided) {
      f.ctl->ks = ks;
      f.ctl->a = a;
      f.ctl->b = b;
      f.ctl->S = f.S_acc[ks];
      f.ctl->done = 1;
    }
    const double de = (double)f.S_acc[ks] / ((double)f.N * (double)f.N * (double)f.Nt);
    const double e = *f.e_io + de;
    *f.e_io = e;
    const int W = f.W, wpr = (W + 63) >> 6;
    const int ay = a / W, ax = a - ay * W, by = b / W, bx = b - by * W;
    f.bits[(size_t)ay * wpr + (ax >> 6)] &= ~(1ull << (ax & 63));
    f.bits[(size_t)by * wpr + (bx >> 6)] |= 1ull << (bx & 63);
    st->pos1[f.slot[ks].x] = b;
    st->pos0[f.slot[ks].y] = a;
    st->last_a = a;
    st->last_b = b;
    r.k = ks;
    r.a = a;
    r.b = b;
    r.de = de;
    r.e = e;
  } else {
    st->last_a = -1;
    st->last_b = -1;
    r.k = -1;
    r.a = -1;
    r.b = -1;
    r.de = 0.0;
    r.e = *f.e_io;
  }
  *out = r;
  *f.k_sel = ks;
  st->step += 1;
}

// Energy sum of one term: dL (Nt (dL + 2L) - 2 N T); every partial sum of a candidate stays in
// int64 under the bound lpf_anneal_create checks.
__device__ __forceinline__ int64_t energy_term(int d, int64_t L, int64_t T, int64_t N,
                                               int64_t Nt) {
  return (int64_t)d * (Nt * ((int64_t)d + 2 * L) - 2 * N * T);
}

}  // namespace lpf
