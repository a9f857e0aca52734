// One annealing step's evaluation in rounds, with early exit.
//
// The K candidates of a step are evaluated in evaluation order (draw order, or the learned
// ranking when an order array is given), in rounds of 64 and then the rest (at most 8192 each),
// so that a step whose first candidates are accepted costs one small round.  Each round is an
// evaluation kernel (recount method here, records method in k_rec.hip, the two-point probability
// descriptor in k_s2.hip) that adds every candidate's integer energy sum
// S = sum dL (Nt (dL + 2L) - 2 N T) into S_acc and stores its dL (int16 per term and candidate).
// The Metropolis test of Alg. "annealing" (accept iff de <= 0 or U < exp(-de / T),
// de = S / (N^2 Nt), eq. (LSE)) is applied in evaluation order to a round's candidates at the start
// of the next round (round 0), by k_round_decide (middle rounds), or at the end of the step (last
// round), and the first accepted candidate is recorded.  Rounds after an acceptance return at
// once.  The step's result is the first accepted candidate over all K, exactly as if every
// candidate had been evaluated.
#include <limits.h>
#include <math.h>

#include "delta_dev.h"
#include "step_dev.h"

namespace lpf {

// Zero the step's control block and energy sums (a fill kernel, so the step can be captured).
__global__ void k_step_reset(StepCtl *__restrict__ ctl, int64_t *__restrict__ S_acc, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) S_acc[i] = 0;
  if (i == 0) {
    ctl->done = 0;
    ctl->ks = -1;
    ctl->a = -1;
    ctl->b = -1;
    ctl->S = 0;
  }
}

template <bool LDS>
__global__ void __launch_bounds__(256)
k_round_delta(const uint32_t *__restrict__ Eg, DeltaGeo geo, const uint64_t *__restrict__ bits,
              int W, int H, const int2 *__restrict__ cand, int K, int k0, int C,
              const DeltaVec *__restrict__ vecs, const int32_t *__restrict__ chunk_off,
              const uint32_t *__restrict__ runs, unsigned phase_mask, int nv,
              const uint32_t *__restrict__ counts, const uint32_t *__restrict__ target, int64_t N,
              int64_t Nt, int64_t *__restrict__ S_acc, int16_t *__restrict__ dl,
              StepCtl *__restrict__ ctl, const int32_t *__restrict__ order,
              const double *__restrict__ U, const double *__restrict__ Tp, int pi0, int pC) {
  extern __shared__ uint32_t lds[];
  __shared__ int s_prev;
  if (prev_round_accepted(S_acc, nullptr, cand, U, order, pi0, pC, Tp,
                          (double)N * (double)N * (double)Nt, ctl, &s_prev))
    return;
  const int kr = blockIdx.x * blockDim.x + threadIdx.x;  // index within the round
  const int i = k0 + kr;                                 // evaluation position
  bool ok = kr < C && i < K;
  const int k = ok && order ? order[i] : i;              // candidate (draw index)
  const bool in = ok;
  int a = -1, b = -1;
  if (ok) {
    const int2 ab = cand[k];
    a = ab.x;
    b = ab.y;
  }
  Cand cf[3];
  lane_candidate(bits, W, H, a, b, ok, cf);
  const uint32_t *E;
  if constexpr (LDS) {
    for (int i = threadIdx.x; i < geo.total; i += blockDim.x) lds[i] = Eg[i];
    __syncthreads();
    E = lds;
  } else {
    E = Eg;
  }
  const int c = blockIdx.y;
  const int v0 = chunk_off[c], v1 = chunk_off[c + 1];
  int64_t S = 0;
  for (int j = v0; j < v1; ++j) {
    const DeltaVec dv = vecs[j];
    int d1, d0;
    vector_delta<LDS>(E, geo, dv, runs, cf, d1, d0);
    if (!ok) {
      d1 = 0;
      d0 = 0;
    }
    int p = 0;
    if (phase_mask & 1) {
      const size_t t = (size_t)p * nv + dv.idx;
      S += energy_term(d0, counts[t], target[t], N, Nt);
      if (in && dl) dl[t * K + k] = (int16_t)d0;
      ++p;
    }
    if (phase_mask & 2) {
      const size_t t = (size_t)p * nv + dv.idx;
      S += energy_term(d1, counts[t], target[t], N, Nt);
      if (in && dl) dl[t * K + k] = (int16_t)d1;
    }
  }
  if (in) add_acc(&S_acc[k], S);
}

// Decision for the round's candidates k0 .. k0 + C - 1 (one workgroup).
__global__ void __launch_bounds__(1024)
k_round_decide(const int64_t *__restrict__ S_acc, const int2 *__restrict__ cand,
               const double *__restrict__ U, int k0, int C, const double *__restrict__ Tp,
               int64_t N, int64_t Nt, StepCtl *__restrict__ ctl,
               const int32_t *__restrict__ order) {
  __shared__ int s_first;
  if (ctl->done) return;
  const double T = *Tp;
  if (threadIdx.x == 0) s_first = INT_MAX;
  __syncthreads();
  const double scale = (double)N * (double)N * (double)Nt;
  for (int base = 0; base < C; base += blockDim.x) {
    const int kr = base + threadIdx.x;
    const int k = kr < C ? (order ? order[k0 + kr] : k0 + kr) : 0;
    if (kr < C && cand[k].x >= 0) {
      const double de = (double)S_acc[k] / scale;
      if (de <= 0.0 || U[k] < exp(-de / T)) atomicMin(&s_first, kr);
    }
    __syncthreads();
    const int f = s_first;
    __syncthreads();
    if (f != INT_MAX) break;
  }
  if (threadIdx.x == 0 && s_first != INT_MAX) {
    const int ks = order ? order[k0 + s_first] : k0 + s_first;
    const int2 ab = cand[ks];
    ctl->ks = ks;
    ctl->a = ab.x;
    ctl->b = ab.y;
    ctl->S = S_acc[ks];
    ctl->done = 1;
  }
}

// Step result, running energy, and the accepted interchange applied to counts, image and pixel
// lists (one workgroup).
__global__ void __launch_bounds__(1024) k_step_final(FinalArgs f) {
  __shared__ int s_ks0, s_first;
  if (threadIdx.x == 0) s_ks0 = f.ctl->ks;
  __syncthreads();
  const int ks0 = s_ks0;
  const int ks = step_choice(f, ks0, &s_first);
  step_apply(f, ks, ks0 < 0 && ks >= 0);
}

namespace {

hipError_t launch_round_recount(const StepLaunch &L, const RoundPlan &r, bool decide,
                                hipStream_t stream) {
  dim3 grid((unsigned)((r.C + r.block - 1) / r.block), (unsigned)r.nchunks);
  int16_t *dl = decide ? L.dl : nullptr;
  if (L.use_lds)
    hipLaunchKernelGGL(k_round_delta<true>, grid, dim3(r.block),
                       (size_t)L.geo.total * sizeof(uint32_t), stream, L.E, L.geo, L.bits, L.W,
                       L.H, L.cand, L.K, r.k0, r.C, r.vecs, r.chunk_off, L.runs, L.phase_mask,
                       L.nv, L.counts, L.target, L.N, L.Nt, L.S_acc, dl, L.ctl, L.order, L.U,
                       L.T, decide ? r.pi0 : 0, decide ? r.pC : 0);
  else
    hipLaunchKernelGGL(k_round_delta<false>, grid, dim3(r.block), 0, stream, L.E, L.geo, L.bits,
                       L.W, L.H, L.cand, L.K, r.k0, r.C, r.vecs, r.chunk_off, L.runs,
                       L.phase_mask, L.nv, L.counts, L.target, L.N, L.Nt, L.S_acc, dl, L.ctl,
                       L.order, L.U, L.T, decide ? r.pi0 : 0, decide ? r.pC : 0);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(const StepLaunch &L, hipStream_t stream) {
  hipError_t e;
  if (!L.reset_done) {
    hipLaunchKernelGGL(k_step_reset, dim3((L.K + 255) / 256), dim3(256), 0, stream, L.ctl,
                       L.S_acc, L.K);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // Decisions: round 0 (64 candidates) is decided at the start of round 1 by every workgroup,
  // middle rounds by k_round_decide, the last round by k_step_final.
  const int nr = (int)L.rounds.size();
  for (int j = 0; j < nr; ++j) {
    RoundPlan r = L.rounds[j];
    r.pi0 = 0;
    r.pC = 0;
    if (j == 1 && L.rounds[0].C <= 64) {
      r.pi0 = L.rounds[0].k0;
      r.pC = L.rounds[0].C;
    }
    if (j == 0 && L.fuse_draw)
      e = launch_rec_draw_round0(L, r, stream);
    else if (j == 0 && L.fuse_rank)
      e = launch_rec_rank_round0(L, r, stream);
    else
      e = L.s2        ? launch_s2_round(L, r, true, stream)
          : L.records ? launch_rec_round(L, r, true, stream)
                      : launch_round_recount(L, r, true, stream);
    if (e != hipSuccess) return e;
    const bool decided_later = j == nr - 1 || (j == 0 && L.rounds[0].C <= 64);
    if (!decided_later) {
      hipLaunchKernelGGL(k_round_decide, dim3(1), dim3(std::min(1024, ((r.C + 63) / 64) * 64)), 0,
                         stream, L.S_acc, L.cand, L.U, r.k0, r.C, L.T, L.N, L.Nt, L.ctl, L.order);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  FinalArgs f;
  f.st = L.st;
  f.ctl = L.ctl;
  f.cand = L.cand;
  f.slot = L.slot;
  f.dl = L.dl;
  f.dl_t = L.dl_t;
  f.dl_k = L.dl_k;
  f.nterms = L.nterms;
  f.N = L.N;
  f.Nt = L.Nt;
  f.e_io = L.e;
  f.counts = L.counts_rw;
  f.bits = L.bits_rw;
  f.W = L.W;
  f.k_sel = L.k_sel;
  f.out = L.out;
  f.S_acc = L.S_acc;
  f.U = L.U;
  f.Tp = L.T;
  f.order = L.order;
  f.li0 = nr ? L.rounds[nr - 1].k0 : 0;
  f.lC = nr ? L.rounds[nr - 1].C : 0;
  f.out_base = L.out_base;
  f.S0 = L.fuse_draw || L.fuse_rank ? L.S0 : nullptr;
  // records: the upkeep and the update of ones and records share one launch (with the next
  // step's draws in ranked chains)
  if (L.records && !L.s2)
    return launch_rec_step_end(L.rg, f, L.draw_next ? L.next : nullptr,
                               L.draw_next ? (L.K + 255) / 256 : 0, stream);
  hipLaunchKernelGGL(k_step_final, dim3(1), dim3(1024), 0, stream, f);
  return hipGetLastError();
}

__global__ void k_energy_sum(const int64_t *__restrict__ S_acc, int n, int64_t N, int64_t Nt,
                             double *__restrict__ de) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) de[i] = (double)S_acc[i] / ((double)N * (double)N * (double)Nt);
}

hipError_t launch_energy(const StepLaunch &L, double *de, hipStream_t stream) {
  hipLaunchKernelGGL(k_step_reset, dim3((L.K + 255) / 256), dim3(256), 0, stream, L.ctl, L.S_acc,
                     L.K);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (const RoundPlan &r : L.rounds) {
    e = L.s2        ? launch_s2_round(L, r, false, stream)
        : L.records ? launch_rec_round(L, r, false, stream)
                    : launch_round_recount(L, r, false, stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_energy_sum, dim3((L.K + 255) / 256), dim3(256), 0, stream, L.S_acc, L.K,
                     L.N, L.Nt, de);
  return hipGetLastError();
}

hipError_t prepare_step_kernels(int max_lds_bytes) {
  return hipFuncSetAttribute((const void *)k_round_delta<true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
}

}  // namespace lpf
