// One annealing step's evaluation in rounds, with early exit.
//
// The K candidates of a step are evaluated in draw order, C at a time.  A round launches one
// workgroup per (256 candidates, vector chunk): each lane evaluates one candidate's exact dL
// (int16, kept per candidate as [phase][vector][candidate]) and its integer energy partial
// S = sum dL (Nt (dL + 2L) - 2 N T) over the chunk.  The round's decision kernel sums the
// partials in chunk order, applies the Metropolis test to the round's candidates in draw order
// and records the first accepted one.  Rounds after an acceptance return at once.  The step's
// result is therefore the first accepted candidate over all K, exactly as if every candidate had
// been evaluated, while an early acceptance costs one round.
#include <math.h>

#include "delta_dev.h"

namespace lpf {

__global__ void k_step_reset(StepCtl *__restrict__ ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->done = 0;
    ctl->ks = -1;
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
              int64_t Nt, int64_t *__restrict__ S_part, int16_t *__restrict__ dl,
              const StepCtl *__restrict__ ctl) {
  extern __shared__ uint32_t lds[];
  if (ctl->done) return;  // an earlier round accepted
  const int kr = blockIdx.x * blockDim.x + threadIdx.x;  // index within the round
  const int k = k0 + kr;
  bool ok = kr < C && k < K;
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
  const bool in = kr < C && k < K;
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
      const int64_t L = counts[(size_t)p * nv + dv.idx], T = target[(size_t)p * nv + dv.idx];
      S += (int64_t)d0 * (Nt * ((int64_t)d0 + 2 * L) - 2 * N * T);
      if (in && dl) dl[((size_t)p * nv + dv.idx) * K + k] = (int16_t)d0;
      ++p;
    }
    if (phase_mask & 2) {
      const int64_t L = counts[(size_t)p * nv + dv.idx], T = target[(size_t)p * nv + dv.idx];
      S += (int64_t)d1 * (Nt * ((int64_t)d1 + 2 * L) - 2 * N * T);
      if (in && dl) dl[((size_t)p * nv + dv.idx) * K + k] = (int16_t)d1;
    }
  }
  if (kr < C) S_part[(size_t)c * C + kr] = S;
}

// Decision for the round's candidates k0 .. k0 + C - 1 (one workgroup, C <= 1024).
__global__ void __launch_bounds__(1024)
k_round_decide(const int64_t *__restrict__ S_part, int nchunks, int K, int k0, int C,
               const int2 *__restrict__ cand, const double *__restrict__ U, double T, int64_t N,
               int64_t Nt, StepCtl *__restrict__ ctl) {
  __shared__ int s_first[16];
  __shared__ long long s_S[16];
  if (ctl->done) return;
  const int kr = threadIdx.x, k = k0 + kr;
  bool acc = false;
  int64_t St = 0;
  if (kr < C && k < K && cand[k].x >= 0) {
    for (int c = 0; c < nchunks; ++c) St += S_part[(size_t)c * C + kr];
    const double de = (double)St / ((double)N * (double)N * (double)Nt);
    acc = de <= 0.0 || U[k] < exp(-de / T);
  }
  const uint64_t m = __ballot(acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int first = m ? __ffsll((unsigned long long)m) - 1 : 64;
  if (lane == first) s_S[wave] = St;
  if (lane == 0) s_first[wave] = m ? wave * 64 + first : 0x7fffffff;
  __syncthreads();
  if (threadIdx.x == 0) {
    int f = 0x7fffffff;
    long long Sf = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
      if (s_first[w] < f) {
        f = s_first[w];
        Sf = s_S[w];
      }
    if (f != 0x7fffffff) {
      ctl->ks = k0 + f;
      ctl->S = Sf;
      ctl->done = 1;
    }
  }
}

// Step result, running energy, and the accepted interchange applied to counts, image and pixel
// lists (one workgroup).
__global__ void __launch_bounds__(1024)
k_step_final(AnnealDev *__restrict__ st, const StepCtl *__restrict__ ctl, int K,
             const int2 *__restrict__ cand, const int2 *__restrict__ slot,
             const int16_t *__restrict__ dl, int nterms, int64_t N, int64_t Nt,
             double *__restrict__ e_io, uint32_t *__restrict__ counts, uint64_t *__restrict__ bits,
             int W, int32_t *__restrict__ k_sel, StepResult *__restrict__ out) {
  const int ks = ctl->ks;
  if (ks >= 0)
    for (int t = threadIdx.x; t < nterms; t += blockDim.x)
      counts[t] = (uint32_t)((int32_t)counts[t] + (int32_t)dl[(size_t)t * K + ks]);
  if (threadIdx.x == 0) {
    StepResult r;
    r.step = st->step;
    r.pad = 0;
    if (ks >= 0) {
      const double de = (double)ctl->S / ((double)N * (double)N * (double)Nt);
      const double e = *e_io + de;
      *e_io = e;
      const int a = cand[ks].x, b = cand[ks].y;  // a: phase 1 -> 0, b: phase 0 -> 1
      const int wpr = (W + 63) >> 6;
      const int ay = a / W, ax = a - ay * W, by = b / W, bx = b - by * W;
      bits[(size_t)ay * wpr + (ax >> 6)] &= ~(1ull << (ax & 63));
      bits[(size_t)by * wpr + (bx >> 6)] |= 1ull << (bx & 63);
      st->pos1[slot[ks].x] = b;
      st->pos0[slot[ks].y] = a;
      r.k = ks;
      r.a = a;
      r.b = b;
      r.de = de;
      r.e = e;
    } else {
      r.k = -1;
      r.a = -1;
      r.b = -1;
      r.de = 0.0;
      r.e = *e_io;
    }
    *out = r;
    *k_sel = ks;
    st->step += 1;
  }
}

hipError_t launch_step(const StepLaunch &L, hipStream_t stream) {
  hipLaunchKernelGGL(k_step_reset, dim3(1), dim3(64), 0, stream, L.ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int k0 = 0; k0 < L.K; k0 += L.C) {
    const int C = std::min(L.C, L.K - k0);
    dim3 grid((unsigned)((C + 255) / 256), (unsigned)L.nchunks);
    if (L.use_lds)
      hipLaunchKernelGGL(k_round_delta<true>, grid, dim3(256),
                         (size_t)L.geo.total * sizeof(uint32_t), stream, L.E, L.geo, L.bits, L.W,
                         L.H, L.cand, L.K, k0, C, L.vecs, L.chunk_off, L.runs, L.phase_mask, L.nv,
                         L.counts, L.target, L.N, L.Nt, L.S_part, L.dl, L.ctl);
    else
      hipLaunchKernelGGL(k_round_delta<false>, grid, dim3(256), 0, stream, L.E, L.geo, L.bits,
                         L.W, L.H, L.cand, L.K, k0, C, L.vecs, L.chunk_off, L.runs, L.phase_mask,
                         L.nv, L.counts, L.target, L.N, L.Nt, L.S_part, L.dl, L.ctl);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_round_decide, dim3(1), dim3(((C + 63) / 64) * 64), 0, stream, L.S_part,
                       L.nchunks, L.K, k0, C, L.cand, L.U, L.T, L.N, L.Nt, L.ctl);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_step_final, dim3(1), dim3(1024), 0, stream, L.st, L.ctl, L.K, L.cand,
                     L.slot, L.dl, L.nterms, L.N, L.Nt, L.e, L.counts_rw, L.bits_rw, L.W, L.k_sel,
                     L.out);
  return hipGetLastError();
}

__global__ void k_energy_sum(const int64_t *__restrict__ S_part, int nchunks, int n, int64_t N,
                             int64_t Nt, double *__restrict__ de) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t S = 0;
  for (int c = 0; c < nchunks; ++c) S += S_part[(size_t)c * n + i];
  de[i] = (double)S / ((double)N * (double)N * (double)Nt);
}

hipError_t launch_energy(const StepLaunch &L, double *de, hipStream_t stream) {
  hipLaunchKernelGGL(k_step_reset, dim3(1), dim3(64), 0, stream, L.ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((L.K + 255) / 256), (unsigned)L.nchunks);
  if (L.use_lds)
    hipLaunchKernelGGL(k_round_delta<true>, grid, dim3(256),
                       (size_t)L.geo.total * sizeof(uint32_t), stream, L.E, L.geo, L.bits, L.W,
                       L.H, L.cand, L.K, 0, L.K, L.vecs, L.chunk_off, L.runs, L.phase_mask, L.nv,
                       L.counts, L.target, L.N, L.Nt, L.S_part, (int16_t *)nullptr, L.ctl);
  else
    hipLaunchKernelGGL(k_round_delta<false>, grid, dim3(256), 0, stream, L.E, L.geo, L.bits, L.W,
                       L.H, L.cand, L.K, 0, L.K, L.vecs, L.chunk_off, L.runs, L.phase_mask, L.nv,
                       L.counts, L.target, L.N, L.Nt, L.S_part, (int16_t *)nullptr, L.ctl);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_sum, dim3((L.K + 255) / 256), dim3(256), 0, stream, L.S_part,
                     L.nchunks, L.K, L.N, L.Nt, de);
  return hipGetLastError();
}

hipError_t prepare_step_kernels(int max_lds_bytes) {
  return hipFuncSetAttribute((const void *)k_round_delta<true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
}

}  // namespace lpf
