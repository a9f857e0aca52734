// Throughput probes of the two on-chip resources the counting kernels are bound by: the int32
// vector ALU (the bitwise, funnel-shift and popcount instructions the path product issues) and
// LDS reads.  Each lane runs 8 independent dependency chains so that issue, not latency, limits
// the rate; results go to a sink so that nothing is optimised away.  Used to measure the peaks a
// roofline fraction is quoted against.
#include "lpf_internal.h"

namespace lpf {

constexpr int kProbeChains = 8;

// kind 0: the path product's mix per chain and iteration: two funnel shifts, one 3-input AND,
//         one 3-input OR (4 ops);
// kind 1: 3-input AND only (v_bitop3_b32), 4 per chain and iteration;
// kind 2: funnel shift only (v_alignbit_b32), 4 per chain and iteration;
// kind 3: popcount with accumulate (v_bcnt_u32_b32), 4 per chain and iteration.
template <int KIND>
__global__ void __launch_bounds__(256) k_probe_valu(int64_t iters, uint32_t s0, uint32_t s1,
                                                    uint32_t *__restrict__ sink) {
  uint32_t a[kProbeChains], o[kProbeChains];
#pragma unroll
  for (int i = 0; i < kProbeChains; ++i) {
    a[i] = threadIdx.x * 2654435761u + (uint32_t)i * 40503u + blockIdx.x;
    o[i] = a[i] ^ 0x9e3779b9u;
  }
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kProbeChains; ++i) {
      if constexpr (KIND == 0) {
        const uint32_t t0 = __builtin_amdgcn_alignbit(a[i], o[i], s0);
        const uint32_t t1 = __builtin_amdgcn_alignbit(o[i], a[i], s1);
        a[i] = __builtin_amdgcn_bitop3_b32(a[i], t0, t1, 0x80);
        o[i] = o[i] | t0 | t1;
      } else if constexpr (KIND == 1) {
        a[i] = __builtin_amdgcn_bitop3_b32(a[i], o[i], s0, 0x80);
        o[i] = __builtin_amdgcn_bitop3_b32(o[i], a[i], s1, 0x96);
        a[i] = __builtin_amdgcn_bitop3_b32(a[i], o[i], s1, 0x80);
        o[i] = __builtin_amdgcn_bitop3_b32(o[i], a[i], s0, 0x96);
      } else if constexpr (KIND == 2) {
        a[i] = __builtin_amdgcn_alignbit(a[i], o[i], s0);
        o[i] = __builtin_amdgcn_alignbit(o[i], a[i], s1);
        a[i] = __builtin_amdgcn_alignbit(a[i], o[i], s1);
        o[i] = __builtin_amdgcn_alignbit(o[i], a[i], s0);
      } else {
        a[i] = __popc(o[i]) + a[i];
        o[i] = __popc(a[i]) + o[i];
        a[i] = __popc(o[i]) + a[i];
        o[i] = __popc(a[i]) + o[i];
      }
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kProbeChains; ++i) r ^= a[i] ^ o[i];
  sink[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// LDS reads: 32 KiB per workgroup, each lane reads 16 bytes per access at consecutive addresses
// across the wave (no bank conflicts), 8 accesses per iteration at fixed offsets, each folded
// with two 3-input XORs.  The empty asm statement with a memory clobber keeps the compiler from
// hoisting the loads out of the loop; it emits no instruction.
__global__ void __launch_bounds__(256) k_probe_lds(int64_t iters, uint32_t *__restrict__ sink) {
  __shared__ uint4 buf[2048];
  for (int i = threadIdx.x; i < 2048; i += blockDim.x)
    buf[i] = make_uint4(i * 3u + blockIdx.x, i ^ 0x55u, i + 7u, ~(uint32_t)i);
  __syncthreads();
  uint32_t acc0 = threadIdx.x, acc1 = 0;
  const int p = threadIdx.x;  // blockDim.x == 256
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint4 d = buf[p + u * 256];
      acc0 = __builtin_amdgcn_bitop3_b32(acc0, d.x, d.y, 0x96);
      acc1 = __builtin_amdgcn_bitop3_b32(acc1, d.z, d.w, 0x96);
    }
    __asm__ volatile("" ::: "memory");
  }
  sink[blockIdx.x * blockDim.x + threadIdx.x] = acc0 ^ acc1;
}

hipError_t launch_probe(int kind, int64_t iters, int nwg, uint32_t *sink, hipStream_t stream) {
  const dim3 g(nwg), b(256);
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_probe_valu<0>, g, b, 0, stream, iters, 7u, 25u, sink); break;
    case 1: hipLaunchKernelGGL(k_probe_valu<1>, g, b, 0, stream, iters, 7u, 25u, sink); break;
    case 2: hipLaunchKernelGGL(k_probe_valu<2>, g, b, 0, stream, iters, 7u, 25u, sink); break;
    case 3: hipLaunchKernelGGL(k_probe_valu<3>, g, b, 0, stream, iters, 7u, 25u, sink); break;
    case 4: hipLaunchKernelGGL(k_probe_lds, g, b, 0, stream, iters, sink); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Work of one probe launch: int32 lane-operations (kinds 0-3) or LDS bytes read (kind 4).
double probe_work(int kind, int64_t iters, int nwg) {
  const double lanes = (double)nwg * 256.0;
  if (kind == 4) return lanes * (double)iters * 8.0 * 16.0;
  return lanes * (double)iters * kProbeChains * 4.0;
}

}  // namespace lpf
