// Lineal path function of a periodic 3-D volume (the extension of Sec. 2; with cz = 0 it is the
// sum over the xy-cuts of their 2-D functions, the ensemble of cuts of Sec. 5).
//
// Same bit-parallel product as the 2-D kernel: 32 start voxels of one x-row share a word; for a
// segment voxel (px, py, pz) a lane forms t = bits [32w + px, 32w + px + 32) of row
// (y + py, z + pz) of the extended volume (one v_alignbit_b32) and folds it into A (AND) and O
// (OR); popcount(A & valid) counts phase 1, popcount(~O & valid) phase 0.  Vectors with dx < 0
// are mirrored in x and shifted by |dx| (a translation, which leaves a periodic count unchanged).
// The segment's voxels are generated on the scalar unit (Bresenham with two error terms), one
// wave per vector; lanes own R words of one start row (S lanes per row) and walk all H*D start
// rows in bands.  Rows are read from the extended volume in global memory (it stays in L2 for the
// volume sizes of the paper): a 3-D halo does not fit the LDS.
#include "lpf_internal.h"

namespace lpf {

namespace {

__device__ __forceinline__ uint32_t wave_sum3(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace

// vec[j] = {dx, dy, dz, 0}; counts[p][j] for the phases of phase_mask.  E: H*D rows of we dwords,
// row index z*H + y.
template <int R>
__global__ void __launch_bounds__(256)
k_lpf3(const uint32_t *__restrict__ E, int W, int H, int D, int we, int S,
       const short4 *__restrict__ vec, int nv, unsigned phase_mask, uint32_t *__restrict__ counts) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= nv) return;  // wave-uniform; no barrier in this kernel
  const short4 v = vec[j];
  const int dx = v.x, dy = v.y, dz = v.z;
  const int a0 = dx < 0 ? -dx : dx, a1 = dy < 0 ? -dy : dy, a2 = dz < 0 ? -dz : dz;
  const int s1 = dy < 0 ? -1 : 1, s2 = dz < 0 ? -1 : 1;
  const int n = max(a0, max(a1, a2));
  const int major = a0 == n ? 0 : (a1 == n ? 1 : 2);
  const int rpw = 64 / S;
  const int strip = lane / rpw;
  const int r_in = lane - strip * rpw;
  const int swd = (W + 31) >> 5;
  const uint32_t lastmask = (W & 31) ? ((1u << (W & 31)) - 1u) : 0xffffffffu;
  const int rows = H * D;
  uint32_t c0 = 0, c1 = 0;
  for (int r0 = 0; r0 < rows; r0 += rpw) {
    const int r = r0 + r_in;
    const bool row_ok = r < rows;
    const int z = row_ok ? r / H : 0;
    const int y = row_ok ? r - z * H : 0;
    uint32_t A[R], O[R], mk[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      A[i] = 0xffffffffu;
      O[i] = 0u;
      const int w = strip * R + i;
      const uint32_t mw = (w < swd - 1) ? 0xffffffffu : (w == swd - 1 ? lastmask : 0u);
      mk[i] = row_ok ? mw : 0u;
    }
    // Bresenham: the major coordinate is k, each minor one has its own error term (the
    // rounding of the 2-D segments per minor axis)
    int e0 = n, e1 = n, e2 = n, q0 = 0, q1 = 0, q2 = 0;
    for (int k = 0; k <= n; ++k) {
      if (k > 0) {
        if (major == 0) {
          q0 = k;
        } else {
          e0 += 2 * a0;
          if (e0 >= 2 * n) { e0 -= 2 * n; ++q0; }
        }
        if (major == 1) {
          q1 = k;
        } else {
          e1 += 2 * a1;
          if (e1 >= 2 * n) { e1 -= 2 * n; ++q1; }
        }
        if (major == 2) {
          q2 = k;
        } else {
          e2 += 2 * a2;
          if (e2 >= 2 * n) { e2 -= 2 * n; ++q2; }
        }
      }
      const int px = dx < 0 ? a0 - q0 : q0;  // mirrored and shifted by |dx| when dx < 0
      int yy = y + s1 * q1, zz = z + s2 * q2;
      yy = yy >= H ? yy - H : (yy < 0 ? yy + H : yy);  // |dy| <= H - 1, |dz| <= D - 1
      zz = zz >= D ? zz - D : (zz < 0 ? zz + D : zz);
      const uint32_t *p = E + ((size_t)zz * H + yy) * we + strip * R + (px >> 5);
      const int sh = px & 31;
      uint32_t d[R + 1];
#pragma unroll
      for (int c = 0; c <= R; ++c) d[c] = p[c];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const uint32_t t = __builtin_amdgcn_alignbit(d[i + 1], d[i], sh);
        A[i] &= t;
        O[i] |= t;
      }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      c1 += __popc(A[i] & mk[i]);
      c0 += __popc(~O[i] & mk[i]);
    }
  }
  c0 = wave_sum3(c0);
  c1 = wave_sum3(c1);
  if (lane == 0) {
    int p = 0;
    if (phase_mask & 1u) counts[(size_t)(p++) * nv + j] = c0;
    if (phase_mask & 2u) counts[(size_t)p * nv + j] = c1;
  }
}

hipError_t launch_lpf3(const uint32_t *E, int W, int H, int D, int we, int R, int S,
                       const short4 *vec, int nv, unsigned phase_mask, uint32_t *counts,
                       hipStream_t stream) {
  const dim3 grid((unsigned)((nv + 3) / 4));
#define LPF3(RR)                                                                                \
  hipLaunchKernelGGL(k_lpf3<RR>, grid, dim3(256), 0, stream, E, W, H, D, we, S, vec, nv,      \
                     phase_mask, counts)
  switch (R) {
    case 1: LPF3(1); break;
    case 2: LPF3(2); break;
    case 4: LPF3(4); break;
    case 8: LPF3(8); break;
    case 16: LPF3(16); break;
    default: return hipErrorInvalidValue;
  }
#undef LPF3
  return hipGetLastError();
}

}  // namespace lpf
