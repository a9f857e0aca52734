// Lineal path function of a periodic 3-D volume (the extension of Sec. 2; with cz = 0 it is the
// sum over the xy-cuts of their 2-D functions, the ensemble of cuts of Sec. 6.3).
//
// Same bit-parallel product as the 2-D kernel: 32 start voxels of one x-row share a word; for a
// segment voxel (px, py, pz) a lane forms t = bits [32w + px, 32w + px + 32) of row
// (y + py, z + pz) of the extended volume (one v_alignbit_b32) and folds it into A (AND) and O
// (OR); popcount(A & valid) counts phase 1, popcount(~O & valid) phase 0.  Vectors with dx < 0
// are mirrored in x and shifted by |dx| (a translation, which leaves a periodic count unchanged).
// The segment's voxels are generated on the scalar unit (Bresenham with two error terms), one
// wave per vector; lanes own R words of one start row (S lanes per row) and walk all H*D start
// rows in bands.  Rows are read from the extended volume in global memory (it stays in L2 for the
// volume sizes of the paper) by k_lpf3, or, when a slab of planes with its cz-plane halo fits,
// from LDS by k_lpf3_slab.
#include "lpf_internal.h"

namespace lpf {

namespace {

__device__ __forceinline__ uint32_t wave_sum3(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace

// vec[j] = {dx, dy, dz, canonical index}, longest segments first; counts[p][index] for the
// phases of phase_mask.  E: H*D rows of we dwords,
// row index z*H + y.
template <int R>
__global__ void __launch_bounds__(256)
k_lpf3(const uint32_t *__restrict__ E, int W, int H, int D, int we, int S,
       const int4 *__restrict__ vec, int nv, unsigned phase_mask, uint32_t *__restrict__ counts) {
  const int lane = threadIdx.x & 63;
  // wave-uniform vector index: its Bresenham state then lives in scalar registers
  const int j = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (j >= nv) return;  // no barrier in this kernel
  const int4 v = make_int4(__builtin_amdgcn_readfirstlane(vec[j].x),
                           __builtin_amdgcn_readfirstlane(vec[j].y),
                           __builtin_amdgcn_readfirstlane(vec[j].z),
                           __builtin_amdgcn_readfirstlane(vec[j].w));
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
    if (phase_mask & 1u) counts[(size_t)(p++) * nv + v.w] = c0;
    if (phase_mask & 2u) counts[(size_t)p * nv + v.w] = c1;
  }
}

// Slab variant: workgroup (blockIdx.x, blockIdx.y) stages planes Z0 .. Z0 + zb + cz - 1 (mod D),
// Z0 = blockIdx.y * zb, of the extended volume in LDS, each plane with cy periodic halo rows
// above and below (HH = H + 2 cy rows of rst dwords, LDS row cy + y = volume row y), and its
// waves count vectors of vec[v0 .. v1) (vpw per wave; dz >= 0 for canonical vectors, so a segment
// stays in the slab, and |dy| <= cy, so it stays in the halo) over the start rows of planes
// Z0 .. Z0 + zb - 1; the slab's counts are added into counts (zeroed before the launch) with
// integer atomics.  MAJ: the major axis of every vector of the range (0 = x, 1 = y, 2 = z), so
// the voxel walk has no axis branches.
template <int R, int MAJ>
__global__ void __launch_bounds__(512)
k_lpf3_slab(const uint32_t *__restrict__ E, int W, int H, int D, int we, int S, int rst, int zb,
            int cz, int cy, const int4 *__restrict__ vec, int v0, int v1, int vpw, int nv,
            unsigned phase_mask, uint32_t *__restrict__ counts) {
  extern __shared__ uint32_t lds[];
  const int Z0 = blockIdx.y * zb;
  const int planes = min(zb, D - Z0);  // start planes of this slab
  const int staged = planes + cz;
  const int HH = H + 2 * cy;
  for (int i = threadIdx.x; i < staged * HH * we; i += blockDim.x) {
    const int pr = i / we, e = i - pr * we;  // pr = plane * HH + halo row
    const int pl = pr / HH, yh = pr - pl * HH;
    int z = Z0 + pl;
    z = z >= D ? z - D : z;  // cz <= D - 1
    int y = yh - cy;  // in [-cy, H + cy), cy <= H - 1
    y = y < 0 ? y + H : (y >= H ? y - H : y);
    lds[pr * rst + e] = E[((size_t)z * H + y) * we + e];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  // wave-uniform vector indices: the Bresenham state lives in scalar registers
  const int waves = blockDim.x >> 6, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rpw = 64 / S;
  const int strip = lane / rpw;
  const int r_in = lane - strip * rpw;
  const int swd = (W + 31) >> 5;
  const uint32_t lastmask = (W & 31) ? ((1u << (W & 31)) - 1u) : 0xffffffffu;
  const int rows = planes * H;
  constexpr int RPL = R <= 4 ? 2 : 1;
  // vpw vectors per wave, interleaved across the waves (neighbours in the length order)
  for (int jj = 0; jj < vpw; ++jj) {
    const int j = __builtin_amdgcn_readfirstlane(v0 + (blockIdx.x * vpw + jj) * waves + wave);
    if (j >= v1) break;  // after the only barrier
    const int dx = __builtin_amdgcn_readfirstlane(vec[j].x);
    const int dy = __builtin_amdgcn_readfirstlane(vec[j].y);
    const int dz = __builtin_amdgcn_readfirstlane(vec[j].z);
    const int idx = __builtin_amdgcn_readfirstlane(vec[j].w);
    const int a0 = dx < 0 ? -dx : dx, a1 = dy < 0 ? -dy : dy, a2 = dz;
    const int s1 = dy < 0 ? -1 : 1;
    const int n = MAJ == 0 ? a0 : (MAJ == 1 ? a1 : a2);
    // the two minor axes: magnitudes (the major one gets coordinate k)
    const int ma = MAJ == 0 ? a1 : a0;  // minor a: y for MAJ 0, else x
    const int mb = MAJ == 2 ? a1 : a2;  // minor b: y for MAJ 2, else z
    uint32_t c0 = 0, c1 = 0;
    // RPL start rows per lane per band: the scalar voxel walk is shared by their vector work.
    // A voxel's byte offset is the lane's row start (Pq) plus a wave-uniform part; the halo rows
    // make the y wrap unnecessary.  Offsets in bytes, so that they are LDS addresses as they stand.
    for (int r0 = 0; r0 < rows; r0 += rpw * RPL) {
      int Pq[RPL];
      uint32_t A[RPL][R], O[RPL][R], mk[RPL][R];
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = r0 + q * rpw + r_in;
        const bool row_ok = r < rows;
        const int zr = row_ok ? r / H : 0;
        const int yr = row_ok ? r - zr * H : 0;
        Pq[q] = (zr * HH + yr + cy) * rst * 4;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          A[q][i] = 0xffffffffu;
          O[q][i] = 0u;
          const int w = strip * R + i;
          const uint32_t mw = (w < swd - 1) ? 0xffffffffu : (w == swd - 1 ? lastmask : 0u);
          mk[q][i] = row_ok ? mw : 0u;
        }
      }
      const char *base = reinterpret_cast<const char *>(lds + strip * R);
      auto word = [&](int off, int c) -> uint32_t {
        return *reinterpret_cast<const uint32_t *>(base + off + 4 * c);
      };
      // Bresenham state of voxel k: minor coordinates qa, qb with error terms ea, eb; voxels in
      // pairs (two funnel shifts, one 3-input AND, one 3-input OR)
      int ea = n, eb = n, qa = 0, qb = 0;
      auto advance = [&]() {
        ea += 2 * ma;
        if (ea >= 2 * n) { ea -= 2 * n; ++qa; }
        eb += 2 * mb;
        if (eb >= 2 * n) { eb -= 2 * n; ++qb; }
      };
      auto voxel = [&](int k, int (&off)[RPL], int &sh) {
        const int qx = MAJ == 0 ? k : qa;
        const int qy = MAJ == 1 ? k : (MAJ == 0 ? qa : qb);
        const int qz = MAJ == 2 ? k : qb;
        const int px = dx < 0 ? a0 - qx : qx;  // mirrored and shifted by |dx| when dx < 0
        const int su = ((qz * HH + s1 * qy) * rst + (px >> 5)) * 4;  // wave-uniform
#pragma unroll
        for (int q = 0; q < RPL; ++q) off[q] = Pq[q] + su;
        sh = px & 31;
      };
      int k = 0;
      for (; k + 1 <= n; k += 2) {
        int off0[RPL], off1[RPL], sh0, sh1;
        voxel(k, off0, sh0);
        advance();
        voxel(k + 1, off1, sh1);
        advance();
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          uint32_t d0[R + 1], d1[R + 1];
#pragma unroll
          for (int c = 0; c <= R; ++c) {
            d0[c] = word(off0[q], c);
            d1[c] = word(off1[q], c);
          }
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const uint32_t t0 = __builtin_amdgcn_alignbit(d0[i + 1], d0[i], sh0);
            const uint32_t t1 = __builtin_amdgcn_alignbit(d1[i + 1], d1[i], sh1);
            A[q][i] = __builtin_amdgcn_bitop3_b32(A[q][i], t0, t1, 0x80);
            O[q][i] = O[q][i] | t0 | t1;
          }
        }
      }
      if (k == n) {  // odd voxel count: the last voxel alone
        int off[RPL], sh;
        voxel(k, off, sh);
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          uint32_t d[R + 1];
#pragma unroll
          for (int c = 0; c <= R; ++c) d[c] = word(off[q], c);
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const uint32_t t = __builtin_amdgcn_alignbit(d[i + 1], d[i], sh);
            A[q][i] &= t;
            O[q][i] |= t;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < RPL; ++q)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          c1 += __popc(A[q][i] & mk[q][i]);
          c0 += __popc(~O[q][i] & mk[q][i]);
        }
    }
    c0 = wave_sum3(c0);
    c1 = wave_sum3(c1);
    if (lane == 0) {
      int p = 0;
      if (phase_mask & 1u) {
        if (c0) atomicAdd(&counts[(size_t)p * nv + idx], c0);
        ++p;
      }
      if ((phase_mask & 2u) && c1) atomicAdd(&counts[(size_t)p * nv + idx], c1);
    }
  }
}

__global__ void k_lpf3_zero(uint32_t *__restrict__ counts, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counts[i] = 0;
}

hipError_t launch_lpf3_slab(const uint32_t *E, int W, int H, int D, int we, int R, int S, int rst,
                            int zb, int cz, int cy, const int4 *vec, const int *maj_off, int nv,
                            unsigned phase_mask, uint32_t *counts, hipStream_t stream) {
  const int nph = (int)(phase_mask & 1u) + (int)((phase_mask >> 1) & 1u);
  const int64_t nc = (int64_t)nph * nv;
  hipLaunchKernelGGL(k_lpf3_zero, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, stream,
                     counts, nc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int kWaves = 8;
  const int nslab = (D + zb - 1) / zb;
  const size_t lds = (size_t)(zb + cz) * (H + 2 * cy) * rst * sizeof(uint32_t);
  for (int maj = 0; maj < 3; ++maj) {
    const int v0 = maj_off[maj], v1 = maj_off[maj + 1];
    const int cnt = v1 - v0;
    if (cnt <= 0) continue;
    // enough vectors per wave that staging a slab is amortised, while keeping about 2048
    // workgroups
    const int64_t groups_at_1 = ((int64_t)cnt + kWaves - 1) / kWaves;
    const int vpw = (int)std::max<int64_t>(1, std::min<int64_t>(16, groups_at_1 * nslab / 2048));
    const dim3 grid((unsigned)((cnt + kWaves * vpw - 1) / (kWaves * vpw)), (unsigned)nslab);
#define LPF3S(RR, MM)                                                                           \
  hipLaunchKernelGGL((k_lpf3_slab<RR, MM>), grid, dim3(64 * kWaves), lds, stream, E, W, H, D,   \
                     we, S, rst, zb, cz, cy, vec, v0, v1, vpw, nv, phase_mask, counts)
#define LPF3M(RR)                               \
  switch (maj) {                                \
    case 0: LPF3S(RR, 0); break;                \
    case 1: LPF3S(RR, 1); break;                \
    default: LPF3S(RR, 2); break;               \
  }
    switch (R) {
      case 1: LPF3M(1); break;
      case 2: LPF3M(2); break;
      case 4: LPF3M(4); break;
      case 8: LPF3M(8); break;
      case 16: LPF3M(16); break;
      default: return hipErrorInvalidValue;
    }
#undef LPF3M
#undef LPF3S
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t prepare_lpf3_kernels(int max_lds_bytes) {
  const void *fns[] = {
      (const void *)k_lpf3_slab<1, 0>,  (const void *)k_lpf3_slab<1, 1>,
      (const void *)k_lpf3_slab<1, 2>,  (const void *)k_lpf3_slab<2, 0>,
      (const void *)k_lpf3_slab<2, 1>,  (const void *)k_lpf3_slab<2, 2>,
      (const void *)k_lpf3_slab<4, 0>,  (const void *)k_lpf3_slab<4, 1>,
      (const void *)k_lpf3_slab<4, 2>,  (const void *)k_lpf3_slab<8, 0>,
      (const void *)k_lpf3_slab<8, 1>,  (const void *)k_lpf3_slab<8, 2>,
      (const void *)k_lpf3_slab<16, 0>, (const void *)k_lpf3_slab<16, 1>,
      (const void *)k_lpf3_slab<16, 2>};
  hipError_t e = hipSuccess;
  for (const void *f : fns) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       max_lds_bytes);
    if (e == hipSuccess) e = r;
  }
  return e;
}

hipError_t launch_lpf3(const uint32_t *E, int W, int H, int D, int we, int R, int S,
                       const int4 *vec, int nv, unsigned phase_mask, uint32_t *counts,
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
