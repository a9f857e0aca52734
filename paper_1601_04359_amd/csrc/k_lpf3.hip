// Lineal path function of a periodic 3-D volume (the extension of Sec. 2; with cz = 0 it is the
// sum over the xy-cuts of their 2-D functions, the ensemble of cuts of Sec. 6.3).
//
// Same bit-parallel product as the 2-D kernel: 32 start voxels of one x-row share a word; for a
// segment voxel (px, py, pz) a lane forms t = bits [32w + px, 32w + px + 32) of row
// (y + py, z + pz) of the extended volume (one v_alignbit_b32) and folds it into A (AND) and O
// (OR); popcount(A & valid) counts phase 1, popcount(~O & valid) phase 0.  Vectors with dx < 0
// are mirrored in x and shifted by |dx| (a translation, which leaves a periodic count unchanged).
// One wave per vector; lanes own R words of one start row (S lanes per row) and walk all H*D
// start rows in bands.  When a slab of planes with its cz-plane halo fits in LDS, k_lpf3_slab
// reads rows from LDS and the segment's voxels from a table (k_lpf3_walk); otherwise k_lpf3 reads
// rows from the extended volume in global memory (it stays in L2 for the volume sizes of the
// paper) and generates the voxels on the scalar unit (Bresenham with two error terms).
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

// Voxel table of the segments for the slab kernel: vector j (launch order) owns the int2 entries
// walk[woff[j] ...], one per voxel k = 0..n of its segment and one repeat of the last voxel when
// n + 1 is odd (AND and OR are idempotent, so the repeat leaves the product unchanged):
// {byte offset of the voxel's row word in a slab relative to the start row, bit shift px & 31}.
// The slab geometry (ps dwords per plane, rst dwords per row) fixes the offsets.  The 3-D
// digitisation: n = max(|dx|, |dy|, |dz|), the major axis is the first of x, y, z with extent n and
// each minor coordinate follows its own error term (the 2-D rounding per minor axis).
__global__ void k_lpf3_walk(const int4 *__restrict__ vec, int nv, const int *__restrict__ woff,
                            int ps, int rst, int2 *__restrict__ walk) {
  // one wave per vector, one lane per voxel: after k steps an error term started at n and
  // advanced by 2a (less 2n per carry) has carried floor((2ka + n) / 2n) times
  const int j = blockIdx.x * (blockDim.x >> 6) + (int)(threadIdx.x >> 6);
  if (j >= nv) return;
  const int lane = threadIdx.x & 63;
  const int4 v = vec[j];
  const int dx = v.x, dy = v.y, dz = v.z;
  const int a0 = dx < 0 ? -dx : dx, a1 = dy < 0 ? -dy : dy, a2 = dz < 0 ? -dz : dz;
  const int s1 = dy < 0 ? -1 : 1, s2 = dz < 0 ? -1 : 1;
  const int n = max(a0, max(a1, a2));
  const int maj = a0 == n ? 0 : (a1 == n ? 1 : 2);
  const int ma = maj == 0 ? a1 : a0;  // minor a: y for an x-major vector, else x
  const int mb = maj == 2 ? a1 : a2;  // minor b: y for a z-major vector, else z
  int2 *w = walk + woff[j];
  const int cnt = (n + 2) & ~1;  // n + 1 voxels, the last repeated when n + 1 is odd
  for (int i = lane; i < cnt; i += 64) {
    const int k = min(i, n);
    // 2kn + n < 2^32 for n <= 32767
    const int qa = n ? (int)((2u * k * ma + n) / (2u * n)) : 0;
    const int qb = n ? (int)((2u * k * mb + n) / (2u * n)) : 0;
    const int qx = maj == 0 ? k : qa;
    const int qy = maj == 1 ? k : (maj == 0 ? qa : qb);
    const int qz = maj == 2 ? k : qb;
    const int px = dx < 0 ? a0 - qx : qx;  // mirrored and shifted by |dx| when dx < 0
    w[i] = make_int2((s2 * qz * ps + s1 * qy * rst + (px >> 5)) * 4, px & 31);
  }
}

// Slab variant: workgroup (blockIdx.x, blockIdx.y) stages planes Z0 .. Z0 + zb + cz - 1 (mod D),
// Z0 = blockIdx.y * zb, of the extended volume in LDS, each plane with cy periodic halo rows
// above and below (HH = H + 2 cy rows of rst dwords, LDS row cy + y = volume row y; planes ps
// dwords apart, ps >= HH rst, the gap chosen so that start rows on both sides of a plane
// boundary keep the bank pattern of consecutive rows), and its
// waves count vectors of vec[0 .. nv) (vpw per wave; dz >= 0 for canonical vectors, so a segment
// stays in the slab, and |dy| <= cy, so it stays in the halo) over the start rows of planes
// Z0 .. Z0 + zb - 1; the slab's counts are added into counts (zeroed before the launch) with
// integer atomics.  The voxels come from the table of k_lpf3_walk, two per scalar load.  RPL
// start rows per lane share each table load (R <= 4: 2 for short segments, where the per-band
// work weighs more, 1 for long ones).
template <int R, int RPL>
__global__ void __launch_bounds__(512)
k_lpf3_slab(const uint32_t *__restrict__ E, int W, int H, int D, int we, int S, int rst, int ps, int zb,
            int cz, int cy, const int4 *__restrict__ vec, const int *__restrict__ woff,
            const int2 *__restrict__ walk, int vpw, int nv, unsigned phase_mask,
            uint32_t *__restrict__ counts) {
  extern __shared__ uint32_t lds[];
  const int Z0 = blockIdx.y * zb;
  const int planes = min(zb, D - Z0);  // start planes of this slab
  const int staged = planes + cz;
  const int HH = H + 2 * cy;
  {
    // element i = row pr (plane pl, halo row yh) and dword e; the thread's elements advance by
    // blockDim.x, so the row and plane are carried forward instead of divided out each time
    const int step = blockDim.x, dq = step / we, dr = step - dq * we;
    int e = threadIdx.x % we, pr = threadIdx.x / we;
    int pl = pr / HH, yh = pr - pl * HH;
    const int total_rows = staged * HH;
    while (pr < total_rows) {
      int z = Z0 + pl;
      z = z >= D ? z - D : z;  // cz <= D - 1
      int y = yh - cy;  // in [-cy, H + cy), cy <= H - 1
      y = y < 0 ? y + H : (y >= H ? y - H : y);
      lds[pl * ps + yh * rst + e] = E[((size_t)z * H + y) * we + e];
      e += dr;
      int adv = dq;
      if (e >= we) { e -= we; ++adv; }
      pr += adv;
      yh += adv;
      while (yh >= HH) { yh -= HH; ++pl; }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int waves = blockDim.x >> 6, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rpw = 64 / S;
  const int strip = lane / rpw;
  const int r_in = lane - strip * rpw;
  const int swd = (W + 31) >> 5;
  const uint32_t lastmask = (W & 31) ? ((1u << (W & 31)) - 1u) : 0xffffffffu;
  const int rows = planes * H;
  // the lane's words: all-ones, the last word's valid bits, or none past the row
  uint32_t mw[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int w = strip * R + i;
    mw[i] = (w < swd - 1) ? 0xffffffffu : (w == swd - 1 ? lastmask : 0u);
  }
  // start row r0 + q * rpw + r_in of each band: its (plane, row) advance by a fixed step per
  // band, so the LDS row start (Pb, in bytes) is carried forward; a lane past the slab's rows
  // reads the first start row (P0) and counts nothing
  const int bstep = rpw * RPL, dzb = bstep / H, dyb = bstep - dzb * H;
  const int dPb = (dzb * ps + dyb * rst) * 4, wrapP = (ps - H * rst) * 4, P0 = cy * rst * 4;
  int Pf[RPL], yf[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int r = q * rpw + r_in;
    const int zr = r / H;
    yf[q] = r - zr * H;
    Pf[q] = (zr * ps + (yf[q] + cy) * rst) * 4;
  }
  // vpw vectors per wave, interleaved across the waves (neighbours in the length order)
  for (int jj = 0; jj < vpw; ++jj) {
    const int j = __builtin_amdgcn_readfirstlane((blockIdx.x * vpw + jj) * waves + wave);
    if (j >= nv) break;  // after the only barrier
    const int dx = __builtin_amdgcn_readfirstlane(vec[j].x);
    const int dy = __builtin_amdgcn_readfirstlane(vec[j].y);
    const int dz = __builtin_amdgcn_readfirstlane(vec[j].z);
    const int idx = __builtin_amdgcn_readfirstlane(vec[j].w);
    const int n = max(dx < 0 ? -dx : dx, max(dy < 0 ? -dy : dy, dz < 0 ? -dz : dz));
    const int npair = (n + 2) >> 1;
    // two voxels per entry pair: {offset0, shift0, offset1, shift1}
    const int4 *wp = reinterpret_cast<const int4 *>(walk + __builtin_amdgcn_readfirstlane(woff[j]));
    uint32_t c0 = 0, c1 = 0;
    int Pb[RPL], yb[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      Pb[q] = Pf[q];
      yb[q] = yf[q];
    }
    // RPL start rows per lane per band share each scalar table load.  A voxel's byte offset is
    // the lane's row start plus the table's wave-uniform part; the halo rows make the y wrap
    // unnecessary.  A (phase 1: AND of the voxels) and N (phase 0: AND of their complements)
    // start as the lane's valid bits, so the counts need no mask.
    for (int r0 = 0; r0 < rows; r0 += bstep) {
      int Pq[RPL];
      uint32_t A[RPL][R], N[RPL][R];
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const bool row_ok = r0 + q * rpw + r_in < rows;
        Pq[q] = row_ok ? Pb[q] : P0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          A[q][i] = row_ok ? mw[i] : 0u;
          N[q][i] = A[q][i];
        }
        Pb[q] += dPb;
        yb[q] += dyb;
        if (yb[q] >= H) {
          yb[q] -= H;
          Pb[q] += wrapP;
        }
      }
      const char *base = reinterpret_cast<const char *>(lds + strip * R);
      auto word = [&](int off, int c) -> uint32_t {
        return *reinterpret_cast<const uint32_t *>(base + off + 4 * c);
      };
      for (int p = 0; p < npair; ++p) {
        const int4 t = wp[p];
        const int su0 = __builtin_amdgcn_readfirstlane(t.x), sh0 = __builtin_amdgcn_readfirstlane(t.y);
        const int su1 = __builtin_amdgcn_readfirstlane(t.z), sh1 = __builtin_amdgcn_readfirstlane(t.w);
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
          uint32_t d0[R + 1], d1[R + 1];
#pragma unroll
          for (int c = 0; c <= R; ++c) {
            d0[c] = word(Pq[q] + su0, c);
            d1[c] = word(Pq[q] + su1, c);
          }
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const uint32_t t0 = __builtin_amdgcn_alignbit(d0[i + 1], d0[i], sh0);
            const uint32_t t1 = __builtin_amdgcn_alignbit(d1[i + 1], d1[i], sh1);
            A[q][i] = __builtin_amdgcn_bitop3_b32(A[q][i], t0, t1, 0x80);  // A & t0 & t1
            N[q][i] = __builtin_amdgcn_bitop3_b32(N[q][i], t0, t1, 0x10);  // N & ~t0 & ~t1
          }
        }
      }
#pragma unroll
      for (int q = 0; q < RPL; ++q)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          c1 += __popc(A[q][i]);
          c0 += __popc(N[q][i]);
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

hipError_t launch_lpf3_slab(const uint32_t *E, int W, int H, int D, int we, int R, int S, int rst, int ps,
                            int zb, int cz, int cy, const int4 *vec, const int *woff, int2 *walk,
                            bool build, int rpl, int nv, unsigned phase_mask, uint32_t *counts,
                            hipStream_t stream) {
  const int nph = (int)(phase_mask & 1u) + (int)((phase_mask >> 1) & 1u);
  const int64_t nc = (int64_t)nph * nv;
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lpf3_zero, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, stream,
                     counts, nc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (build) {
    hipLaunchKernelGGL(k_lpf3_walk, dim3((unsigned)((nv + 3) / 4)), dim3(256), 0, stream, vec,
                       nv, woff, ps, rst, walk);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  constexpr int kWaves = 8;
  const int nslab = (D + zb - 1) / zb;
  const size_t lds = (size_t)(zb + cz) * ps * sizeof(uint32_t);
  // enough vectors per wave that staging a slab is amortised, while keeping about 2048
  // workgroups; at most 8, so that waves whose segments are long do not trail the launch (the
  // cuts' full in-plane domain, n up to 99: 4.74 ms with 16 per wave, 4.35 ms with 9)
  const int64_t groups_at_1 = ((int64_t)nv + kWaves - 1) / kWaves;
  const int vpw = (int)std::max<int64_t>(1, std::min<int64_t>(8, groups_at_1 * nslab / 2048));
  const dim3 grid((unsigned)((nv + kWaves * vpw - 1) / (kWaves * vpw)), (unsigned)nslab);
#define LPF3S(RR, QQ)                                                                          \
  hipLaunchKernelGGL((k_lpf3_slab<RR, QQ>), grid, dim3(64 * kWaves), lds, stream, E, W, H, D,  \
                     we, S, rst, ps, zb, cz, cy, vec, woff, walk, vpw, nv, phase_mask, counts)
  const bool two = rpl == 2;
  switch (R) {
    case 1: if (two) LPF3S(1, 2); else LPF3S(1, 1); break;
    case 2: if (two) LPF3S(2, 2); else LPF3S(2, 1); break;
    case 4: if (two) LPF3S(4, 2); else LPF3S(4, 1); break;
    case 8: LPF3S(8, 1); break;
    case 16: LPF3S(16, 1); break;
    default: return hipErrorInvalidValue;
  }
#undef LPF3S
  return hipGetLastError();
}

hipError_t prepare_lpf3_kernels(int max_lds_bytes) {
  const void *fns[] = {(const void *)k_lpf3_slab<1, 1>, (const void *)k_lpf3_slab<1, 2>,
                       (const void *)k_lpf3_slab<2, 1>, (const void *)k_lpf3_slab<2, 2>,
                       (const void *)k_lpf3_slab<4, 1>, (const void *)k_lpf3_slab<4, 2>,
                       (const void *)k_lpf3_slab<8, 1>, (const void *)k_lpf3_slab<16, 1>};
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
