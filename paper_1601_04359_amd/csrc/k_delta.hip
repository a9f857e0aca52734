// Exact change of the lineal path function under a pixel interchange (Sec. 4 modification
// operator), for many candidate interchanges at once.
//
// Only translations whose segment covers a swapped pixel can change.  With a the phase-1 pixel
// and b the phase-0 pixel of an interchange, P_p = {p - p_k} the translations whose segment
// covers p, lambda_i the indicator "segment entirely in phase i", J1 = I with b set to 1 and
// J0 = I with a set to 0:
//     dL_1 = sum_{s in P_b} lambda_1(s; J1) - sum_{s in P_a} lambda_1(s; J1)
//     dL_0 = sum_{s in P_a} lambda_0(s; J0) - sum_{s in P_b} lambda_0(s; J0)
// (a translation covering both pixels appears in both sums with the same value and cancels;
// one covering only a or only b sees exactly the old or the new image).
//
// Lanes are candidates; the vector is wave-uniform.  Every vector is evaluated as a "flat" one
// (|dx| >= |dy|): steep first-quadrant vectors on the transposed image, steep second-quadrant
// vectors on the anti-transposed image (x, y) -> (-y, -x), which map segments to segments under
// the digitisation rule.  A flat segment is a stack of m+1 horizontal runs, so P_p is m+1 start
// rows of contiguous start columns; each start row is one 32-bit word of starts, and the path
// product over the segment's pixels is formed with funnel shifts of a 64-bit row window.
#include <algorithm>

#include "lpf_internal.h"

namespace lpf {

// E_X[r][e] (r < H_X + hy, e < we_X): bit j = pixel of image X at ((32e + j) mod W_X, r mod H_X).
// X = 0: the image; X = 1: transposed, X(x,y) = I(y,x); X = 2: anti-transposed,
// X(x,y) = I(-y mod W, -x mod H).  Images 1 and 2 are H wide and W high.
__global__ void k_ext3(const uint64_t *__restrict__ bits, int W, int H, DeltaGeo geo,
                       uint32_t *__restrict__ E) {
  const int img = blockIdx.z;
  const ImgGeo g = img == 0 ? geo.g[0] : (img == 1 ? geo.g[1] : geo.g[2]);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= g.we || r >= g.H + geo.hy) return;
  const int wpr = (W + 63) >> 6;
  const int y = r % g.H;
  uint32_t v = 0;
  int x = (int)(((int64_t)32 * e) % g.W);
  for (int t = 0; t < 32; ++t) {
    int sx, sy;
    if (img == 0) {
      sx = x;
      sy = y;
    } else if (img == 1) {
      sx = y;
      sy = x;
    } else {
      sx = y ? W - y : 0;
      sy = x ? H - x : 0;
    }
    const uint64_t w = bits[(size_t)sy * wpr + (sx >> 6)];
    v |= (uint32_t)((w >> (sx & 63)) & 1ull) << t;
    x = (x + 1 == g.W) ? 0 : x + 1;
  }
  E[(size_t)g.off + (size_t)r * g.we + e] = v;
}

hipError_t launch_ext3(const uint64_t *bits, int W, int H, const DeltaGeo &geo, uint32_t *E,
                       hipStream_t stream) {
  int wemax = std::max(geo.g[0].we, std::max(geo.g[1].we, geo.g[2].we));
  int hmax = std::max(geo.g[0].H, std::max(geo.g[1].H, geo.g[2].H)) + geo.hy;
  dim3 grid((wemax + 63) / 64, hmax, 3);
  hipLaunchKernelGGL(k_ext3, grid, dim3(64), 0, stream, bits, W, H, geo, E);
  return hipGetLastError();
}

__device__ __forceinline__ int pixel_value(const uint64_t *__restrict__ bits, int W, int q) {
  const int wpr = (W + 63) >> 6;
  const int y = q / W, x = q - y * W;
  return (int)((bits[(size_t)y * wpr + (x >> 6)] >> (x & 63)) & 1ull);
}

// 64-bit mask of the occurrences of column u + t*W (t >= 0) inside a 64-column window.
__device__ __forceinline__ uint64_t occ_mask(bool on, int u, uint64_t pat) {
  return (on && u < 64) ? (pat << u) : 0ull;
}

// Lane-side state of one candidate in one image frame.
struct Cand {
  int ax, ay, bx, by;
};

// Path products over one window (start pixel p), accumulated into d1/d0 with the given sign.
template <bool LDS>
__device__ __forceinline__ void window_counts(const uint32_t *__restrict__ EX, int WX, int HX,
                                              int we, uint64_t pat, const uint32_t *__restrict__ runs,
                                              int m, const Cand &c, bool at_b, int &d1, int &d0) {
  const int px = at_b ? c.bx : c.ax;
  const int py = at_b ? c.by : c.ay;
  for (int j = 0; j <= m; ++j) {
    const uint32_t rj_ = runs[j];
    const int alpha_j = (int)(rj_ & 0xffffu), beta_j = (int)(rj_ >> 16);
    const int rj = beta_j - alpha_j + 1;
    int srow = py - j;
    srow += srow < 0 ? HX : 0;
    for (int sc = 0; sc < rj; sc += 32) {
      int c0 = px - beta_j + sc;
      c0 += c0 < 0 ? WX : 0;
      uint32_t A = 0xffffffffu, O = 0u;
      for (int jj = 0; jj <= m; ++jj) {
        const uint32_t rr = runs[jj];
        const int alpha = (int)(rr & 0xffffu), beta = (int)(rr >> 16);
        const int row = srow + jj;
        const bool ra = (row == c.ay) || (row == c.ay + HX);
        const bool rb = (row == c.by) || (row == c.by + HX);
        const uint32_t *Er = EX + row * we;
        for (int pc = alpha; pc <= beta; pc += 32) {
          const int base = c0 + pc;
          const int q = base >> 5;
          const uint32_t D0 = Er[q], D1 = Er[q + 1], D2 = Er[q + 2];
          const uint32_t Vlo = __builtin_amdgcn_alignbit(D1, D0, base & 31);
          const uint32_t Vhi = __builtin_amdgcn_alignbit(D2, D1, base & 31);
          int ua = c.ax - base, ub = c.bx - base;
          ua += ua < 0 ? WX : 0;
          ua += ua < 0 ? WX : 0;
          ub += ub < 0 ? WX : 0;
          ub += ub < 0 ? WX : 0;
          const uint64_t ma = occ_mask(ra, ua, pat);  // a forced to 0 for the phase-0 product
          const uint64_t mb = occ_mask(rb, ub, pat);  // b forced to 1 for the phase-1 product
          const int cnt = min(beta - pc, 31);
          if (__any((ma | mb) != 0ull)) {
            const uint32_t Alo = Vlo | (uint32_t)mb, Ahi = Vhi | (uint32_t)(mb >> 32);
            const uint32_t Olo = Vlo & ~(uint32_t)ma, Ohi = Vhi & ~(uint32_t)(ma >> 32);
            for (int t = 0; t <= cnt; ++t) {
              A &= __builtin_amdgcn_alignbit(Ahi, Alo, t);
              O |= __builtin_amdgcn_alignbit(Ohi, Olo, t);
            }
          } else {
            for (int t = 0; t <= cnt; ++t) {
              const uint32_t w = __builtin_amdgcn_alignbit(Vhi, Vlo, t);
              A &= w;
              O |= w;
            }
          }
        }
      }
      const int left = rj - sc;
      const uint32_t valid = left >= 32 ? 0xffffffffu : ((1u << left) - 1u);
      const int c1 = __popc(A & valid), c0n = __popc(~O & valid);
      if (at_b) {
        d1 += c1;
        d0 -= c0n;
      } else {
        d1 -= c1;
        d0 += c0n;
      }
    }
  }
}

template <int MODE, bool LDS>
__global__ void __launch_bounds__(256)
k_delta(const uint32_t *__restrict__ Eg, DeltaGeo geo, const uint64_t *__restrict__ bits, int W,
        int H, const int2 *__restrict__ cand, int K, const DeltaVec *__restrict__ vecs,
        const int32_t *__restrict__ chunk_off, const uint32_t *__restrict__ runs,
        unsigned phase_mask, int nv, int32_t *__restrict__ delta_out,
        const uint32_t *__restrict__ counts, const uint32_t *__restrict__ target, int64_t N,
        int64_t Nt, int64_t *__restrict__ S_part, uint32_t *__restrict__ counts_rw,
        const int32_t *__restrict__ k_sel) {
  extern __shared__ uint32_t lds[];
  int k;
  bool ok;
  if (MODE == 2) {
    const int ks = *k_sel;
    if (ks < 0) return;  // no candidate accepted: nothing to apply
    k = ks;
    ok = threadIdx.x == 0 && blockIdx.x == 0;
  } else {
    k = blockIdx.x * blockDim.x + threadIdx.x;
    ok = k < K;
  }
  int a = -1, b = -1;
  if (ok) {
    const int2 ab = cand[k];
    a = ab.x;
    b = ab.y;
  }
  const int64_t NN = (int64_t)W * H;
  ok = ok && a >= 0 && b >= 0 && a < NN && b < NN && a != b;
  if (ok) {
    const int va = pixel_value(bits, W, a), vb = pixel_value(bits, W, b);
    ok = va != vb;
    if (va == 0) {
      const int t = a;
      a = b;
      b = t;
    }
  }
  if (!ok) {
    a = 0;
    b = 0;
  }
  Cand cf[3];
  {
    const int ay = a / W, ax = a - ay * W, by = b / W, bx = b - by * W;
    cf[0] = Cand{ax, ay, bx, by};
    cf[1] = Cand{ay, ax, by, bx};
    cf[2] = Cand{ay ? H - ay : 0, ax ? W - ax : 0, by ? H - by : 0, bx ? W - bx : 0};
  }
  const uint32_t *E;
  if constexpr (LDS) {
    for (int i = threadIdx.x; i < geo.total; i += blockDim.x) lds[i] = Eg[i];
    __syncthreads();
    E = lds;
  } else {
    E = Eg;
  }
  const int chunk = blockIdx.y;
  const int vb0 = chunk_off[chunk], vb1 = chunk_off[chunk + 1];
  const int nph = (phase_mask & 1) + ((phase_mask >> 1) & 1);
  int64_t S = 0;
  for (int j = vb0; j < vb1; ++j) {
    const DeltaVec dv = vecs[j];
    const int img = dv.img;
    const ImgGeo g = img == 0 ? geo.g[0] : (img == 1 ? geo.g[1] : geo.g[2]);
    const Cand c = img == 0 ? cf[0] : (img == 1 ? cf[1] : cf[2]);
    const uint64_t pat = g.pat;
    int d1 = 0, d0 = 0;
    const uint32_t *EX = E + g.off;
    window_counts<LDS>(EX, g.W, g.H, g.we, pat, runs + dv.run_off, dv.m, c, false, d1, d0);
    window_counts<LDS>(EX, g.W, g.H, g.we, pat, runs + dv.run_off, dv.m, c, true, d1, d0);
    if (!ok) {
      d1 = 0;
      d0 = 0;
    }
    if (MODE == 0) {
      if (k < K) {
        int p = 0;
        if (phase_mask & 1) delta_out[((size_t)k * nph + p++) * nv + dv.idx] = d0;
        if (phase_mask & 2) delta_out[((size_t)k * nph + p) * nv + dv.idx] = d1;
      }
    } else if (MODE == 1) {
      int p = 0;
      if (phase_mask & 1) {
        const int64_t L = counts[(size_t)p * nv + dv.idx], T = target[(size_t)p * nv + dv.idx];
        S += (int64_t)d0 * (Nt * ((int64_t)d0 + 2 * L) - 2 * N * T);
        ++p;
      }
      if (phase_mask & 2) {
        const int64_t L = counts[(size_t)p * nv + dv.idx], T = target[(size_t)p * nv + dv.idx];
        S += (int64_t)d1 * (Nt * ((int64_t)d1 + 2 * L) - 2 * N * T);
      }
    } else {
      if (ok) {
        int p = 0;
        if (phase_mask & 1) {
          counts_rw[(size_t)p * nv + dv.idx] += (uint32_t)d0;
          ++p;
        }
        if (phase_mask & 2) counts_rw[(size_t)p * nv + dv.idx] += (uint32_t)d1;
      }
    }
  }
  if (MODE == 1 && k < K) S_part[(size_t)chunk * K + k] = S;
}

template <int MODE>
static hipError_t launch_delta_mode(const DeltaLaunch &L, hipStream_t stream) {
  const bool lds = L.use_lds;
  dim3 block(256);
  dim3 grid(MODE == 2 ? 1 : (unsigned)((L.K + 255) / 256), (unsigned)L.nchunks);
  size_t sh = lds ? (size_t)L.geo.total * sizeof(uint32_t) : 0;
  if (lds)
    hipLaunchKernelGGL((k_delta<MODE, true>), grid, block, sh, stream, L.E, L.geo, L.bits, L.W, L.H,
                       L.cand, L.K, L.vecs, L.chunk_off, L.runs, L.phase_mask, L.nv, L.delta_out,
                       L.counts, L.target, L.N, L.Nt, L.S_part, L.counts_rw, L.k_sel);
  else
    hipLaunchKernelGGL((k_delta<MODE, false>), grid, block, 0, stream, L.E, L.geo, L.bits, L.W,
                       L.H, L.cand, L.K, L.vecs, L.chunk_off, L.runs, L.phase_mask, L.nv,
                       L.delta_out, L.counts, L.target, L.N, L.Nt, L.S_part, L.counts_rw, L.k_sel);
  return hipGetLastError();
}

hipError_t launch_delta(int mode, const DeltaLaunch &L, hipStream_t stream) {
  switch (mode) {
    case 0: return launch_delta_mode<0>(L, stream);
    case 1: return launch_delta_mode<1>(L, stream);
    case 2: return launch_delta_mode<2>(L, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t prepare_delta_kernels(int max_lds_bytes) {
  hipError_t e = hipSuccess;
  const void *fns[] = {(const void *)k_delta<0, true>, (const void *)k_delta<1, true>,
                       (const void *)k_delta<2, true>};
  for (const void *f : fns) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
    if (r != hipSuccess) e = r;
  }
  return e;
}

}  // namespace lpf
