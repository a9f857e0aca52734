// Device helpers of the pixel-interchange delta (shared by k_delta.hip and k_step.hip).
#pragma once

#include "lpf_internal.h"

namespace lpf {

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


// Candidate (a, b) of lane `ok`: checks the indices, orders the pair so that a is the phase-1
// pixel, and expresses both pixels in the three image frames.  Invalid pairs become (0, 0) with
// ok = false (their results are discarded).
__device__ __forceinline__ void lane_candidate(const uint64_t *__restrict__ bits, int W, int H,
                                               int a, int b, bool &ok, Cand (&cf)[3]) {
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
  const int ay = a / W, ax = a - ay * W, by = b / W, bx = b - by * W;
  cf[0] = Cand{ax, ay, bx, by};
  cf[1] = Cand{ay, ax, by, bx};
  cf[2] = Cand{ay ? H - ay : 0, ax ? W - ax : 0, by ? H - by : 0, bx ? W - bx : 0};
}

// dL of one vector for one candidate (phase 1 in d1, phase 0 in d0).
template <bool LDS>
__device__ __forceinline__ void vector_delta(const uint32_t *__restrict__ E, const DeltaGeo &geo,
                                             const DeltaVec &dv, const uint32_t *__restrict__ runs,
                                             const Cand (&cf)[3], int &d1, int &d0) {
  const int img = dv.img;
  const ImgGeo g = img == 0 ? geo.g[0] : (img == 1 ? geo.g[1] : geo.g[2]);
  const Cand c = img == 0 ? cf[0] : (img == 1 ? cf[1] : cf[2]);
  d1 = 0;
  d0 = 0;
  const uint32_t *EX = E + g.off;
  window_counts<LDS>(EX, g.W, g.H, g.we, g.pat, runs + dv.run_off, dv.m, c, false, d1, d0);
  window_counts<LDS>(EX, g.W, g.H, g.we, g.pat, runs + dv.run_off, dv.m, c, true, d1, d0);
}

}  // namespace lpf
