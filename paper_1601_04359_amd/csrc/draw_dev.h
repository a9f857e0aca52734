// Candidate draws of an annealing step (Alg. "annealing": a phase-1 pixel a and a phase-0 pixel
// b to interchange, and the uniform of the step's Metropolis test), shared by k_propose and the
// records method's first round, which draws its own candidates again so that it does not wait for
// k_propose: the draw is a pure function of (step, k, seed) and the pixel lists.
#pragma once

#include <stdint.h>

#include "lpf_internal.h"

namespace lpf {

// Philox-4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

__device__ __forceinline__ int bit_at(const uint64_t *__restrict__ bits, int wpr, int x, int y) {
  return (int)((bits[(size_t)y * wpr + (x >> 6)] >> (x & 63)) & 1ull);
}

// A pixel with a periodic 4-neighbour of the other phase.
__device__ __forceinline__ bool interfacial(const uint64_t *__restrict__ bits, int W, int H, int q) {
  const int wpr = (W + 63) >> 6;
  const int y = q / W, x = q - y * W;
  const int v = bit_at(bits, wpr, x, y);
  const int xl = x ? x - 1 : W - 1, xr = x + 1 == W ? 0 : x + 1;
  const int yu = y ? y - 1 : H - 1, yd = y + 1 == H ? 0 : y + 1;
  return bit_at(bits, wpr, xl, y) != v || bit_at(bits, wpr, xr, y) != v ||
         bit_at(bits, wpr, x, yu) != v || bit_at(bits, wpr, x, yd) != v;
}

// First i with cw[i] > u (cw: inclusive prefix sums, n > 0 entries).
__device__ __forceinline__ int upper_index(const double *__restrict__ cw, int n, double u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cw[mid] > u) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// A list slot uniform in [0, n) from the high half of a 64-bit draw.
__device__ __forceinline__ int uniform_slot(uint64_t r, int n) {
  return (int)(((r >> 32) * (uint64_t)n) >> 32);
}

// Tag of step `step` in ProposeArgs::pre (never 0, the value of a cleared entry).
__device__ __forceinline__ int pre_tag(uint64_t step) { return (int)(step & 0x3fffffffull) + 1; }

// Pixels a (read from the phase-1 list) and b (from the phase-0 list) as the lists hold them
// after the interchange (sa, sb) whose writes a read may or may not have seen (sa < 0: none):
// see draw_candidate_at.
__device__ __forceinline__ void after_interchange(int &a, int &b, int sa, int sb) {
  if (sa >= 0) {
    a = a == sa || a == sb ? sb : a;
    b = b == sb || b == sa ? sa : b;
  }
}

// Candidate k of step `step`: ctr = {step, k, 0, 0}, key = {seed, 0x6c7066}.
// proposal 0: a, b uniform in the phase-1 / phase-0 lists; 1: as 0, void (a = b = -1) unless
// both pixels are interfacial; 2 (learned): with probability eps (r3) as 0, otherwise a drawn
// with probability proportional to the weights whose inclusive prefix sums are cw1 (over pos1)
// and b likewise with cw0 (over pos0), by inversion of r0, r1.  ia, ib: the list slots; u = r2.
// (sa, sb), sa >= 0: an interchange being applied in the same launch (the draws of the next step
// in the launch that ends this one), whose two list writes may or may not be visible: a's slot
// of the phase-1 list holds sa before and sb after it, b's slot of the phase-0 list sb before and
// sa after, and no other slot holds either pixel, so a read of either value there is taken as
// the value after it.  Not with proposal 1, which reads the image.
__device__ __forceinline__ void draw_candidate_at(const ProposeArgs &p, uint64_t step, int k,
                                                  int sa, int sb, int &a, int &b, int &ia,
                                                  int &ib, double &u) {
  const AnnealDev *st = p.st;
  uint64_t c[4] = {step, (uint64_t)k, 0ull, 0ull};
  philox4x64_10(c, p.seed, 0x6c7066ull);
  const int n1 = st->n1, n0 = st->n0;
  const double u3 = (double)(c[3] >> 11) * (1.0 / 9007199254740992.0);
  if (p.proposal == 2 && !(u3 < p.eps)) {
    const double ua = (double)(c[0] >> 11) * (1.0 / 9007199254740992.0) * p.cw1[n1 - 1];
    const double ub = (double)(c[1] >> 11) * (1.0 / 9007199254740992.0) * p.cw0[n0 - 1];
    ia = upper_index(p.cw1, n1, ua);
    ib = upper_index(p.cw0, n0, ub);
  } else {
    ia = uniform_slot(c[0], n1);
    ib = uniform_slot(c[1], n0);
  }
  a = st->pos1[ia];
  b = st->pos0[ib];
  after_interchange(a, b, sa, sb);
  if (p.proposal == 1 && !(interfacial(p.bits, p.W, p.H, a) && interfacial(p.bits, p.W, p.H, b))) {
    a = -1;
    b = -1;
  }
  u = (double)(c[2] >> 11) * (1.0 / 9007199254740992.0);
}

// Candidate k of the current step.
__device__ __forceinline__ void draw_candidate(const ProposeArgs &p, int k, int &a, int &b,
                                               int &ia, int &ib, double &u) {
  draw_candidate_at(p, p.st->step, k, -1, -1, a, b, ia, ib, u);
}

// Draw k (< K) into cand / slot / U; also zeroes its energy sum (S_acc) and, for k = 0, the
// step's control block and the step's temperature (T_cur: T_sched[step - T_base], else T).
// a, b: the draw (-1 when k >= K).
__device__ __forceinline__ void propose_draw(const ProposeArgs &p, int k, int &a, int &b) {
  if (p.ctl && k == 0) {
    p.ctl->done = 0;
    p.ctl->ks = -1;
    p.ctl->a = -1;
    p.ctl->b = -1;
    p.ctl->S = 0;
  }
  if (p.T_cur && k == 0)
    *p.T_cur = p.T_sched ? p.T_sched[(int64_t)p.st->step - p.T_base] : p.T;
  a = -1;
  b = -1;
  if (k >= p.K) return;
  if (p.S_acc) p.S_acc[k] = 0;
  int ia, ib;
  double u;
  draw_candidate(p, k, a, b, ia, ib, u);
  p.cand[k] = make_int2(a, b);
  p.slot[k] = make_int2(ia, ib);
  p.U[k] = u;
}

// The next step's uniform candidate k (< 64) for its round 0, drawn during this step: the same
// draw with the step counter advanced (a phase-preserving interchange keeps n1 and n0), its
// pixels read from the lists as they are before this step's interchange (round0_candidate
// corrects the one that the interchange moves).
__device__ __forceinline__ void pre_draw(const ProposeArgs &p, int k) {
  const AnnealDev *st = p.st;
  const uint64_t next = st->step + 1;
  uint64_t c[4] = {next, (uint64_t)k, 0ull, 0ull};
  philox4x64_10(c, p.seed, 0x6c7066ull);
  const int a = st->pos1[uniform_slot(c[0], st->n1)], b = st->pos0[uniform_slot(c[1], st->n0)];
  p.pre[(int)(next & 1ull) * 64 + k] = make_int4(a, b, pre_tag(next), 0);
}

// Candidate k (< 64) of the current step for round 0: from the previous step's pre_draw when
// it was written for this step, else drawn here.  Only a and b are produced.
__device__ __forceinline__ void round0_candidate(const ProposeArgs &p, int k, int &a, int &b) {
  if (p.pre && p.proposal == 0) {
    // both parities are read at once, beside the state, so that no load waits on the step
    const int4 q0 = p.pre[k], q1 = p.pre[64 + k];
    const AnnealDev *st = p.st;
    const int tag = pre_tag(st->step);
    const int4 q = q0.z == tag ? q0 : q1;
    if (q.z == tag) {
      // the previous step's interchange put its b at its a's slot of the phase-1 list and its a
      // at its b's slot of the phase-0 list (the lists hold distinct pixels, so a pixel read
      // before it equals that a exactly when it was read at that slot)
      a = q.x == st->last_a ? st->last_b : q.x;
      b = q.y == st->last_b ? st->last_a : q.y;
      return;
    }
  }
  int ia, ib;
  double u;
  draw_candidate(p, k, a, b, ia, ib, u);
}

}  // namespace lpf
