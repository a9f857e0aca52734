// Placement-state records: exact evaluation of interchange candidates by reading two
// contiguous records per candidate (the annealer's evaluation method when they fit in memory).
//
// For vector v and placement x let ones(v, x) be the number of phase-1 pixels on x + path(v)
// (n + 1 pixels).  x counts for phase 1 iff ones = n + 1 and for phase 0 iff ones = 0 (Sec. 2.2
// definition).  An interchange of a (phase 1 -> 0) and b (phase 0 -> 1) lowers ones by one on
// P_a = {a - p_k} and raises it by one on P_b, and leaves P_a ∩ P_b unchanged, so
//   dL1(v) = #{x in P_b \ P_a : ones = n} - #{x in P_a \ P_b : ones = n + 1},
//   dL0(v) = #{x in P_a \ P_b : ones = 1} - #{x in P_b \ P_a : ones = 0}.
// The record of pixel q stores, at bit off(v) + k, the state of placement q - p_k: plane A
// ([ones == 1] for phase 0, [ones == n + 1] for phase 1) and plane B ([ones == 0], [ones == n]).
// A candidate therefore reads plane A of a and plane B of b over [off(v), off(v) + n] for every
// v: a contiguous, coalesced read of 2 * nph * sum(n + 1) bits, with lanes running over vectors.
// Placements in P_a ∩ P_b (only when a and b are within the vector's reach) are taken out of
// both sums with a membership test on the digitised path.  After an accepted interchange the
// ones field is updated on P_a and P_b, and record bits flip only where a placement's state
// changed.
#include "draw_dev.h"
#include "rank_dev.h"
#include "step_dev.h"

namespace lpf {

namespace {

__device__ __forceinline__ int wrapi(int v, int n) {  // v in (-n, 2n)
  v += v < 0 ? n : 0;
  v -= v >= n ? n : 0;
  return v;
}

__device__ __forceinline__ int pix_dx(int32_t p) { return (int)(int16_t)(p & 0xffff); }
__device__ __forceinline__ int pix_dy(int32_t p) { return p >> 16; }

__device__ __forceinline__ int image_bit(const uint64_t *__restrict__ bits, int wpr, int x, int y) {
  return (int)((bits[(size_t)y * wpr + (x >> 6)] >> (x & 63)) & 1ull);
}

// Set bits of the 64-bit window x[0..2] >> sh, first len (<= 64) of them.
__device__ __forceinline__ int popcount_window(const uint32_t (&x)[3], uint32_t sh, int len) {
  const uint32_t lo = __builtin_amdgcn_alignbit(x[1], x[0], sh);
  const uint32_t hi = __builtin_amdgcn_alignbit(x[2], x[1], sh);
  const uint64_t v = ((uint64_t)hi << 32) | lo;
  return __popcll(len == 64 ? v : v & ((1ull << len) - 1ull));
}

// Byte of placement (x, y) in a vector's plane of ones: 8 x 8-pixel tiles of 64 bytes, row-major
// inside a tile and over tiles, so that the placements along a path (which step through rows as
// often as through columns) share cache lines.
__device__ __forceinline__ int64_t ones_at(const RecGeo &g, int x, int y) {
  return ((int64_t)(y >> 3) * ((g.W + 7) >> 3) + (x >> 3)) * 64 + ((y & 7) << 3) + (x & 7);
}

// Number of set bits j of `plane` with off <= j < off + len.
__device__ __forceinline__ int popcount_range(const uint32_t *__restrict__ plane, int off, int len) {
  int c = 0;
  for (int s = 0; s < len; s += 32) {
    const int j = off + s;
    const int w = j >> 5;
    uint32_t x = __builtin_amdgcn_alignbit(plane[w + 1], plane[w], (uint32_t)(j & 31));
    const int l = len - s;
    if (l < 32) x &= (1u << l) - 1u;
    c += __popc(x);
  }
  return c;
}

__device__ __forceinline__ int plane_bit(const uint32_t *__restrict__ plane, int j) {
  return (int)((plane[j >> 5] >> (j & 31)) & 1u);
}

// Is (rx, ry), taken modulo (W, H), a pixel of the digitised path of v = (dx, dy) (n = max
// extent, dy >= 0)?  The path is the segment's pixel set of Sec. 2.2 with the minor coordinate
// sgn(m) floor((2 i |m| + n) / (2 n)), i = 0..n, of the major step i; its extents are below
// (W, H), so the residues are unique.
__device__ __forceinline__ bool on_path(int rx, int ry, int dx, int dy, int n, int W, int H) {
  int rxm = rx % W;
  rxm += rxm < 0 ? W : 0;
  int rym = ry % H;
  rym += rym < 0 ? H : 0;
  const int adx = dx < 0 ? -dx : dx;
  if (adx >= dy) {  // major axis x (also v = 0)
    const int i = dx >= 0 ? rxm : (rxm ? W - rxm : 0);
    if (i > n) return false;
    const int f = n ? (2 * i * dy + n) / (2 * n) : 0;  // n <= 254 for the records
    return rym == f;
  }
  const int i = rym;
  if (i > n) return false;
  const int g = (2 * i * adx + n) / (2 * n);
  const int gx = dx < 0 ? (g ? W - g : 0) : g;
  return rxm == gx;
}

// The plane conditions: side 0 (A) / 1 (B), phase 0 / 1.
__device__ __forceinline__ bool plane_cond(int side, int phase, int o, int n) {
  return side == 0 ? (phase ? o == n + 1 : o == 1) : (phase ? o == n : o == 0);
}

// Record layout for a phase mask: planes A of the kept phases, then planes B (phase 0 first).
template <unsigned MASK>
struct Planes {
  static constexpr int nph = MASK == 3u ? 2 : 1;
  static constexpr int n = 2 * nph;
  static __device__ __forceinline__ constexpr int side(int pl) { return pl / nph; }
  static __device__ __forceinline__ constexpr int phase(int pl) {
    return nph == 2 ? pl % 2 : (MASK == 2u ? 1 : 0);
  }
};

}  // namespace

// Records build, in three launches.  (1) k_rec_ext: the packed image (and the position set)
// as rows of 32-bit words extended periodically (bit x = pixel x mod W, ew words per row).
// (2) k_rec_cond: per vector and 32 consecutive placements x of a row, the count ones(v, x) in
// bit slices (one 32-bit word per count bit, a ripple add per path pixel), from which the ones
// bytes and the plane conditions follow (ones = 0, 1, n, n + 1); the conditions are stored as
// rows of cw words extended periodically past W, so that any 64 placements starting below W
// are three consecutive words.  (3) k_rec_fill: the record bit j = off(v) + k of pixel q is the
// condition of placement q - p_k, so for 64 consecutive pixels of a row lane t (bit j0 + t) reads
// the 64-bit window of its vector's condition row that starts at q0 - p_t; a bit transpose
// across the wave (lanes t x bits over q into lanes q x bits over t) then gives each pixel's 64
// record bits, which are staged in LDS and written per pixel as contiguous dwords.
__global__ void __launch_bounds__(256)
k_rec_ext(RecGeo g, const uint64_t *__restrict__ bits) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nsrc = g.sample ? 2 : 1;
  if (i >= g.H * g.ew * nsrc) return;
  const int src = i / (g.H * g.ew), r = i - src * g.H * g.ew;
  const int y = r / g.ew, w = r - y * g.ew;
  const uint64_t *img = src ? g.sample : bits;
  const int wpr = (g.W + 63) >> 6;
  uint32_t o = 0;
  for (int b = 0; b < 32; ++b) {
    int x = 32 * w + b;
    while (x >= g.W) x -= g.W;
    o |= (uint32_t)image_bit(img, wpr, x, y) << b;
  }
  g.ext[(size_t)src * g.H * g.ew + (size_t)y * g.ew + w] = o;
}

// The 32 bits starting at bit s (0 <= s < W) of an extended row.
__device__ __forceinline__ uint32_t ext_window32(const uint32_t *row, int s) {
  return __builtin_amdgcn_alignbit(row[(s >> 5) + 1], row[s >> 5], (uint32_t)(s & 31));
}

// Bit-sliced count c (nb slices) equal to K, per bit position.
__device__ __forceinline__ uint32_t count_eq(const uint32_t (&c)[8], int nb, int K) {
  uint32_t e = ~0u;
#pragma unroll
  for (int b = 0; b < 8; ++b)
    if (b < nb) e &= ((K >> b) & 1) ? c[b] : ~c[b];
  return ((K >> nb) == 0) ? e : 0u;
}

// Lanes over (row y, word xw) of vector blockIdx.x: placements x = 32 xw + i (taken mod W).
template <unsigned MASK>
__global__ void __launch_bounds__(256)
k_rec_cond(RecGeo g) {
  using P = Planes<MASK>;
  const int v = blockIdx.x;
  const int t = blockIdx.y * blockDim.x + threadIdx.x;
  if (t >= g.H * g.cw) return;
  const int y = t / g.cw, xw = t - y * g.cw;
  const int4 m = g.meta[v];
  const int n = m.y, nb = 32 - __clz(n + 1);  // count bits for 0 .. n + 1 (n <= 254)
  uint32_t c[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) c[b] = 0u;
  for (int j = 0; j <= n; ++j) {
    const int32_t p = g.pix[m.x + j];
    const int yy = wrapi(y + pix_dy(p), g.H);
    int s = 32 * xw + pix_dx(p);
    while (s < 0) s += g.W;
    while (s >= g.W) s -= g.W;
    uint32_t carry = ext_window32(g.ext + (size_t)yy * g.ew, s);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (b < nb) {
        const uint32_t t2 = c[b] & carry;
        c[b] ^= carry;
        carry = t2;
      }
    }
  }
  int s0 = 32 * xw;
  while (s0 >= g.W) s0 -= g.W;
  const uint32_t in = g.sample ? ext_window32(g.ext + (size_t)(g.H + y) * g.ew, s0) : ~0u;
#pragma unroll
  for (int pl = 0; pl < P::n; ++pl) {
    const int K = P::side(pl) == 0 ? (P::phase(pl) ? n + 1 : 1) : (P::phase(pl) ? n : 0);
    g.cond[((size_t)(v * P::n + pl) * g.H + y) * g.cw + xw] = count_eq(c, nb, K) & in;
  }
  // ones bytes of the placements below W (outside the position set: + 128, n <= 126)
  for (int i = 0; i < 32; ++i) {
    const int x = 32 * xw + i;
    if (x >= g.W) break;
    int o = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b)
      if (b < nb) o |= (int)((c[b] >> i) & 1u) << b;
    if (!((in >> i) & 1u)) o += 128;
    g.ones[(size_t)v * g.oplane + ones_at(g, x, y)] = (uint8_t)o;
  }
}

// x's 64 bits transposed across the wave (lane i gets bit i of every lane, lane t in bit t).
// Every lane must be active.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x, int lane) {
  auto step = [&](uint64_t y, int S, uint64_t msk) {
    return (lane & S) ? ((x & ~msk) | ((y & ~msk) >> S)) : ((x & msk) | ((y & msk) << S));
  };
  x = step(xor_lane64<32>(x), 32, 0x00000000FFFFFFFFull);
  x = step(xor_lane64<16>(x), 16, 0x0000FFFF0000FFFFull);
  x = step(xor_lane64<8>(x), 8, 0x00FF00FF00FF00FFull);
  x = step(xor_lane64<4>(x), 4, 0x0F0F0F0F0F0F0F0Full);
  x = step(xor_lane64<2>(x), 2, 0x3333333333333333ull);
  x = step(xor_lane64<1>(x), 1, 0x5555555555555555ull);
  return x;
}

// Workgroup (row segment of 64 pixels, 32-dword tile of the record): each wave takes 64-bit
// chunks of the tile in turn.
template <unsigned MASK>
__global__ void __launch_bounds__(256)
k_rec_fill(RecGeo g) {
  using P = Planes<MASK>;
  __shared__ uint32_t tile[P::n][64][33];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nseg = (g.W + 63) >> 6;
  const int qy = (int)blockIdx.x / nseg, qx0 = ((int)blockIdx.x - qy * nseg) * 64;
  const int w0 = blockIdx.y * 32;
  const int nw = min(32, g.Rw - w0);
  const int nwaves = (int)(blockDim.x >> 6);
  for (int ch = wv; 2 * ch < nw; ch += nwaves) {
    const int j = (w0 + 2 * ch) * 32 + lane;  // this lane's record bit
    uint64_t seg[P::n];
#pragma unroll
    for (int pl = 0; pl < P::n; ++pl) seg[pl] = 0ull;
    if (j < g.Mc) {
      const int v = g.vbit[j] >> 8;
      const int32_t p = g.pix[j];
      const int yy = wrapi(qy - pix_dy(p), g.H);
      int x0 = qx0 - pix_dx(p);
      while (x0 < 0) x0 += g.W;
      while (x0 >= g.W) x0 -= g.W;
      const int sh = x0 & 31;
#pragma unroll
      for (int pl = 0; pl < P::n; ++pl) {
        const uint32_t *r = g.cond + ((size_t)(v * P::n + pl) * g.H + yy) * g.cw + (x0 >> 5);
        const uint32_t r0 = r[0], r1 = r[1], r2 = r[2];
        seg[pl] = ((uint64_t)__builtin_amdgcn_alignbit(r2, r1, (uint32_t)sh) << 32) |
                  __builtin_amdgcn_alignbit(r1, r0, (uint32_t)sh);
      }
    }
#pragma unroll
    for (int pl = 0; pl < P::n; ++pl) {
      const uint64_t tr = wave_transpose64(seg[pl], lane);  // lane = pixel qx0 + lane
      tile[pl][lane][2 * ch] = (uint32_t)tr;
      tile[pl][lane][2 * ch + 1] = (uint32_t)(tr >> 32);
    }
  }
  __syncthreads();
  // write out: wave wv writes pixels wv, wv + nwaves, ...; lanes over the tile's dwords
  for (int pq = wv; pq < 64 && qx0 + pq < g.W; pq += nwaves) {
    uint32_t *R = g.rec + ((size_t)qy * g.W + qx0 + pq) * g.rstride + w0;
    if (lane < nw)
#pragma unroll
      for (int pl = 0; pl < P::n; ++pl) R[(size_t)pl * g.Rw + lane] = tile[pl][pq][lane];
  }
}

// Is d (|d| < M) within [-r, r] modulo M?
__device__ __forceinline__ bool within_small(int d, int M, int r) {
  const int m = d < 0 ? d + M : d;
  return m <= r || M - m <= r;
}

// Placements of vector v (m = meta[v], n = m.y > 0) through s whose other end s + (DX, DY) is on
// their path as well: x = s - p_k with x + p_j = s + (DX, DY) for some j.  Along the major axis
// p_j - p_k has the index difference t = j - k, so t is fixed modulo the period by (DX, DY):
// t = t0 for k <= n - t0 and t = t0 - P for k >= P - t0 (range 0 and 1).  The minor coordinate
// of point k is floor((2 k e + n) / 2n) (e the minor extent), so with the error term
// r_k = (2 k e + n) mod 2n and 2 t e = q 2n + rho (0 <= rho < 2n) the minor difference of
// points k + t and k is q when r_k < 2n - rho and q + 1 otherwise; a range holds placements
// only when one of the two equals the minor part of (DX, DY) modulo its period: those k with
// r_k < th (lo) or r_k >= th (hi).
struct BothRange {
  int k0, k1, th;
  bool lo, hi;
};
__device__ __forceinline__ void both_ranges(const RecGeo &g, int4 m, int DX, int DY,
                                            BothRange (&r)[2], int &mext) {
  const int n = m.y, dxv = m.z, dyv = m.w;
  const int adx = dxv < 0 ? -dxv : dxv;
  const bool xm = adx >= dyv;
  const int sx = dxv < 0 ? -1 : 1;
  const int Pm = xm ? g.W : g.H, Qm = xm ? g.H : g.W;
  int t0 = xm ? sx * DX : DY;  // in (-Pm, Pm)
  t0 += t0 < 0 ? Pm : 0;
  int mm = xm ? DY : sx * DX;  // in (-Qm, Qm)
  mm += mm < 0 ? Qm : 0;
  mext = xm ? dyv : adx;
  const int n2 = 2 * n;
#pragma unroll
  for (int ps = 0; ps < 2; ++ps) {
    const int t = ps == 0 ? t0 : t0 - Pm;
    r[ps].k0 = ps == 0 ? 0 : Pm - t0;
    r[ps].k1 = ps == 0 ? n - t0 : n;
    const int T2 = 2 * t * mext;
    int q = T2 / n2, rho = T2 - q * n2;
    if (rho < 0) {  // floor division
      rho += n2;
      --q;
    }
    const bool any = r[ps].k0 <= r[ps].k1;
    r[ps].lo = any && (q == mm || q == mm - Qm);
    r[ps].hi = any && (q + 1 == mm || q + 1 == mm - Qm);
    r[ps].th = n2 - rho;
  }
}

// Bit k set for each such placement, for n + 1 <= 64, from the error-term masks (one load per
// range that can hold any).
__device__ __forceinline__ uint64_t both_mask(const RecGeo &g, int4 m, int v, int DX, int DY) {
  BothRange r[2];
  int mext;
  both_ranges(g, m, DX, DY, r, mext);
  const uint64_t *E = g.emask + (2 * (int64_t)m.x - v);
  uint64_t both = 0;
#pragma unroll
  for (int ps = 0; ps < 2; ++ps) {
    if (!r[ps].lo && !r[ps].hi) continue;
    const uint64_t ge = E[r[ps].th];
    const uint64_t range = ((~0ull) >> (63 - r[ps].k1)) & ((~0ull) << r[ps].k0);
    both |= range & ((r[ps].hi ? ge : 0ull) | (r[ps].lo ? ~ge : 0ull));
  }
  return both;
}

// hit(k) for each such placement, walking the error terms (paths of any length).
template <class F>
__device__ __forceinline__ void both_walk(const RecGeo &g, int4 m, int DX, int DY, F &&hit) {
  BothRange r[2];
  int mext;
  both_ranges(g, m, DX, DY, r, mext);
  const int n = m.y, n2 = 2 * n;
  for (int ps = 0; ps < 2; ++ps) {
    if (!r[ps].lo && !r[ps].hi) continue;
    int e = (n + 2 * r[ps].k0 * mext) % n2;
    for (int kk = r[ps].k0; kk <= r[ps].k1; ++kk) {
      if (kk > r[ps].k0) {
        e += 2 * mext;
        e -= e >= n2 ? n2 : 0;
      }
      if (e >= r[ps].th ? r[ps].hi : r[ps].lo) hit(kk);
    }
  }
}

// Bits sh .. sh + 63 of three consecutive words.
__device__ __forceinline__ uint64_t window64(const uint32_t (&x)[3], uint32_t sh) {
  return ((uint64_t)__builtin_amdgcn_alignbit(x[2], x[1], sh) << 32) |
         __builtin_amdgcn_alignbit(x[1], x[0], sh);
}

// Exact dL of interchange (a, b) for vector v, one entry per kept phase.  Invalid or same-phase
// pairs change nothing.
// ORDERED: the pair is known to be (phase-1 pixel, phase-0 pixel), as the annealer's draws are,
// so the image is not read.
template <unsigned MASK, bool ORDERED>
__device__ __forceinline__ void rec_delta(const RecGeo &g, const uint64_t *__restrict__ bits,
                                          int a, int b, int v, int4 m, int (&d)[2]) {
  using P = Planes<MASK>;
  d[0] = 0;
  d[1] = 0;
  const int64_t N = (int64_t)g.W * g.H;
  if (a < 0 || b < 0 || a >= N || b >= N || a == b || v >= g.nv) return;
  int ay = a / g.W, ax = a - ay * g.W, by = b / g.W, bx = b - by * g.W;
  if (!ORDERED) {
    const int wpr = (g.W + 63) >> 6;
    const int va = image_bit(bits, wpr, ax, ay), vb = image_bit(bits, wpr, bx, by);
    if (va == vb) return;
    if (va == 0) {  // a leaves phase 1, b enters it
      int t = a; a = b; b = t;
      t = ax; ax = bx; bx = t;
      t = ay; ay = by; by = t;
    }
  }
  const int off = m.x, n = m.y, len = n + 1;
  const uint32_t *RA = g.rec + (size_t)a * g.rstride;                 // planes A of a
  const uint32_t *RB = g.rec + (size_t)b * g.rstride + P::nph * g.Rw;  // planes B of b
  const uint32_t *RBa = g.rec + (size_t)a * g.rstride + P::nph * g.Rw;  // planes B of a
  // placements in P_a ∩ P_b keep their count (a leaves phase 1, b enters it); they exist only
  // when b - a lies within the vector's box.  Such a placement holds b (phase 0), so for phase 1
  // only the sum over P_b can count it, by [ones = n], which plane B of a records for it too;
  // it holds a (phase 1), so for phase 0 only the sum over P_a can, by [ones = 1] of plane A
  // of a.  Both are taken out of dL.
  const int DX = bx - ax, DY = by - ay;
  if (len <= 64) {
    // a range of up to 64 bits spans three words (planes carry two padding words): every
    // plane's words are requested before any is used, so the record reads overlap; the words
    // of planes B of a that a placement in both sets needs are requested with them
    const int w = off >> 5;
    const uint32_t sh = (uint32_t)(off & 31);
    uint32_t xa[P::nph][3], xb[P::nph][3], xc[P::nph][3];
#pragma unroll
    for (int p = 0; p < P::nph; ++p)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        xa[p][i] = RA[(size_t)p * g.Rw + w + i];
        xb[p][i] = RB[(size_t)p * g.Rw + w + i];
      }
    const bool near = n > 0 && within_small(DX, g.W, m.z < 0 ? -m.z : m.z) &&
                      within_small(DY, g.H, m.w);
#pragma unroll
    for (int p = 0; p < P::nph; ++p)
#pragma unroll
      for (int i = 0; i < 3; ++i) xc[p][i] = 0u;
    if (near) {
#pragma unroll
      for (int p = 0; p < P::nph; ++p)
        if (P::phase(p))
#pragma unroll
          for (int i = 0; i < 3; ++i) xc[p][i] = RBa[(size_t)p * g.Rw + w + i];
    }
#pragma unroll
    for (int p = 0; p < P::nph; ++p) {
      const int cA = popcount_window(xa[p], sh, len), cB = popcount_window(xb[p], sh, len);
      d[p] = P::phase(p) ? cB - cA : cA - cB;
    }
    if (near) {
      const uint64_t both = both_mask(g, m, v, DX, DY);  // bit k: a - p_k lies in P_b too
#pragma unroll
      for (int p = 0; p < P::nph; ++p)
        d[p] -= __popcll(both & window64(P::phase(p) ? xc[p] : xa[p], sh));
    }
    return;
  }
#pragma unroll
  for (int p = 0; p < P::nph; ++p) {
    const int cA = popcount_range(RA + (size_t)p * g.Rw, off, len);
    const int cB = popcount_range(RB + (size_t)p * g.Rw, off, len);
    d[p] = P::phase(p) ? cB - cA : cA - cB;
  }
  if (within_small(DX, g.W, m.z < 0 ? -m.z : m.z) && within_small(DY, g.H, m.w))
    both_walk(g, m, DX, DY, [&](int k) {
#pragma unroll
      for (int s = 0; s < P::nph; ++s)
        d[s] -= P::phase(s) ? plane_bit(RBa + (size_t)s * g.Rw, off + k)
                            : plane_bit(RA + (size_t)s * g.Rw, off + k);
    });
}

// One round: block (vector block, candidate slot); the slots stride over the round's evaluation
// positions k0 .. k0 + C - 1 (candidate order[i], or i without an order).  Lanes run over
// vectors; the candidate is uniform.  Each block adds its part of a candidate's
// energy sum into S_acc[k] and stores the candidate's dL when dl is given.
template <unsigned MASK, bool ORDERED>
__global__ void __launch_bounds__(256)
k_rec_round(RecGeo g, const uint64_t *__restrict__ bits, const int2 *__restrict__ cand, int K,
            int k0, int C, const uint32_t *__restrict__ counts,
            const uint32_t *__restrict__ target, int64_t N, int64_t Nt,
            int64_t *__restrict__ S_acc, int16_t *__restrict__ dl, int64_t dl_t, int64_t dl_k,
            StepCtl *__restrict__ ctl, const int32_t *__restrict__ order,
            const double *__restrict__ U, const double *__restrict__ Tp, int pi0, int pC,
            const int64_t *__restrict__ S0) {
  using P = Planes<MASK>;
  __shared__ long long s_part[4];
  __shared__ int s_prev;
  if (prev_round_accepted(S_acc, S0, cand, U, order, pi0, pC, Tp,
                          (double)N * (double)N * (double)Nt, ctl, &s_prev))
    return;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const bool vin = v < g.nv;
  // candidate-independent operands first, so that their loads overlap the candidate's
  // loads at a clamped index, without a branch, so that they overlap what follows; lanes past
  // the last vector contribute nothing (rec_delta returns zeros for them)
  const int vc = vin ? v : g.nv - 1;
  const int4 m = g.meta[vc];
  int64_t Lc[2] = {0, 0}, Tc[2] = {0, 0};
#pragma unroll
  for (int p = 0; p < P::nph; ++p) {
    Lc[p] = counts[(size_t)p * g.nv + vc];
    Tc[p] = target[(size_t)p * g.nv + vc];
  }
  for (int kr = blockIdx.y; kr < C; kr += gridDim.y) {
    if (k0 + kr >= K) break;
    const int k = order ? order[k0 + kr] : k0 + kr;  // candidate (draw index)
    const int2 ab = cand[k];
    int d[2];
    rec_delta<MASK, ORDERED>(g, bits, ab.x, ab.y, v, m, d);
    int64_t S = 0;
    if (vin) {
#pragma unroll
      for (int p = 0; p < P::nph; ++p) {
        S += energy_term(d[p], Lc[p], Tc[p], N, Nt);
        if (dl) dl[(int64_t)((size_t)p * g.nv + v) * dl_t + (int64_t)k * dl_k] = (int16_t)d[p];
      }
    }
    // block sum (int64: exact), one accumulation per block
    S = wave_sum63_i64(S);
    if ((threadIdx.x & 63) == 63) s_part[threadIdx.x >> 6] = S;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long tot = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += s_part[w];
      add_acc(&S_acc[k], tot);
    }
    __syncthreads();
  }
}

// Round 0 of a step in the launch of the step's draws (unranked draws, K > 64): workgroups
// [0, nprop) are the draws of k_propose (propose_draw); workgroup nprop draws the next step's
// first 64 uniform candidates (pre_draw); workgroup nprop + 1 + kr * nvb + vb takes vector block
// vb of draw kr < C0, which it takes from the previous step's pre_draw or draws again itself (the
// same counter gives the same draw, so it does not wait for the draw blocks), and adds its block
// sum into S0[kr] instead of S_acc, which the draw blocks are zeroing.  S0 is zero at the start
// of every step (cleared at allocation and by the end of each step); round 1 reads it when it
// decides round 0.
template <unsigned MASK>
__global__ void __launch_bounds__(256)
k_rec_draw_round0(RecGeo g, ProposeArgs p, int nprop, int C0, const uint32_t *__restrict__ counts,
                  const uint32_t *__restrict__ target, int64_t N, int64_t Nt,
                  int64_t *__restrict__ S0, int16_t *__restrict__ dl, int64_t dl_t,
                  int64_t dl_k) {
  using P = Planes<MASK>;
  __shared__ long long s_part[4];
  if ((int)blockIdx.x < nprop) {
    int a, b;
    propose_draw(p, (int)(blockIdx.x * blockDim.x + threadIdx.x), a, b);
    return;
  }
  if ((int)blockIdx.x == nprop) {  // the next step's round-0 candidates
    if (p.pre && p.proposal == 0 && threadIdx.x < 64) pre_draw(p, (int)threadIdx.x);
    return;
  }
  const int nvb = (g.nv + 255) >> 8;
  const int bi = (int)blockIdx.x - nprop - 1, kr = bi / nvb, vb = bi - kr * nvb;
  if (kr >= C0) return;
  const int v = vb * 256 + (int)threadIdx.x;
  const bool vin = v < g.nv;
  // loads at a clamped index, without a branch, so that they overlap what follows; lanes past
  // the last vector contribute nothing (rec_delta returns zeros for them)
  const int vc = vin ? v : g.nv - 1;
  const int4 m = g.meta[vc];
  int64_t Lc[2] = {0, 0}, Tc[2] = {0, 0};
#pragma unroll
  for (int q = 0; q < P::nph; ++q) {
    Lc[q] = counts[(size_t)q * g.nv + vc];
    Tc[q] = target[(size_t)q * g.nv + vc];
  }
  int a, b;
  round0_candidate(p, kr, a, b);
  int d[2];
  rec_delta<MASK, true>(g, p.bits, a, b, v, m, d);
  int64_t S = 0;
  if (vin) {
#pragma unroll
    for (int q = 0; q < P::nph; ++q) {
      S += energy_term(d[q], Lc[q], Tc[q], N, Nt);
      dl[(int64_t)((size_t)q * g.nv + v) * dl_t + (int64_t)kr * dl_k] = (int16_t)d[q];
    }
  }
  S = wave_sum63_i64(S);
  if ((threadIdx.x & 63) == 63) s_part[threadIdx.x >> 6] = S;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += s_part[w];
    add_acc(&S0[kr], tot);
  }
}

// Round 0 of a ranked step together with the merge of the ranking (records method, K > 64,
// after k_propose or the previous step's end wrote the rank keys and workgroup lists): every
// workgroup merges the lists itself (merge_lists16).  Workgroup 0 writes the evaluation order for
// the later rounds (the best 64, then the other draws of [0, R) in draw order, then R .. K - 1);
// workgroup 1 + kr * nvb + vb evaluates vector block vb of the kr-th best draw and adds its block
// sum into S0[kr] (zero at the start of every step; round 1 reads it when it decides round 0).
// The launch also does the step's resets, which a draw made by the previous step's end does not.
template <unsigned MASK>
__global__ void __launch_bounds__(256)
k_rec_rank_round0(RecGeo g, const uint64_t *__restrict__ lists, const uint64_t *__restrict__ keys,
                  int K, int32_t *__restrict__ order, const uint64_t *__restrict__ bits,
                  const int2 *__restrict__ cand, int C0, const uint32_t *__restrict__ counts,
                  const uint32_t *__restrict__ target, int64_t N, int64_t Nt,
                  int64_t *__restrict__ S_acc, int64_t *__restrict__ S0,
                  int16_t *__restrict__ dl, int64_t dl_t, int64_t dl_k,
                  StepCtl *__restrict__ ctl, const AnnealDev *__restrict__ st,
                  double *__restrict__ T_cur, const double *__restrict__ T_sched, int64_t T_base,
                  double T_value) {
  using P = Planes<MASK>;
  constexpr int kPer = kRankMax / 256;  // draws of [0, R) per thread in the compaction
  // the step's resets: energy sums of the later rounds (spread over all workgroups; round 0
  // adds into S0), and in workgroup 0 the control block, the next step's number and the step's
  // temperature
  for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < K; i += (int)(gridDim.x * blockDim.x))
    S_acc[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint64_t step = st->step;
    ctl->done = 0;
    ctl->ks = -1;
    ctl->a = -1;
    ctl->b = -1;
    ctl->S = 0;
    ctl->next_step = step + 1;
    *T_cur = T_sched ? T_sched[(int64_t)step - T_base] : T_value;
  }
  __shared__ uint64_t sl[2][64];
  __shared__ uint64_t s_key;
  __shared__ int s_cnt[kPer][4];
  __shared__ long long s_part[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int R = min(K, kRankMax), T = min(R, kRankTop), nl = (R + 255) >> 8;
  if (blockIdx.x == 0) {
    // this thread's keys are requested before the merge, so that their latency overlaps it
    uint64_t kk[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int i = j * 256 + (int)threadIdx.x;
      kk[j] = i < R ? keys[i] : 0ull;
    }
    const uint64_t m = merge_lists16(lists, nl, sl);
    if (w == 0) {
      if (lane < T) order[lane] = (int32_t)~(uint32_t)m;
      if (lane == T - 1) s_key = m;  // the T-th best key: every other draw is below it
    }
    __syncthreads();
    const uint64_t thr = s_key;
    // the other draws of [0, R) in draw order: every wave's count per slice j first, then the
    // positions from their prefix sums (one barrier for all slices)
    uint64_t bal[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int i = j * 256 + (int)threadIdx.x;
      bal[j] = __ballot(i < R && kk[j] < thr);
      if (lane == 0) s_cnt[j][w] = __popcll(bal[j]);
    }
    __syncthreads();
    int base = T;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      int before = 0, total = 0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        before += v < w ? s_cnt[j][v] : 0;
        total += s_cnt[j][v];
      }
      if ((bal[j] >> lane) & 1ull) {
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal[j] >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)bal[j], 0u));
        order[base + before + below] = j * 256 + (int)threadIdx.x;
      }
      base += total;
    }
    for (int i = R + (int)threadIdx.x; i < K; i += 256) order[i] = i;
    return;
  }
  const uint64_t m = merge_lists16(lists, nl, sl);
  const int nvb = (g.nv + 255) >> 8;
  const int bi = (int)blockIdx.x - 1, kr = bi / nvb, vb = bi - kr * nvb;
  if (w == 0 && lane == kr) s_key = m;
  __syncthreads();
  if (kr >= C0 || kr >= T) return;
  const int k = (int)~(uint32_t)s_key;  // draw index of the kr-th best
  const int v = vb * 256 + (int)threadIdx.x;
  const bool vin = v < g.nv;
  // loads at a clamped index, without a branch, so that they overlap what follows; lanes past
  // the last vector contribute nothing (rec_delta returns zeros for them)
  const int vc = vin ? v : g.nv - 1;
  const int4 mv = g.meta[vc];
  int64_t Lc[2] = {0, 0}, Tc[2] = {0, 0};
#pragma unroll
  for (int q = 0; q < P::nph; ++q) {
    Lc[q] = counts[(size_t)q * g.nv + vc];
    Tc[q] = target[(size_t)q * g.nv + vc];
  }
  const int2 ab = cand[k];
  int d[2];
  rec_delta<MASK, true>(g, bits, ab.x, ab.y, v, mv, d);
  int64_t S = 0;
  if (vin) {
#pragma unroll
    for (int q = 0; q < P::nph; ++q) {
      S += energy_term(d[q], Lc[q], Tc[q], N, Nt);
      dl[(int64_t)((size_t)q * g.nv + v) * dl_t + (int64_t)k * dl_k] = (int16_t)d[q];
    }
  }
  S = wave_sum63_i64(S);
  if ((threadIdx.x & 63) == 63) s_part[threadIdx.x >> 6] = S;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) tot += s_part[q];
    add_acc(&S0[kr], tot);
  }
}

// The accepted interchange (a now in phase 0, b in phase 1) applied to ones and the records of
// vector v on one side (side 0: the placements through a, 1: through b), by one wave.  Lane k
// takes placement x_k = s - p_k (s = a or b), updates ones(v, x_k) and finds which plane bits of
// x_k change; those bits live in the records of the pixels x_k + p_j at bit off + j, j = 0..n.
// Placements in both P_a and P_b keep their count and are left alone.
//
// For n + 1 <= 64 (upd_load, then upd_apply, so that a wave can issue the loads of several
// pairs before it applies any) the flips are merged before they are issued: with j = k + d the
// record pixel is s + (p_{k+d} - p_k), whose major part is d and whose minor part is q_d or
// q_d + 1: with the minor extent e, 2 d e = q_d 2n + rho_d (0 <= rho_d < 2n) and the error term
// r_k = (2 k e + n) mod 2n of point k, it is q_d + 1 exactly when r_k >= 2n - rho_d.  So lane d
// splits the changed k into those two classes (one compare per changed k against the error term
// that lane k holds) and flips each class's mask << (off + d) with at most three atomic XORs per
// plane, instead of one per (k, j).  Longer paths flip bit by bit (upd_long).
struct UpdPair {
  int v, side;
  int4 m;         // meta[v]
  int32_t pk;     // p_lane (lane <= n)
  uint8_t *op;    // ones byte of the lane's placement
  int o0;         // its value before the interchange
  uint64_t keep;  // placements in both P_a and P_b (bit k)
};

template <unsigned MASK>
__device__ __forceinline__ void upd_load(const RecGeo &g, int a, int b, UpdPair &u) {
  const int lane = threadIdx.x & 63;
  const int n = u.m.y;
  const int ay = a / g.W, ax = a - ay * g.W, by = b / g.W, bx = b - by * g.W;
  const int sx = u.side ? bx : ax, sy = u.side ? by : ay;
  const int ox = u.side ? ax - bx : bx - ax, oy = u.side ? ay - by : by - ay;
  const bool near = within_small(ox, g.W, u.m.z < 0 ? -u.m.z : u.m.z) && within_small(oy, g.H, u.m.w);
  u.keep = near && n > 0 ? both_mask(g, u.m, u.v, ox, oy) : 0ull;
  const int x = wrapi(sx - pix_dx(u.pk), g.W), y = wrapi(sy - pix_dy(u.pk), g.H);
  u.op = g.ones + (size_t)u.v * g.oplane + ones_at(g, x, y);
  u.o0 = lane <= n ? (int)*u.op : 0;
}

template <unsigned MASK>
__device__ __forceinline__ void upd_apply(const RecGeo &g, int a, int b, const UpdPair &u) {
  using P = Planes<MASK>;
  const int lane = threadIdx.x & 63;
  const int off = u.m.x, n = u.m.y;
  const int ay = a / g.W, ax = a - ay * g.W, by = b / g.W, bx = b - by * g.W;
  const int sx = u.side ? bx : ax, sy = u.side ? by : ay;
  unsigned chg = 0;
  if (lane <= n && !((u.keep >> lane) & 1ull)) {
    const int o0 = u.o0, o1 = u.side ? o0 + 1 : o0 - 1;
    *u.op = (uint8_t)o1;
#pragma unroll
    for (int pl = 0; pl < P::n; ++pl)
      if (plane_cond(P::side(pl), P::phase(pl), o0, n) != plane_cond(P::side(pl), P::phase(pl), o1, n))
        chg |= 1u << pl;
  }
  uint64_t M[P::n], any = 0;
#pragma unroll
  for (int pl = 0; pl < P::n; ++pl) {
    M[pl] = __ballot((chg >> pl) & 1u);
    any |= M[pl];
  }
  if (!any) return;
  const int adx = u.m.z < 0 ? -u.m.z : u.m.z;
  const bool xm = adx >= u.m.w;
  const int sgn = u.m.z < 0 ? -1 : 1, mext = xm ? u.m.w : adx, n2 = 2 * n;
  const int ek = n > 0 && lane <= n ? (2 * lane * mext + n) % n2 : 0;  // error term of point lane
  // this lane's offsets d = dd - n, dd = lane and lane + 64 (when dd <= 2n): q_d and the
  // threshold 2n - rho_d of class q_d + 1 (none for d = 0)
  int q[2], th[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int d = lane + 64 * h - n;
    q[h] = 0;
    th[h] = INT_MAX;
    if (d != 0 && d <= n) {  // then n > 0
      const int T2 = 2 * d * mext;
      int qq = T2 / n2, rho = T2 - qq * n2;
      if (rho < 0) {  // floor division
        rho += n2;
        --qq;
      }
      q[h] = qq;
      th[h] = n2 - rho;
    }
  }
  uint64_t c1[2] = {0ull, 0ull};  // changed k of class q_d + 1
  for (uint64_t t = any; t; t &= t - 1) {
    const int k = __ffsll((unsigned long long)t) - 1;  // uniform
    const int e = __builtin_amdgcn_readlane(ek, k);
    c1[0] |= (uint64_t)(e >= th[0]) << k;
    c1[1] |= (uint64_t)(e >= th[1]) << k;
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int dd = lane + 64 * h;
    if (dd > 2 * n) continue;
    const int d = dd - n;
    const int k0 = d < 0 ? -d : 0, k1 = d > 0 ? n - d : n;
    const uint64_t range = ((~0ull) >> (63 - k1)) & ((~0ull) << k0);
    const int base = off + d, sh = base & 31;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const uint64_t cls = range & (c ? c1[h] : ~c1[h]);
      if (!(cls & any)) continue;
      const int mn = q[h] + c;
      const int qx = wrapi(sx + (xm ? sgn * d : sgn * mn), g.W);
      const int qy = wrapi(sy + (xm ? mn : d), g.H);
      uint32_t *R = g.rec + ((size_t)qy * g.W + qx) * g.rstride + (base >> 5);
#pragma unroll
      for (int pl = 0; pl < P::n; ++pl) {
        const uint64_t cm = M[pl] & cls;
        if (!cm) continue;
        const uint32_t w0 = (uint32_t)(cm << sh);
        const uint32_t w1 = (uint32_t)((cm << sh) >> 32);
        const uint32_t w2 = sh ? (uint32_t)(cm >> (64 - sh)) : 0u;
        uint32_t *Rp = R + (size_t)pl * g.Rw;
        if (w0) atomicXor(Rp, w0);
        if (w1) atomicXor(Rp + 1, w1);
        if (w2) atomicXor(Rp + 2, w2);
      }
    }
  }
}

// The same for a path of more than 64 pixels, bit by bit.
template <unsigned MASK>
__device__ __forceinline__ void upd_long(const RecGeo &g, int a, int b, int v, int side, int4 m) {
  using P = Planes<MASK>;
  const int lane = threadIdx.x & 63;
  const int off = m.x, n = m.y;
  const int ay = a / g.W, ax = a - ay * g.W, by = b / g.W, bx = b - by * g.W;
  const int sx = side ? bx : ax, sy = side ? by : ay;
  const int ox = side ? ax - bx : bx - ax, oy = side ? ay - by : by - ay;
  const bool near = within_small(ox, g.W, m.z < 0 ? -m.z : m.z) && within_small(oy, g.H, m.w);
  for (int kc = 0; kc <= n; kc += 64) {
    const int k = kc + lane;
    if (k > n) continue;
    const int32_t pk = g.pix[off + k];
    if (near && on_path(ox + pix_dx(pk), oy + pix_dy(pk), m.z, m.w, n, g.W, g.H)) continue;
    const int x = wrapi(sx - pix_dx(pk), g.W), y = wrapi(sy - pix_dy(pk), g.H);
    uint8_t *op = g.ones + (size_t)v * g.oplane + ones_at(g, x, y);
    const int o0 = (int)*op, o1 = side ? o0 + 1 : o0 - 1;
    *op = (uint8_t)o1;
    unsigned chg = 0;
#pragma unroll
    for (int pl = 0; pl < P::n; ++pl)
      if (plane_cond(P::side(pl), P::phase(pl), o0, n) != plane_cond(P::side(pl), P::phase(pl), o1, n))
        chg |= 1u << pl;
    if (!chg) continue;
    for (int j = 0; j <= n; ++j) {
      const int32_t pj = g.pix[off + j];
      const int qx = wrapi(x + pix_dx(pj), g.W), qy = wrapi(y + pix_dy(pj), g.H);
      uint32_t *R = g.rec + ((size_t)qy * g.W + qx) * g.rstride;
      const int bit = off + j;
#pragma unroll
      for (int pl = 0; pl < P::n; ++pl)
        if (chg & (1u << pl)) atomicXor(R + (size_t)pl * g.Rw + (bit >> 5), 1u << (bit & 31));
    }
  }
}

// End of a step under the records method: workgroups 0 .. nupd - 1 apply the accepted
// interchange to ones and records (upd_load and upd_apply, upd_long for paths of 64 pixels or
// more), workgroup nupd does the step's upkeep
// (step_apply).  Each workgroup takes the step's decision itself (ctl->ks, or the same scan of the
// last round), so one launch replaces the upkeep kernel followed by the update kernel: the upkeep
// touches counts, image bits, pixel lists and energy, none of which the update reads.
// The update waves stride over the 2 nv (vector, side) pairs, so that the launch stays within
// what the device holds at once (a second round of workgroups would repeat the whole latency
// chain of decision, load and flips).
// PRE: the wave's first PRE (vector, side) pairs are prefetched (1 when every pair has its own
// wave).  DRAW: workgroups past nupd (ranked chains) draw the next step with the arguments *nxp:
// candidates, rank keys and each 256-draw workgroup's best 64, from the pixel lists as this
// step's interchange leaves them (draw_candidate_at), so that the next step needs no launch of
// its draws.
template <unsigned MASK, int PRE, bool DRAW>
__global__ void __launch_bounds__(256)
k_rec_step_end(RecGeo g, FinalArgs f, int nupd, const ProposeArgs *__restrict__ nxp) {
  __shared__ int s_first;
  __shared__ uint64_t sl[2][64];
  // the wave's first PRE (vector, side) pairs: vectors and path pixels do not depend on the
  // decision, so they are loaded first, at clamped indices (no branch), to overlap its reads
  constexpr int kPre = PRE;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wid0 = (int)blockIdx.x * 4 + wave;
  const int stride = 4 * nupd, npairs = 2 * g.nv;
  UpdPair u[kPre];
#pragma unroll
  for (int i = 0; i < kPre; ++i) {
    const int wid = min(wid0 + i * stride, npairs - 1);
    u[i].v = wid >> 1;
    u[i].side = wid & 1;
    u[i].m = g.meta[u[i].v];
  }
#pragma unroll
  for (int i = 0; i < kPre; ++i) u[i].pk = g.pix[u[i].m.x + min(lane, u[i].m.y)];
  // done, ks, a, b of an earlier round's decision in one load (nothing in this launch writes
  // the control block: the upkeep is told not to)
  const int4 c4 = *reinterpret_cast<const int4 *>(f.ctl);
  const int ks0 = c4.y;
  if (DRAW && (int)blockIdx.x > nupd) {
    // the draw does not depend on this step's decision, only its correction for the step's
    // interchange does: the counter-based draw and its list reads go first
    const ProposeArgs &nx = *nxp;
    const int db = (int)blockIdx.x - nupd - 1, k = db * 256 + (int)threadIdx.x;
    const bool in = k < nx.K;
    int a = -1, b = -1, ia = 0, ib = 0;
    double u = 0.0;
    if (in) draw_candidate_at(nx, f.ctl->next_step, k, -1, -1, a, b, ia, ib, u);
    const int ks = step_choice(f, ks0, &s_first);
    const int2 sab = ks < 0 ? make_int2(-1, -1) : ks0 >= 0 ? make_int2(c4.z, c4.w) : f.cand[ks];
    if (in) {
      after_interchange(a, b, sab.x, sab.y);
      nx.cand[k] = make_int2(a, b);
      nx.slot[k] = make_int2(ia, ib);
      nx.U[k] = u;
    }
    if (nx.rank_score && db * 256 < min(nx.K, kRankMax)) {
      const bool ranked = k < min(nx.K, kRankMax);
      const uint64_t key = ranked ? rank_key(a, b, k, nx.rank_score) : 0ull;
      if (ranked) nx.rank_keys[k] = key;
      block_top64(key, sl, nx.rank_lists + (size_t)db * kRankTop);
    }
    return;
  }
  const int ks = step_choice(f, ks0, &s_first);
  // counts += dL shared by all nupd + 1 workgroups (one term per thread at most sizes)
  step_counts(f, ks, (int)blockIdx.x, nupd + 1);
  if ((int)blockIdx.x == nupd) {
    step_apply(f, ks, false, false);
    return;
  }
  if (ks < 0) return;
  const int2 ab = ks0 >= 0 ? make_int2(c4.z, c4.w) : f.cand[ks];
  // the loads of every prefetched pair are issued before any pair is applied
#pragma unroll
  for (int i = 0; i < kPre; ++i)
    if (wid0 + i * stride < npairs && u[i].m.y < 64) upd_load<MASK>(g, ab.x, ab.y, u[i]);
#pragma unroll
  for (int i = 0; i < kPre; ++i) {
    if (wid0 + i * stride >= npairs) break;
    if (u[i].m.y < 64)
      upd_apply<MASK>(g, ab.x, ab.y, u[i]);
    else
      upd_long<MASK>(g, ab.x, ab.y, u[i].v, u[i].side, u[i].m);
  }
  for (int wid = wid0 + kPre * stride; wid < npairs; wid += stride) {
    UpdPair w;
    w.v = wid >> 1;
    w.side = wid & 1;
    w.m = g.meta[w.v];
    if (w.m.y < 64) {
      w.pk = g.pix[w.m.x + min(lane, w.m.y)];
      upd_load<MASK>(g, ab.x, ab.y, w);
      upd_apply<MASK>(g, ab.x, ab.y, w);
    } else {
      upd_long<MASK>(g, ab.x, ab.y, w.v, w.side, w.m);
    }
  }
}

#define LPF_REC_MASK_SWITCH(mask, CALL) \
  switch (mask) {                             \
    case 1u: CALL(1u); break;                 \
    case 2u: CALL(2u); break;                 \
    default: CALL(3u); break;                 \
  }

// The two parities' arguments of the next-step draws into device memory (kernel arguments are
// copied at the launch, so the host structs need not outlive it).
__global__ void k_rec_set_next(ProposeArgs *__restrict__ dst, ProposeArgs a0, ProposeArgs a1) {
  if (threadIdx.x == 0) {
    dst[0] = a0;
    dst[1] = a1;
  }
}

hipError_t launch_rec_set_next(ProposeArgs *dst, const ProposeArgs &a0, const ProposeArgs &a1,
                               hipStream_t stream) {
  hipLaunchKernelGGL(k_rec_set_next, dim3(1), dim3(64), 0, stream, dst, a0, a1);
  return hipGetLastError();
}

hipError_t launch_rec_build(const RecGeo &g, const uint64_t *bits, hipStream_t stream) {
  const int next = g.H * g.ew * (g.sample ? 2 : 1);
  hipLaunchKernelGGL(k_rec_ext, dim3((unsigned)((next + 255) / 256)), dim3(256), 0, stream, g, bits);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 gc((unsigned)g.nv, (unsigned)((g.H * g.cw + 255) / 256));
  const dim3 gf((unsigned)(g.H * ((g.W + 63) / 64)), (unsigned)((g.Rw + 31) / 32));
#define LPF_BUILD(M)                                                              \
  hipLaunchKernelGGL(k_rec_cond<M>, gc, dim3(256), 0, stream, g);                 \
  if ((e = hipGetLastError()) == hipSuccess)                                      \
    hipLaunchKernelGGL(k_rec_fill<M>, gf, dim3(256), 0, stream, g);
  LPF_REC_MASK_SWITCH(g.mask, LPF_BUILD)
#undef LPF_BUILD
  return e != hipSuccess ? e : hipGetLastError();
}

// One wave per (vector, side) pair when that many workgroups are resident at once; otherwise
// 1024 workgroups whose waves stride over the pairs.  A grid beyond what the device holds queues
// a second wave of workgroups, which repeats the launch's whole latency chain (decision, loads,
// flips); and when the pairs need more than one pass anyway, 1024 workgroups measured faster
// than the resident maximum (fewer workgroups to dispatch, each taking the decision).
int rec_end_workgroups(const RecGeo &g, int cus) {
  const int need = (2 * g.nv + 3) / 4;
  int per_cu = 0;
  hipError_t e = hipSuccess;
#define LPF_OCC(M) \
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rec_step_end<M, 1, true>, 256, 0)
  LPF_REC_MASK_SWITCH(g.mask, LPF_OCC)
#undef LPF_OCC
  // the step's upkeep workgroup runs beside the update workgroups, and up to 64 workgroups of
  // the next step's draws in ranked chains
  if (e == hipSuccess && need + 1 + 64 <= per_cu * cus) return need;
  return std::min(need, 1024);
}

hipError_t launch_rec_step_end(const RecGeo &g, const FinalArgs &f, const ProposeArgs *next,
                               int ndraw, hipStream_t stream) {
  const int nupd = g.end_wgs > 0 ? g.end_wgs : std::min((2 * g.nv + 3) / 4, 1024);
  // pairs per wave: with more than one, the first three are prefetched together
  const bool one = 2 * g.nv <= 4 * nupd;
  const ProposeArgs *nx = next;
  if (!next) ndraw = 0;
  const dim3 grid((unsigned)(nupd + 1 + ndraw));
#define LPF_END_D(M, D)                                                                       \
  if (one)                                                                                     \
    hipLaunchKernelGGL((k_rec_step_end<M, 1, D>), grid, dim3(256), 0, stream, g, f, nupd, nx); \
  else                                                                                         \
    hipLaunchKernelGGL((k_rec_step_end<M, 3, D>), grid, dim3(256), 0, stream, g, f, nupd, nx);
#define LPF_END(M)       \
  if (nx) {              \
    LPF_END_D(M, true)   \
  } else {               \
    LPF_END_D(M, false)  \
  }
  LPF_REC_MASK_SWITCH(g.mask, LPF_END)
#undef LPF_END_D
#undef LPF_END
  return hipGetLastError();
}

hipError_t launch_rec_round(const StepLaunch &L, const RoundPlan &r, bool decide,
                            hipStream_t stream) {
  // about 512 workgroups: a round after an accepting round is all early exits, whose cost grows
  // with the grid (2 048 workgroups took 0.8 us longer per step); a round that does evaluate
  // strides its candidates over them
  const int nvb = (L.rg.nv + 255) / 256;
  const int gy = std::max(1, std::min(std::min(r.C, 512), (512 + nvb - 1) / nvb));
  const dim3 grid((unsigned)nvb, (unsigned)gy);
  int16_t *dl = decide ? L.dl : nullptr;
  // round 1 after a round 0 evaluated with the draws or the ranking's merge: its sums are in S0
  const int64_t *S0 = decide && (L.fuse_draw || L.fuse_rank) && r.pC > 0 ? L.S0 : nullptr;
#define LPF_ROUND_O(M, O)                                                                      \
  hipLaunchKernelGGL((k_rec_round<M, O>), grid, dim3(256), 0, stream, L.rg, L.bits, L.cand, L.K, \
                     r.k0, r.C, L.counts, L.target, L.N, L.Nt, L.S_acc, dl, L.dl_t, L.dl_k,   \
                     L.ctl, L.order, L.U, L.T, decide ? r.pi0 : 0, decide ? r.pC : 0, S0)
#define LPF_ROUND(M)               \
  if (L.ordered)                   \
    LPF_ROUND_O(M, true);          \
  else                             \
    LPF_ROUND_O(M, false);
  LPF_REC_MASK_SWITCH(L.rg.mask, LPF_ROUND)
#undef LPF_ROUND
#undef LPF_ROUND_O
  return hipGetLastError();
}

hipError_t launch_rec_draw_round0(const StepLaunch &L, const RoundPlan &r, hipStream_t stream) {
  const int nprop = (L.draw.K + 255) / 256;
  const int nvb = (L.rg.nv + 255) / 256;
  const unsigned grid = (unsigned)(nprop + 1 + nvb * r.C);
#define LPF_R0(M)                                                                            \
  hipLaunchKernelGGL(k_rec_draw_round0<M>, dim3(grid), dim3(256), 0, stream, L.rg, L.draw, nprop, \
                     r.C, L.counts, L.target, L.N, L.Nt, L.S0, L.dl, L.dl_t, L.dl_k)
  LPF_REC_MASK_SWITCH(L.rg.mask, LPF_R0)
#undef LPF_R0
  return hipGetLastError();
}

hipError_t launch_rec_rank_round0(const StepLaunch &L, const RoundPlan &r, hipStream_t stream) {
  const int nvb = (L.rg.nv + 255) / 256;
  const unsigned grid = (unsigned)(1 + nvb * r.C);
#define LPF_RR0(M)                                                                             \
  hipLaunchKernelGGL(k_rec_rank_round0<M>, dim3(grid), dim3(256), 0, stream, L.rg,               \
                     L.rank_keys + kRankMax, L.rank_keys, L.K, L.order_rw, L.bits, L.cand, r.C, \
                     L.counts, L.target, L.N, L.Nt, L.S_acc, L.S0, L.dl, L.dl_t, L.dl_k, L.ctl, \
                     L.st, L.T_cur, L.T_sched, L.T_base, L.T_value)
  LPF_REC_MASK_SWITCH(L.rg.mask, LPF_RR0)
#undef LPF_RR0
  return hipGetLastError();
}

#undef LPF_REC_MASK_SWITCH

}  // namespace lpf
