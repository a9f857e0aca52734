// Full evaluation of the lineal path function on gfx950.
//
// The paper's Alg. "L2_eval" tests, for every segment and every translation, the segment's
// pixels one by one.  Here 32 translations (start pixels) share one 32-bit word: for a segment
// with pixels p_k = (px_k, py_k) (translated so that every offset is >= 0, which leaves the
// count unchanged on a periodic image), a lane owning start word w of row y forms
//     t_k = bits [32w + px_k, 32w + px_k + 32) of row y + py_k      (one v_alignbit_b32)
//     A   = AND_k t_k    -> bit b set   <=> every pixel of the segment is phase 1
//     O   = OR_k  t_k    -> bit b clear <=> every pixel of the segment is phase 0
// and popcounts A and ~O.  Both phases share the aligned word.  The segment's pixels are
// generated on the scalar unit (the vector is wave-uniform), so px_k and py_k live in SGPRs.
//
// Periodicity (Sec. 2.1) is handled by an extended image E: row y of E holds row y of the image
// followed by wrapped copies, so bit j of E row y is pixel (j mod W, y).  Rows wrap when they are
// staged into LDS.  This replaces the paper's 2x2-tiled image A and translation table C.
#include "lpf_internal.h"

namespace lpf {

// ------------------------------------------------------------------------------------ pack
__global__ void k_pack(const uint8_t *__restrict__ img, int W, int H, int wpr,
                       uint64_t *__restrict__ bits) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y;
  if (j >= wpr || y >= H) return;
  const uint8_t *row = img + (size_t)y * W;
  uint64_t w = 0;
  int x0 = j * 64;
  int nb = min(64, W - x0);
  for (int b = 0; b < nb; ++b) w |= (uint64_t)(row[x0 + b] != 0) << b;
  bits[(size_t)y * wpr + j] = w;
}

hipError_t launch_pack(const uint8_t *img, int W, int H, uint64_t *bits, hipStream_t stream) {
  int wpr = (W + 63) / 64;
  dim3 grid((wpr + 63) / 64, H);
  hipLaunchKernelGGL(k_pack, grid, dim3(64), 0, stream, img, W, H, wpr, bits);
  return hipGetLastError();
}

// ------------------------------------------------------------------------- extended image
// E[r][e], e < we, r < rows: bit b = pixel ((32e + b) mod W, r mod H).
__global__ void k_ext(const uint32_t *__restrict__ src, int W, int H, int src_stride, int we,
                      int rows, uint32_t *__restrict__ E) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  int y = blockIdx.y;
  if (e >= we || y >= rows) return;
  const uint32_t *row = src + (size_t)(y % H) * src_stride;
  int s = (int)(((int64_t)32 * e) % W);
  uint32_t v;
  if (s + 32 <= W) {
    int q = s >> 5, sh = s & 31;
    uint32_t lo = row[q];
    uint32_t hi = sh ? row[q + 1] : 0u;  // q + 1 < ceil(W/32) whenever sh != 0 here
    v = __builtin_amdgcn_alignbit(hi, lo, sh);
  } else {
    v = 0;
    int x = s;
    for (int b = 0; b < 32; ++b) {
      v |= ((row[x >> 5] >> (x & 31)) & 1u) << b;
      x = (x + 1 == W) ? 0 : x + 1;
    }
  }
  E[(size_t)y * we + e] = v;
}

hipError_t launch_ext(const uint64_t *bits, int W, int H, int we, uint32_t *ext,
                      hipStream_t stream, int rows) {
  if (rows < H) rows = H;
  int src_stride = 2 * ((W + 63) / 64);
  dim3 grid((we + 63) / 64, rows);
  hipLaunchKernelGGL(k_ext, grid, dim3(64), 0, stream, reinterpret_cast<const uint32_t *>(bits),
                     W, H, src_stride, we, rows, ext);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------ full kernel
//
// Chains.  Every segment path is taken from (0,0) in the order of its major axis, and the first
// l + 1 pixels of the path of a vector v are, up to a translation, often the whole path of a
// shorter vector u of the domain: u is one of the "shorter overlapping segments" of v that the
// paper's enhanced evaluation builds on (Sec. 3.2).  The counts are translation invariant on a
// periodic image, so one walk of v's path gives the count of u as well, read off the running
// product after pixel l.  The host cuts the domain into chains (a walked vector and the vectors
// whose paths are its prefixes, in increasing l; every vector in exactly one chain), which
// removes more than half of the pixel work of the per-vector walk (at cutoff 128: 1 272 832
// instead of 2 862 081 pixels per 32 start pixels).
//
// A workgroup owns one bin of chains and counts them over every row tile of the image; its
// waves split the work as (chain group, band group): wave w walks the chains j = cw, cw + nwc,
// ... of the bin over the bands bw, bw + nwb, ... of the tile (cw = w / nwb, bw = w % nwb).  At a
// member's end the wave sums its popcounts (both phases packed in one word) across lanes and one
// lane adds them into the member's count slot in LDS; after the last tile the workgroup writes
// each member's count once.

// Vector i of the canonical half domain: [0,cx] x [0,cy] row by row, then [-cx,-1] x [1,cy].
__device__ __forceinline__ VecDesc canonical_vec(int i, int cx, int cy) {
  const int n1 = (cx + 1) * (cy + 1);
  VecDesc v;
  v.idx = i;
  if (i < n1) {
    const int dy = i / (cx + 1);
    v.dy = (int16_t)dy;
    v.dx = (int16_t)(i - dy * (cx + 1));
  } else {
    const int r = i - n1;
    const int dy = r / cx;
    v.dy = (int16_t)(1 + dy);
    v.dx = (int16_t)(-cx + (r - dy * cx));
  }
  return v;
}

// Sum over the wave of v, valid in lane 63 (DPP: within quads, half rows and rows, then row
// broadcasts 15 and 31).  Every lane must be active.
__device__ __forceinline__ uint32_t wave_sum63(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return v;
}

// Count of vector `idx` = (dx, dy) for phase slot p, in the image's output layout (the GRID
// layout also fills -v, eq. (symmetry)).
__device__ __forceinline__ void put_count(const FullImg &I, int p, int idx, int dx, int dy,
                                          uint32_t c) {
  if (I.layout == 0) {
    I.out[(size_t)p * I.nv + idx] = c;
  } else {
    const int gw = 2 * I.cx + 1;
    const size_t g = (size_t)gw * (2 * I.cy + 1);
    I.out[(size_t)p * g + (size_t)(dy + I.cy) * gw + (dx + I.cx)] = c;
    I.out[(size_t)p * g + (size_t)(I.cy - dy) * gw + (I.cx - dx)] = c;
  }
}

// Valid start pixels of a lane's words, computed when a member's count is taken (not kept in
// registers during the walk): word w = w0 + i of the row is full below the last word, the last
// word keeps the bits below W mod 32, rows past the tile have none; with a Monte-Carlo position
// set only its members count (its extended row read at the walked vector's shift).
struct LaneMask {
  int w0, swd;
  uint32_t lastmask;
  bool row_ok;
  const uint32_t *srow;  // the position set's extended row at this lane's first word, or null
  int so, ssh;
};

template <bool SAMPLE>
__device__ __forceinline__ uint32_t lane_mask(const LaneMask &L, int i) {
  const int w = L.w0 + i;
  uint32_t mw = (w < L.swd - 1) ? 0xffffffffu : (w == L.swd - 1 ? L.lastmask : 0u);
  if (!L.row_ok) mw = 0u;
  if constexpr (SAMPLE) {
    if (L.row_ok) mw &= __builtin_amdgcn_alignbit(L.srow[L.so + i + 1], L.srow[L.so + i], L.ssh);
  }
  return mw;
}

// Walk of one chain for the lane's R words of one row: A &= t, O |= t over the walked vector's
// pixels; after pixel l of each member the wave's counts go to the member's slot.
// XM: x is the major axis.  Q2: dx < 0 (mirrored in x and shifted by |dx|, a translation).
// Pixels are taken in pairs: two funnel shifts, one 3-input AND (v_bitop3_b32) and one 3-input
// OR (v_or3_b32) per word; when both pixels of a pair read the same dwords (same row, same word
// column) the dwords are loaded once.  A pair never straddles a member's end.
//
// SKIP (the paper's "enhanced" evaluation, Sec. 3.2): a member whose count over the wave's rows
// is zero for every requested phase has no occurrence there, so neither has any longer member of
// the chain (later pixels only clear A and set O); the walk stops at that member.  The test reads
// the count the member's emission has just summed.  Far from the next member the wave also
// tests, after 32, 64, 128, ... pixels, whether any start pixel can still count.
// FULL (wave-uniform): every bit of the lane's words is a start pixel (mk all ones), so the
// popcounts need no mask.
template <int R, bool XM, bool Q2, bool SKIP, bool CANON, bool SAMPLE>
__device__ __forceinline__ void walk_chain(const uint32_t *__restrict__ base, int rst, int adx,
                                           int n, int m, const MemDesc *__restrict__ mems,
                                           int m0, int nm, int lw, uint32_t (&A)[R],
                                           uint32_t (&O)[R], const LaneMask &lm, bool full,
                                           unsigned phase_mask, uint32_t *__restrict__ slots,
                                           int lane) {
  int err = n, q = 0;
  auto advance = [&]() {
    err += 2 * m;
    if (err >= 2 * n) {
      err -= 2 * n;
      ++q;
    }
  };
  auto pixel = [&](int k, int &off, int &sh) {
    const int X = XM ? k : q;
    const int Y = XM ? q : k;
    const int px = Q2 ? adx - X : X;
    off = Y * rst + (px >> 5);
    sh = px & 31;
  };
  int mi = 0;
  int next_l = CANON ? lw : __builtin_amdgcn_readfirstlane(mems[m0].l);
  // the next pixel index with work beside the path product: a member's end, or (SKIP) a
  // liveness test; one compare per pixel pair either way
  int next_test = 32;
  int next_ev = SKIP ? min(next_l, next_test) : next_l;
  int k = 0;
  for (;;) {
    // the next two pixels, or one when a second would pass the member's end; one pixel is taken
    // as a pair of equal pixels (A & t & t = A & t), so that the vector code has a single path
    // and the accumulators stay in place
    int off0, sh0, off1, sh1;
    pixel(k, off0, sh0);
    advance();
    if (k + 1 <= next_l) {
      pixel(k + 1, off1, sh1);
      advance();
      k += 2;
    } else {
      off1 = off0;
      sh1 = sh0;
      k += 1;
    }
    const uint32_t *p0 = base + off0;
    const uint32_t *p1 = base + off1;
    uint32_t d0[R + 1], d1[R + 1];
#pragma unroll
    for (int c = 0; c <= R; ++c) {
      d0[c] = p0[c];
      d1[c] = p1[c];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const uint32_t t0 = __builtin_amdgcn_alignbit(d0[i + 1], d0[i], sh0);
      const uint32_t t1 = __builtin_amdgcn_alignbit(d1[i + 1], d1[i], sh1);
      A[i] = __builtin_amdgcn_bitop3_b32(A[i], t0, t1, 0x80);
      O[i] = O[i] | t0 | t1;
    }
    if constexpr (SKIP) {
      if (k - 1 < next_ev) continue;
    }
    if (k - 1 == next_l) {
      // member mi ends at pixel next_l: phase 0 in the low half-word, phase 1 in the high one
      // (a lane counts at most 32 R <= 512 start pixels, a wave at most 32 768)
      uint32_t p0 = 0, p1 = 0;
      if (full) {
        if (phase_mask & 2u) {
#pragma unroll
          for (int i = 0; i < R; ++i) p1 += __popc(A[i]);
        }
        if (phase_mask & 1u) {
#pragma unroll
          for (int i = 0; i < R; ++i) p0 += __popc(~O[i]);
        }
      } else {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const uint32_t mk = lane_mask<SAMPLE>(lm, i);
          if (phase_mask & 2u) p1 += __popc(A[i] & mk);
          if (phase_mask & 1u) p0 += __popc(~O[i] & mk);
        }
      }
      const uint32_t s = wave_sum63(p0 | (p1 << 16));
      if (lane == 63 && s) {
        atomicAdd(slots + 2 * mi, s & 0xffffu);
        atomicAdd(slots + 2 * mi + 1, s >> 16);
      }
      if (++mi == nm) return;
      if constexpr (SKIP) {
        if (__builtin_amdgcn_readlane(s, 63) == 0u) return;
      }
      next_l = __builtin_amdgcn_readfirstlane(mems[m0 + mi].l);
    } else if constexpr (SKIP) {
      // test after 32, 64, 128, ... pixels, when the next member is still far, whether any start
      // pixel can still count for a requested phase (a set bit of A, a clear bit of O, if valid)
      next_test = 2 * k;
      if (next_l - k >= 16) {
        uint32_t live = 0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const uint32_t mk = full ? 0xffffffffu : lane_mask<SAMPLE>(lm, i);
          if (phase_mask & 2u) live |= A[i] & mk;
          if (phase_mask & 1u) live |= ~O[i] & mk;
        }
        if (!__any(live != 0u)) return;
      }
    }
    next_ev = SKIP ? min(next_l, next_test) : next_l;
  }
}

// One work item: bin `bin` of image I (one workgroup).  lds: staged rows; slots: two count
// words per member of the bin, zeroed here and added into by the waves over every band and row
// tile; each count is then written once.
// CANON: no chain tables; bin b takes the canonical vectors b, b + nbins, b + 2 nbins, ... as
// chains of one member each (interleaving spreads long and short vectors evenly).
// GLOB: rows are read from the extended image in device memory (one tile, I.lds_rows rows of
// E with a periodic halo), for halos too large for LDS; only the count slots live in LDS.
// SAMPLE: I.sample holds a Monte-Carlo position set (the approximation's instance).
template <int R, bool SKIP, bool CANON = false, bool GLOB = false, bool SAMPLE = false>
__device__ __forceinline__ void process_item(const FullImg &I, int bin, int wpg,
                                             unsigned phase_mask, uint32_t *__restrict__ lds,
                                             uint32_t *__restrict__ slots) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rpw = 64 / I.S;
  const int strip = lane / rpw;
  const int r_in = lane - strip * rpw;
  const int swd = (I.W + 31) >> 5;
  const uint32_t lastmask = (I.W & 31) ? ((1u << (I.W & 31)) - 1u) : 0xffffffffu;
  int cb, ce, mb, nmb;
  if constexpr (CANON) {
    cb = 0;
    ce = bin < I.nv ? (I.nv - 1 - bin) / I.nbins + 1 : 0;
    mb = 0;
    nmb = ce;
  } else {
    cb = I.bin_off[bin];
    ce = I.bin_off[bin + 1];
    mb = cb < ce ? I.chains[cb].m0 : 0;
    nmb = cb < ce ? I.chains[ce - 1].m0 + I.chains[ce - 1].nm - mb : 0;
  }
  for (int t = threadIdx.x; t < 2 * nmb; t += blockDim.x) slots[t] = 0u;
  const int nwb = I.nwb;
  const int nwc = wpg / nwb;
  const int cw = wave / nwb, bw = wave - cw * nwb;
  for (int t_id = 0; t_id < I.ntiles; ++t_id) {
    const int Y0 = t_id * I.tile;
    const int rows_here = min(I.tile, I.H - Y0);
    __syncthreads();  // slots zeroed; every wave is done with the previous tile
    if constexpr (!GLOB) {
      // Stage rows Y0 .. Y0 + lds_rows - 1 (mod H) of E.
      for (int i = threadIdx.x; i < I.lds_rows * I.we; i += blockDim.x) {
        const int r = i / I.we;
        const int e = i - r * I.we;
        const int y = (Y0 + r) % I.H;
        lds[r * I.rst + e] = I.E[(size_t)y * I.we + e];
      }
      __syncthreads();
    }
    const int nbands = (rows_here + rpw - 1) / rpw;
    for (int j = cb + cw; j < ce; j += nwc) {
      int dx, dy, m0, nm, lw;
      if constexpr (CANON) {
        const VecDesc v = canonical_vec(bin + j * I.nbins, I.cx, I.cy);
        dx = v.dx;
        dy = v.dy;
        m0 = j;
        nm = 1;
        lw = max(dx < 0 ? -dx : dx, dy);
      } else {
        const ChainDesc c = I.chains[j];
        dx = c.dx;
        dy = c.dy;
        m0 = c.m0;
        nm = c.nm;
        lw = c.lw;
      }
      const int adx = dx < 0 ? -dx : dx;
      const int n = adx > dy ? adx : dy;
      const bool xm = adx >= dy;
      const int m = xm ? dy : adx;
      uint32_t *cs = slots + 2 * (m0 - mb);
      for (int band = bw; band < nbands; band += nwb) {
        const int row = band * rpw + r_in;
        const uint32_t *base =
            (GLOB ? I.E + (size_t)(Y0 + row) * I.rst : lds + row * I.rst) + strip * R;
        const bool row_ok = row < rows_here;
        uint32_t A[R], O[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
          A[i] = 0xffffffffu;
          O[i] = 0u;
        }
        // Monte-Carlo approximation: only start pixels of the position set count.  Lane bit b of
        // word w stands for the placement whose first pixel is 32w + b (+ |dx| of the walked
        // vector when it is mirrored: the members share its frame), so the set's extended row is
        // read at that shift.
        LaneMask lmk;
        lmk.w0 = strip * R;
        lmk.swd = swd;
        lmk.lastmask = lastmask;
        lmk.row_ok = row_ok;
        lmk.srow = SAMPLE ? I.sample + (size_t)(Y0 + (row_ok ? row : 0)) * I.sample_stride + strip * R
                          : nullptr;
        lmk.so = dx < 0 ? (adx >> 5) : 0;
        lmk.ssh = dx < 0 ? (adx & 31) : 0;
        // every bit of every lane's words a start pixel: no masks at the members' counts
        const bool lane_full = row_ok && !SAMPLE &&
                               (strip * R + R - 1 < swd - 1 ||
                                (strip * R + R - 1 == swd - 1 && lastmask == 0xffffffffu));
        const bool full = __all(lane_full);
        const MemDesc *md = I.mems;
        if (xm) {
          if (dx < 0) walk_chain<R, true, true, SKIP, CANON, SAMPLE>(base, I.rst, adx, n, m, md, m0, nm, lw, A, O, lmk, full, phase_mask, cs, lane);
          else walk_chain<R, true, false, SKIP, CANON, SAMPLE>(base, I.rst, adx, n, m, md, m0, nm, lw, A, O, lmk, full, phase_mask, cs, lane);
        } else {
          if (dx < 0) walk_chain<R, false, true, SKIP, CANON, SAMPLE>(base, I.rst, adx, n, m, md, m0, nm, lw, A, O, lmk, full, phase_mask, cs, lane);
          else walk_chain<R, false, false, SKIP, CANON, SAMPLE>(base, I.rst, adx, n, m, md, m0, nm, lw, A, O, lmk, full, phase_mask, cs, lane);
        }
      }
    }
  }
  __syncthreads();  // every wave's additions are in the slots
  for (int t = threadIdx.x; t < nmb; t += blockDim.x) {
    int idx, dx, dy;
    if constexpr (CANON) {
      const VecDesc v = canonical_vec(bin + t * I.nbins, I.cx, I.cy);
      idx = v.idx;
      dx = v.dx;
      dy = v.dy;
    } else {
      const MemDesc md = I.mems[mb + t];
      idx = md.idx;
      dx = md.dx;
      dy = md.dy;
    }
    int p = 0;
    if (phase_mask & 1) put_count(I, p++, idx, dx, dy, slots[2 * t]);
    if (phase_mask & 2) put_count(I, p, idx, dx, dy, slots[2 * t + 1]);
  }
}

// One image, one workgroup per bin.  At most 128 registers per lane (four waves per SIMD): at
// the usual staging sizes LDS already limits a CU to two workgroups of eight waves.
template <int R, bool SKIP, bool GLOB = false, bool SAMPLE = false>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4)))
k_lpf_full(FullImg I, int wpg, unsigned phase_mask, int cnt_off) {
  extern __shared__ uint32_t lds[];
  process_item<R, SKIP, false, GLOB, SAMPLE>(I, blockIdx.x, wpg, phase_mask, lds, lds + cnt_off);
}

// One image without chain tables (canonical vectors interleaved over the bins).
template <int R>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4)))
k_lpf_full_canon(FullImg I, int wpg, unsigned phase_mask, int cnt_off) {
  extern __shared__ uint32_t lds[];
  process_item<R, false, true>(I, blockIdx.x, wpg, phase_mask, lds, lds + cnt_off);
}

// Many images, persistent workgroups drawing work items (image, bin) from a device counter in
// descending cost order until the list is exhausted (every wave reaches the exit test).  The
// counts pool is read from `args` (written before each replay of the captured launch); image i's
// counts start at counts_off[i].
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4)))
k_lpf_batch(const FullImg *__restrict__ imgs, const BatchArgs *__restrict__ args,
            const int64_t *__restrict__ counts_off, const int2 *__restrict__ items, int n_items,
            int *__restrict__ counter, int wpg, unsigned phase_mask, int cnt_off) {
  extern __shared__ uint32_t lds[];
  __shared__ int s_item;
  uint32_t *const counts = args->counts;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= n_items) break;
    const int2 w = items[it];
    FullImg I = imgs[w.x];
    I.out = counts + counts_off[w.x];
    if (!I.glob) {
      switch (I.R) {
        case 1: process_item<1, false>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
        case 2: process_item<2, false>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
        case 4: process_item<4, false>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
        case 8: process_item<8, false>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
        default: process_item<16, false>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
      }
    } else {
      switch (I.R) {
        case 1: process_item<1, false, false, true>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
        case 2: process_item<2, false, false, true>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
        case 4: process_item<4, false, false, true>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
        case 8: process_item<8, false, false, true>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
        default: process_item<16, false, false, true>(I, w.y, wpg, phase_mask, lds, lds + cnt_off); break;
      }
    }
    __syncthreads();  // the item's counts are written and its rows no longer read
  }
}

__global__ void k_reset_counter(int *counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = 0;
}

size_t full_lds_bytes(const FullShape &sh, int wpg) {
  (void)wpg;
  const size_t stage = sh.glob ? 0 : (size_t)sh.lds_rows * sh.rst * sizeof(uint32_t);
  return stage + (size_t)kSlotWords * sizeof(uint32_t);
}

// The launch shape the kernel assumes: nwb waves per chain dividing the workgroup's waves.
static bool shape_ok(const FullImg &I, const FullShape &sh) {
  return sh.wpg >= 1 && sh.wpg <= 16 && I.nwb >= 1 && sh.wpg % I.nwb == 0 && sh.nbins >= 1 &&
         I.nbins == sh.nbins && I.R == sh.R && 64 % I.S == 0;
}

template <int R, bool SKIP>
static hipError_t launch_full_r(const FullImg &I, const FullShape &sh, unsigned phase_mask,
                                hipStream_t stream) {
  if (!shape_ok(I, sh) || I.glob != sh.glob) return hipErrorInvalidValue;
  const size_t lds = full_lds_bytes(sh, sh.wpg);
  const int cnt_off = sh.glob ? 0 : sh.lds_rows * sh.rst;
  const dim3 g(sh.nbins), b(64 * sh.wpg);
  if constexpr (SKIP) {  // the enhanced evaluation has no Monte-Carlo variant
    if (I.sample) return hipErrorInvalidValue;
    if (sh.glob)
      hipLaunchKernelGGL((k_lpf_full<R, true, true>), g, b, lds, stream, I, sh.wpg, phase_mask, cnt_off);
    else
      hipLaunchKernelGGL((k_lpf_full<R, true>), g, b, lds, stream, I, sh.wpg, phase_mask, cnt_off);
  } else if (I.sample) {
    if (sh.glob)
      hipLaunchKernelGGL((k_lpf_full<R, false, true, true>), g, b, lds, stream, I, sh.wpg, phase_mask, cnt_off);
    else
      hipLaunchKernelGGL((k_lpf_full<R, false, false, true>), g, b, lds, stream, I, sh.wpg, phase_mask, cnt_off);
  } else {
    if (sh.glob)
      hipLaunchKernelGGL((k_lpf_full<R, false, true>), g, b, lds, stream, I, sh.wpg, phase_mask, cnt_off);
    else
      hipLaunchKernelGGL((k_lpf_full<R, false>), g, b, lds, stream, I, sh.wpg, phase_mask, cnt_off);
  }
  return hipGetLastError();
}

template <bool SKIP>
static hipError_t launch_full_s(const FullImg &I, const FullShape &sh, unsigned phase_mask,
                                hipStream_t stream) {
  switch (sh.R) {
    case 1: return launch_full_r<1, SKIP>(I, sh, phase_mask, stream);
    case 2: return launch_full_r<2, SKIP>(I, sh, phase_mask, stream);
    case 4: return launch_full_r<4, SKIP>(I, sh, phase_mask, stream);
    case 8: return launch_full_r<8, SKIP>(I, sh, phase_mask, stream);
    case 16: return launch_full_r<16, SKIP>(I, sh, phase_mask, stream);
    default: return hipErrorInvalidValue;
  }
}

template <int R>
static hipError_t launch_canon_r(const FullImg &I, const FullShape &sh, unsigned phase_mask,
                                 hipStream_t stream) {
  if (!shape_ok(I, sh) || sh.glob) return hipErrorInvalidValue;
  const size_t lds = full_lds_bytes(sh, sh.wpg);
  const int cnt_off = sh.lds_rows * sh.rst;
  hipLaunchKernelGGL((k_lpf_full_canon<R>), dim3(sh.nbins), dim3(64 * sh.wpg), lds, stream, I,
                     sh.wpg, phase_mask, cnt_off);
  return hipGetLastError();
}

hipError_t launch_full_canon(const FullImg &I, const FullShape &sh, unsigned phase_mask,
                             hipStream_t stream) {
  switch (sh.R) {
    case 1: return launch_canon_r<1>(I, sh, phase_mask, stream);
    case 2: return launch_canon_r<2>(I, sh, phase_mask, stream);
    case 4: return launch_canon_r<4>(I, sh, phase_mask, stream);
    case 8: return launch_canon_r<8>(I, sh, phase_mask, stream);
    case 16: return launch_canon_r<16>(I, sh, phase_mask, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_full(const FullImg &I, const FullShape &sh, unsigned phase_mask, bool skip,
                       hipStream_t stream) {
  return skip ? launch_full_s<true>(I, sh, phase_mask, stream)
              : launch_full_s<false>(I, sh, phase_mask, stream);
}

// Workgroups of one full-evaluation kernel resident per CU (registers and LDS of the launch).
int full_wgs_per_cu(int R, bool skip, int wpg, size_t lds_bytes) {
  const void *f = nullptr;
  switch (R) {
    case 1: f = skip ? (const void *)k_lpf_full<1, true> : (const void *)k_lpf_full<1, false>; break;
    case 2: f = skip ? (const void *)k_lpf_full<2, true> : (const void *)k_lpf_full<2, false>; break;
    case 4: f = skip ? (const void *)k_lpf_full<4, true> : (const void *)k_lpf_full<4, false>; break;
    case 8: f = skip ? (const void *)k_lpf_full<8, true> : (const void *)k_lpf_full<8, false>; break;
    default: f = skip ? (const void *)k_lpf_full<16, true> : (const void *)k_lpf_full<16, false>; break;
  }
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64 * wpg, lds_bytes) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

hipError_t launch_batch(const FullImg *imgs, const BatchArgs *args, const int64_t *counts_off,
                        const int2 *items, int n_items, int *counter, int wpg,
                        unsigned phase_mask, size_t lds_bytes, int cnt_off, int n_wg,
                        hipStream_t stream) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, stream, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lpf_batch, dim3(n_wg), dim3(64 * wpg), lds_bytes, stream, imgs, args,
                     counts_off, items, n_items, counter, wpg, phase_mask, cnt_off);
  return hipGetLastError();
}

// The buffers of one lpf_batch call, written on the call's stream before the captured launch.
__global__ void k_batch_args(BatchArgs *args, const uint64_t *pool, uint32_t *counts) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    args->pool = pool;
    args->counts = counts;
  }
}

hipError_t launch_batch_args(BatchArgs *args, const uint64_t *pool, uint32_t *counts,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_batch_args, dim3(1), dim3(64), 0, stream, args, pool, counts);
  return hipGetLastError();
}

// E for many images in one launch: image b's rows at ext_off[b], we[b] dwords per row; the
// packed images at args->pool + bits_off[b].
__global__ void k_ext_batch(const FullImg *__restrict__ imgs, const BatchArgs *__restrict__ args,
                            const int64_t *__restrict__ bits_off, uint32_t *__restrict__ ext,
                            const int64_t *__restrict__ ext_off) {
  const int b = blockIdx.z;
  const FullImg I = imgs[b];
  const uint64_t *const pool = args->pool;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (e >= I.we || y >= (I.glob ? I.lds_rows : I.H)) return;
  const uint32_t *row = reinterpret_cast<const uint32_t *>(pool + bits_off[b]) +
                        (size_t)(y % I.H) * 2 * ((I.W + 63) / 64);
  const int W = I.W;
  const int s = (int)(((int64_t)32 * e) % W);
  uint32_t v;
  if (s + 32 <= W) {
    const int q = s >> 5, sh = s & 31;
    v = __builtin_amdgcn_alignbit(sh ? row[q + 1] : 0u, row[q], sh);
  } else {
    v = 0;
    int x = s;
    for (int t = 0; t < 32; ++t) {
      v |= ((row[x >> 5] >> (x & 31)) & 1u) << t;
      x = (x + 1 == W) ? 0 : x + 1;
    }
  }
  ext[ext_off[b] + (size_t)y * I.we + e] = v;
}

hipError_t launch_ext_batch(const FullImg *imgs, int n_images, int max_we, int max_h,
                            const BatchArgs *args, const int64_t *bits_off, uint32_t *ext,
                            const int64_t *ext_off, hipStream_t stream) {
  dim3 grid((max_we + 63) / 64, max_h, n_images);
  hipLaunchKernelGGL(k_ext_batch, grid, dim3(64), 0, stream, imgs, args, bits_off, ext, ext_off);
  return hipGetLastError();
}

hipError_t prepare_full_kernels(int max_lds_bytes) {
  hipError_t e = hipSuccess;
  const void *fns[] = {(const void *)k_lpf_full<1, false>, (const void *)k_lpf_full<2, false>,
                       (const void *)k_lpf_full<4, false>, (const void *)k_lpf_full<8, false>,
                       (const void *)k_lpf_full<16, false>, (const void *)k_lpf_full<1, true>,
                       (const void *)k_lpf_full<2, true>, (const void *)k_lpf_full<4, true>,
                       (const void *)k_lpf_full<8, true>, (const void *)k_lpf_full<16, true>,
                       (const void *)k_lpf_full<1, false, true>, (const void *)k_lpf_full<2, false, true>,
                       (const void *)k_lpf_full<4, false, true>, (const void *)k_lpf_full<8, false, true>,
                       (const void *)k_lpf_full<16, false, true>, (const void *)k_lpf_full<1, true, true>,
                       (const void *)k_lpf_full<2, true, true>, (const void *)k_lpf_full<4, true, true>,
                       (const void *)k_lpf_full<8, true, true>, (const void *)k_lpf_full<16, true, true>,
                       (const void *)k_lpf_full<1, false, false, true>, (const void *)k_lpf_full<2, false, false, true>,
                       (const void *)k_lpf_full<4, false, false, true>, (const void *)k_lpf_full<8, false, false, true>,
                       (const void *)k_lpf_full<16, false, false, true>, (const void *)k_lpf_full<1, false, true, true>,
                       (const void *)k_lpf_full<2, false, true, true>, (const void *)k_lpf_full<4, false, true, true>,
                       (const void *)k_lpf_full<8, false, true, true>, (const void *)k_lpf_full<16, false, true, true>,
                       (const void *)k_lpf_full_canon<1>, (const void *)k_lpf_full_canon<2>,
                       (const void *)k_lpf_full_canon<4>, (const void *)k_lpf_full_canon<8>,
                       (const void *)k_lpf_full_canon<16>};
  for (const void *f : fns) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
    if (r != hipSuccess) e = r;
  }
  // the batch kernel also holds one static LDS word
  hipError_t r = hipFuncSetAttribute((const void *)k_lpf_batch,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     max_lds_bytes - kBatchStaticLds);
  if (r != hipSuccess) e = r;
  return e;
}

}  // namespace lpf
