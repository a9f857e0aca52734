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

#include "delta_dev.h"

namespace lpf {

// E_X[r][e] (r < H_X + hy, e < we_X): bit j = pixel of image X at ((32e + j) mod W_X, r mod H_X).
// X = 0: the image; X = 1: transposed, X(x,y) = I(y,x); X = 2: anti-transposed,
// X(x,y) = I(-y mod W, -x mod H).  Images 1 and 2 are H wide and W high.
__global__ void k_ext3(const uint64_t *__restrict__ bits, int W, int H, DeltaGeo geo,
                       uint32_t *__restrict__ E, const int32_t *__restrict__ only_if) {
  if (only_if && *only_if < 0) return;  // the image did not change
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
  hipLaunchKernelGGL(k_ext3, grid, dim3(64), 0, stream, bits, W, H, geo, E, nullptr);
  return hipGetLastError();
}

hipError_t launch_ext3_if(const uint64_t *bits, int W, int H, const DeltaGeo &geo, uint32_t *E,
                          const int32_t *flag, hipStream_t stream) {
  int wemax = std::max(geo.g[0].we, std::max(geo.g[1].we, geo.g[2].we));
  int hmax = std::max(geo.g[0].H, std::max(geo.g[1].H, geo.g[2].H)) + geo.hy;
  dim3 grid((wemax + 63) / 64, hmax, 3);
  hipLaunchKernelGGL(k_ext3, grid, dim3(64), 0, stream, bits, W, H, geo, E, flag);
  return hipGetLastError();
}

// dL for n candidate interchanges (lanes) and the vectors of chunk blockIdx.y, written to
// delta_out[k][p][idx].
template <bool LDS>
__global__ void __launch_bounds__(256)
k_delta(const uint32_t *__restrict__ Eg, DeltaGeo geo, const uint64_t *__restrict__ bits, int W,
        int H, const int2 *__restrict__ cand, int K, const DeltaVec *__restrict__ vecs,
        const int32_t *__restrict__ chunk_off, const uint32_t *__restrict__ runs,
        unsigned phase_mask, int nv, int32_t *__restrict__ delta_out) {
  extern __shared__ uint32_t lds[];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  bool ok = k < K;
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
  const int chunk = blockIdx.y;
  const int vb0 = chunk_off[chunk], vb1 = chunk_off[chunk + 1];
  const int nph = (phase_mask & 1) + ((phase_mask >> 1) & 1);
  for (int j = vb0; j < vb1; ++j) {
    const DeltaVec dv = vecs[j];
    int d1, d0;
    vector_delta<LDS>(E, geo, dv, runs, cf, d1, d0);
    if (!ok) {
      d1 = 0;
      d0 = 0;
    }
    if (k < K) {
      int p = 0;
      if (phase_mask & 1) delta_out[((size_t)k * nph + p++) * nv + dv.idx] = d0;
      if (phase_mask & 2) delta_out[((size_t)k * nph + p) * nv + dv.idx] = d1;
    }
  }
}

hipError_t launch_delta(const DeltaLaunch &L, hipStream_t stream) {
  dim3 block(256);
  dim3 grid((unsigned)((L.K + 255) / 256), (unsigned)L.nchunks);
  if (L.use_lds)
    hipLaunchKernelGGL(k_delta<true>, grid, block, (size_t)L.geo.total * sizeof(uint32_t), stream,
                       L.E, L.geo, L.bits, L.W, L.H, L.cand, L.K, L.vecs, L.chunk_off, L.runs,
                       L.phase_mask, L.nv, L.delta_out);
  else
    hipLaunchKernelGGL(k_delta<false>, grid, block, 0, stream, L.E, L.geo, L.bits, L.W, L.H,
                       L.cand, L.K, L.vecs, L.chunk_off, L.runs, L.phase_mask, L.nv, L.delta_out);
  return hipGetLastError();
}

// ---- offset rows ----
// Frames of the offset-row delta: frame 0 row r = y + cy holds x along its bits, frame 1 row
// r = x + cx holds y; bit B + u is minor coordinate u, both coordinates periodic.
__global__ void k_dframe(const uint64_t *__restrict__ bits, int W, int H, DiagGeo g,
                         uint32_t *__restrict__ F) {
  const int f = blockIdx.z;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= g.we[f] || r >= g.rows[f]) return;
  const int wpr = (W + 63) >> 6;
  const int Pr = f == 0 ? H : W, Pm = f == 0 ? W : H;
  int maj = (r - g.rowoff[f]) % Pr;
  maj += maj < 0 ? Pr : 0;
  int u = (32 * e - g.B[f]) % Pm;
  u += u < 0 ? Pm : 0;
  uint32_t v = 0;
  for (int t = 0; t < 32; ++t) {
    const int x = f == 0 ? u : maj, y = f == 0 ? maj : u;
    v |= (uint32_t)((bits[(size_t)y * wpr + (x >> 6)] >> (x & 63)) & 1ull) << t;
    u = u + 1 == Pm ? 0 : u + 1;
  }
  F[(size_t)g.off[f] + (size_t)r * g.we[f] + e] = v;
}

hipError_t launch_dframe(const uint64_t *bits, int W, int H, const DiagGeo &g, uint32_t *F,
                         hipStream_t stream) {
  const int we = std::max(g.we[0], g.we[1]), rows = std::max(g.rows[0], g.rows[1]);
  hipLaunchKernelGGL(k_dframe, dim3((we + 63) / 64, rows, 2), dim3(64), 0, stream, bits, W, H, g,
                     F);
  return hipGetLastError();
}

namespace {

// Lane state of one side (the pixel s whose placements are evaluated) in one frame: dword of
// its row and its minor bit; for the other pixel q of the interchange, the two row offsets du
// (from s) that can hold it, and its minor offset from s reduced to [0, P).
struct SideFrame {
  int row, minb, du1, du2, dqn;
};

__device__ __forceinline__ SideFrame side_frame(const DiagGeo &g, int f, int sx, int sy, int qx,
                                                int qy, int W, int H) {
  const int Pr = f == 0 ? H : W, Pm = f == 0 ? W : H;
  const int sr = f == 0 ? sy : sx, sm = f == 0 ? sx : sy;
  const int qr = f == 0 ? qy : qx, qm = f == 0 ? qx : qy;
  // row s + du holds q iff du = q - s modulo Pr; |du| <= cutoff < Pr leaves two candidates
  const int dr = qr - sr;  // in (-Pr, Pr)
  const int du2 = dr > 0 ? dr - Pr : dr + Pr;
  int dq = qm - sm;
  dq += dq < 0 ? Pm : 0;
  return SideFrame{g.off[f] + (sr + g.rowoff[f]) * g.we[f], sm + g.B[f], dr, du2, dq};
}

// Bits of the window (origin o, frame row offset du) that hold the other pixel q.
__device__ __forceinline__ uint32_t other_bits(const SideFrame &s, int du, int o, int Pm,
                                               uint32_t pat) {
  const bool on_row = du == s.du1 || du == s.du2;
  int t = s.dqn - o;  // in (-Pm, 2 Pm)
  t += t < 0 ? Pm : 0;
  t -= t >= Pm ? Pm : 0;
  return (on_row && t < 32) ? pat << t : 0u;
}

__device__ __forceinline__ uint32_t window(const uint32_t *__restrict__ F, const SideFrame &s,
                                           int du_dw, int o) {
  const int pos = s.minb + o;
  const uint32_t *p = F + s.row + du_dw + (pos >> 5);
  return __builtin_amdgcn_alignbit(p[1], p[0], (uint32_t)pos);
}

}  // namespace

// Rows r0 .. r1 - 1 of one placement block of a group of NG (a multiple of 4, >= G) vectors on
// one side (0: placements through a, 1: through b), added into dl0 / dl1 with the side's sign.
// The product that sees the other pixel's change is A on side 0 (b set in J1) and O on side 1
// (a cleared in J0).
template <unsigned MASK, int NG>
__device__ __forceinline__ void side_rows(const uint32_t *__restrict__ F,
                                          const DiagRow *__restrict__ rows, int r0, int r1,
                                          const SideFrame &sx, int side, int sr, int we, int Pm,
                                          uint32_t pat, uint32_t V, int (&dl0)[kDiagG],
                                          int (&dl1)[kDiagG]) {
  constexpr bool P0 = (MASK & 1u) != 0, P1 = (MASK & 2u) != 0;
  const bool patch = side == 0 ? P1 : P0;
  uint32_t A[NG], O[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    A[g] = 0xffffffffu;
    O[g] = 0u;
  }
  // table row values (wave-uniform, scalar registers); with both products (the longer row
  // evaluation) the next row's are loaded while this one is evaluated, which measured 7% faster
  // there and 13% slower with one product (more scalar registers, fewer waves)
  constexpr bool kPrefetch = false;
  struct RowVals {
    int d, o;
    uint32_t valid, hs[NG], jp[NG / 4];
  };
  auto load_row = [&](int r, RowVals &v) {
    const DiagRow &R = rows[r];
    v.d = R.d;
    v.o = R.o;
    v.valid = R.valid;
#pragma unroll
    for (int g = 0; g < NG; ++g) v.hs[g] = R.hs[g];
#pragma unroll
    for (int g = 0; g < NG / 4; ++g) v.jp[g] = R.jp[g];
  };
  RowVals cur;
  if (kPrefetch && r0 < r1) load_row(r0, cur);
  for (int r = r0; r < r1; ++r) {
    RowVals nxt;
    if constexpr (kPrefetch)
      load_row(min(r + 1, r1 - 1), nxt);  // the last iteration reads its own row again
    else
      load_row(r, cur);
    const int du = sr * cur.d, o = cur.o;
    const uint32_t valid = cur.valid;
    const uint32_t *hs = cur.hs, *jp = cur.jp;
    const uint32_t w = window(F, sx, du * we, o);
    const uint32_t q = patch ? other_bits(sx, du, o, Pm, pat) : 0u;
    const uint32_t wA = side == 0 ? (w | q) : w, wO = side == 0 ? w : (w & ~q);
    // the pixel word of vector g's placements in window x: bit t from window bit j + 1 where
    // hs has t, else from bit j
    auto word = [&](int g, uint32_t x) {
      const uint32_t jj = (jp[g >> 2] >> (8 * (g & 3))) & 0xffu;
      return __builtin_amdgcn_bitop3_b32(hs[g], (uint32_t)__builtin_amdgcn_sbfe((int)x, jj + 1, 1),
                                         (uint32_t)__builtin_amdgcn_sbfe((int)x, jj, 1), 0xCA);
    };
    // With both products, one word serves both; a row where some lane's other pixel is in the
    // window (rare) keeps the patched product's accumulators before the row and redoes it after.
    const bool split = P0 && P1 && __builtin_amdgcn_ballot_w64(q != 0u) != 0;
    uint32_t keep[NG];
    if (split) {
#pragma unroll
      for (int g = 0; g < NG; ++g) keep[g] = side == 0 ? A[g] : O[g];
    }
    const uint32_t x = (P0 && P1) ? w : (P1 ? wA : wO);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const uint32_t t = word(g, x);
      if constexpr (P1) A[g] = __builtin_amdgcn_bitop3_b32(A[g], t, valid, 0xD0);  // A & (t | ~valid)
      if constexpr (P0) O[g] = __builtin_amdgcn_bitop3_b32(O[g], t, valid, 0xF8);  // O | (t & valid)
    }
    if (split) {
      if (side == 0) {
#pragma unroll
        for (int g = 0; g < NG; ++g)
          A[g] = __builtin_amdgcn_bitop3_b32(keep[g], word(g, wA), valid, 0xD0);
      } else {
#pragma unroll
        for (int g = 0; g < NG; ++g)
          O[g] = __builtin_amdgcn_bitop3_b32(keep[g], word(g, wO), valid, 0xF8);
      }
    }
    if constexpr (kPrefetch) cur = nxt;
  }
  // dL1 = (through b) - (through a) for phase 1, the reverse for phase 0
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if (P1) {
      const int c = __popc(A[g] & V);
      dl1[g] += side == 0 ? -c : c;
    }
    if (P0) {
      const int c = __popc(~O[g] & V);
      dl0[g] += side == 0 ? c : -c;
    }
  }
}

// dL of candidate interchanges (lanes: BS per workgroup) for the vector groups of chunk
// blockIdx.y.  All waves of a workgroup read the same table rows through the scalar cache; with
// one product, 16 waves per workgroup (fewer chunks per CU) measured 7 % faster than 4 at
// 128^2 / cutoff 32, with both (122 registers) 10 % slower at 256^2 / cutoff 48.  With J1 = I with b set to 1 and J0 = I with a cleared (a the phase-1 pixel):
//   dL1 = sum_{P_b} lambda1(J1) - sum_{P_a} lambda1(J1),  dL0 = sum_{P_a} lambda0(J0) - sum_{P_b} lambda0(J0)
// (a placement in both sets counts the same on both sides and cancels).  The pixel s itself
// (d = 0) is 1 in J1 and 0 in J0 on either side, so it never decides a product and is skipped;
// the only other changed pixel is b in side a's J1 and a in side b's J0.
template <unsigned MASK, bool LDS, int BS>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4)))
k_delta_diag(const uint32_t *__restrict__ Fg, DiagGeo geo, const uint64_t *__restrict__ bits,
             int W, int H, const int2 *__restrict__ cand, int K,
             const DiagGroup *__restrict__ groups, const int32_t *__restrict__ chunk_off,
             const DiagRow *__restrict__ rows, int nv, int32_t *__restrict__ out) {
  extern __shared__ uint32_t lds[];
  constexpr bool P0 = (MASK & 1u) != 0, P1 = (MASK & 2u) != 0;
  constexpr int nph = (P0 ? 1 : 0) + (P1 ? 1 : 0);
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  bool ok = k < K;
  int a = 0, b = 0;
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
  const int ay = a / W, ax = a - ay * W, by = b / W, bx = b - by * W;
  const uint32_t *F;
  if constexpr (LDS) {
    for (int i = threadIdx.x; i < geo.total; i += blockDim.x) lds[i] = Fg[i];
    __syncthreads();
    F = lds;
  } else {
    F = Fg;
  }
  const int c0 = chunk_off[blockIdx.y], c1 = chunk_off[blockIdx.y + 1];
  for (int gi = c0; gi < c1; ++gi) {
    const DiagGroup &gr = groups[gi];
    const int G = gr.G, n = gr.n, f = gr.frame, sr = gr.sr, nb = gr.nb, row0 = gr.row0;
    // lane state in the group's frame (recomputed per group: fewer live registers); side 0:
    // placements through a (other pixel b), side 1: through b (other pixel a)
    const SideFrame s0 = side_frame(geo, f, ax, ay, bx, by, W, H);
    const SideFrame s1 = side_frame(geo, f, bx, by, ax, ay, W, H);
    const int we = f == 0 ? geo.we[0] : geo.we[1];
    const int Pm = f == 0 ? W : H;
    const uint32_t pat = f == 0 ? geo.pat[0] : geo.pat[1];
    int dl0[kDiagG], dl1[kDiagG];
#pragma unroll
    for (int g = 0; g < kDiagG; ++g) {
      dl0[g] = 0;
      dl1[g] = 0;
    }
    const int ng4 = (G + 3) >> 2;
    for (int bl = 0; bl < nb; ++bl) {
      const int r0 = row0 + gr.boff[bl], r1 = row0 + gr.boff[bl + 1];
      // placements of the block
      const int nk = min(31, n - 32 * bl);
      const uint32_t V = nk == 31 ? 0xffffffffu : ((1u << (nk + 1)) - 1u);
      // side 0 (placements through a) and side 1 (through b) in turn: the accumulators of one
      // side only are live; the vector count is a compile-time multiple of 4
      for (int side = 0; side < 2; ++side) {
        const SideFrame &sx = side == 0 ? s0 : s1;
        switch (ng4) {
          case 1: side_rows<MASK, 4>(F, rows, r0, r1, sx, side, sr, we, Pm, pat, V, dl0, dl1); break;
          case 2: side_rows<MASK, 8>(F, rows, r0, r1, sx, side, sr, we, Pm, pat, V, dl0, dl1); break;
          case 3: side_rows<MASK, 12>(F, rows, r0, r1, sx, side, sr, we, Pm, pat, V, dl0, dl1); break;
          default: side_rows<MASK, 16>(F, rows, r0, r1, sx, side, sr, we, Pm, pat, V, dl0, dl1); break;
        }
      }
    }
    if (k < K) {
      int32_t *ok_out = out + (size_t)k * nph * nv;
#pragma unroll
      for (int g4 = 0; g4 < kDiagG; g4 += 4) {
        if (g4 >= G) break;
#pragma unroll
        for (int g = g4; g < g4 + 4; ++g) {
          if (g < G) {
            const int idx = gr.idx[g];
            int p = 0;
            if (P0) ok_out[(size_t)(p++) * nv + idx] = ok ? dl0[g] : 0;
            if (P1) ok_out[(size_t)p * nv + idx] = ok ? dl1[g] : 0;
          }
        }
      }
    }
  }
}

hipError_t launch_delta_diag(const DiagLaunch &L, hipStream_t stream) {
  const size_t lds = L.use_lds ? (size_t)L.geo.total * sizeof(uint32_t) : 0;
#define LPF_DIAG(M, BS)                                                                         \
  {                                                                                             \
    const dim3 grid((unsigned)((L.K + BS - 1) / BS), (unsigned)L.nchunks), block(BS);           \
    if (L.use_lds)                                                                              \
      hipLaunchKernelGGL((k_delta_diag<M, true, BS>), grid, block, lds, stream, L.F, L.geo,     \
                         L.bits, L.W, L.H, L.cand, L.K, L.groups, L.chunk_off, L.rows, L.nv,    \
                         L.delta_out);                                                          \
    else                                                                                        \
      hipLaunchKernelGGL((k_delta_diag<M, false, BS>), grid, block, 0, stream, L.F, L.geo,      \
                         L.bits, L.W, L.H, L.cand, L.K, L.groups, L.chunk_off, L.rows, L.nv,    \
                         L.delta_out);                                                          \
  }
  switch (L.phase_mask) {
    case 1: LPF_DIAG(1u, 1024); break;
    case 2: LPF_DIAG(2u, 1024); break;
    case 3: LPF_DIAG(3u, 256); break;
    default: return hipErrorInvalidValue;
  }
#undef LPF_DIAG
  return hipGetLastError();
}

hipError_t prepare_delta_kernels(int max_lds_bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)k_delta<true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_delta_diag<1u, true, 1024>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_delta_diag<2u, true, 1024>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_delta_diag<3u, true, 256>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
  return e;
}

}  // namespace lpf
