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

hipError_t prepare_delta_kernels(int max_lds_bytes) {
  return hipFuncSetAttribute((const void *)k_delta<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             max_lds_bytes);
}

}  // namespace lpf
