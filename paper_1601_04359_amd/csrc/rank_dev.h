// Learned ranking of a step's candidates on the device (shared by k_anneal.hip and k_rec.hip).
#pragma once

#include <math.h>
#include <stdint.h>

#include "lpf_internal.h"

namespace lpf {

// Evaluation order of a step's candidates (learned ranking): the kRankTop draws with the highest
// predicted gain score[a] + score[b] (fp32; void draws and NaN lowest; ties by draw index) among
// the first R = min(K, kRankMax), best first, then every other draw in draw order.  Each
// 256-draw workgroup (of k_propose, or k_rank_blocks) sorts its keys per wave (bitonic, across
// lanes) and merges the four wave lists into its best 64; k_rank_merge (or, in a records chain,
// every workgroup of round 0, k_rec_rank_round0) merges the workgroup lists, and the remaining
// draws are compacted in draw order with ballot prefix counts.

// 64-bit rank key: the gain in an order-preserving unsigned encoding (void draws and NaN as -inf,
// -0 as +0) above the complement of the draw index, so that a larger key ranks first and equal
// gains go to the earlier draw.  Every real key exceeds 0, the key of an empty slot.
__device__ __forceinline__ uint64_t rank_key(int a, int b, int i, const float *__restrict__ score) {
  float g = -INFINITY;
  if (a >= 0 && b >= 0) {
    const float s = score[a] + score[b];
    g = s == s ? s : -INFINITY;
    if (g == 0.0f) g = 0.0f;
  }
  const uint32_t u = __float_as_uint(g);
  const uint32_t o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((uint64_t)o << 32) | (uint64_t)(~(uint32_t)i);
}

// Value of lane (lane ^ S): DPP for S = 1, 2 (quad permutations) and 8 (row rotation by 8),
// ds_bpermute otherwise.  Like every cross-lane read here, call it with the whole wave active.
template <int S>
__device__ __forceinline__ uint32_t xor_lane32(uint32_t v) {
  if constexpr (S == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
  else if constexpr (S == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
  else if constexpr (S == 8) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);
  else return (uint32_t)__shfl_xor((int)v, S);
}

template <int S>
__device__ __forceinline__ uint64_t xor_lane64(uint64_t v) {
  return ((uint64_t)xor_lane32<S>((uint32_t)(v >> 32)) << 32) | xor_lane32<S>((uint32_t)v);
}

__device__ __forceinline__ uint64_t lane64(uint64_t v, int src) {
  return ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(v >> 32), src) << 32) |
         (uint32_t)__shfl((int)(uint32_t)v, src);
}

// Compare-exchange steps STRIDE, STRIDE/2, ..., 1 of the bitonic network at block size SIZE over
// NC independent columns (one key per lane each); blocks with (lane & SIZE) == 0 end descending.
template <int SIZE, int STRIDE, int NC>
__device__ __forceinline__ void bitonic_steps(uint64_t (&k)[NC], int lane) {
  if constexpr (STRIDE > 0) {
    const bool take_max = ((lane & STRIDE) == 0) == ((lane & SIZE) == 0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const uint64_t p = xor_lane64<STRIDE>(k[c]);
      k[c] = (take_max == (p > k[c])) ? p : k[c];
    }
    bitonic_steps<SIZE, STRIDE / 2, NC>(k, lane);
  }
}

// Sort each column descending across the 64 lanes.
template <int SIZE, int NC>
__device__ __forceinline__ void wave_sort_desc(uint64_t (&k)[NC], int lane) {
  if constexpr (SIZE <= 64) {
    bitonic_steps<SIZE, SIZE / 2, NC>(k, lane);
    wave_sort_desc<SIZE * 2, NC>(k, lane);
  }
}

// Best 64 of two descending columns, descending: lane l takes the larger of a[l] and b[63 - l]
// (a bitonic sequence holding the 64 largest), then a bitonic merge.
__device__ __forceinline__ uint64_t merge_top64(uint64_t a, uint64_t b_rev, int lane) {
  uint64_t m[1] = {a > b_rev ? a : b_rev};
  bitonic_steps<64, 32, 1>(m, lane);
  return m[0];
}

// Best 64 keys of a 256-thread workgroup (one key per thread), descending, into list[0..63].
// Called by every thread of the workgroup; sl is 2 x 64 keys of LDS.
__device__ __forceinline__ void block_top64(uint64_t key, uint64_t (*sl)[64],
                                            uint64_t *__restrict__ list) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t k[1] = {key};
  wave_sort_desc<2, 1>(k, lane);
  uint64_t m = k[0];
  if (w >= 2) sl[w - 2][lane] = m;
  __syncthreads();
  if (w < 2) m = merge_top64(m, sl[w][63 - lane], lane);
  __syncthreads();
  if (w == 1) sl[0][lane] = m;
  __syncthreads();
  if (w == 0) list[lane] = merge_top64(m, sl[0][63 - lane], lane);
}

// Best 64 keys of the kRankMax / 256 = 16 workgroup lists (nl of them present, 64 keys each,
// descending), descending, in the lanes of wave 0 of a 256-thread workgroup.  Called by every
// thread of the workgroup; sl is 2 x 64 keys of LDS.
__device__ __forceinline__ uint64_t merge_lists16(const uint64_t *__restrict__ lists, int nl,
                                                  uint64_t (*sl)[64]) {
  static_assert(kRankMax / 256 == 16 && kRankTop == 64, "merge_lists16: 16 lists of 64");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t c[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int li = 4 * w + j;
    c[j] = li < nl ? lists[li * kRankTop + lane] : 0ull;
  }
  // lane shuffles outside conditional expressions (see xor_lane32)
  const uint64_t r1 = lane64(c[1], 63 - lane), r3 = lane64(c[3], 63 - lane);
  uint64_t m2[2] = {c[0] > r1 ? c[0] : r1, c[2] > r3 ? c[2] : r3};
  bitonic_steps<64, 32, 2>(m2, lane);
  const uint64_t r = lane64(m2[1], 63 - lane);
  uint64_t m = merge_top64(m2[0], r, lane);
  if (w >= 2) sl[w - 2][lane] = m;
  __syncthreads();
  if (w < 2) m = merge_top64(m, sl[w][63 - lane], lane);
  __syncthreads();
  if (w == 1) sl[0][lane] = m;
  __syncthreads();
  if (w == 0) m = merge_top64(m, sl[0][63 - lane], lane);
  return m;
}

}  // namespace lpf
