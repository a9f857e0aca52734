// Internal declarations shared by the HIP sources of liblpf (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpf {

// One entry of a launch plan's vector list: the vector and its canonical index in D_c.
struct VecDesc {
  int16_t dx, dy;
  int32_t idx;
};

// Tile shape of the full-evaluation kernel.
//   R       consecutive 32-pixel words of one row owned by a lane
//   S       lanes per image row (R*S >= ceil(W/32)); a wave covers 64/S rows per band
//   wpg     waves per workgroup
//   tile    start rows per workgroup (row tile); ntiles = ceil(H / tile)
//   rst     LDS row stride in dwords (>= we), chosen against bank conflicts
//   we      dwords per row of the extended image: S*R + (cx >> 5) + 1
//   lds_rows rows staged in LDS per workgroup: tile + cy + 64/S
struct FullShape {
  int R, S, wpg, tile, ntiles, rst, we, lds_rows;
  int nbins;  // wave-level vector bins per tile
};

// Kernel launchers (defined in k_full.hip).  All enqueue on `stream` and return the HIP status.
hipError_t launch_pack(const uint8_t *img, int W, int H, uint64_t *bits, hipStream_t stream);
hipError_t launch_ext(const uint64_t *bits, int W, int H, int we, uint32_t *ext,
                      hipStream_t stream);
hipError_t launch_full(const FullShape &sh, const uint32_t *ext, int W, int H, int cy,
                       const VecDesc *vecs, const int32_t *bin_off, unsigned phase_mask,
                       uint32_t *out, int nv, hipStream_t stream);
hipError_t launch_finish(const uint32_t *part, int ntiles, int nph, int nv, const int16_t *dxdy,
                         int cx, int cy, int layout, uint32_t *out, hipStream_t stream);
hipError_t prepare_full_kernels(int max_lds_bytes);

}  // namespace lpf
