"""Entire lineal path function (LPF) of periodic two-phase images on AMD MI355X (gfx950).

Havelka, Kucerova & Sykora, arXiv:1601.04359.  The compute path is liblpf.so (hand-written HIP
kernels behind the C ABI of include/lpf.h); this package is its thin Python binding.  Counts are
returned as torch int32 tensors holding the C ABI's uint32 values (all counts are < 2^31).
"""
from __future__ import annotations

import torch

from . import _abi
from ._abi import (LPF_BOTH, LPF_OUT_GRID, LPF_OUT_HALF, LPF_PHASE0, LPF_PHASE1, LpfError,
                   counts_shape, lpf_num_vectors, lpf_vectors)


def packed_words(W: int, H: int) -> int:
    return ((W + 63) // 64) * H


class Context:
    """Owns an lpf_ctx (scratch memory, launch plans) on one device; use one per stream."""

    def __init__(self, device: int = 0):
        self.device = device
        self.handle = _abi.lpf_ctx_create(device)

    def close(self) -> None:
        if self.handle:
            _abi.lpf_ctx_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- marshalling helpers: allocate outputs on the device, then call the C ABI --------------
    def pack(self, img: torch.Tensor, stream=None) -> torch.Tensor:
        """uint8 (H, W) device image -> packed int64 words (H, ceil(W/64))."""
        H, W = img.shape
        bits = torch.empty((H, (W + 63) // 64), dtype=torch.int64, device=img.device)
        _abi.lpf_pack(self.handle, img.contiguous(), W, H, bits, stream)
        return bits

    def full(self, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
             phase_mask: int = LPF_BOTH, layout: int = LPF_OUT_HALF, out=None,
             stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(counts_shape(cx, cy, phase_mask, layout), dtype=torch.int32,
                              device=bits.device)
        _abi.lpf_full(self.handle, bits, W, H, cx, cy, phase_mask, layout, out, stream)
        return out

    def set_full_shape(self, R: int = 0, S: int = 0, waves_per_group: int = 0,
                       lds_bytes: int = 0) -> None:
        _abi.lpf_set_full_shape(self.handle, R, S, waves_per_group, lds_bytes)
