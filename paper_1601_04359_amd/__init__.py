"""Entire lineal path function (LPF) of periodic two-phase images on AMD MI355X (gfx950).

Havelka, Kucerova & Sykora, arXiv:1601.04359.  The compute path is liblpf.so (hand-written HIP
kernels behind the C ABI of include/lpf.h); this package is its thin Python binding.  Counts are
returned as torch int32 tensors holding the C ABI's uint32 values (all counts are < 2^31).
"""
from __future__ import annotations

import torch

from . import _abi
from ._abi import (LPF_BOTH, LPF_DELTA_AUTO, LPF_DELTA_RECORDS, LPF_DELTA_RECOUNT, LPF_DELTA_S2,
                   LPF_OUT_GRID, LPF_OUT_HALF, LPF_PHASE0, LPF_PHASE1,
                   LPF_PROP_INTERFACIAL, LPF_PROP_LEARNED, LPF_PROP_UNIFORM, LpfError,
                   counts_shape, lpf_num_vectors, lpf_vectors)

import numpy as _np

# host view of lpf_step_result records (an int64 tensor of shape (n, 5) on the device)
STEP_DTYPE = _np.dtype([("k", _np.int32), ("a", _np.int32), ("b", _np.int32), ("pad", _np.int32),
                        ("de", _np.float64), ("e", _np.float64), ("step", _np.uint64)])


def step_records(t: torch.Tensor) -> _np.ndarray:
    return t.detach().cpu().numpy().view(STEP_DTYPE).reshape(-1)


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

    def full_enhanced(self, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                      phase_mask: int = LPF_BOTH, layout: int = LPF_OUT_HALF, out=None,
                      stream=None) -> torch.Tensor:
        """Same counts as full(), with segments abandoned once no start pixel can still count."""
        if out is None:
            out = torch.empty(counts_shape(cx, cy, phase_mask, layout), dtype=torch.int32,
                              device=bits.device)
        _abi.lpf_full_enhanced(self.handle, bits, W, H, cx, cy, phase_mask, layout, out, stream)
        return out

    def pack3d(self, vol: torch.Tensor, stream=None) -> torch.Tensor:
        """uint8 (D, H, W) device volume -> packed int64 rows (D*H, ceil(W/64))."""
        D, H, W = vol.shape
        return self.pack(vol.reshape(D * H, W), stream)

    def full3d(self, bits: torch.Tensor, W: int, H: int, D: int, cx: int, cy: int, cz: int,
               phase_mask: int = LPF_BOTH, out=None, stream=None) -> torch.Tensor:
        """Counts int32 (nph, |D_c|) of a periodic volume over the canonical 3-D vectors
        (lpf_vectors3); cz = 0 gives the sum of the xy-cuts' 2-D functions."""
        if out is None:
            nph = (phase_mask & 1) + ((phase_mask >> 1) & 1)
            out = torch.empty((nph, _abi.lpf_num_vectors3(cx, cy, cz)), dtype=torch.int32,
                              device=bits.device)
        _abi.lpf_full3d(self.handle, bits, W, H, D, cx, cy, cz, phase_mask, out, stream)
        return out

    def full_sampled(self, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                     sample: torch.Tensor, phase_mask: int = LPF_BOTH, layout: int = LPF_OUT_HALF,
                     out=None, stream=None) -> torch.Tensor:
        """Monte-Carlo approximation in counts: segments tested only at the start pixels set in
        the packed mask `sample` (pack() of a uint8 mask)."""
        if out is None:
            out = torch.empty(counts_shape(cx, cy, phase_mask, layout), dtype=torch.int32,
                              device=bits.device)
        _abi.lpf_full_sampled(self.handle, bits, W, H, cx, cy, phase_mask, layout,
                              sample.contiguous(), out, stream)
        return out

    def s2(self, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
           phase_mask: int = LPF_BOTH, layout: int = LPF_OUT_HALF, out=None,
           stream=None) -> torch.Tensor:
        """Two-point counts W*H*S2 (eq. (S2dis)) in the layout of full()."""
        if out is None:
            out = torch.empty(counts_shape(cx, cy, phase_mask, layout), dtype=torch.int32,
                              device=bits.device)
        _abi.lpf_s2(self.handle, bits, W, H, cx, cy, phase_mask, layout, out, stream)
        return out

    def s2_delta_swap(self, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                      swaps: torch.Tensor, phase_mask: int = LPF_BOTH, out=None,
                      stream=None) -> torch.Tensor:
        """delta int32 (n, nph, |D_c|) of the two-point counts for interchanges (n, 2)."""
        n = swaps.shape[0]
        nph = (phase_mask & 1) + ((phase_mask >> 1) & 1)
        if out is None:
            out = torch.empty((n, nph, lpf_num_vectors(cx, cy)), dtype=torch.int32,
                              device=bits.device)
        _abi.lpf_s2_delta_swap(self.handle, bits, W, H, cx, cy, phase_mask, swaps.contiguous(),
                               n, out, stream)
        return out

    def delta_swap(self, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                   swaps: torch.Tensor, phase_mask: int = LPF_BOTH, out=None,
                   stream=None) -> torch.Tensor:
        """delta int32 (n, nph, |D_c|) = L(I') - L(I) for interchanges swaps (n, 2) int32."""
        n = swaps.shape[0]
        nph = (phase_mask & 1) + ((phase_mask >> 1) & 1)
        if out is None:
            out = torch.empty((n, nph, lpf_num_vectors(cx, cy)), dtype=torch.int32,
                              device=bits.device)
        _abi.lpf_delta_swap(self.handle, bits, W, H, cx, cy, phase_mask, swaps.contiguous(), n,
                            out, stream)
        return out

    def batch(self, images, phase_mask: int = LPF_BOTH, layout: int = LPF_OUT_HALF,
              stream=None):
        """images: list of (bits tensor, W, H, cx, cy).  Packs them into one pool, runs lpf_batch
        and returns (counts_pool, offsets, pool, descs); counts of image i are
        counts_pool[offsets[i] : offsets[i] + size_i] in the layout's order."""
        descs = (_abi.lpf_image_desc * len(images))()
        off_b, off_c, offs = 0, 0, []
        for i, (bits, W, H, cx, cy) in enumerate(images):
            descs[i].W, descs[i].H, descs[i].cx, descs[i].cy = W, H, cx, cy
            descs[i].bits_off, descs[i].counts_off = off_b, off_c
            offs.append(off_c)
            off_b += bits.numel()
            off_c += int(torch.Size(counts_shape(cx, cy, phase_mask, layout)).numel())
        dev = images[0][0].device
        pool = torch.cat([b.reshape(-1) for (b, *_r) in images]).contiguous()
        counts = torch.empty(max(off_c, 1), dtype=torch.int32, device=dev)
        _abi.lpf_batch(self.handle, pool, descs, phase_mask, layout, counts, stream)
        return counts, offs, pool, descs

    def autotune(self, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                 phase_mask: int = LPF_BOTH, stream=None) -> float:
        return _abi.lpf_autotune_full(self.handle, bits, W, H, cx, cy, phase_mask, stream)

    def tuned_shape(self, W: int, H: int, cx: int, cy: int):
        return _abi.lpf_get_tuned_shape(self.handle, W, H, cx, cy)

    def set_full_shape(self, R: int = 0, S: int = 0, waves_per_group: int = 0,
                       lds_bytes: int = 0) -> None:
        _abi.lpf_set_full_shape(self.handle, R, S, waves_per_group, lds_bytes)


class Anneal:
    """A device-resident annealing chain (anneal_step); the tensors below are its state.

    bits (packed cell, updated in place), counts (int32 [nph][|D_c|]), e (float64 [1]) are
    allocated here and owned by this object; target (int32 [nph][|D_c|]) is the caller's.
    descriptor "lpf" (the lineal path function) or "s2" (two-point counts, lpf_anneal_create_s2;
    target then holds Context.s2 counts of the original).  sample: a packed position set of the
    cell for the Monte-Carlo approximation (lpf_anneal_create_sampled; target then holds the
    original's sampled counts and Nt its number of positions)."""

    def __init__(self, ctx: Context, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                 phase_mask: int, target: torch.Tensor, Nt: int, seed: int, step0: int = 0,
                 pos: torch.Tensor | None = None, n1: int = 0, stream=None,
                 descriptor: str = "lpf", sample: torch.Tensor | None = None):
        if descriptor not in ("lpf", "s2"):
            raise ValueError("descriptor is 'lpf' or 's2'")
        if sample is not None and descriptor != "lpf":
            raise ValueError("a position set applies to the lineal path function only")
        self.descriptor = descriptor
        self.sample = None if sample is None else sample.contiguous()
        self.ctx, self.W, self.H, self.cx, self.cy, self.phase_mask = ctx, W, H, cx, cy, phase_mask
        dev = bits.device
        self.bits = bits.clone().contiguous()
        self.counts = torch.empty(counts_shape(cx, cy, phase_mask, LPF_OUT_HALF), dtype=torch.int32,
                                  device=dev)
        self.target = target.contiguous()
        self.e = torch.zeros(1, dtype=torch.float64, device=dev)
        if self.sample is not None:
            self.handle = _abi.lpf_anneal_create_sampled(
                ctx.handle, self.bits, W, H, cx, cy, phase_mask, self.sample, self.counts,
                self.target, Nt, seed, step0, pos, n1, self.e, stream)
        else:
            self.handle = _abi.lpf_anneal_create(ctx.handle, self.bits, W, H, cx, cy, phase_mask,
                                                 self.counts, self.target, Nt, seed, step0, pos,
                                                 n1, self.e, stream, s2=descriptor == "s2")

    def step(self, n_candidates: int, T: float, out: torch.Tensor,
             proposal: int = LPF_PROP_UNIFORM, stream=None) -> None:
        """One step; its record goes to `out` (a device int64 tensor row of 5 elements)."""
        _abi.anneal_step(self.handle, n_candidates, proposal, T, out, stream)

    def run(self, n_candidates: int, Ts, proposal: int = LPF_PROP_UNIFORM,
            stream=None) -> torch.Tensor:
        """len(Ts) steps, one anneal_step call each; records (n, 5) int64 on the device."""
        recs = torch.empty((len(Ts), 5), dtype=torch.int64, device=self.bits.device)
        for i, T in enumerate(Ts):
            _abi.anneal_step(self.handle, n_candidates, proposal, float(T), recs[i], stream)
        return recs

    def run_schedule(self, n_candidates: int, Ts, proposal: int = LPF_PROP_UNIFORM,
                     stream=None) -> torch.Tensor:
        """The same steps in one lpf_anneal_run call (temperatures uploaded once; graph replays
        for uniform and interfacial proposals)."""
        dev = self.bits.device
        T = torch.as_tensor(Ts, dtype=torch.float64).to(dev).contiguous()
        recs = torch.empty((T.numel(), 5), dtype=torch.int64, device=dev)
        self._T_sched = T  # alive until the stream has consumed it
        _abi.lpf_anneal_run(self.handle, n_candidates, proposal, T, recs, stream)
        return recs

    def set_proposal(self, net=None, scores: torch.Tensor | None = None, beta: float = 1.0,
                     eps_uniform: float = 0.1, refresh: int = 1, rank: bool = False) -> None:
        """Learned proposals from a ProposalNet (scored on the current cell) or a score field,
        re-scored every `refresh` learned draws; with `rank` the step's candidates are evaluated
        by descending predicted gain."""
        self._scores = scores  # keep the caller's field alive
        self._net = net
        _abi.lpf_anneal_set_proposal(self.handle, net.handle if net is not None else None,
                                     scores, beta, eps_uniform, refresh, int(bool(rank)))

    def set_method(self, method: int) -> None:
        """Candidate evaluation method: LPF_DELTA_AUTO, LPF_DELTA_RECOUNT or LPF_DELTA_RECORDS."""
        _abi.lpf_anneal_set_method(self.handle, method)

    @property
    def method(self) -> int:
        return _abi.lpf_anneal_get_method(self.handle)

    def propose(self, K: int, proposal: int = LPF_PROP_UNIFORM, stream=None) -> torch.Tensor:
        out = torch.empty((K, 2), dtype=torch.int32, device=self.bits.device)
        _abi.lpf_anneal_propose(self.handle, K, proposal, out, stream)
        return out

    def delta_energy(self, swaps: torch.Tensor, stream=None) -> torch.Tensor:
        n = swaps.shape[0]
        de = torch.empty(n, dtype=torch.float64, device=self.bits.device)
        _abi.lpf_anneal_delta_energy(self.handle, swaps.contiguous(), n, de, stream)
        return de

    def export(self, stream=None):
        pos = torch.empty(self.W * self.H, dtype=torch.int32, device=self.bits.device)
        n1, nxt = _abi.lpf_anneal_export(self.handle, pos, stream)
        return pos, n1, nxt

    def close(self) -> None:
        if getattr(self, "handle", 0):
            _abi.lpf_anneal_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cnn_samples(img_idx, a, b, y, device) -> torch.Tensor:
    """Pack interchange samples as the C ABI's lpf_cnn_sample records (int32 x3, float32)."""
    n = len(a)
    rec = _np.zeros((n, 4), _np.int32)
    rec[:, 0] = _np.asarray(img_idx, _np.int32)
    rec[:, 1] = _np.asarray(a, _np.int32)
    rec[:, 2] = _np.asarray(b, _np.int32)
    rec[:, 3] = _np.asarray(y, _np.float32).view(_np.int32)
    return torch.from_numpy(rec).to(device)


class ProposalNet:
    """The swap-proposal CNN (lpf_cnn_*): scores every pixel of W x H cells."""

    def __init__(self, ctx: Context, W: int, H: int, max_batch: int, max_samples: int,
                 params: torch.Tensor | None = None, stream=None):
        self.ctx, self.W, self.H = ctx, W, H
        self.max_batch, self.max_samples = max_batch, max_samples
        self.handle = _abi.lpf_cnn_create(ctx.handle, W, H, max_batch, max_samples,
                                          None if params is None else params.contiguous(), stream)
        self.t = 0

    def params(self, stream=None) -> torch.Tensor:
        out = torch.empty(_abi.LPF_CNN_PARAMS, dtype=torch.float32, device="cuda")
        _abi.lpf_cnn_get_params(self.handle, out, stream)
        return out

    def set_params(self, p: torch.Tensor, stream=None) -> None:
        _abi.lpf_cnn_set_params(self.handle, p.contiguous(), stream)
        self.t = 0

    def forward(self, bits: torch.Tensor, batch: int, out=None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty((batch, self.H, self.W), dtype=torch.float32, device=bits.device)
        _abi.lpf_cnn_forward(self.handle, bits.contiguous(), batch, out, stream)
        return out

    def grad(self, bits: torch.Tensor, batch: int, samples: torch.Tensor, stream=None):
        g = torch.empty(_abi.LPF_CNN_PARAMS, dtype=torch.float32, device=bits.device)
        loss = torch.empty(1, dtype=torch.float32, device=bits.device)
        _abi.lpf_cnn_grad(self.handle, bits.contiguous(), batch, samples, samples.shape[0], g,
                          loss, stream)
        return g, loss

    def adam(self, grad: torch.Tensor, lr: float, stream=None) -> None:
        self.t += 1
        _abi.lpf_cnn_adam(self.handle, grad, self.t, lr, stream=stream)

    def close(self) -> None:
        if getattr(self, "handle", 0):
            _abi.lpf_cnn_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
