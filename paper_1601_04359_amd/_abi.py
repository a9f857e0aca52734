"""ctypes binding of liblpf (include/lpf.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Tensors are PyTorch tensors
used as device memory; the stream is torch's current stream unless one is given.  All compute
runs in the HIP kernels of liblpf.so; when the library is missing this module raises at import.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblpf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"liblpf.so not built at {LIB_PATH}; run `python paper_1601_04359_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

LPF_OK = 0
LPF_E_INVAL = -22
LPF_E_NOMEM = -12
LPF_E_DEVICE = -5
LPF_E_UNSUPPORTED = -95
LPF_PHASE0, LPF_PHASE1, LPF_BOTH = 1, 2, 3
LPF_OUT_HALF, LPF_OUT_GRID = 0, 1
LPF_DELTA_AUTO, LPF_DELTA_RECOUNT, LPF_DELTA_RECORDS, LPF_DELTA_S2 = 0, 1, 2, 3
LPF_SWAP_AUTO, LPF_SWAP_RUNS = 0, 1

_P = ctypes.c_void_p
_i32, _i64, _u32, _u64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint, ctypes.c_uint64


class LpfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"liblpf status {status}: {msg}")
        self.status = status


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("lpf_ctx_create", _i32, _i32, ctypes.POINTER(_P))
_sig("lpf_ctx_destroy", None, _P)
_sig("lpf_last_error", ctypes.c_char_p)
_sig("lpf_num_vectors", _i64, _i32, _i32)
_sig("lpf_vectors", _i32, _i32, _i32, _P)
_sig("lpf_pack", _i32, _P, _P, _i32, _i32, _P, _P)
_sig("lpf_full", _i32, _P, _P, _i32, _i32, _i32, _i32, _u32, _i32, _P, _P)
_sig("lpf_full_enhanced", _i32, _P, _P, _i32, _i32, _i32, _i32, _u32, _i32, _P, _P)
_sig("lpf_full_noalloc", _i32, _P, _P, _i32, _i32, _i32, _i32, _u32, _i32, _P, _P)
_sig("lpf_chain_stats", _i32, _i32, _i32, _P)
_sig("lpf_plan_check", _i32, _i32, _i32, _i64, _P)
_sig("lpf_peak_probe", _i32, _P, _i32, _i64, _i32, _P, ctypes.POINTER(ctypes.c_double), _P)
_sig("lpf_set_full_shape", _i32, _P, _i32, _i32, _i32, _i32)
_sig("lpf_delta_swap", _i32, _P, _P, _i32, _i32, _i32, _i32, _u32, _P, _i32, _P, _P)
_sig("lpf_set_delta_method", _i32, _P, _i32)
_sig("lpf_anneal_create", _i32, _P, _P, _i32, _i32, _i32, _i32, _u32, _P, _P, _i64, _u64, _u64,
     _P, _i32, _P, ctypes.POINTER(_P), _P)
_sig("lpf_anneal_create_s2", _i32, _P, _P, _i32, _i32, _i32, _i32, _u32, _P, _P, _i64, _u64, _u64,
     _P, _i32, _P, ctypes.POINTER(_P), _P)
_sig("lpf_s2", _i32, _P, _P, _i32, _i32, _i32, _i32, _u32, _i32, _P, _P)
_sig("lpf_num_vectors3", _i64, _i32, _i32, _i32)
_sig("lpf_vectors3", _i32, _i32, _i32, _i32, _P)
_sig("lpf_full3d", _i32, _P, _P, _i32, _i32, _i32, _i32, _i32, _i32, _u32, _P, _P)
_sig("lpf_full_sampled", _i32, _P, _P, _i32, _i32, _i32, _i32, _u32, _i32, _P, _P, _P)
_sig("lpf_anneal_create_sampled", _i32, _P, _P, _i32, _i32, _i32, _i32, _u32, _P, _P, _P, _i64,
     _u64, _u64, _P, _i32, _P, ctypes.POINTER(_P), _P)
_sig("lpf_s2_delta_swap", _i32, _P, _P, _i32, _i32, _i32, _i32, _u32, _P, _i32, _P, _P)
_sig("anneal_step", _i32, _P, _i32, _i32, ctypes.c_double, _P, _P)
_sig("lpf_anneal_run", _i32, _P, _i32, _i32, _P, _i32, _P, _P)
_sig("lpf_rank", _i32, _P, _P, _P, _i32, _P, _P)
_sig("lpf_anneal_export", _i32, _P, _P, ctypes.POINTER(_i32), ctypes.POINTER(_u64), _P)
_sig("lpf_anneal_destroy", None, _P)

_sig("lpf_batch", _i32, _P, _P, _P, _i32, _u32, _i32, _P, _P)
_sig("lpf_autotune_full", _i32, _P, _P, _i32, _i32, _i32, _i32, _u32, _P,
     ctypes.POINTER(ctypes.c_double))
_sig("lpf_get_tuned_shape", _i32, _P, _i32, _i32, _i32, _i32, ctypes.POINTER(_i32),
     ctypes.POINTER(_i32), ctypes.POINTER(_i32))

_sig("lpf_cnn_create", _i32, _P, _i32, _i32, _i32, _i32, _P, ctypes.POINTER(_P), _P)
_sig("lpf_cnn_set_params", _i32, _P, _P, _P)
_sig("lpf_cnn_get_params", _i32, _P, _P, _P)
_sig("lpf_cnn_forward", _i32, _P, _P, _i32, _P, _P)
_sig("lpf_cnn_grad", _i32, _P, _P, _i32, _P, _i32, _P, _P, _P)
_sig("lpf_cnn_adam", _i32, _P, _P, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
     ctypes.c_float, _P)
_sig("lpf_cnn_destroy", None, _P)
LPF_CNN_PARAMS = 4961
_sig("lpf_anneal_set_proposal", _i32, _P, _P, _P, ctypes.c_float, ctypes.c_float, _i32, _i32)
_sig("lpf_anneal_propose", _i32, _P, _i32, _i32, _P, _P)
_sig("lpf_anneal_delta_energy", _i32, _P, _P, _i32, _P, _P)
_sig("lpf_anneal_set_method", _i32, _P, _i32)
_sig("lpf_anneal_get_method", _i32, _P)

LPF_PROP_UNIFORM, LPF_PROP_INTERFACIAL, LPF_PROP_LEARNED = 0, 1, 2


class lpf_image_desc(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("H", ctypes.c_int32), ("cx", ctypes.c_int32),
                ("cy", ctypes.c_int32), ("bits_off", ctypes.c_int64), ("counts_off", ctypes.c_int64)]
STEP_RESULT_BYTES = 40  # lpf_step_result: int32 x4, double x2, uint64


def lib() -> ctypes.CDLL:
    return _lib


def _check(status: int) -> None:
    if status != LPF_OK:
        raise LpfError(status, _lib.lpf_last_error().decode())


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dev(t: torch.Tensor, dtype, name: str) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.data_ptr() % 8:
        raise ValueError(f"{name}: must be 8-byte aligned")
    return t.data_ptr()


def lpf_ctx_create(device: int = 0) -> int:
    h = _P()
    _check(_lib.lpf_ctx_create(device, ctypes.byref(h)))
    return h.value


def lpf_ctx_destroy(ctx: int) -> None:
    _lib.lpf_ctx_destroy(ctx)


def lpf_num_vectors(cx: int, cy: int) -> int:
    return int(_lib.lpf_num_vectors(cx, cy))


def lpf_vectors(cx: int, cy: int):
    import numpy as np
    n = lpf_num_vectors(cx, cy)
    if n < 0:
        raise LpfError(LPF_E_INVAL, "negative cutoff")
    out = np.zeros((n, 2), np.int16)
    _check(_lib.lpf_vectors(cx, cy, out.ctypes.data_as(_P)))
    return out


def lpf_pack(ctx: int, img: torch.Tensor, W: int, H: int, bits: torch.Tensor, stream=None) -> None:
    if img.numel() != W * H or bits.numel() != ((W + 63) // 64) * H:
        raise ValueError("lpf_pack: buffer sizes do not match W, H")
    _check(_lib.lpf_pack(ctx, _dev(img, torch.uint8, "img"), W, H,
                         _dev(bits, torch.int64, "bits"), _stream(stream)))


def counts_shape(cx: int, cy: int, phase_mask: int, layout: int):
    nph = (phase_mask & 1) + ((phase_mask >> 1) & 1)
    if layout == LPF_OUT_HALF:
        return (nph, lpf_num_vectors(cx, cy))
    return (nph, 2 * cy + 1, 2 * cx + 1)


def lpf_full(ctx: int, bits: torch.Tensor, W: int, H: int, cx: int, cy: int, phase_mask: int,
             out_layout: int, counts: torch.Tensor, stream=None) -> None:
    if bits.numel() != ((W + 63) // 64) * H:
        raise ValueError("lpf_full: bits size does not match W, H")
    shp = counts_shape(cx, cy, phase_mask, out_layout) if 0 <= cx and 0 <= cy else None
    if shp is not None and counts.numel() != int(torch.Size(shp).numel()):
        raise ValueError(f"lpf_full: counts must hold {shp} elements")
    _check(_lib.lpf_full(ctx, _dev(bits, torch.int64, "bits"), W, H, cx, cy, phase_mask,
                         out_layout, _dev(counts, torch.int32, "counts"), _stream(stream)))


def lpf_full_enhanced(ctx: int, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                      phase_mask: int, out_layout: int, counts: torch.Tensor,
                      stream=None) -> None:
    if bits.numel() != ((W + 63) // 64) * H:
        raise ValueError("lpf_full_enhanced: bits size does not match W, H")
    shp = counts_shape(cx, cy, phase_mask, out_layout) if 0 <= cx and 0 <= cy else None
    if shp is not None and counts.numel() != int(torch.Size(shp).numel()):
        raise ValueError(f"lpf_full_enhanced: counts must hold {shp} elements")
    _check(_lib.lpf_full_enhanced(ctx, _dev(bits, torch.int64, "bits"), W, H, cx, cy,
                                  phase_mask, out_layout, _dev(counts, torch.int32, "counts"),
                                  _stream(stream)))


def lpf_full_noalloc(ctx: int, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                     phase_mask: int, out_layout: int, counts: torch.Tensor,
                     stream=None) -> None:
    if bits.numel() != ((W + 63) // 64) * H:
        raise ValueError("lpf_full_noalloc: bits size does not match W, H")
    shp = counts_shape(cx, cy, phase_mask, out_layout) if 0 <= cx and 0 <= cy else None
    if shp is not None and counts.numel() != int(torch.Size(shp).numel()):
        raise ValueError(f"lpf_full_noalloc: counts must hold {shp} elements")
    _check(_lib.lpf_full_noalloc(ctx, _dev(bits, torch.int64, "bits"), W, H, cx, cy,
                                 phase_mask, out_layout, _dev(counts, torch.int32, "counts"),
                                 _stream(stream)))


def lpf_chain_stats(cx: int, cy: int) -> dict:
    """Chains lpf_full walks for a cutoff (host computation, no device)."""
    out = (ctypes.c_int64 * 4)()
    st = _lib.lpf_chain_stats(cx, cy, ctypes.cast(out, _P))
    if st != LPF_OK:
        raise LpfError(st, f"lpf_chain_stats({cx}, {cy})")
    return {"vectors": out[0], "chains": out[1], "walk": out[2], "path_pixels": out[3]}


def lpf_plan_check(cx: int, cy: int, nb_want: int) -> dict:
    """Host check of lpf_full's launch plan (no device); raises LpfError when a check fails."""
    out = (ctypes.c_int64 * 4)()
    st = _lib.lpf_plan_check(cx, cy, nb_want, ctypes.cast(out, _P))
    if st != LPF_OK:
        raise LpfError(st, f"lpf_plan_check({cx}, {cy}, {nb_want})")
    return {"bins": out[0], "pieces": out[1], "max_members": out[2], "walk": out[3]}


def lpf_peak_probe(ctx: int, kind: int, iters: int, nwg: int, sink: torch.Tensor,
                   stream=None) -> float:
    """Enqueue one throughput probe; returns its lane-operations (kinds 0-3) or LDS bytes (4)."""
    if sink.numel() < nwg * 256:
        raise ValueError("lpf_peak_probe: sink must hold nwg * 256 uint32")
    work = ctypes.c_double(0.0)
    _check(_lib.lpf_peak_probe(ctx, kind, iters, nwg, _dev(sink, torch.int32, "sink"),
                               ctypes.byref(work), _stream(stream)))
    return work.value


def lpf_delta_swap(ctx: int, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                   phase_mask: int, swaps: torch.Tensor, n: int, delta: torch.Tensor,
                   stream=None) -> None:
    if swaps.numel() != 2 * n:
        raise ValueError("lpf_delta_swap: swaps must hold n pairs")
    nph = (phase_mask & 1) + ((phase_mask >> 1) & 1)
    if n and delta.numel() != n * nph * lpf_num_vectors(cx, cy):
        raise ValueError("lpf_delta_swap: delta must hold n * nph * |D_c| elements")
    _check(_lib.lpf_delta_swap(ctx, _dev(bits, torch.int64, "bits"), W, H, cx, cy, phase_mask,
                               _dev(swaps, torch.int32, "swaps") if n else None, n,
                               _dev(delta, torch.int32, "delta") if n else None, _stream(stream)))


def lpf_set_delta_method(ctx: int, method: int) -> None:
    _check(_lib.lpf_set_delta_method(ctx, method))


def lpf_s2(ctx: int, bits: torch.Tensor, W: int, H: int, cx: int, cy: int, phase_mask: int,
           out_layout: int, counts: torch.Tensor, stream=None) -> None:
    if bits.numel() != ((W + 63) // 64) * H:
        raise ValueError("lpf_s2: bits size does not match W, H")
    shp = counts_shape(cx, cy, phase_mask, out_layout) if 0 <= cx and 0 <= cy else None
    if shp is not None and counts.numel() != int(torch.Size(shp).numel()):
        raise ValueError(f"lpf_s2: counts must hold {shp} elements")
    _check(_lib.lpf_s2(ctx, _dev(bits, torch.int64, "bits"), W, H, cx, cy, phase_mask,
                       out_layout, _dev(counts, torch.int32, "counts"), _stream(stream)))


def lpf_num_vectors3(cx: int, cy: int, cz: int) -> int:
    return int(_lib.lpf_num_vectors3(cx, cy, cz))


def lpf_vectors3(cx: int, cy: int, cz: int):
    import numpy as np
    n = lpf_num_vectors3(cx, cy, cz)
    if n < 0:
        raise ValueError("lpf_vectors3: negative cutoff")
    out = np.zeros((n, 3), np.int16)
    _check(_lib.lpf_vectors3(cx, cy, cz, out.ctypes.data_as(_P)))
    return out


def lpf_full3d(ctx: int, bits: torch.Tensor, W: int, H: int, D: int, cx: int, cy: int, cz: int,
               phase_mask: int, counts: torch.Tensor, stream=None) -> None:
    if bits.numel() != ((W + 63) // 64) * H * D:
        raise ValueError("lpf_full3d: bits size does not match W, H, D")
    nph = (phase_mask & 1) + ((phase_mask >> 1) & 1)
    if min(cx, cy, cz) >= 0 and counts.numel() != nph * lpf_num_vectors3(cx, cy, cz):
        raise ValueError("lpf_full3d: counts must hold nph * |D_c| elements")
    _check(_lib.lpf_full3d(ctx, _dev(bits, torch.int64, "bits"), W, H, D, cx, cy, cz, phase_mask,
                           _dev(counts, torch.int32, "counts"), _stream(stream)))


def lpf_full_sampled(ctx: int, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                     phase_mask: int, out_layout: int, sample: torch.Tensor, counts: torch.Tensor,
                     stream=None) -> None:
    if bits.numel() != ((W + 63) // 64) * H or sample.numel() != bits.numel():
        raise ValueError("lpf_full_sampled: bits / sample sizes do not match W, H")
    shp = counts_shape(cx, cy, phase_mask, out_layout) if 0 <= cx and 0 <= cy else None
    if shp is not None and counts.numel() != int(torch.Size(shp).numel()):
        raise ValueError(f"lpf_full_sampled: counts must hold {shp} elements")
    _check(_lib.lpf_full_sampled(ctx, _dev(bits, torch.int64, "bits"), W, H, cx, cy, phase_mask,
                                 out_layout, _dev(sample, torch.int64, "sample"),
                                 _dev(counts, torch.int32, "counts"), _stream(stream)))


def lpf_anneal_create_sampled(ctx: int, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                              phase_mask: int, sample: torch.Tensor, counts: torch.Tensor,
                              target: torch.Tensor, Nt: int, seed: int, step0: int, pos, n1: int,
                              e: torch.Tensor, stream=None) -> int:
    if sample.numel() != bits.numel():
        raise ValueError("lpf_anneal_create_sampled: sample must be packed like bits")
    h = _P()
    _check(_lib.lpf_anneal_create_sampled(
        ctx, _dev(bits, torch.int64, "bits"), W, H, cx, cy, phase_mask,
        _dev(sample, torch.int64, "sample"), _dev(counts, torch.int32, "counts"),
        _dev(target, torch.int32, "target"), Nt, seed, step0,
        _dev(pos, torch.int32, "pos") if pos is not None else None, n1,
        _dev(e, torch.float64, "e"), ctypes.byref(h), _stream(stream)))
    return h.value


def lpf_s2_delta_swap(ctx: int, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                      phase_mask: int, swaps: torch.Tensor, n: int, delta: torch.Tensor,
                      stream=None) -> None:
    if swaps.numel() != 2 * n:
        raise ValueError("lpf_s2_delta_swap: swaps must hold n pairs")
    nph = (phase_mask & 1) + ((phase_mask >> 1) & 1)
    if n and delta.numel() != n * nph * lpf_num_vectors(cx, cy):
        raise ValueError("lpf_s2_delta_swap: delta must hold n * nph * |D_c| elements")
    _check(_lib.lpf_s2_delta_swap(ctx, _dev(bits, torch.int64, "bits"), W, H, cx, cy,
                                  phase_mask, _dev(swaps, torch.int32, "swaps") if n else None, n,
                                  _dev(delta, torch.int32, "delta") if n else None,
                                  _stream(stream)))


def lpf_anneal_create(ctx: int, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                      phase_mask: int, counts: torch.Tensor, target: torch.Tensor, Nt: int,
                      seed: int, step0: int, pos, n1: int, e: torch.Tensor, stream=None,
                      s2: bool = False) -> int:
    h = _P()
    fn = _lib.lpf_anneal_create_s2 if s2 else _lib.lpf_anneal_create
    _check(fn(
        ctx, _dev(bits, torch.int64, "bits"), W, H, cx, cy, phase_mask,
        _dev(counts, torch.int32, "counts"), _dev(target, torch.int32, "target"), Nt, seed, step0,
        _dev(pos, torch.int32, "pos") if pos is not None else None, n1,
        _dev(e, torch.float64, "e"), ctypes.byref(h), _stream(stream)))
    return h.value


def lpf_rank(ctx: int, cand: torch.Tensor, score: torch.Tensor, order: torch.Tensor,
             stream=None) -> None:
    K = cand.numel() // 2
    if cand.numel() != 2 * K or order.numel() != K:
        raise ValueError("lpf_rank: cand must be (K, 2) and order K elements")
    _check(_lib.lpf_rank(ctx, _dev(cand, torch.int32, "cand"), _dev(score, torch.float32, "score"),
                         K, _dev(order, torch.int32, "order"), _stream(stream)))


def lpf_anneal_run(st: int, n_candidates: int, proposal: int, T_sched: torch.Tensor,
                   out: torch.Tensor, stream=None) -> None:
    n = T_sched.numel()
    if out.device.type != "cuda" or out.dtype != torch.int64 or out.numel() < 5 * n:
        raise ValueError("lpf_anneal_run: out must be a device int64 tensor of >= 5 * n elements")
    if n == 0:
        return
    _check(_lib.lpf_anneal_run(st, n_candidates, proposal, _dev(T_sched, torch.float64, "T_sched"),
                               n, _dev(out, torch.int64, "out"), _stream(stream)))


def anneal_step(st: int, n_candidates: int, proposal: int, T: float, out: torch.Tensor,
                stream=None) -> None:
    if out.device.type != "cuda" or out.dtype != torch.int64 or out.numel() < 5:
        raise ValueError("anneal_step: out must be a device int64 tensor of >= 5 elements")
    _check(_lib.anneal_step(st, n_candidates, proposal, float(T), out.data_ptr(), _stream(stream)))


def lpf_anneal_export(st: int, pos: torch.Tensor | None, stream=None):
    n1 = _i32()
    nxt = _u64()
    _check(_lib.lpf_anneal_export(st, _dev(pos, torch.int32, "pos") if pos is not None else None,
                                  ctypes.byref(n1), ctypes.byref(nxt), _stream(stream)))
    return n1.value, nxt.value


def lpf_anneal_destroy(st: int) -> None:
    _lib.lpf_anneal_destroy(st)


def lpf_batch(ctx: int, bits_pool: torch.Tensor, descs, phase_mask: int, out_layout: int,
              counts_pool: torch.Tensor, stream=None) -> None:
    """descs: a ctypes array of lpf_image_desc (host)."""
    _check(_lib.lpf_batch(ctx, _dev(bits_pool, torch.int64, "bits_pool"), ctypes.byref(descs),
                          len(descs), phase_mask, out_layout,
                          _dev(counts_pool, torch.int32, "counts_pool"), _stream(stream)))


def lpf_autotune_full(ctx: int, bits: torch.Tensor, W: int, H: int, cx: int, cy: int,
                      phase_mask: int, stream=None) -> float:
    ms = ctypes.c_double()
    _check(_lib.lpf_autotune_full(ctx, _dev(bits, torch.int64, "bits"), W, H, cx, cy, phase_mask,
                                  _stream(stream), ctypes.byref(ms)))
    return ms.value


def lpf_get_tuned_shape(ctx: int, W: int, H: int, cx: int, cy: int):
    R, wpg, lds = _i32(), _i32(), _i32()
    _check(_lib.lpf_get_tuned_shape(ctx, W, H, cx, cy, ctypes.byref(R), ctypes.byref(wpg),
                                    ctypes.byref(lds)))
    return R.value, wpg.value, lds.value


def lpf_set_full_shape(ctx: int, R: int = 0, S: int = 0, waves_per_group: int = 0,
                       lds_bytes: int = 0) -> None:
    _check(_lib.lpf_set_full_shape(ctx, R, S, waves_per_group, lds_bytes))


def lpf_cnn_create(ctx: int, W: int, H: int, max_batch: int, max_samples: int, params=None,
                   stream=None) -> int:
    h = _P()
    _check(_lib.lpf_cnn_create(ctx, W, H, max_batch, max_samples,
                               _dev(params, torch.float32, "params") if params is not None else None,
                               ctypes.byref(h), _stream(stream)))
    return h.value


def lpf_cnn_set_params(net: int, params: torch.Tensor, stream=None) -> None:
    _check(_lib.lpf_cnn_set_params(net, _dev(params, torch.float32, "params"), _stream(stream)))


def lpf_cnn_get_params(net: int, params: torch.Tensor, stream=None) -> None:
    _check(_lib.lpf_cnn_get_params(net, _dev(params, torch.float32, "params"), _stream(stream)))


def lpf_cnn_forward(net: int, bits: torch.Tensor, batch: int, scores: torch.Tensor,
                    stream=None) -> None:
    _check(_lib.lpf_cnn_forward(net, _dev(bits, torch.int64, "bits"), batch,
                                _dev(scores, torch.float32, "scores"), _stream(stream)))


def lpf_cnn_grad(net: int, bits: torch.Tensor, batch: int, samples: torch.Tensor, n: int,
                 grad: torch.Tensor, loss: torch.Tensor, stream=None) -> None:
    """samples: int32 tensor (n, 4) holding (img, a, b, float32 bits of y)."""
    _check(_lib.lpf_cnn_grad(net, _dev(bits, torch.int64, "bits"), batch,
                             _dev(samples, torch.int32, "samples"), n,
                             _dev(grad, torch.float32, "grad"), _dev(loss, torch.float32, "loss"),
                             _stream(stream)))


def lpf_cnn_adam(net: int, grad: torch.Tensor, t: int, lr: float, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8, stream=None) -> None:
    _check(_lib.lpf_cnn_adam(net, _dev(grad, torch.float32, "grad"), t, lr, beta1, beta2, eps,
                             _stream(stream)))


def lpf_cnn_destroy(net: int) -> None:
    _lib.lpf_cnn_destroy(net)


def lpf_anneal_set_proposal(st: int, net: int | None, scores: torch.Tensor | None, beta: float,
                            eps_uniform: float, refresh: int = 1, rank: int = 0) -> None:
    _check(_lib.lpf_anneal_set_proposal(
        st, net, _dev(scores, torch.float32, "scores") if scores is not None else None,
        beta, eps_uniform, refresh, rank))


def lpf_anneal_propose(st: int, K: int, proposal: int, cand: torch.Tensor, stream=None) -> None:
    if cand.numel() < 2 * K:
        raise ValueError("lpf_anneal_propose: cand must hold K pairs")
    _check(_lib.lpf_anneal_propose(st, K, proposal, _dev(cand, torch.int32, "cand"),
                                   _stream(stream)))


def lpf_anneal_delta_energy(st: int, swaps: torch.Tensor, n: int, de: torch.Tensor,
                            stream=None) -> None:
    if swaps.numel() != 2 * n or de.numel() < n:
        raise ValueError("lpf_anneal_delta_energy: sizes")
    _check(_lib.lpf_anneal_delta_energy(st, _dev(swaps, torch.int32, "swaps"), n,
                                        _dev(de, torch.float64, "de"), _stream(stream)))


def lpf_anneal_set_method(st: int, method: int) -> None:
    _check(_lib.lpf_anneal_set_method(st, method))


def lpf_anneal_get_method(st: int) -> int:
    m = _lib.lpf_anneal_get_method(st)
    if m < 0:
        raise LpfError(LPF_E_INVAL, _lib.lpf_last_error().decode())
    return m
