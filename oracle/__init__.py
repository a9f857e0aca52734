"""CPU oracle for the entire lineal path function -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may import
this package.  The product package never imports it, and it imports nothing from the product.

The arithmetic lives in ``lpf_oracle.c`` (plain definitions from Havelka, Kucerova & Sykora,
arXiv:1601.04359: Sec. 2.2 segments and symmetry, Alg. "L2_eval", Sec. 4 interchange operator,
Alg. "annealing" with eq. (LSE), and the two-point probability of Sec. 2.1, eq. (S2dis), with
its interchange update); ``brute.py`` is a second, independent pure-Python/numpy
implementation for tiny images that pins it.  This module only marshals numpy arrays.

Parity unpinned: the pixel choice on Bresenham tie vectors (reading R1 in ``lpf_oracle.c``) is
a convention that no passage of the paper fixes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblpf_oracle.so")
_lib = None


def build() -> None:
    subprocess.run(["sh", os.path.join(_HERE, "build.sh")], check=True)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u32, u64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint, ctypes.c_uint64
    lib.oracle_bresenham.argtypes = [i32, i32, P, P]
    lib.oracle_bresenham.restype = i32
    lib.oracle_num_vectors.argtypes = [i32, i32]
    lib.oracle_num_vectors.restype = i64
    lib.oracle_vectors.argtypes = [i32, i32, P]
    lib.oracle_vectors.restype = i32
    lib.oracle_lpf_vectors.argtypes = [P, i32, i32, P, i64, u32, P, i32]
    lib.oracle_lpf_vectors.restype = i32
    lib.oracle_lpf.argtypes = [P, i32, i32, i32, i32, u32, i32, P, i32]
    lib.oracle_lpf.restype = i32
    lib.oracle_delta_swap_full.argtypes = [P, i32, i32, i32, i32, u32, P, i32, P, i32]
    lib.oracle_delta_swap_full.restype = i32
    lib.oracle_delta_swap.argtypes = [P, i32, i32, i32, i32, u32, P, i32, P, i32]
    lib.oracle_delta_swap.restype = i32
    lib.oracle_philox4x64.argtypes = [P, P, P]
    lib.oracle_philox4x64.restype = None
    lib.oracle_lse.argtypes = [P, P, i64, i64, i64]
    lib.oracle_lse.restype = ctypes.c_double
    lib.oracle_anneal_run.argtypes = [P, i32, i32, i32, i32, u32, P, P, i64, u64, u64, i32, i32,
                                      P, i32, P, P, P, P, i32]
    lib.oracle_anneal_run.restype = i32
    lib.oracle_anneal_run_desc.argtypes = [P, i32, i32, i32, i32, u32, i32, P, P, i64, u64, u64,
                                           i32, i32, P, i32, P, P, P, P, i32]
    lib.oracle_anneal_run_desc.restype = i32
    lib.oracle_anneal_run_ranked.argtypes = [P, i32, i32, i32, i32, u32, P, P, i64, u64, u64,
                                             i32, i32, P, i32, P, P, P, P, P, i32]
    lib.oracle_anneal_run_ranked.restype = i32
    lib.oracle_lpf_sampled.argtypes = [P, i32, i32, i32, i32, u32, P, P, i32]
    lib.oracle_lpf_sampled.restype = i32
    lib.oracle_delta_swap_sampled.argtypes = [P, i32, i32, i32, i32, u32, P, P, i32, P, i32]
    lib.oracle_delta_swap_sampled.restype = i32
    lib.oracle_anneal_run_sampled.argtypes = [P, i32, i32, i32, i32, u32, P, P, P, i64, u64, u64,
                                              i32, i32, P, i32, P, P, P, P, i32]
    lib.oracle_anneal_run_sampled.restype = i32
    lib.oracle_bresenham3.argtypes = [i32, i32, i32, P, P, P]
    lib.oracle_bresenham3.restype = i32
    lib.oracle_num_vectors3.argtypes = [i32, i32, i32]
    lib.oracle_num_vectors3.restype = i64
    lib.oracle_vectors3.argtypes = [i32, i32, i32, P]
    lib.oracle_vectors3.restype = i32
    lib.oracle_lpf3_vectors.argtypes = [P, i32, i32, i32, P, i64, u32, P, i32]
    lib.oracle_lpf3_vectors.restype = i32
    lib.oracle_lpf3.argtypes = [P, i32, i32, i32, i32, i32, i32, u32, P, i32]
    lib.oracle_lpf3.restype = i32
    lib.oracle_s2_vectors.argtypes = [P, i32, i32, P, i64, u32, P, i32]
    lib.oracle_s2_vectors.restype = i32
    lib.oracle_s2.argtypes = [P, i32, i32, i32, i32, u32, i32, P, i32]
    lib.oracle_s2.restype = i32
    lib.oracle_s2_delta_swap.argtypes = [P, i32, i32, i32, i32, u32, P, i32, P, i32]
    lib.oracle_s2_delta_swap.restype = i32
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _img(img) -> np.ndarray:
    a = np.ascontiguousarray(img, dtype=np.uint8)
    if a.ndim != 2:
        raise ValueError("image must be 2-D (H, W)")
    return a


def nphases(phase_mask: int) -> int:
    return (phase_mask & 1) + ((phase_mask >> 1) & 1)


def bresenham(dx: int, dy: int) -> np.ndarray:
    """Pixels (px, py) of the digitised segment from (0,0) to (dx,dy): shape (n+1, 2)."""
    n = max(abs(dx), abs(dy))
    px = np.zeros(n + 1, np.int32)
    py = np.zeros(n + 1, np.int32)
    m = _load().oracle_bresenham(int(dx), int(dy), _ptr(px), _ptr(py))
    assert m == n + 1
    return np.stack([px, py], axis=1)


def num_vectors(cx: int, cy: int) -> int:
    return int(_load().oracle_num_vectors(cx, cy))


def vectors(cx: int, cy: int) -> np.ndarray:
    """Canonical half domain, int16 (|D_c|, 2) of (dx, dy)."""
    out = np.zeros((num_vectors(cx, cy), 2), np.int16)
    rc = _load().oracle_vectors(cx, cy, _ptr(out))
    if rc:
        raise ValueError("bad cutoff")
    return out


def lpf(img, cx: int, cy: int, phase_mask: int = 3, layout: int = 0, nthreads: int = 0) -> np.ndarray:
    """Counts uint32 [nph][|D_c|] (layout 0) or [nph][2cy+1][2cx+1] (layout 1)."""
    a = _img(img)
    H, W = a.shape
    nph = nphases(phase_mask)
    if layout == 0:
        out = np.zeros((nph, num_vectors(cx, cy)), np.uint32)
    else:
        out = np.zeros((nph, 2 * cy + 1, 2 * cx + 1), np.uint32)
    rc = _load().oracle_lpf(_ptr(a), W, H, cx, cy, phase_mask, layout, _ptr(out), nthreads)
    if rc:
        raise ValueError(f"oracle_lpf failed ({rc})")
    return out


def lpf_vectors(img, dxdy, phase_mask: int = 3, nthreads: int = 0) -> np.ndarray:
    a = _img(img)
    H, W = a.shape
    v = np.ascontiguousarray(dxdy, dtype=np.int16).reshape(-1, 2)
    out = np.zeros((nphases(phase_mask), len(v)), np.uint32)
    rc = _load().oracle_lpf_vectors(_ptr(a), W, H, _ptr(v), len(v), phase_mask, _ptr(out), nthreads)
    if rc:
        raise ValueError(f"oracle_lpf_vectors failed ({rc})")
    return out


def delta_swap(img, cx: int, cy: int, swaps, phase_mask: int = 3, full: bool = False,
               nthreads: int = 0) -> np.ndarray:
    """delta int32 [n][nph][|D_c|] = L(I') - L(I) for each interchange (a, b)."""
    a = _img(img)
    H, W = a.shape
    sw = np.ascontiguousarray(swaps, dtype=np.int32).reshape(-1, 2)
    out = np.zeros((len(sw), nphases(phase_mask), num_vectors(cx, cy)), np.int32)
    fn = _load().oracle_delta_swap_full if full else _load().oracle_delta_swap
    rc = fn(_ptr(a), W, H, cx, cy, phase_mask, _ptr(sw), len(sw), _ptr(out), nthreads)
    if rc:
        raise ValueError(f"oracle delta failed ({rc})")
    return out


def _sample(sample, shape) -> np.ndarray:
    m = np.ascontiguousarray(sample, dtype=np.uint8)
    if m.shape != shape:
        raise ValueError("sample mask must have the image's shape")
    return m


def lpf_sampled(img, cx: int, cy: int, sample, phase_mask: int = 3,
                nthreads: int = 0) -> np.ndarray:
    """Monte-Carlo approximation in counts: uint32 [nph][|D_c|], segments tested only at the start
    positions where the (H, W) mask `sample` is nonzero."""
    a = _img(img)
    H, W = a.shape
    m = _sample(sample, a.shape)
    out = np.zeros((nphases(phase_mask), num_vectors(cx, cy)), np.uint32)
    rc = _load().oracle_lpf_sampled(_ptr(a), W, H, cx, cy, phase_mask, _ptr(m), _ptr(out), nthreads)
    if rc:
        raise ValueError(f"oracle_lpf_sampled failed ({rc})")
    return out


def delta_swap_sampled(img, cx: int, cy: int, sample, swaps, phase_mask: int = 3,
                       nthreads: int = 0) -> np.ndarray:
    a = _img(img)
    H, W = a.shape
    m = _sample(sample, a.shape)
    sw = np.ascontiguousarray(swaps, dtype=np.int32).reshape(-1, 2)
    out = np.zeros((len(sw), nphases(phase_mask), num_vectors(cx, cy)), np.int32)
    rc = _load().oracle_delta_swap_sampled(_ptr(a), W, H, cx, cy, phase_mask, _ptr(m), _ptr(sw),
                                           len(sw), _ptr(out), nthreads)
    if rc:
        raise ValueError(f"oracle_delta_swap_sampled failed ({rc})")
    return out


def s2(img, cx: int, cy: int, phase_mask: int = 3, layout: int = 0, nthreads: int = 0) -> np.ndarray:
    """Two-point counts W*H*S2 (eq. (S2dis)), uint32 [nph][|D_c|] (layout 0) or
    [nph][2cy+1][2cx+1] (layout 1)."""
    a = _img(img)
    H, W = a.shape
    nph = nphases(phase_mask)
    if layout == 0:
        out = np.zeros((nph, num_vectors(cx, cy)), np.uint32)
    else:
        out = np.zeros((nph, 2 * cy + 1, 2 * cx + 1), np.uint32)
    rc = _load().oracle_s2(_ptr(a), W, H, cx, cy, phase_mask, layout, _ptr(out), nthreads)
    if rc:
        raise ValueError(f"oracle_s2 failed ({rc})")
    return out


def s2_vectors(img, dxdy, phase_mask: int = 3, nthreads: int = 0) -> np.ndarray:
    a = _img(img)
    H, W = a.shape
    v = np.ascontiguousarray(dxdy, dtype=np.int16).reshape(-1, 2)
    out = np.zeros((nphases(phase_mask), len(v)), np.uint32)
    rc = _load().oracle_s2_vectors(_ptr(a), W, H, _ptr(v), len(v), phase_mask, _ptr(out), nthreads)
    if rc:
        raise ValueError(f"oracle_s2_vectors failed ({rc})")
    return out


def s2_delta_swap(img, cx: int, cy: int, swaps, phase_mask: int = 3,
                  nthreads: int = 0) -> np.ndarray:
    """delta int32 [n][nph][|D_c|] = C(I') - C(I) of the two-point counts per interchange."""
    a = _img(img)
    H, W = a.shape
    sw = np.ascontiguousarray(swaps, dtype=np.int32).reshape(-1, 2)
    out = np.zeros((len(sw), nphases(phase_mask), num_vectors(cx, cy)), np.int32)
    rc = _load().oracle_s2_delta_swap(_ptr(a), W, H, cx, cy, phase_mask, _ptr(sw), len(sw),
                                      _ptr(out), nthreads)
    if rc:
        raise ValueError(f"oracle_s2_delta_swap failed ({rc})")
    return out


DESC_LPF, DESC_S2 = 0, 1


def bresenham3(dx: int, dy: int, dz: int) -> np.ndarray:
    """Voxels (px, py, pz) of the digitised 3-D segment: shape (n+1, 3)."""
    n = max(abs(dx), abs(dy), abs(dz))
    p = [np.zeros(n + 1, np.int32) for _ in range(3)]
    m = _load().oracle_bresenham3(int(dx), int(dy), int(dz), *(_ptr(a) for a in p))
    assert m == n + 1
    return np.stack(p, axis=1)


def num_vectors3(cx: int, cy: int, cz: int) -> int:
    return int(_load().oracle_num_vectors3(cx, cy, cz))


def vectors3(cx: int, cy: int, cz: int) -> np.ndarray:
    """Canonical 3-D half domain, int16 (n, 3) of (dx, dy, dz)."""
    out = np.zeros((num_vectors3(cx, cy, cz), 3), np.int16)
    if _load().oracle_vectors3(cx, cy, cz, _ptr(out)):
        raise ValueError("bad cutoff")
    return out


def lpf3(vol, cx: int, cy: int, cz: int, phase_mask: int = 3, nthreads: int = 0) -> np.ndarray:
    """Counts uint32 [nph][|D_c|] of a periodic volume vol[z][y][x] (uint8)."""
    a = np.ascontiguousarray(vol, dtype=np.uint8)
    if a.ndim != 3:
        raise ValueError("volume must be 3-D (D, H, W)")
    D, H, W = a.shape
    out = np.zeros((nphases(phase_mask), num_vectors3(cx, cy, cz)), np.uint32)
    rc = _load().oracle_lpf3(_ptr(a), W, H, D, cx, cy, cz, phase_mask, _ptr(out), nthreads)
    if rc:
        raise ValueError(f"oracle_lpf3 failed ({rc})")
    return out


def philox4x64(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    _load().oracle_philox4x64(_ptr(c), _ptr(k), _ptr(out))
    return out


def lse(counts, target, N: int, Nt: int) -> float:
    c = np.ascontiguousarray(counts, dtype=np.uint32).ravel()
    t = np.ascontiguousarray(target, dtype=np.uint32).ravel()
    return float(_load().oracle_lse(_ptr(c), _ptr(t), c.size, N, Nt))


STEP_DTYPE = np.dtype([("k", np.int32), ("a", np.int32), ("b", np.int32), ("pad", np.int32),
                       ("de", np.float64), ("e", np.float64)])


class AnnealState:
    """Host copy of an annealing chain: image, counts, target counts, pixel lists, error."""

    def __init__(self, img, cx, cy, phase_mask, target, Nt, seed, nthreads=0,
                 descriptor: int = DESC_LPF, sample=None):
        self.img = _img(img).copy()
        self.H, self.W = self.img.shape
        self.cx, self.cy, self.phase_mask = cx, cy, phase_mask
        self.target = np.ascontiguousarray(target, dtype=np.uint32).copy()
        self.Nt = int(Nt)
        self.seed = int(seed)
        self.step = 0
        self.nthreads = nthreads
        flat = self.img.ravel()
        self.pos1 = np.flatnonzero(flat == 1).astype(np.int32)
        self.pos0 = np.flatnonzero(flat == 0).astype(np.int32)
        self.descriptor = descriptor
        self.sample = None if sample is None else _sample(sample, self.img.shape).copy()
        if self.sample is not None:
            if descriptor != DESC_LPF:
                raise ValueError("a position set applies to the lineal path function only")
            self.counts = lpf_sampled(self.img, cx, cy, self.sample, phase_mask, nthreads)
        elif descriptor == DESC_LPF:
            self.counts = lpf(self.img, cx, cy, phase_mask, 0, nthreads)
        elif descriptor == DESC_S2:
            self.counts = s2(self.img, cx, cy, phase_mask, 0, nthreads)
        else:
            raise ValueError("descriptor")
        self.N = self.W * self.H if self.sample is None else int(np.count_nonzero(self.sample))
        self.e = lse(self.counts, self.target, self.N, self.Nt)

    def run(self, nsteps: int, K: int, Ts, proposal: int = 0, score=None) -> np.ndarray:
        """nsteps steps of K draws each; with `score` (float32 per pixel) every step evaluates
        its draws in the ranked order of that field (reading R18) instead of draw order."""
        Ts = np.ascontiguousarray(Ts, dtype=np.float64)
        assert Ts.size == nsteps
        res = np.zeros(nsteps, STEP_DTYPE)
        e = np.array([self.e], np.float64)
        if score is not None:
            if self.sample is not None or self.descriptor != DESC_LPF:
                raise ValueError("the ranked order is implemented for the plain lineal path chain")
            sc = np.ascontiguousarray(score, dtype=np.float32).reshape(-1)
            assert sc.size == self.W * self.H
            rc = _load().oracle_anneal_run_ranked(
                _ptr(self.img), self.W, self.H, self.cx, self.cy, self.phase_mask,
                _ptr(self.counts), _ptr(self.target), self.Nt, self.seed, self.step, nsteps, K,
                _ptr(Ts), proposal, _ptr(sc), _ptr(self.pos1), _ptr(self.pos0), _ptr(e),
                _ptr(res), self.nthreads)
        elif self.sample is not None:
            rc = _load().oracle_anneal_run_sampled(
                _ptr(self.img), self.W, self.H, self.cx, self.cy, self.phase_mask,
                _ptr(self.sample), _ptr(self.counts), _ptr(self.target), self.Nt, self.seed,
                self.step, nsteps, K, _ptr(Ts), proposal, _ptr(self.pos1), _ptr(self.pos0), _ptr(e),
                _ptr(res), self.nthreads)
        else:
            rc = _load().oracle_anneal_run_desc(
                _ptr(self.img), self.W, self.H, self.cx, self.cy, self.phase_mask,
                self.descriptor, _ptr(self.counts), _ptr(self.target), self.Nt, self.seed,
                self.step, nsteps, K, _ptr(Ts), proposal, _ptr(self.pos1), _ptr(self.pos0), _ptr(e),
                _ptr(res), self.nthreads)
        if rc:
            raise ValueError(f"oracle_anneal_run failed ({rc})")
        self.e = float(e[0])
        self.step += nsteps
        return res


def lpf3_vectors(vol, v3, phase_mask: int = 3, nthreads: int = 0) -> np.ndarray:
    """Counts uint32 [nph][n] of a periodic volume for the vectors v3 (n, 3) of (dx, dy, dz)."""
    a = np.ascontiguousarray(vol, dtype=np.uint8)
    D, H, W = a.shape
    v = np.ascontiguousarray(v3, dtype=np.int16).reshape(-1, 3)
    out = np.zeros((nphases(phase_mask), len(v)), np.uint32)
    rc = _load().oracle_lpf3_vectors(_ptr(a), W, H, D, _ptr(v), len(v), phase_mask, _ptr(out),
                                     nthreads)
    if rc:
        raise ValueError(f"oracle_lpf3_vectors failed ({rc})")
    return out
