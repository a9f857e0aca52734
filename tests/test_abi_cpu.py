"""C-ABI checks that need no GPU: the library loads, exports what include/*.h declares, and its
host-side logic (vector enumeration, argument checks) behaves as documented."""
from __future__ import annotations

import ctypes
import glob
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(lpf_\w+|anneal_\w+)\s*\(", src,
                             flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_declared_symbols():
    from paper_1601_04359_amd import _abi
    names = _declared_symbols()
    assert {"lpf_full", "lpf_pack", "lpf_ctx_create", "lpf_vectors"} <= names
    lib = _abi.lib()
    for n in sorted(names):
        assert hasattr(lib, n), f"{n} declared in include/ but not exported"


@pytest.mark.parametrize("cx,cy", [(0, 0), (16, 16), (5, 9), (128, 128), (40, 3)])
def test_vectors_match_oracle_enumeration(cx, cy):
    from paper_1601_04359_amd import _abi
    assert _abi.lpf_num_vectors(cx, cy) == oracle.num_vectors(cx, cy)
    assert np.array_equal(_abi.lpf_vectors(cx, cy), oracle.vectors(cx, cy))


def test_num_vectors_negative():
    from paper_1601_04359_amd import _abi
    assert _abi.lpf_num_vectors(-1, 3) == -1


def test_argument_errors_without_device():
    from paper_1601_04359_amd import _abi
    lib = _abi.lib()
    # NULL context: rejected before any HIP call, message names the argument
    st = lib.lpf_full(None, None, 8, 8, 1, 1, 3, 0, None, None)
    assert st == _abi.LPF_E_INVAL
    assert b"ctx" in lib.lpf_last_error()
    assert lib.lpf_vectors(-1, 0, None) == _abi.LPF_E_INVAL
    assert b"cutoff" in lib.lpf_last_error()
    assert lib.lpf_set_full_shape(None, 8, 2, 8, 0) == _abi.LPF_E_INVAL
    h = ctypes.c_void_p()
    assert lib.lpf_ctx_create(-1, ctypes.byref(h)) == _abi.LPF_E_INVAL
    assert lib.lpf_ctx_create(0, None) == _abi.LPF_E_INVAL


def test_python_binding_checks():
    import torch
    from paper_1601_04359_amd import _abi
    with pytest.raises(ValueError):
        _abi._dev(torch.zeros(4, dtype=torch.int64), torch.int64, "bits")  # host tensor
    with pytest.raises(ValueError):
        _abi.lpf_full(0, torch.zeros(3, dtype=torch.int64), 8, 8, 1, 1, 3, 0,
                      torch.zeros(1, dtype=torch.int32))


def test_new_entry_points_reject_null_before_any_device_call():
    from paper_1601_04359_amd import _abi
    lib = _abi.lib()
    assert lib.lpf_full_enhanced(None, None, 8, 8, 1, 1, 3, 0, None, None) == _abi.LPF_E_INVAL
    assert b"ctx" in lib.lpf_last_error()
    assert lib.lpf_anneal_set_method(None, 2) == _abi.LPF_E_INVAL
    assert b"state" in lib.lpf_last_error()
    assert lib.lpf_anneal_get_method(None) == -1
    assert lib.lpf_anneal_set_proposal(None, None, None, 1.0, 0.1, 1, 0) == _abi.LPF_E_INVAL


def test_s2_entry_points_reject_bad_arguments_before_any_device_call():
    import ctypes
    from paper_1601_04359_amd import _abi
    lib = _abi.lib()
    assert lib.lpf_s2(None, None, 8, 8, 1, 1, 3, 0, None, None) == _abi.LPF_E_INVAL
    assert b"ctx" in lib.lpf_last_error()
    assert lib.lpf_s2_delta_swap(None, None, 8, 8, 1, 1, 3, None, 1, None, None) == _abi.LPF_E_INVAL
    h = ctypes.c_void_p()
    assert lib.lpf_anneal_create_s2(None, None, 8, 8, 1, 1, 3, None, None, 1, 0, 0, None, 0, None,
                                    ctypes.byref(h), None) == _abi.LPF_E_INVAL
    assert lib.lpf_anneal_create_s2(None, None, 8, 8, 1, 1, 3, None, None, 1, 0, 0, None, 0, None,
                                    None, None) == _abi.LPF_E_INVAL
    assert b"out" in lib.lpf_last_error()


def test_sampled_entry_points_reject_bad_arguments_before_any_device_call():
    import ctypes
    from paper_1601_04359_amd import _abi
    lib = _abi.lib()
    assert lib.lpf_full_sampled(None, None, 8, 8, 1, 1, 3, 0, None, None, None) == _abi.LPF_E_INVAL
    assert b"sample" in lib.lpf_last_error()
    h = ctypes.c_void_p(1)
    assert lib.lpf_anneal_create_sampled(None, None, 8, 8, 1, 1, 3, None, None, None, 1, 0, 0,
                                         None, 0, None, ctypes.byref(h), None) == _abi.LPF_E_INVAL
    assert h.value is None


def test_bench_counts_match_oracle_paths():
    # the benchmark's algorithmic work: M_c from the oracle's digitisation, ops = N/32 (3 M_c +
    # 2 |D_c|) for both phases (7.088e10 at 512^2, cutoff 128)
    import bench
    for cx, cy in ((16, 16), (128, 128), (5, 9)):
        n = np.array([len(oracle.bresenham(int(dx), int(dy))) for dx, dy in oracle.vectors(cx, cy)])
        assert bench.path_pixels(cx, cy) == int(n.sum())
    assert bench.ops_alg(512, 512, 128, 128, 2) == 70879584256.0


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_3d_entry_points_on_the_host():
    from paper_1601_04359_amd import _abi
    lib = _abi.lib()
    assert _abi.lpf_num_vectors3(-1, 0, 0) == -1
    for c in ((0, 0, 0), (3, 2, 1), (5, 0, 4), (4, 4, 4)):
        assert _abi.lpf_num_vectors3(*c) == oracle.num_vectors3(*c)
        assert np.array_equal(_abi.lpf_vectors3(*c), oracle.vectors3(*c))
    assert lib.lpf_full3d(None, None, 8, 8, 8, 1, 1, 1, 3, None, None) == _abi.LPF_E_INVAL
    assert b"ctx" in lib.lpf_last_error()
