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


def _chain_stats_reference(cx, cy):
    """Chains from the definition: a vector is walked when its digitised path (oracle
    digitisation) is not, up to a translation, a proper prefix of another vector's path; the
    walk is the sum of the walked paths' pixel counts."""
    def norm(pix):
        x0 = min(int(x) for x, y in pix if y == 0)
        return frozenset((int(x) - x0, int(y)) for x, y in pix)
    vecs = oracle.vectors(cx, cy)
    paths = [oracle.bresenham(int(dx), int(dy)) for dx, dy in vecs]
    prefixes = set()
    for p in paths:
        for l in range(len(p) - 1):
            prefixes.add(norm(p[:l + 1]))
    walked = [p for p in paths if norm(p) not in prefixes]
    return {"vectors": len(vecs), "chains": len(walked), "walk": sum(len(p) for p in walked),
            "path_pixels": sum(len(p) for p in paths)}


@pytest.mark.parametrize("cx,cy", [(0, 0), (1, 1), (0, 7), (7, 0), (5, 9), (16, 16), (40, 3),
                                   (32, 32)])
def test_chain_stats_match_definition(cx, cy):
    from paper_1601_04359_amd import _abi
    assert _abi.lpf_chain_stats(cx, cy) == _chain_stats_reference(cx, cy)


def test_chain_stats_headline_cutoff():
    # cutoff 128: the walk of the chains is 1 272 832 pixels per start word against
    # M_c = 2 862 081 for one walk per vector (M_c pinned by the closed form of the memory count)
    from paper_1601_04359_amd import _abi
    s = _abi.lpf_chain_stats(128, 128)
    assert s["vectors"] == 33025 and s["path_pixels"] == 2862081
    assert s["chains"] == 11200 and s["walk"] == 1272832


@pytest.mark.parametrize("cx,cy,nb", [(0, 0, 1), (1, 1, 4), (5, 9, 8), (16, 16, 64),
                                      (40, 300, 512), (128, 128, 512), (255, 255, 1),
                                      (512, 512, 256)])
def test_full_plan_checks(cx, cy, nb):
    # the launch plan of lpf_full (host logic): every vector exactly once, each one the walked
    # path's pixel l with that path's first l + 1 pixels as its own path, bins within their slots
    from paper_1601_04359_amd import _abi
    r = _abi.lpf_plan_check(cx, cy, nb)
    assert r["bins"] >= 1 and r["max_members"] <= 256
    assert r["walk"] >= _abi.lpf_chain_stats(cx, cy)["walk"]
