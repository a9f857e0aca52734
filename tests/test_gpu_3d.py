"""3-D volumes on the GPU (lpf_full3d) against the CPU oracle, bit for bit; with cz = 0 against
the sum of the 2-D functions of the xy-cuts (the ensemble of cuts of Sec. 6.3)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1601_04359_amd import Context
    c = Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = [(1, 1, 1, 0, 0, 0), (5, 4, 3, 4, 3, 2), (12, 10, 8, 11, 9, 7), (37, 5, 3, 20, 4, 2),
         (70, 6, 5, 40, 5, 4), (100, 4, 4, 99, 3, 3), (33, 33, 7, 6, 6, 6), (1, 9, 8, 0, 8, 7),
         (20, 3, 100, 4, 2, 10),  # many bands of start rows over short planes
         (200, 6, 5, 10, 2, 3), (300, 4, 4, 40, 2, 2)]  # 8 and 16 words per lane


@pytest.mark.parametrize("W,H,D,cx,cy,cz", CASES)
def test_full3d_matches_oracle(ctx, W, H, D, cx, cy, cz):
    import torch
    print(f"[gpu] lpf3 {W}x{H}x{D} c=({cx},{cy},{cz})", flush=True)
    vol = wl.gaussian_field_3d(W, H, D, 1.2, 0.5, W * H + D) if W * H * D > 8 else \
        np.array([[[1]]], np.uint8)
    bits = ctx.pack3d(_dev(vol))
    want = oracle.lpf3(vol, cx, cy, cz, 3) if W * H * D > 1 else None
    for mask in (1, 2, 3):
        got = ctx.full3d(bits, W, H, D, cx, cy, cz, mask)
        torch.cuda.synchronize()
        if want is None:  # a single phase-1 voxel
            assert got.cpu().numpy().tolist() == {1: [[0]], 2: [[1]], 3: [[0], [1]]}[mask]
            continue
        sel = {1: [0], 2: [1], 3: [0, 1]}[mask]
        assert np.array_equal(got.cpu().numpy().astype(np.uint32), want[sel]), mask


def test_full3d_same_cutoff_other_shapes(ctx):
    # one cutoff, volumes whose plane geometry differs (halo rows, row words) in turn: the cached
    # voxel table follows the shape of each call
    import torch
    for W, H, D in ((20, 6, 5), (70, 9, 5), (20, 6, 5), (40, 6, 4)):
        print(f"[gpu] lpf3 {W}x{H}x{D} c=(3,2,2) after other shapes", flush=True)
        vol = wl.gaussian_field_3d(W, H, D, 1.2, 0.5, W + H + D)
        got = ctx.full3d(ctx.pack3d(_dev(vol)), W, H, D, 3, 2, 2, 3)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy().astype(np.uint32), oracle.lpf3(vol, 3, 2, 2, 3))


def test_vectors3_match_oracle():
    from paper_1601_04359_amd import _abi
    for c in ((0, 0, 0), (3, 2, 1), (5, 0, 4), (7, 7, 7)):
        assert np.array_equal(_abi.lpf_vectors3(*c), oracle.vectors3(*c))


def test_dz0_is_the_ensemble_of_cuts(ctx):
    # 100 x 100 x 100 bone-like volume, full in-plane domain: the sum of 100 lpf_full calls
    import torch
    print("[gpu] lpf3 100^3 c=(99,99,0) vs 100 cuts", flush=True)
    vol = wl.gaussian_field_3d(100, 100, 100, 2.0, 0.5, 7)
    dv = _dev(vol)
    got = ctx.full3d(ctx.pack3d(dv), 100, 100, 100, 99, 99, 0, 3).long()
    want = torch.zeros_like(got)
    for z in range(100):
        want += ctx.full(ctx.pack(dv[z].contiguous()), 100, 100, 99, 99, 3).long()
    torch.cuda.synchronize()
    assert torch.equal(got, want)


def test_full3d_bone_volume_sampled_vectors(ctx):
    # the bench volume: 100^3, cutoff 16 on every axis; a sample of vectors from the oracle
    import torch
    print("[gpu] lpf3 100^3 c=16 sampled", flush=True)
    vol = wl.gaussian_field_3d(100, 100, 100, 2.0, 0.5, 7)
    got = ctx.full3d(ctx.pack3d(_dev(vol)), 100, 100, 100, 16, 16, 16, 3)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.uint32)
    v = oracle.vectors3(16, 16, 16)
    pick = np.unique(np.concatenate([[0, 1, len(v) - 1],
                                     np.random.default_rng(3).integers(0, len(v), 60)]))
    assert np.array_equal(got[:, pick], oracle.lpf3_vectors(vol, v[pick], 3))
    n1 = int(vol.sum())
    assert got[1, 0] == n1 and got[0, 0] == vol.size - n1


def test_full3d_global_rows_path(ctx):
    # planes too large for cz + 1 of them in LDS (256 x 256 rows, cz = 18): rows from global
    # memory; sampled vectors against the oracle
    import torch
    print("[gpu] lpf3 256x256x20 c=(3,3,18) global rows", flush=True)
    vol = wl.gaussian_field_3d(256, 256, 20, 1.5, 0.45, 9)
    got = ctx.full3d(ctx.pack3d(_dev(vol)), 256, 256, 20, 3, 3, 18, 3)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.uint32)
    v = oracle.vectors3(3, 3, 18)
    pick = np.unique(np.concatenate([[0, len(v) - 1],
                                     np.random.default_rng(4).integers(0, len(v), 40)]))
    assert np.array_equal(got[:, pick], oracle.lpf3_vectors(vol, v[pick], 3))
