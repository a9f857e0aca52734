"""Pins of the oracle's 3-D extension (Sec. 2: the extension to three dimensions; Sec. 6.3: a 3-D
specimen described by an ensemble of 2-D cuts), on the CPU."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads as wl


@pytest.mark.parametrize("cx,cy,cz", [(0, 0, 0), (2, 1, 1), (3, 3, 2), (5, 0, 4), (0, 4, 3)])
def test_half_domain3_is_one_of_each_pair(cx, cy, cz):
    v = [tuple(map(int, r)) for r in oracle.vectors3(cx, cy, cz)]
    assert len(v) == len(set(v)) == oracle.num_vectors3(cx, cy, cz)
    assert set(v) == brute.half_domain3(cx, cy, cz)
    box = (2 * cx + 1) * (2 * cy + 1) * (2 * cz + 1)
    assert len(v) == (box + 1) // 2
    # the dz = 0 part is the 2-D half domain in its own order
    n2 = oracle.num_vectors(cx, cy)
    assert np.array_equal(oracle.vectors3(cx, cy, cz)[:n2, :2], oracle.vectors(cx, cy))


def test_bresenham3_matches_exact_rounding_and_2d():
    for dx in range(-7, 8):
        for dy in range(-7, 8):
            for dz in range(-6, 7):
                got = [tuple(map(int, r)) for r in oracle.bresenham3(dx, dy, dz)]
                assert got == brute.path3(dx, dy, dz), (dx, dy, dz)
    for dx in range(-20, 21):
        for dy in range(-20, 21):
            p3 = oracle.bresenham3(dx, dy, 0)
            assert not p3[:, 2].any()
            assert np.array_equal(p3[:, :2], oracle.bresenham(dx, dy))


def test_bresenham3_commutes_with_axis_permutations():
    # the digitisation treats the axes alike: permuting the vector permutes its voxels
    # (ties between the major extents pick the same voxels either way)
    for dx in range(-6, 7):
        for dy in range(-6, 7):
            for dz in range(-6, 7):
                p = oracle.bresenham3(dx, dy, dz)
                for perm in ((1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)):
                    d = (dx, dy, dz)
                    q = oracle.bresenham3(*(d[i] for i in perm))
                    assert np.array_equal(q, p[:, perm]), (d, perm)


VOLS = {
    "random_7x5x4": lambda: wl.random_binary(7, 5 * 4, 0.5, 1).reshape(4, 5, 7),
    "field_12x10x8": lambda: wl.gaussian_field_3d(12, 10, 8, 1.5, 0.5, 2),
    "field_9x9x9": lambda: wl.gaussian_field_3d(9, 9, 9, 1.0, 0.4, 3),
}


@pytest.mark.parametrize("name", sorted(VOLS))
def test_lpf3_against_brute_force(name):
    vol = VOLS[name]()
    D, H, W = vol.shape
    cx, cy, cz = min(W - 1, 4), min(H - 1, 3), min(D - 1, 3)
    got = oracle.lpf3(vol, cx, cy, cz)
    for i, (dx, dy, dz) in enumerate(oracle.vectors3(cx, cy, cz)):
        for ph in (0, 1):
            assert got[ph, i] == brute.lpf3_vector(vol, int(dx), int(dy), int(dz), ph)


@pytest.mark.parametrize("name", sorted(VOLS))
def test_dz0_is_the_ensemble_of_2d_cuts(name):
    # paths with dz = 0 stay in one xy-cut: L3(dx, dy, 0) = sum over the cuts of their 2-D L
    vol = VOLS[name]()
    D, H, W = vol.shape
    cx, cy = W - 1, H - 1
    got = oracle.lpf3(vol, cx, cy, 0)
    want = sum(oracle.lpf(vol[z], cx, cy).astype(np.int64) for z in range(D))
    assert np.array_equal(got.astype(np.int64), want)


def test_axis_swap_and_closed_forms():
    vol = VOLS["field_12x10x8"]()
    D, H, W = vol.shape
    c = 4
    # swapping x and y of the volume swaps dx and dy (vectors with dz > 0 stay canonical)
    a = oracle.lpf3(vol, c, c, 3)
    b = oracle.lpf3(vol.transpose(0, 2, 1).copy(), c, c, 3)
    va = [tuple(map(int, r)) for r in oracle.vectors3(c, c, 3)]
    idx = {v: i for i, v in enumerate(va)}
    for i, (dx, dy, dz) in enumerate(va):
        if dz > 0:
            assert np.array_equal(a[:, i], b[:, idx[(dy, dx, dz)]])
    # v = 0 counts the voxels of each phase
    n1 = int(vol.sum())
    assert a[1, 0] == n1 and a[0, 0] == vol.size - n1
    # layers: phase = z mod 2; in-plane segments see one layer, the others cross both
    lay = np.broadcast_to((np.arange(6) % 2)[:, None, None], (6, 5, 7)).astype(np.uint8).copy()
    L = oracle.lpf3(lay, 3, 2, 2)
    for i, (dx, dy, dz) in enumerate(oracle.vectors3(3, 2, 2)):
        assert L[1, i] == (lay.size // 2 if dz == 0 else 0)
        assert L[0, i] == (lay.size // 2 if dz == 0 else 0)
