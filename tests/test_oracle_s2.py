"""Pins of the oracle's two-point probability (Sec. 2.1, eq. (S2dis)) and of its interchange
update and annealing chain, on the CPU.

The oracle evaluates the definition's double sum.  It is pinned against the FFT route the paper
uses (numpy's FFT, oracle/brute.py), against the lineal path function on unit steps (a segment of
two pixels is its two end points), against eq. (S2add), and against closed forms.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads as wl

IMAGES = {
    "random_13x17": lambda: wl.random_binary(17, 13, 0.4, 1),
    "disks_40x24": lambda: wl.boolean_disks(40, 24, 3.0, 0.45, 2),
    "squares_30x30": lambda: wl.square_particles(30, 30, 4, 8, 3),
    "stripes_9x20": lambda: wl.stripes(9, 20, 3, 1, vertical=False),
    "ragged_1x7": lambda: wl.random_binary(7, 1, 0.5, 4),
    "ragged_5x1": lambda: wl.random_binary(1, 5, 0.5, 5),
}


@pytest.mark.parametrize("name", sorted(IMAGES))
def test_s2_equals_fft_route_on_whole_domain(name):
    # the paper's evaluation: IDFT(DFT(chi) conj(DFT(chi))) / (W H), times W H
    img = IMAGES[name]()
    H, W = img.shape
    g = oracle.s2(img, W - 1, H - 1, 3, layout=1)
    for ph in (0, 1):
        f = brute.s2_fft(img, ph)
        dy, dx = np.mgrid[-(H - 1):H, -(W - 1):W]
        assert np.array_equal(g[ph].astype(np.int64), f[dy % H, dx % W]), (name, ph)


@pytest.mark.parametrize("name", ["random_13x17", "disks_40x24", "squares_30x30"])
def test_half_layout_matches_grid_and_symmetry(name):
    img = IMAGES[name]()
    H, W = img.shape
    cx, cy = min(W - 1, 9), min(H - 1, 7)
    half = oracle.s2(img, cx, cy, 3, 0)
    grid = oracle.s2(img, cx, cy, 3, 1)
    v = oracle.vectors(cx, cy).astype(int)
    for p in range(2):
        assert np.array_equal(half[p], grid[p][v[:, 1] + cy, v[:, 0] + cx])
        # C(-v) = C(v): the autocorrelation of a periodic image is even (every grid entry is
        # evaluated separately, so this is a check, not a construction)
        assert np.array_equal(grid[p], grid[p][::-1, ::-1])
    # phase selection: single-phase masks give the corresponding rows
    assert np.array_equal(oracle.s2(img, cx, cy, 1, 0)[0], half[0])
    assert np.array_equal(oracle.s2(img, cx, cy, 2, 0)[0], half[1])


@pytest.mark.parametrize("name", sorted(IMAGES))
def test_unit_steps_equal_lpf(name):
    # a segment with |dx|, |dy| <= 1 has exactly its two end points (Sec. 2.2), so L = N S2
    img = IMAGES[name]()
    H, W = img.shape
    cx, cy = min(W - 1, 1), min(H - 1, 1)
    assert np.array_equal(oracle.s2(img, cx, cy, 3, 0), oracle.lpf(img, cx, cy, 3, 0))


@pytest.mark.parametrize("name", sorted(IMAGES))
def test_phase_relation_eq_s2add(name):
    # eq. (S2add) times W H: C_0(v) - C_1(v) = N_0 - N_1 for every v
    img = IMAGES[name]()
    H, W = img.shape
    n1 = int(img.sum())
    n0 = W * H - n1
    c = oracle.s2(img, W - 1, H - 1, 3, 0).astype(np.int64)
    assert np.all(c[0] - c[1] == n0 - n1)
    # v = 0: S2 is the volume fraction
    assert c[0][0] == n0 and c[1][0] == n1


def test_closed_forms():
    # checkerboard of unit squares: both end points in phase 1 iff dx + dy is even
    W, H = 12, 8
    img = wl.checkerboard(W, H, 1)
    c = oracle.s2(img, W - 1, H - 1, 2, 1)[0]
    dy, dx = np.mgrid[-(H - 1):H, -(W - 1):W]
    assert np.array_equal(c, np.where((dx + dy) % 2 == 0, W * H // 2, 0))
    # a single phase-1 pixel: C_1(v) = [v = 0 mod (W, H)], C_0(v) = N - 2 + C_1(v)
    W, H = 7, 5
    img = np.zeros((H, W), np.uint8)
    img[3, 2] = 1
    c = oracle.s2(img, W - 1, H - 1, 3, 1).astype(np.int64)
    dy, dx = np.mgrid[-(H - 1):H, -(W - 1):W]
    one = ((dx % W == 0) & (dy % H == 0)).astype(np.int64)
    assert np.array_equal(c[1], one)
    assert np.array_equal(c[0], W * H - 2 + one)
    # vertical stripes of width w, period P: rows are constant, so C_1(dx, dy) = H * #{x: both}
    W, H, P, w = 12, 5, 6, 2
    img = wl.stripes(W, H, P, w, vertical=True)
    c = oracle.s2(img, W - 1, H - 1, 2, 1)[0]
    for dx in range(-(W - 1), W):
        both = sum(1 for x in range(W) if x % P < w and (x + dx) % P < w)
        assert np.all(c[:, dx + W - 1] == H * both)


def _swaps(img, n, seed, extra=()):
    g = np.random.default_rng(seed)
    ones = np.flatnonzero(img.ravel() == 1)
    zeros = np.flatnonzero(img.ravel() == 0)
    sw = [(int(g.choice(ones)), int(g.choice(zeros))) for _ in range(n)]
    return np.array(list(sw) + list(extra), np.int32)


@pytest.mark.parametrize("W,H,cx,cy", [(9, 7, 8, 6), (16, 12, 15, 11), (20, 10, 5, 9),
                                       (6, 6, 5, 5), (1, 9, 0, 8)])
def test_s2_delta_equals_two_full_evaluations(W, H, cx, cy):
    img = wl.random_binary(W, H, 0.5, W * 31 + H)
    if img.min() == img.max():
        img.flat[0] ^= 1
    extra = []
    ones = np.flatnonzero(img.ravel() == 1)
    zeros = np.flatnonzero(img.ravel() == 0)
    a = int(ones[0])
    # partners at special offsets: neighbours, b - a = a - b mod (W, H), the same pixel pair twice
    for off in (1, W, W // 2, (H // 2) * W, (H // 2) * W + W // 2):
        b = (a + off) % (W * H)
        if img.flat[b] == 0:
            extra.append((a, b))
    extra.append((a, int(zeros[-1])))
    sw = _swaps(img, 24, W + H, extra)
    got = oracle.s2_delta_swap(img, cx, cy, sw, 3)
    base = oracle.s2(img, cx, cy, 3, 0).astype(np.int64)
    for s, (a, b) in enumerate(sw):
        img2 = img.copy().ravel()
        img2[a], img2[b] = img2[b], img2[a]
        ref = oracle.s2(img2.reshape(H, W), cx, cy, 3, 0).astype(np.int64) - base
        assert np.array_equal(got[s], ref), (s, a, b)
        # N_1 is unchanged by an interchange, so both phases change alike (eq. (S2add))
        assert np.array_equal(got[s][0], got[s][1])
    # single-phase masks
    assert np.array_equal(oracle.s2_delta_swap(img, cx, cy, sw, 2)[:, 0], got[:, 1])
    assert np.array_equal(oracle.s2_delta_swap(img, cx, cy, sw, 1)[:, 0], got[:, 0])


def _lse_exact(counts, target, N, Nt):
    return sum((Fraction(int(t), Nt) - Fraction(int(c), N)) ** 2
               for c, t in zip(counts.ravel(), target.ravel()))


@pytest.mark.parametrize("mask,K", [(3, 16), (2, 5), (1, 40)])
def test_s2_chain_is_exact(mask, K):
    # every accepted step's de is the exact change of eq. (LSE) on S2 counts, the final counts are
    # the S2 of the final image, and rejected candidates leave the state unchanged
    tgt = wl.square_particles(40, 40, 4, 16, 7)
    W = H = 20
    cx = cy = 6
    target = oracle.s2(tgt, cx, cy, mask, 0)
    cell = wl.random_cell(W, H, int(tgt.sum()) // 4, 8)
    st = oracle.AnnealState(cell, cx, cy, mask, target, 1600, 11, descriptor=oracle.DESC_S2)
    e0 = st.e
    prev = st.counts.copy()
    img_prev = st.img.copy()
    res = []
    for _ in range(6):
        r = st.run(10, K, np.full(10, 2e-4))
        res.append(r)
    res = np.concatenate(res)
    assert np.array_equal(st.counts, oracle.s2(st.img, cx, cy, mask, 0))
    exact = _lse_exact(st.counts, target, W * H, 1600)
    assert math.isclose(st.e, float(exact), rel_tol=1e-9, abs_tol=1e-15)
    acc = res[res["k"] >= 0]
    assert len(acc) > 0
    assert st.e < e0
    # replay the accepted interchanges one by one
    img = img_prev.ravel().copy()
    e_prev = _lse_exact(prev, target, W * H, 1600)
    for r in acc:
        assert img[r["a"]] == 1 and img[r["b"]] == 0
        img[r["a"]], img[r["b"]] = 0, 1
        e_now = _lse_exact(oracle.s2(img.reshape(H, W), cx, cy, mask, 0), target, W * H, 1600)
        assert math.isclose(r["de"], float(e_now - e_prev), rel_tol=1e-9, abs_tol=1e-15)
        e_prev = e_now
    assert np.array_equal(img.reshape(H, W), st.img)
