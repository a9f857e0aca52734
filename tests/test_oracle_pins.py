"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test checks the oracle against something other than itself: values the paper prints,
closed forms, invariants of the definition, and an independent brute force (oracle/brute.py).
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(key: str) -> float:
    with open(os.path.join(GOLDEN, "paper_counts.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line and line.split()[0] == key:
                return float(line.split()[1])
    raise KeyError(key)


# ---------------------------------------------------------------- segment domain (eq. segments)

@pytest.mark.parametrize("W,H", [(1, 1), (2, 3), (5, 5), (10, 7), (64, 64), (100, 100)])
def test_domain_size_full(W, H):
    # |D| = 2HW - H - W + 1 (Sec. 2.2, eq. (segments))
    assert oracle.num_vectors(W - 1, H - 1) == 2 * H * W - H - W + 1
    assert len(oracle.vectors(W - 1, H - 1)) == 2 * H * W - H - W + 1


@pytest.mark.parametrize("cx,cy", [(0, 0), (3, 0), (0, 4), (16, 16), (5, 9)])
def test_domain_matches_symmetry_filter(cx, cy):
    # canonical half = one representative of each {v, -v} pair of the cutoff grid
    v = [tuple(map(int, r)) for r in oracle.vectors(cx, cy)]
    assert v == brute.half_domain(cx, cy)
    full = {(dx, dy) for dx in range(-cx, cx + 1) for dy in range(-cy, cy + 1)}
    cover = set(v) | {(-a, -b) for (a, b) in v}
    assert cover == full


# ------------------------------------------------------- segment lengths (memory formula M)

def _path_len_sum(W, H, quadrant_only=False):
    tot = 0
    for dx, dy in oracle.vectors(W - 1, H - 1):
        if quadrant_only and dx < 0:
            continue
        tot += len(oracle.bresenham(int(dx), int(dy)))
    return tot


@pytest.mark.parametrize("W", [1, 2, 3, 10, 31])
def test_memory_formula_square(W):
    # M = (4W^3 - 4W + 3) / 3 for W = H (Sec. 3.1, memory of the segment table)
    assert 3 * _path_len_sum(W, W) == 4 * W**3 - 4 * W + 3


@pytest.mark.parametrize("W,H", [(3, 5), (4, 9), (7, 8)])
def test_memory_formula_rect(W, H):
    # M = W(3H^2 + 3H + W^2 - 1)/3 - W(W+1)/2 - H(H+1)/2 + 1 for W <= H (Sec. 3.1)
    M = Fraction(W * (3 * H * H + 3 * H + W * W - 1), 3) - Fraction(W * (W + 1), 2) \
        - Fraction(H * (H + 1), 2) + 1
    assert _path_len_sum(W, H) == M


def test_paper_op_count_100():
    # Sec. 6.3: one standard evaluation of one phase at 100 x 100 px takes 6.716e9 operations,
    # i.e. WH times the pixel count of the segments of the first rectangle of eq. (segments).
    W = H = 100
    ops = W * H * _path_len_sum(W, H, quadrant_only=True)
    assert abs(ops - _golden("ops_standard_l2_100x100")) <= 0.0005e9  # 4 significant digits
    # the S2 figure printed beside it is WH ln(WH) + WH (Sec. 2.1)
    s2 = W * H * math.log(W * H) + W * H
    assert abs(s2 - _golden("ops_s2_100x100")) < 0.0005e5


# ------------------------------------------------------------------------- digitisation (R1)

def test_bresenham_vs_closed_form():
    for dx in range(-40, 41):
        for dy in range(-40, 41):
            p = [tuple(map(int, r)) for r in oracle.bresenham(dx, dy)]
            assert p == brute.path(dx, dy, "up"), (dx, dy)


def test_bresenham_structure():
    for dx in range(-25, 26):
        for dy in range(-25, 26):
            p = oracle.bresenham(dx, dy)
            n = max(abs(dx), abs(dy))
            assert len(p) == n + 1
            assert tuple(p[0]) == (0, 0) and tuple(p[-1]) == (dx, dy)
            steps = np.abs(np.diff(p, axis=0))
            assert np.all(steps.max(axis=1) == 1) and np.all(steps <= 1)


def test_bresenham_nontie_is_unique_nearest():
    # away from ties the digitisation is the unique nearest-pixel set, independent of the rule
    for dx in range(0, 33):
        for dy in range(0, 33):
            n, m = max(dx, dy), min(dx, dy)
            g = math.gcd(n, m) if n else 1
            tie = n > 0 and (n // g) % 2 == 0 and m > 0
            if not tie:
                assert brute.path(dx, dy, "up") == brute.path(dx, dy, "down")
                assert [tuple(map(int, r)) for r in oracle.bresenham(dx, dy)] == brute.path(dx, dy, "down")


# ---------------------------------------------------------------------- invariants of L

def _imgs():
    return [
        wl.random_binary(12, 9, 0.6, 11),
        wl.random_binary(16, 16, 0.4, 12),
        wl.boolean_disks(24, 20, 3.0, 0.5, 13),
        wl.small_boolean_64(),
    ]


@pytest.mark.parametrize("k", range(4))
def test_l_zero_is_phase_count(k):
    img = _imgs()[k]
    c = oracle.lpf(img, 3, 3, 3)
    # eq. (l2zero): L(0) = phi^i, i.e. N_i translations
    assert c[0, 0] == int((img == 0).sum()) and c[1, 0] == int((img == 1).sum())


@pytest.mark.parametrize("k", range(4))
def test_unit_steps_equal_s2_and_upper_bound(k):
    img = _imgs()[k]
    H, W = img.shape
    cx, cy = min(6, W - 1), min(6, H - 1)
    c = oracle.lpf(img, cx, cy, 3)
    v = oracle.vectors(cx, cy)
    for ph in (0, 1):
        s2 = brute.s2_fft(img, ph)  # N * S2 via the FFT route of Sec. 2.1
        for i, (dx, dy) in enumerate(v):
            ref = s2[dy % H, dx % W]
            if max(abs(dx), abs(dy)) <= 1:
                assert c[ph, i] == ref, (ph, dx, dy)
            assert c[ph, i] <= ref


@pytest.mark.parametrize("k", range(4))
def test_phase_identity_unit_steps(k):
    # eq. (S2add) times N: L_1(u) - L_0(u) = N_1 - N_0 for unit steps u
    img = _imgs()[k]
    c = oracle.lpf(img, 1, 1, 3).astype(np.int64)
    d = int((img == 1).sum()) - int((img == 0).sum())
    assert np.all(c[1] - c[0] == d)


@pytest.mark.parametrize("k", range(4))
def test_nested_monotonicity(k):
    # a longer segment containing a shorter one (up to translation) cannot be found more often
    img = _imgs()[k]
    H, W = img.shape
    cx, cy = min(8, W - 1), min(8, H - 1)
    c = oracle.lpf(img, cx, cy, 3)
    vs = [tuple(map(int, r)) for r in oracle.vectors(cx, cy)]
    paths = {v: set(map(tuple, oracle.bresenham(*v).tolist())) for v in vs}
    idx = {v: i for i, v in enumerate(vs)}
    checked = 0
    for u in vs:
        for v in vs:
            if len(paths[v]) <= len(paths[u]):
                continue
            pu = paths[u]
            for t in paths[v]:
                if {(x + t[0], y + t[1]) for (x, y) in pu} <= paths[v]:
                    assert np.all(c[:, idx[v]] <= c[:, idx[u]]), (u, v)
                    checked += 1
                    break
    assert checked > 100


def test_axis_monotone():
    img = wl.small_boolean_64()
    c = oracle.lpf(img, 20, 20, 3, layout=1)
    for ph in (0, 1):
        row = c[ph, 20, 20:]  # (d, 0), d = 0..20
        col = c[ph, 20:, 20]  # (0, d)
        assert np.all(np.diff(row.astype(np.int64)) <= 0)
        assert np.all(np.diff(col.astype(np.int64)) <= 0)


@pytest.mark.parametrize("P,a", [(8, 3), (6, 1), (10, 5), (4, 2)])
def test_stripes_closed_form(P, a):
    W, H = 5 * P, 7
    img = wl.stripes(W, H, P, a)
    c = oracle.lpf(img, W - 1, H - 1, 3)
    for i, (dx, dy) in enumerate(oracle.vectors(W - 1, H - 1)):
        adx = abs(int(dx))
        assert c[1, i] == H * (W // P) * max(0, a - adx)
        assert c[0, i] == H * (W // P) * max(0, P - a - adx)


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5])
def test_checkerboard_closed_form(s):
    W = H = 4 * s
    img = wl.checkerboard(W, H, s)
    c = oracle.lpf(img, W - 1, H - 1, 3)
    N = W * H
    hits = 0
    for i, (dx, dy) in enumerate(oracle.vectors(W - 1, H - 1)):
        ax, ay = abs(int(dx)), abs(int(dy))
        if ax < s and ay < s:
            ref = Fraction(N, 2 * s * s) * ((s - ax) * (s - ay) + min(ax, ay))
        elif ax == ay:
            ref = Fraction(N, 2 * s)
        else:
            continue
        hits += 1
        assert c[0, i] == ref and c[1, i] == ref, (dx, dy)
    assert hits >= s * s


@pytest.mark.parametrize("kx,ky", [(2, 1), (1, 3), (2, 2)])
def test_tiling(kx, ky):
    img = wl.random_binary(9, 7, 0.55, 21)
    big = np.tile(img, (ky, kx))
    a = oracle.lpf(img, 8, 6, 3).astype(np.int64)
    b = oracle.lpf(big, 8, 6, 3).astype(np.int64)
    assert np.array_equal(b, kx * ky * a)


def test_translation_and_complement():
    img = wl.random_binary(13, 11, 0.5, 31)
    a = oracle.lpf(img, 7, 6, 3)
    b = oracle.lpf(np.roll(img, (3, -5), axis=(0, 1)), 7, 6, 3)
    assert np.array_equal(a, b)
    c = oracle.lpf(1 - img, 7, 6, 3)
    assert np.array_equal(a[0], c[1]) and np.array_equal(a[1], c[0])


def test_dihedral():
    img = wl.random_binary(14, 14, 0.6, 41)
    n = 14
    cx = cy = 9
    c = oracle.lpf(img, cx, cy, 3, layout=1)
    ct = oracle.lpf(img.T.copy(), cx, cy, 3, layout=1)
    ys, xs = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    anti = img[(-xs) % n, (-ys) % n]  # I_A(x, y) = I(-y, -x)
    ca = oracle.lpf(anti, cx, cy, 3, layout=1)
    for dx, dy in oracle.vectors(cx, cy):
        dx, dy = int(dx), int(dy)
        if dx >= 0:
            assert np.array_equal(ct[:, dx + cy, dy + cx], c[:, dy + cy, dx + cx])
        else:
            assert np.array_equal(ca[:, -dx + cy, -dy + cx], c[:, dy + cy, dx + cx])


def test_grid_layout_symmetry():
    img = wl.random_binary(10, 12, 0.5, 51)
    half = oracle.lpf(img, 5, 4, 3, layout=0)
    grid = oracle.lpf(img, 5, 4, 3, layout=1)
    for i, (dx, dy) in enumerate(oracle.vectors(5, 4)):
        assert np.array_equal(grid[:, dy + 4, dx + 5], half[:, i])
        assert np.array_equal(grid[:, -dy + 4, -dx + 5], half[:, i])


# ------------------------------------------------------------------------------ brute force

def test_exhaustive_4x4():
    # every 4 x 4 image, full domain, both phases, against a vectorised form of brute.py
    n = 4
    bits = (np.arange(1 << 16)[:, None] >> np.arange(16)[None, :]) & 1
    imgs = bits.reshape(-1, n, n).astype(np.uint8)
    vs = brute.half_domain(n - 1, n - 1)
    ref = np.zeros((len(imgs), 2, len(vs)), np.uint32)
    for ph in (0, 1):
        ind = imgs == ph
        for j, (dx, dy) in enumerate(vs):
            acc = np.ones_like(ind)
            for (px, py) in set(brute.path(dx, dy)):
                acc &= np.roll(ind, shift=(-py, -px), axis=(1, 2))
            ref[:, ph, j] = acc.sum(axis=(1, 2))
    got = np.stack([oracle.lpf(im, n - 1, n - 1, 3, nthreads=1) for im in imgs])
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("seed", range(6))
def test_random_8x8_vs_brute(seed):
    img = wl.random_binary(8, 8, 0.3 + 0.08 * seed, 100 + seed)
    assert np.array_equal(oracle.lpf(img, 7, 7, 3), brute.lpf(img, 7, 7, 3))


@pytest.mark.parametrize("shape", [(5, 9), (11, 6), (7, 13)])
def test_random_rect_vs_brute(shape):
    H, W = shape
    img = wl.random_binary(W, H, 0.65, 7 * W + H)
    for cx, cy in [(W - 1, H - 1), (2, 4), (0, 3)]:
        if cx <= W - 1 and cy <= H - 1:
            assert np.array_equal(oracle.lpf(img, cx, cy, 3), brute.lpf(img, cx, cy, 3))


def test_tie_vectors_depend_on_rule():
    # documents that the tie-vector pixel choice is a convention (parity unpinned there)
    img = wl.random_binary(8, 8, 0.7, 7)
    a = brute.lpf(img, 7, 7, 3, "up")
    b = brute.lpf(img, 7, 7, 3, "down")
    assert not np.array_equal(a, b)


def test_phase_mask_subsets():
    img = wl.random_binary(10, 10, 0.5, 3)
    both = oracle.lpf(img, 4, 4, 3)
    assert np.array_equal(oracle.lpf(img, 4, 4, 1)[0], both[0])
    assert np.array_equal(oracle.lpf(img, 4, 4, 2)[0], both[1])


def test_lpf_vectors_matches_full():
    img = wl.random_binary(20, 17, 0.5, 5)
    v = oracle.vectors(6, 5)
    sel = v[::3]
    a = oracle.lpf_vectors(img, sel, 3)
    b = oracle.lpf(img, 6, 5, 3)[:, ::3]
    assert np.array_equal(a, b)


# ----------------------------------------------------------------------------------- delta

@pytest.mark.parametrize("seed", range(3))
def test_delta_restricted_equals_two_evaluations(seed):
    img = wl.random_binary(12, 10, 0.5, 200 + seed)
    g = np.random.default_rng(seed)
    sw = g.integers(0, img.size, size=(12, 2)).astype(np.int32)
    sw[0] = [5, 5]  # a == b
    for cx, cy in [(11, 9), (4, 3)]:
        a = oracle.delta_swap(img, cx, cy, sw, 3)
        b = oracle.delta_swap(img, cx, cy, sw, 3, full=True)
        assert np.array_equal(a, b)
        assert not np.any(a[0])


def test_delta_near_pairs():
    # swaps whose segments overlap (P_a and P_b intersect)
    img = wl.random_binary(9, 9, 0.5, 77)
    ones = np.flatnonzero(img.ravel() == 1)
    zeros = np.flatnonzero(img.ravel() == 0)
    sw = []
    for a in ones[:6]:
        d = np.abs(zeros - a)
        sw.append([a, zeros[np.argmin(d)]])
    sw = np.array(sw, np.int32)
    assert np.array_equal(oracle.delta_swap(img, 8, 8, sw, 3),
                          oracle.delta_swap(img, 8, 8, sw, 3, full=True))


# ---------------------------------------------------------------------------------- Philox

def test_philox_matches_numpy():
    # numpy's Philox (4x64, 10 rounds) advances its counter before each block
    for key in [(0, 0), (1604, 0x6C7066), (2**64 - 1, 12345)]:
        for start in [0, 5, 2**40]:
            g = np.random.Philox(counter=np.array([start, 0, 0, 0], np.uint64),
                                 key=np.array(key, np.uint64))
            raw = g.random_raw(8).astype(np.uint64)
            o1 = oracle.philox4x64([start + 1, 0, 0, 0], key)
            o2 = oracle.philox4x64([start + 2, 0, 0, 0], key)
            assert np.array_equal(np.concatenate([o1, o2]), raw)
