"""Pins of the oracle's Monte-Carlo approximation (Sec. 3, opening paragraph: segments compared
with the image at a chosen set X of start positions only), its interchange update and the chain
it drives, on the CPU."""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads as wl


def _img(W, H, seed):
    img = wl.random_binary(W, H, 0.55, seed)
    if img.min() == img.max():
        img.flat[0] ^= 1
    return img


@pytest.mark.parametrize("W,H,cx,cy", [(12, 10, 11, 9), (17, 9, 6, 8), (1, 7, 0, 6), (30, 30, 8, 8)])
def test_all_positions_give_the_entire_function(W, H, cx, cy):
    img = _img(W, H, W + H)
    full = np.ones((H, W), np.uint8)
    assert np.array_equal(oracle.lpf_sampled(img, cx, cy, full), oracle.lpf(img, cx, cy))
    assert not oracle.lpf_sampled(img, cx, cy, np.zeros((H, W), np.uint8)).any()


def test_disjoint_position_sets_add_up():
    W, H, cx, cy = 19, 13, 7, 6
    img = _img(W, H, 3)
    part = np.random.default_rng(4).integers(0, 3, (H, W))
    total = sum(oracle.lpf_sampled(img, cx, cy, (part == k).astype(np.uint8)).astype(np.int64)
                for k in range(3))
    assert np.array_equal(total, oracle.lpf(img, cx, cy))


def test_single_position_matches_brute_path():
    # X = {x}: the count is 1 exactly when the digitised segment at x lies in the phase
    W, H, cx, cy = 11, 9, 5, 4
    img = _img(W, H, 5)
    vs = brute.half_domain(cx, cy)
    for (x, y) in [(0, 0), (10, 8), (4, 3)]:
        m = np.zeros((H, W), np.uint8)
        m[y, x] = 1
        got = oracle.lpf_sampled(img, cx, cy, m)
        for i, (dx, dy) in enumerate(vs):
            on = [img[(y + py) % H, (x + px) % W] for (px, py) in brute.path(dx, dy)]
            for ph in (0, 1):
                assert got[ph, i] == int(all(v == ph for v in on)), (x, y, dx, dy, ph)


def test_translations_of_a_position_set_average_to_the_function():
    # sum over all periodic translations t of the counts at X + t = |X| * L (each start pixel is
    # covered |X| times); an exact identity of the definition
    W, H, cx, cy = 10, 8, 6, 5
    img = _img(W, H, 6)
    X = wl.sample_positions(W, H, 7, 8)
    tot = np.zeros((2, oracle.num_vectors(cx, cy)), np.int64)
    for ty in range(H):
        for tx in range(W):
            tot += oracle.lpf_sampled(img, cx, cy, np.roll(X, (ty, tx), (0, 1)))
    assert np.array_equal(tot, 7 * oracle.lpf(img, cx, cy).astype(np.int64))


def test_translation_invariance():
    # counts of image I at X equal counts of I rolled by t at X rolled by t
    W, H, cx, cy = 14, 9, 7, 8
    img = _img(W, H, 9)
    X = wl.sample_positions(W, H, 20, 10)
    a = oracle.lpf_sampled(img, cx, cy, X)
    b = oracle.lpf_sampled(np.roll(img, (3, 5), (0, 1)), cx, cy, np.roll(X, (3, 5), (0, 1)))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("W,H,cx,cy,n", [(9, 7, 8, 6, 10), (16, 12, 10, 11, 60), (20, 10, 5, 9, 200)])
def test_sampled_delta_equals_two_sampled_evaluations(W, H, cx, cy, n):
    img = _img(W, H, W * H)
    X = wl.sample_positions(W, H, n, n)
    rng = np.random.default_rng(n)
    ones = np.flatnonzero(img.ravel() == 1)
    zeros = np.flatnonzero(img.ravel() == 0)
    sw = np.stack([rng.choice(ones, 30), rng.choice(zeros, 30)], 1).astype(np.int32)
    got = oracle.delta_swap_sampled(img, cx, cy, X, sw, 3)
    base = oracle.lpf_sampled(img, cx, cy, X).astype(np.int64)
    for s, (a, b) in enumerate(sw):
        img2 = img.copy().ravel()
        img2[a], img2[b] = img2[b], img2[a]
        ref = oracle.lpf_sampled(img2.reshape(H, W), cx, cy, X).astype(np.int64) - base
        assert np.array_equal(got[s], ref), s
    # the full set gives the entire function's delta
    full = np.ones((H, W), np.uint8)
    assert np.array_equal(oracle.delta_swap_sampled(img, cx, cy, full, sw, 3),
                          oracle.delta_swap(img, cx, cy, sw, 3))


def _lse_exact(counts, target, N, Nt):
    return sum((Fraction(int(t), Nt) - Fraction(int(c), N)) ** 2
               for c, t in zip(counts.ravel(), target.ravel()))


@pytest.mark.parametrize("n_cell,n_tgt", [(10, 100), (100, 1000), (144, 400)])
def test_sampled_chain_matches_reference(n_cell, n_tgt):
    # the chain on the approximation (Sec. 5, reconstruction from the approximated function):
    # target = counts of the original at its own N positions over Nt = N, cell counts at the
    # cell's positions, objective eq. (LSE) with the cell's N; replayed with full evaluations
    tgt = wl.checkerboard(40, 40, 5)
    Xt = wl.sample_positions(40, 40, n_tgt, 1)
    cx = cy = 5
    target = oracle.lpf_sampled(tgt, cx, cy, Xt)
    cell = wl.random_cell(12, 12, 72, 2)
    Xc = wl.sample_positions(12, 12, n_cell, 3)
    st = oracle.AnnealState(cell, cx, cy, 3, target, n_tgt, 17, sample=Xc)
    assert st.N == n_cell
    e0 = st.e
    res = st.run(40, 16, 1e-3 * 0.9 ** np.arange(40))
    acc = res[res["k"] >= 0]
    assert len(acc) > 3
    img = cell.ravel().copy()
    e_prev = _lse_exact(oracle.lpf_sampled(cell, cx, cy, Xc), target, n_cell, n_tgt)
    assert math.isclose(e0, float(e_prev), rel_tol=1e-12)
    for r in acc:
        img[r["a"]], img[r["b"]] = 0, 1
        e_now = _lse_exact(oracle.lpf_sampled(img.reshape(12, 12), cx, cy, Xc), target, n_cell, n_tgt)
        assert math.isclose(r["de"], float(e_now - e_prev), rel_tol=1e-9, abs_tol=1e-15)
        e_prev = e_now
    assert np.array_equal(img.reshape(12, 12), st.img)
    assert np.array_equal(st.counts, oracle.lpf_sampled(st.img, cx, cy, Xc))
