"""Pins of the oracle's annealing step (Sec. 4, Alg. "annealing", eq. (LSE)) on the CPU.

The reference route below shares nothing with oracle_anneal_run: its random stream is numpy's
Philox bit generator, its deltas come from two full evaluations, its energy change is the exact
rational difference of eq. (LSE) before and after, and acceptance uses math.exp.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as wl

KEY_TAG = 0x6C7066


def _block(seed, step, k):
    # numpy advances the counter before producing a block: start from (counter - 1)
    assert step > 0
    ctr = np.array([step - 1, k, 0, 0], np.uint64)
    g = np.random.Philox(counter=ctr, key=np.array([seed, KEY_TAG], np.uint64))
    return [int(x) for x in g.random_raw(4)]


def _lse_exact(counts, target, N, Nt):
    return sum((Fraction(int(t), Nt) - Fraction(int(c), N)) ** 2
               for c, t in zip(counts.ravel(), target.ravel()))


def _ranked(cands, score):
    # reading R18, by sorting: the min(64, R) largest fp32 keys among the first R = min(K, 4096)
    # draws (equal keys by draw index; void draws and NaN keys lowest), then the rest in order
    K = len(cands)
    R = min(K, 4096)
    key = np.full(R, -np.inf)
    for k in range(R):
        a, b = cands[k][0], cands[k][1]
        if a >= 0:
            v = np.float32(score[a]) + np.float32(score[b])
            key[k] = -np.inf if np.isnan(v) else float(v) + 0.0  # -0 and +0 are one key
    top = list(np.lexsort((np.arange(R), -key))[:min(R, 64)])
    return top + [k for k in range(K) if k not in set(top)]


def _reference_chain(img, cx, cy, mask, target, Nt, seed, step0, nsteps, K, Ts, proposal,
                     descriptor=oracle.DESC_LPF, score=None):
    img = img.copy()
    H, W = img.shape
    N = W * H
    flat = img.ravel()
    pos1 = list(np.flatnonzero(flat == 1))
    pos0 = list(np.flatnonzero(flat == 0))
    evaluate = oracle.lpf if descriptor == oracle.DESC_LPF else oracle.s2
    counts = evaluate(img, cx, cy, mask).astype(np.int64)
    out = []
    def itf(q):
        x, y = q % W, q // W
        v = img[y, x]
        return (img[y, (x + 1) % W] != v or img[y, (x - 1) % W] != v or
                img[(y + 1) % H, x] != v or img[(y - 1) % H, x] != v)

    for s in range(nsteps):
        res = (-1, -1, -1)
        draws = []
        for k in range(K):
            r = _block(seed, step0 + s, k)
            ia = ((r[0] >> 32) * len(pos1)) >> 32
            ib = ((r[1] >> 32) * len(pos0)) >> 32
            U = (r[2] >> 11) * 2.0**-53
            a, b = int(pos1[ia]), int(pos0[ib])
            if proposal == 1 and not (itf(a) and itf(b)):
                a = b = -1
            draws.append((a, b, ia, ib, U))
        order = range(K) if score is None else _ranked(draws, score)
        for k in order:
            a, b, ia, ib, U = draws[k]
            if a < 0:
                continue
            img2 = img.copy()
            img2.flat[a], img2.flat[b] = 0, 1
            dl = evaluate(img2, cx, cy, mask).astype(np.int64) - counts
            de_exact = _lse_exact(counts + dl, target, N, Nt) - _lse_exact(counts, target, N, Nt)
            # the oracle rounds the exact rational once (integer sum / N^2 Nt)
            de = float(de_exact)
            if de <= 0 or U < math.exp(-de / Ts[s]):
                counts += dl
                img.flat[a], img.flat[b] = 0, 1
                pos1[ia], pos0[ib] = b, a
                res = (k, a, b)
                break
        out.append(res)
    return out, img, counts


@pytest.mark.parametrize("proposal", [0, 1])
def test_anneal_matches_reference_chain(proposal):
    tgt = wl.boolean_disks(32, 32, 3.0, 0.4, 5)
    cx = cy = 5
    mask = 3
    target = oracle.lpf(tgt, cx, cy, mask)
    Nt = tgt.size
    cell = wl.random_cell(12, 12, int(round(0.4 * 144)), 9)
    seed = 77
    nsteps, K = 25, 16
    Ts = 2e-4 * 0.9 ** np.arange(nsteps)
    st = oracle.AnnealState(cell, cx, cy, mask, target, Nt, seed)
    # numpy cannot be stepped back to counter (0, 0, 0, 0): start both chains at step 1
    st.step = 1
    res = st.run(nsteps, K, Ts, proposal)
    ref, img_ref, counts_ref = _reference_chain(cell, cx, cy, mask, target, Nt, seed, 1,
                                                nsteps, K, Ts, proposal)
    got = [(int(r["k"]), int(r["a"]), int(r["b"])) for r in res]
    assert got == ref
    assert np.array_equal(st.img, img_ref)
    assert np.array_equal(st.counts.astype(np.int64), counts_ref)
    assert sum(r[0] >= 0 for r in got) > 3


@pytest.mark.parametrize("proposal,mask", [(0, 3), (1, 3), (0, 2)])
def test_s2_anneal_matches_reference_chain(proposal, mask):
    # the same chain with the two-point probability as the descriptor (Sec. 2.1; Secs. 5 and 6.1)
    tgt = wl.square_particles(40, 40, 4, 16, 5)
    cx = cy = 5
    target = oracle.s2(tgt, cx, cy, mask)
    Nt = tgt.size
    cell = wl.random_cell(14, 14, int(round(0.16 * 196)), 9)
    seed = 78
    nsteps, K = 25, 16
    Ts = 2e-4 * 0.9 ** np.arange(nsteps)
    st = oracle.AnnealState(cell, cx, cy, mask, target, Nt, seed, descriptor=oracle.DESC_S2)
    st.step = 1
    res = st.run(nsteps, K, Ts, proposal)
    ref, img_ref, counts_ref = _reference_chain(cell, cx, cy, mask, target, Nt, seed, 1,
                                                nsteps, K, Ts, proposal, oracle.DESC_S2)
    got = [(int(r["k"]), int(r["a"]), int(r["b"])) for r in res]
    assert got == ref
    assert np.array_equal(st.img, img_ref)
    assert np.array_equal(st.counts.astype(np.int64), counts_ref)
    assert sum(r[0] >= 0 for r in got) > 3


def test_anneal_invariants():
    tgt = wl.boolean_disks(48, 48, 4.0, 0.35, 6)
    cx = cy = 6
    target = oracle.lpf(tgt, cx, cy, 2)
    cell = wl.random_cell(16, 16, int(round(0.35 * 256)), 3)
    st = oracle.AnnealState(cell, cx, cy, 2, target, tgt.size, 1234)
    e0 = st.e
    res = st.run(40, 32, np.full(40, 1e-5))
    # counts track the image, volume fraction is preserved, pixel lists are consistent
    assert np.array_equal(st.counts, oracle.lpf(st.img, cx, cy, 2))
    assert int(st.img.sum()) == int(cell.sum())
    assert set(st.pos1.tolist()) == set(np.flatnonzero(st.img.ravel() == 1).tolist())
    assert set(st.pos0.tolist()) == set(np.flatnonzero(st.img.ravel() == 0).tolist())
    # the running error equals eq. (LSE) recomputed from the counts (up to rounding)
    e_now = oracle.lse(st.counts, target, 256, tgt.size)
    assert abs(st.e - e_now) <= 1e-12 * max(1.0, e0)
    exact = float(_lse_exact(st.counts.astype(np.int64), target, 256, tgt.size))
    assert abs(e_now - exact) <= 1e-12 * exact
    # accepted steps report their own energy change
    acc = res[res["k"] >= 0]
    assert len(acc) > 0
    assert np.allclose(np.cumsum(acc["de"]) + e0, acc["e"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("K,proposal", [(5, 0), (16, 1), (100, 0), (100, 1)])
def test_ranked_anneal_matches_reference_chain(K, proposal):
    # the chain that evaluates each step's draws in the ranked order of a fixed score field
    # (reading R18) against the reference route with the order taken by sorting
    tgt = wl.boolean_disks(32, 32, 3.0, 0.4, 6)
    cx = cy = 4
    mask = 3
    target = oracle.lpf(tgt, cx, cy, mask)
    cell = wl.random_cell(12, 12, int(round(0.4 * 144)), 10)
    g = np.random.default_rng(K + 7 * proposal)
    score = np.round(g.normal(size=144), 1).astype(np.float32)  # many equal keys
    score[::11] = -0.0
    score[5::13] = 0.0
    score[7] = np.nan
    seed = 91
    nsteps = 20
    Ts = 1e-4 * 0.85 ** np.arange(nsteps)
    st = oracle.AnnealState(cell, cx, cy, mask, target, tgt.size, seed)
    st.step = 1
    res = st.run(nsteps, K, Ts, proposal, score=score)
    ref, img_ref, counts_ref = _reference_chain(cell, cx, cy, mask, target, tgt.size, seed, 1,
                                                nsteps, K, Ts, proposal, score=score)
    got = [(int(r["k"]), int(r["a"]), int(r["b"])) for r in res]
    assert got == ref
    assert np.array_equal(st.img, img_ref)
    assert np.array_equal(st.counts.astype(np.int64), counts_ref)
    # the order matters: some accepted draw is not the first acceptable one in draw order
    plain = oracle.AnnealState(cell, cx, cy, mask, target, tgt.size, seed)
    plain.step = 1
    pres = plain.run(nsteps, K, Ts, proposal)
    if K > 5:
        assert [int(r["k"]) for r in pres] != [r[0] for r in ref]
