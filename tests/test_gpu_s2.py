"""Two-point probability on the GPU (lpf_s2, lpf_s2_delta_swap, S2 annealing chains) against the
CPU oracle: counts and deltas bit for bit, chains step for step."""
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


def _dev(img):
    import torch
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def _unpack(bits, W, H):
    b = bits.cpu().numpy().view(np.uint64).reshape(H, -1)
    out = np.zeros((H, W), np.uint8)
    for x in range(W):
        out[:, x] = (b[:, x // 64] >> np.uint64(x % 64)) & np.uint64(1)
    return out


RAGGED = [(1, 1, 0, 0), (7, 1, 6, 0), (1, 9, 0, 8), (5, 7, 4, 6), (37, 23, 36, 22),
          (33, 31, 32, 30), (50, 50, 49, 49), (96, 64, 95, 63), (130, 70, 40, 30),
          (200, 40, 199, 39), (100, 100, 99, 99), (65, 3, 64, 2), (257, 9, 256, 8)]


@pytest.mark.parametrize("W,H,cx,cy", RAGGED)
def test_s2_matches_oracle(ctx, W, H, cx, cy):
    import torch
    print(f"[gpu] s2 {W}x{H} c=({cx},{cy})", flush=True)
    img = wl.random_binary(W, H, 0.45, W * 131 + H)
    bits = ctx.pack(_dev(img))
    for mask in (1, 2, 3):
        for layout in (0, 1):
            got = ctx.s2(bits, W, H, cx, cy, mask, layout)
            torch.cuda.synchronize()
            want = oracle.s2(img, cx, cy, mask, layout)
            assert np.array_equal(got.cpu().numpy().astype(np.uint32), want), (mask, layout)


@pytest.mark.parametrize("name", ["squares", "disks", "checker", "stripes", "all_one_but_one"])
def test_s2_structured_images(ctx, name):
    import torch
    print(f"[gpu] s2 structured {name}", flush=True)
    img = {
        "squares": lambda: wl.square_particles(100, 100, 4, 100, 5),
        "disks": lambda: wl.boolean_disks(96, 80, 5.0, 0.4, 6),
        "checker": lambda: wl.checkerboard(64, 64, 1),
        "stripes": lambda: wl.stripes(90, 33, 7, 3),
        "all_one_but_one": lambda: 1 - np.eye(1, 45 * 37, 700, dtype=np.uint8).reshape(37, 45),
    }[name]()
    H, W = img.shape
    bits = ctx.pack(_dev(img))
    got = ctx.s2(bits, W, H, W - 1, H - 1, 3, 1)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().astype(np.uint32), oracle.s2(img, W - 1, H - 1, 3, 1))


def test_s2_unit_steps_equal_lpf(ctx):
    import torch
    img = wl.rsa_512()
    bits = ctx.pack(_dev(img))
    a = ctx.s2(bits, 512, 512, 1, 1, 3, 0)
    b = ctx.full(bits, 512, 512, 1, 1, 3, 0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("side,c", [(512, 128), (1024, 512), (4000, 3)])
def test_s2_full_size_sampled(ctx, side, c):
    # the bench sizes: every count of a sample of vectors (both phases) from the oracle
    import torch
    print(f"[gpu] s2 {side}x{side if side < 4000 else 5} c={c} sampled", flush=True)
    if side == 512:
        img = wl.rsa_512()
    elif side == 1024:
        img = wl.boolean_disks(1024, 1024, 8.0, 0.35, 9)
    else:
        img = wl.random_binary(side, 5, 0.5, 10)
    H, W = img.shape
    cx, cy = c, min(c, H - 1)
    bits = ctx.pack(_dev(img))
    got = ctx.s2(bits, W, H, cx, cy, 3, 0).cpu().numpy().astype(np.uint32)
    v = oracle.vectors(cx, cy)
    rng = np.random.default_rng(side)
    pick = np.unique(np.concatenate([[0, 1, len(v) - 1], rng.integers(0, len(v), 120)]))
    want = oracle.s2_vectors(img, v[pick], 3)
    assert np.array_equal(got[:, pick], want)
    # eq. (S2add) holds for every vector
    n1 = int(img.sum())
    assert np.all(got[0].astype(np.int64) - got[1] == W * H - 2 * n1)


@pytest.mark.parametrize("W,H,cx,cy,mask", [(9, 7, 8, 6, 3), (16, 12, 15, 11, 3),
                                            (40, 24, 10, 9, 2), (6, 6, 5, 5, 1),
                                            (1, 9, 0, 8, 3), (128, 128, 32, 32, 3)])
def test_s2_delta_matches_oracle(ctx, W, H, cx, cy, mask):
    import torch
    print(f"[gpu] s2 delta {W}x{H} c=({cx},{cy}) mask={mask}", flush=True)
    img = wl.random_binary(W, H, 0.5, W * 17 + H)
    if img.min() == img.max():
        img.flat[0] ^= 1
    N = W * H
    rng = np.random.default_rng(N)
    sw = rng.integers(0, N, (300, 2)).astype(np.int32)  # includes same-phase pairs
    ones = np.flatnonzero(img.ravel() == 1)
    a = int(ones[0])
    extra = [(a, a), (a, (a + 1) % N), (a, (a + W) % N), (a, (a + W // 2) % N),
             (a, (a + (H // 2) * W + W // 2) % N)]
    sw = np.concatenate([sw, np.array(extra, np.int32)])
    bits = ctx.pack(_dev(img))
    got = ctx.s2_delta_swap(bits, W, H, cx, cy, torch.from_numpy(sw).cuda(), mask)
    torch.cuda.synchronize()
    # the oracle reads a swap of two same-phase pixels as no change, like the kernel
    want = oracle.s2_delta_swap(img, cx, cy, sw, mask)
    assert np.array_equal(got.cpu().numpy(), want)


def _s2_problem(cell_side, tgt_side, c, mask, seed):
    tgt = wl.square_particles(tgt_side, tgt_side, 4, int(0.16 * tgt_side * tgt_side) // 16, seed)
    target = oracle.s2(tgt, c, c, mask)
    cell = wl.random_cell(cell_side, cell_side, int(round(0.16 * cell_side * cell_side)), seed + 1)
    return tgt, target, cell


def _gpu_chain(ctx, cell, cx, cy, mask, target, Nt, seed):
    import torch
    from paper_1601_04359_amd import Anneal
    H, W = cell.shape
    bits = ctx.pack(_dev(cell))
    t = torch.from_numpy(target.astype(np.int32)).cuda()
    return Anneal(ctx, bits, W, H, cx, cy, mask, t, Nt, seed, descriptor="s2")


@pytest.mark.parametrize("proposal,mask,K,side,c", [(0, 3, 64, 20, 6), (1, 3, 200, 20, 6),
                                                   (0, 2, 64, 25, 12), (0, 1, 333, 16, 15),
                                                   (0, 3, 4096, 50, 24)])
def test_s2_chain_matches_oracle(ctx, proposal, mask, K, side, c):
    import torch
    from paper_1601_04359_amd import LPF_DELTA_S2, step_records
    print(f"[gpu] s2 chain proposal={proposal} mask={mask} K={K} {side}x{side} c={c}", flush=True)
    tgt, target, cell = _s2_problem(side, 2 * side, c, mask, 40 + K)
    seed, nsteps = 7, 50
    Ts = 1e-4 * 0.9 ** np.arange(nsteps)
    ch = _gpu_chain(ctx, cell, c, c, mask, target, tgt.size, seed)
    assert ch.method == LPF_DELTA_S2
    recs = step_records(ch.run(K, Ts, proposal))
    torch.cuda.synchronize()
    ref = oracle.AnnealState(cell, c, c, mask, target, tgt.size, seed,
                             descriptor=oracle.DESC_S2)
    e0 = ref.e
    rres = ref.run(nsteps, K, Ts, proposal)
    got = [(int(r["k"]), int(r["a"]), int(r["b"])) for r in recs]
    want = [(int(r["k"]), int(r["a"]), int(r["b"])) for r in rres]
    assert got == want
    assert np.array_equal(recs["de"], rres["de"]) and np.array_equal(recs["e"], rres["e"])
    assert sum(k >= 0 for k, _, _ in got) > 5
    assert np.array_equal(_unpack(ch.bits, side, side), ref.img)
    assert np.array_equal(ch.counts.cpu().numpy().astype(np.uint32), ref.counts)
    assert float(ch.e.cpu()[0]) == ref.e
    assert ref.e < e0
    ch.close()


def test_s2_chain_ragged_cell(ctx):
    # 21 x 17 cell, cutoffs (20, 16): every shift of the cell, b - a = a - b cases included
    import torch
    from paper_1601_04359_amd import step_records
    print("[gpu] s2 chain ragged 21x17 c=(20,16)", flush=True)
    tgt = wl.square_particles(42, 34, 4, 14, 3)
    target = oracle.s2(tgt, 20, 16, 3)
    cell = wl.random_cell(21, 17, int(tgt.mean() * 21 * 17), 4)
    Ts = 1e-3 * 0.9 ** np.arange(30)
    ch = _gpu_chain(ctx, cell, 20, 16, 3, target, tgt.size, 5)
    recs = step_records(ch.run(100, Ts))
    torch.cuda.synchronize()
    ref = oracle.AnnealState(cell, 20, 16, 3, target, tgt.size, 5, descriptor=oracle.DESC_S2)
    rres = ref.run(30, 100, Ts)
    assert np.array_equal(recs[["k", "a", "b"]], rres[["k", "a", "b"]])
    assert np.array_equal(recs["e"], rres["e"])
    assert np.array_equal(ch.counts.cpu().numpy().astype(np.uint32), ref.counts)
    ch.close()


def test_s2_delta_energy_exact(ctx):
    # lpf_anneal_delta_energy on an S2 chain: the exact change of eq. (LSE) on S2 counts
    import torch
    from fractions import Fraction
    print("[gpu] s2 delta energy", flush=True)
    tgt, target, cell = _s2_problem(24, 48, 8, 3, 11)
    ch = _gpu_chain(ctx, cell, 8, 8, 3, target, tgt.size, 1)
    rng = np.random.default_rng(5)
    ones = np.flatnonzero(cell.ravel() == 1)
    zeros = np.flatnonzero(cell.ravel() == 0)
    sw = np.stack([rng.choice(ones, 40), rng.choice(zeros, 40)], 1).astype(np.int32)
    de = ch.delta_energy(torch.from_numpy(sw).cuda()).cpu().numpy()
    N, Nt = cell.size, tgt.size
    base = oracle.s2(cell, 8, 8, 3).astype(np.int64)
    dl = oracle.s2_delta_swap(cell, 8, 8, sw, 3).astype(np.int64)
    for i in range(len(sw)):
        S = int(np.sum(dl[i] * (Nt * (dl[i] + 2 * base) - 2 * N * target.astype(np.int64))))
        assert de[i] == S / (N * N * Nt)
        exact = sum((Fraction(int(t), Nt) - Fraction(int(c), N)) ** 2
                    for c, t in zip((base + dl[i]).ravel(), target.ravel())) - \
            sum((Fraction(int(t), Nt) - Fraction(int(c), N)) ** 2
                for c, t in zip(base.ravel(), target.ravel()))
        assert abs(de[i] - float(exact)) <= 1e-12 * max(1.0, abs(float(exact)))
    ch.close()


def test_s2_learned_chain_stays_exact(ctx):
    # learned proposals on an S2 chain: counts stay the S2 of the cell and e stays eq. (LSE)
    import torch
    from paper_1601_04359_amd import LPF_PROP_LEARNED, step_records
    print("[gpu] s2 learned chain", flush=True)
    tgt, target, cell = _s2_problem(32, 64, 10, 3, 21)
    ch = _gpu_chain(ctx, cell, 10, 10, 3, target, tgt.size, 2)
    scores = torch.from_numpy(np.random.default_rng(3).standard_normal(32 * 32).astype(np.float32)).cuda()
    ch.set_proposal(scores=scores, beta=2.0, eps_uniform=0.2, refresh=3, rank=True)
    recs = step_records(ch.run(256, np.full(60, 5e-5), LPF_PROP_LEARNED))
    torch.cuda.synchronize()
    img = _unpack(ch.bits, 32, 32)
    assert int(img.sum()) == int(cell.sum())
    want = oracle.s2(img, 10, 10, 3)
    assert np.array_equal(ch.counts.cpu().numpy().astype(np.uint32), want)
    e = oracle.lse(want, target, 32 * 32, tgt.size)
    assert abs(float(ch.e.cpu()[0]) - e) <= 1e-12 * max(1.0, e)
    assert (recs["k"] >= 0).sum() > 5
    ch.close()
