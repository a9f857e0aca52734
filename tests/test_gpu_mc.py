"""Monte-Carlo approximation on the GPU (lpf_full_sampled, sampled annealing chains) against the
CPU oracle: counts bit for bit, chains step for step."""
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


def _unpack(bits, W, H):
    b = bits.cpu().numpy().view(np.uint64).reshape(H, -1)
    out = np.zeros((H, W), np.uint8)
    for x in range(W):
        out[:, x] = (b[:, x // 64] >> np.uint64(x % 64)) & np.uint64(1)
    return out


def _grid_from_half(half, cx, cy):
    v = oracle.vectors(cx, cy).astype(int)
    g = np.zeros((half.shape[0], 2 * cy + 1, 2 * cx + 1), np.uint32)
    for p in range(half.shape[0]):
        g[p, v[:, 1] + cy, v[:, 0] + cx] = half[p]
        g[p, cy - v[:, 1], cx - v[:, 0]] = half[p]
    return g


CASES = [(1, 1, 0, 0, 1), (7, 1, 6, 0, 3), (1, 9, 0, 8, 4), (37, 23, 36, 22, 50),
         (64, 64, 16, 16, 1), (64, 64, 16, 16, 4096), (130, 70, 40, 30, 700),
         (100, 100, 99, 99, 100), (256, 256, 64, 64, 500)]


@pytest.mark.parametrize("W,H,cx,cy,n", CASES)
def test_sampled_matches_oracle(ctx, W, H, cx, cy, n):
    import torch
    print(f"[gpu] sampled {W}x{H} c=({cx},{cy}) n={n}", flush=True)
    img = wl.boolean_disks(W, H, 3.0, 0.45, W + H) if W * H > 100 else wl.random_binary(W, H, 0.5, 3)
    X = wl.sample_positions(W, H, n, W * H + n)
    bits, sb = ctx.pack(_dev(img)), ctx.pack(_dev(X))
    want = oracle.lpf_sampled(img, cx, cy, X, 3)
    for mask in (1, 2, 3):
        sel = {1: [0], 2: [1], 3: [0, 1]}[mask]
        got = ctx.full_sampled(bits, W, H, cx, cy, sb, mask, 0)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy().astype(np.uint32), want[sel]), mask
    grid = ctx.full_sampled(bits, W, H, cx, cy, sb, 3, 1)
    torch.cuda.synchronize()
    assert np.array_equal(grid.cpu().numpy().astype(np.uint32), _grid_from_half(want, cx, cy))


def test_sampled_full_set_equals_full_and_sets_add_up(ctx):
    import torch
    print("[gpu] sampled 512x512 c=128 additivity", flush=True)
    img = wl.rsa_512()
    bits = ctx.pack(_dev(img))
    full = ctx.full(bits, 512, 512, 128, 128, 3)
    ones = ctx.pack(_dev(np.ones((512, 512), np.uint8)))
    assert torch.equal(ctx.full_sampled(bits, 512, 512, 128, 128, ones, 3), full)
    part = np.random.default_rng(1).integers(0, 3, (512, 512))
    tot = sum(ctx.full_sampled(bits, 512, 512, 128, 128,
                               ctx.pack(_dev((part == k).astype(np.uint8))), 3).long()
              for k in range(3))
    torch.cuda.synchronize()
    assert torch.equal(tot, full.long())


def test_sampled_row_tiled_image(ctx):
    # an image needing several row tiles (LDS count slots), with a 30-position set
    import torch
    print("[gpu] sampled 1024x512 c=300 (row tiles)", flush=True)
    img = wl.boolean_disks(1024, 512, 6.0, 0.35, 12)
    X = wl.sample_positions(1024, 512, 30, 13)
    bits, sb = ctx.pack(_dev(img)), ctx.pack(_dev(X))
    got = ctx.full_sampled(bits, 1024, 512, 300, 300, sb, 3)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().astype(np.uint32),
                          oracle.lpf_sampled(img, 300, 300, X, 3))


def _chain(ctx, cell, c, mask, target, Nt, seed, X):
    import torch
    from paper_1601_04359_amd import Anneal
    H, W = cell.shape
    return Anneal(ctx, ctx.pack(_dev(cell)), W, H, c, c, mask, _dev(target.astype(np.int32)),
                  Nt, seed, sample=ctx.pack(_dev(X)))


@pytest.mark.parametrize("n_cell,mask,K,proposal", [(10, 3, 64, 0), (100, 3, 200, 0),
                                                    (144, 2, 64, 1), (50, 1, 333, 0)])
def test_sampled_chain_matches_oracle(ctx, n_cell, mask, K, proposal):
    import torch
    from paper_1601_04359_amd import LPF_DELTA_RECORDS, step_records
    print(f"[gpu] sampled chain n={n_cell} mask={mask} K={K} proposal={proposal}", flush=True)
    tgt = wl.checkerboard(40, 40, 5)
    Xt = wl.sample_positions(40, 40, 400, 1)
    c = 5
    target = oracle.lpf_sampled(tgt, c, c, Xt, mask)
    cell = wl.random_cell(12, 12, 72, 2)
    Xc = wl.sample_positions(12, 12, n_cell, 3)
    Ts = 1e-3 * 0.9 ** np.arange(40)
    ch = _chain(ctx, cell, c, mask, target, 400, 17, Xc)
    assert ch.method == LPF_DELTA_RECORDS
    recs = step_records(ch.run(K, Ts, proposal))
    torch.cuda.synchronize()
    ref = oracle.AnnealState(cell, c, c, mask, target, 400, 17, sample=Xc)
    rres = ref.run(40, K, Ts, proposal)
    assert np.array_equal(recs[["k", "a", "b"]], rres[["k", "a", "b"]])
    assert np.array_equal(recs["de"], rres["de"]) and np.array_equal(recs["e"], rres["e"])
    assert np.array_equal(_unpack(ch.bits, 12, 12), ref.img)
    assert np.array_equal(ch.counts.cpu().numpy().astype(np.uint32), ref.counts)
    assert (recs["k"] >= 0).sum() > 3
    ch.close()


def test_full_position_set_chain_equals_plain_chain(ctx):
    # X = every pixel: the sampled chain is the entire-function chain, step for step
    import torch
    from paper_1601_04359_amd import Anneal, step_records
    print("[gpu] sampled chain with every position", flush=True)
    tgt = wl.boolean_disks(48, 48, 3.0, 0.4, 21)
    target = oracle.lpf(tgt, 5, 5, 3)
    cell = wl.random_cell(16, 16, int(0.4 * 256), 22)
    Ts = 3e-4 * 0.93 ** np.arange(50)
    a = _chain(ctx, cell, 5, 3, target, tgt.size, 99, np.ones((16, 16), np.uint8))
    b = Anneal(ctx, ctx.pack(_dev(cell)), 16, 16, 5, 5, 3, _dev(target.astype(np.int32)),
               tgt.size, 99)
    ra, rb = step_records(a.run(64, Ts)), step_records(b.run(64, Ts))
    torch.cuda.synchronize()
    assert np.array_equal(ra, rb)
    assert torch.equal(a.counts, b.counts) and torch.equal(a.bits, b.bits)
    a.close()
    b.close()


def test_sampled_delta_energy_exact(ctx):
    import torch
    print("[gpu] sampled delta energy", flush=True)
    tgt = wl.square_particles(40, 40, 4, 16, 3)
    Xt = wl.sample_positions(40, 40, 300, 4)
    c = 6
    target = oracle.lpf_sampled(tgt, c, c, Xt, 3)
    cell = wl.random_cell(20, 20, 64, 5)
    Xc = wl.sample_positions(20, 20, 37, 6)
    ch = _chain(ctx, cell, c, 3, target, 300, 1, Xc)
    rng = np.random.default_rng(7)
    ones, zeros = np.flatnonzero(cell.ravel() == 1), np.flatnonzero(cell.ravel() == 0)
    sw = np.stack([rng.choice(ones, 50), rng.choice(zeros, 50)], 1).astype(np.int32)
    de = ch.delta_energy(_dev(sw)).cpu().numpy()
    base = oracle.lpf_sampled(cell, c, c, Xc, 3).astype(np.int64)
    dl = oracle.delta_swap_sampled(cell, c, c, Xc, sw, 3).astype(np.int64)
    N, Nt, T = 37, 300, target.astype(np.int64)
    for i in range(len(sw)):
        S = int(np.sum(dl[i] * (Nt * (dl[i] + 2 * base) - 2 * N * T)))
        assert de[i] == S / (N * N * Nt)
    ch.close()


def test_sampled_chain_rejects_recount_and_large_cutoff(ctx):
    import torch
    from paper_1601_04359_amd import LPF_DELTA_RECOUNT, LpfError
    cell = wl.random_cell(16, 16, 100, 1)
    X = wl.sample_positions(16, 16, 20, 2)
    t = np.zeros((2, oracle.num_vectors(5, 5)), np.uint32)
    ch = _chain(ctx, cell, 5, 3, t, 100, 1, X)
    with pytest.raises(LpfError):
        ch.set_method(LPF_DELTA_RECOUNT)
    ch.close()
    big = wl.random_cell(300, 300, 40000, 3)
    t2 = np.zeros((2, oracle.num_vectors(127, 127)), np.uint32)
    with pytest.raises(LpfError):
        _chain(ctx, big, 127, 3, t2, 100, 1, wl.sample_positions(300, 300, 10, 4))
