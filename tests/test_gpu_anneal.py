"""GPU annealing chain (anneal_step) against the CPU oracle's chain."""
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


def _problem(cell_side, tgt_side, cx, mask, seed, phi=0.4, r=3.0):
    tgt = wl.boolean_disks(tgt_side, tgt_side, r, phi, seed)
    target = oracle.lpf(tgt, cx, cx, mask)
    cell = wl.random_cell(cell_side, cell_side, int(round(phi * cell_side * cell_side)), seed + 1)
    return tgt, target, cell


METHODS = {"recount": 1, "records": 2}


def _gpu_chain(ctx, cell, cx, mask, target, Nt, seed, step0=0, pos=None, n1=0, method=0, cy=None):
    import torch
    from paper_1601_04359_amd import Anneal
    H, W = cell.shape
    bits = ctx.pack(torch.from_numpy(cell).cuda())
    t = torch.from_numpy(target.astype(np.int32)).cuda()
    ch = Anneal(ctx, bits, W, H, cx, cx if cy is None else cy, mask, t, Nt, seed, step0, pos, n1)
    if method:
        ch.set_method(method)
        assert ch.method == method
    return ch


def _unpack(bits, W, H):
    b = bits.cpu().numpy().view(np.uint64).reshape(H, -1)
    out = np.zeros((H, W), np.uint8)
    for x in range(W):
        out[:, x] = (b[:, x // 64] >> np.uint64(x % 64)) & np.uint64(1)
    return out


@pytest.mark.parametrize("method", ["recount", "records"])
@pytest.mark.parametrize("proposal,mask,K", [(0, 3, 64), (1, 3, 200), (0, 2, 64), (0, 1, 333)])
def test_chain_matches_oracle(ctx, proposal, mask, K, method):
    import torch
    from paper_1601_04359_amd import step_records
    print(f"[gpu] anneal chain proposal={proposal} mask={mask} K={K} {method}", flush=True)
    tgt, target, cell = _problem(16, 48, 5, mask, 21)
    seed, nsteps = 99, 60
    Ts = 3e-4 * 0.93 ** np.arange(nsteps)
    ch = _gpu_chain(ctx, cell, 5, mask, target, tgt.size, seed, method=METHODS[method])
    recs = step_records(ch.run(K, Ts, proposal))
    torch.cuda.synchronize()
    ref = oracle.AnnealState(cell, 5, 5, mask, target, tgt.size, seed)
    e0 = ref.e
    rres = ref.run(nsteps, K, Ts, proposal)
    got = [(int(r["k"]), int(r["a"]), int(r["b"])) for r in recs]
    want = [(int(r["k"]), int(r["a"]), int(r["b"])) for r in rres]
    assert got == want
    assert np.array_equal(recs["step"], np.arange(nsteps))
    assert np.array_equal(recs["de"], rres["de"]) and np.array_equal(recs["e"], rres["e"])
    assert sum(k >= 0 for k, _, _ in got) > 5
    assert np.array_equal(_unpack(ch.bits, 16, 16), ref.img)
    assert np.array_equal(ch.counts.cpu().numpy().astype(np.uint32), ref.counts)
    assert float(ch.e.cpu()[0]) == ref.e
    assert ref.e < e0
    ch.close()


def test_resume_from_export(ctx):
    import torch
    from paper_1601_04359_amd import step_records
    tgt, target, cell = _problem(16, 48, 4, 3, 31)
    seed, K = 5, 32
    Ts = np.full(40, 2e-4)
    one = _gpu_chain(ctx, cell, 4, 3, target, tgt.size, seed)
    r_all = step_records(one.run(K, Ts))
    first = _gpu_chain(ctx, cell, 4, 3, target, tgt.size, seed)
    r_a = step_records(first.run(K, Ts[:20]))
    pos, n1, nxt = first.export()
    assert nxt == 20
    second = _gpu_chain(ctx, _unpack(first.bits, 16, 16), 4, 3, target, tgt.size, seed,
                        step0=nxt, pos=pos, n1=n1)
    second.e.copy_(first.e)
    r_b = step_records(second.run(K, Ts[20:]))
    torch.cuda.synchronize()
    both = np.concatenate([r_a, r_b])
    assert np.array_equal(both[["k", "a", "b"]], r_all[["k", "a", "b"]])
    assert np.array_equal(second.bits.cpu(), one.bits.cpu())
    assert np.array_equal(second.counts.cpu(), one.counts.cpu())
    for c in (one, first, second):
        c.close()


@pytest.mark.parametrize("method", ["recount", "records"])
def test_ragged_cell_long_vectors(ctx, method):
    # a 21 x 17 cell with cutoffs (20, 16): segments wrap around the cell and many candidates
    # have both pixels on one placement's segment; chain equals the oracle's
    import torch
    from paper_1601_04359_amd import step_records
    print(f"[gpu] anneal ragged 21x17 c=(20,16) {method}", flush=True)
    tgt = wl.boolean_disks(40, 40, 3.0, 0.45, 7)
    target = oracle.lpf(tgt, 20, 16, 3)
    cell = wl.random_cell(21, 17, int(round(0.45 * 21 * 17)), 8)
    Ts = 2e-3 * 0.9 ** np.arange(30)
    ch = _gpu_chain(ctx, cell, 20, 3, target, tgt.size, 4, method=METHODS[method], cy=16)
    recs = step_records(ch.run(100, Ts))
    torch.cuda.synchronize()
    ref = oracle.AnnealState(cell, 20, 16, 3, target, tgt.size, 4)
    rres = ref.run(30, 100, Ts)
    assert [(int(r["k"]), int(r["a"]), int(r["b"])) for r in recs] == \
        [(int(r["k"]), int(r["a"]), int(r["b"])) for r in rres]
    assert np.array_equal(recs["de"], rres["de"])
    assert np.array_equal(ch.counts.cpu().numpy().astype(np.uint32), ref.counts)
    ch.close()


def test_records_long_paths(ctx):
    # cutoff (80, 1) on a 150 x 40 cell: paths of up to 81 pixels, longer than one wave, take the
    # bit-by-bit record update; the shorter ones the merged one; K = 70 runs round 0 in the launch
    # of the draws and a second round of 6.  Started from a crop of the target at T ~ 0, this seed
    # has steps accepted in round 0, steps accepted in round 1 and steps with no acceptance.
    import torch
    from paper_1601_04359_amd import step_records
    print("[gpu] anneal records long paths 150x40 c=(80,1)", flush=True)
    tgt = wl.boolean_disks(300, 80, 3.0, 0.4, 17)
    target = oracle.lpf(tgt, 80, 1, 3)
    cell = np.ascontiguousarray(tgt[:40, :150])
    Ts = np.full(60, 1e-9)
    ch = _gpu_chain(ctx, cell, 80, 3, target, tgt.size, 16, method=METHODS["records"], cy=1)
    recs = step_records(ch.run(70, Ts))
    torch.cuda.synchronize()
    ref = oracle.AnnealState(cell, 80, 1, 3, target, tgt.size, 16)
    rres = ref.run(60, 70, Ts)
    assert [(int(r["k"]), int(r["a"]), int(r["b"])) for r in recs] == \
        [(int(r["k"]), int(r["a"]), int(r["b"])) for r in rres]
    assert np.array_equal(recs["de"], rres["de"])
    k = recs["k"]
    assert (k >= 64).sum() >= 1 and (k < 0).sum() >= 1 and ((k >= 0) & (k < 64)).sum() >= 20
    assert np.array_equal(ch.counts.cpu().numpy().astype(np.uint32), ref.counts)
    # the records after the updates still give the exact change of further interchanges
    img = _unpack(ch.bits, 150, 40)
    rng = np.random.default_rng(3)
    ones, zeros = np.flatnonzero(img.ravel() == 1), np.flatnonzero(img.ravel() == 0)
    sw = np.stack([rng.choice(ones, 20), rng.choice(zeros, 20)], 1).astype(np.int32)
    de = ch.delta_energy(torch.from_numpy(sw).cuda()).cpu().numpy()
    base = oracle.lpf(img, 80, 1, 3).astype(np.int64)
    dl = oracle.delta_swap(img, 80, 1, sw, 3).astype(np.int64)
    N, Nt, T = img.size, tgt.size, target.astype(np.int64)
    for i in range(len(sw)):
        S = int(np.sum(dl[i] * (Nt * (dl[i] + 2 * base) - 2 * N * T)))
        assert de[i] == S / (N * N * Nt)
    ch.close()


@pytest.mark.parametrize("method", ["recount", "records"])
def test_three_rounds(ctx, method):
    # K = 9000: rounds of 64, 8192 and 744 (round 0 decided in round 1, round 1 by the middle
    # decision, round 2 at the end of the step).  From a crop of the target at T ~ 0 this seed
    # accepts in round 0 (20 steps), round 1 (47), round 2 (steps 64 and 66) and none (1).
    import torch
    from paper_1601_04359_amd import step_records
    print(f"[gpu] anneal three rounds K=9000 {method}", flush=True)
    tgt = wl.boolean_disks(48, 48, 3.0, 0.4, 21)
    target = oracle.lpf(tgt, 5, 5, 3)
    cell = np.ascontiguousarray(tgt[:16, :16])
    Ts = np.full(70, 1e-12)
    ch = _gpu_chain(ctx, cell, 5, 3, target, tgt.size, 2, method=METHODS[method])
    recs = step_records(ch.run(9000, Ts))
    torch.cuda.synchronize()
    ref = oracle.AnnealState(cell, 5, 5, 3, target, tgt.size, 2)
    rres = ref.run(70, 9000, Ts)
    assert [(int(r["k"]), int(r["a"]), int(r["b"])) for r in recs] == \
        [(int(r["k"]), int(r["a"]), int(r["b"])) for r in rres]
    assert np.array_equal(recs["de"], rres["de"])
    k = recs["k"]
    assert (k >= 8256).sum() >= 1 and ((k >= 64) & (k < 8256)).sum() >= 10 and (k < 0).sum() >= 1
    assert np.array_equal(ch.counts.cpu().numpy().astype(np.uint32), ref.counts)
    ch.close()


def test_records_agree_with_recount(ctx):
    # after many accepted interchanges (incremental record updates), the records method's exact
    # energy changes of random and neighbouring interchanges equal the recount method's, and the
    # counts equal a fresh full evaluation
    import torch
    from paper_1601_04359_amd import LPF_DELTA_RECORDS, LPF_DELTA_RECOUNT
    print("[gpu] anneal records vs recount 48x40 c=(9,7)", flush=True)
    tgt = wl.boolean_disks(96, 96, 4.0, 0.35, 11)
    target = oracle.lpf(tgt, 9, 7, 3)
    cell = wl.random_cell(48, 40, int(round(0.35 * 48 * 40)), 12)
    ch = _gpu_chain(ctx, cell, 9, 3, target, tgt.size, 6, method=LPF_DELTA_RECORDS, cy=7)
    ch.run(64, np.full(300, 1e-2))       # hot: most steps accept
    torch.cuda.synchronize()
    assert torch.equal(ctx.full(ch.bits, 48, 40, 9, 7, 3), ch.counts)
    img = _unpack(ch.bits, 48, 40).ravel()
    g = np.random.default_rng(3)
    ones, zeros = np.flatnonzero(img == 1), np.flatnonzero(img == 0)
    a = g.choice(ones, 600)
    b = g.choice(zeros, 600)
    near = (a[:300] + g.integers(-3, 4, 300) + 48 * g.integers(-3, 4, 300)) % img.size
    b[:300] = np.where(img[near] == 0, near, b[:300])
    sw = torch.from_numpy(np.stack([a, b], 1).astype(np.int32)).cuda()
    de_rec = ch.delta_energy(sw).cpu().numpy()
    ch.set_method(LPF_DELTA_RECOUNT)
    de_cnt = ch.delta_energy(sw).cpu().numpy()
    assert np.array_equal(de_rec, de_cnt)
    # and against the oracle's deltas through the integer energy formula of eq. (LSE)
    swn = sw.cpu().numpy()[:60]
    dl = oracle.delta_swap(_unpack(ch.bits, 48, 40), 9, 7, swn, 3).astype(object)
    L = ch.counts.cpu().numpy().astype(object)
    T = target.astype(object)
    N, Nt = 48 * 40, tgt.size
    for i in range(len(swn)):
        S = int(np.sum(dl[i] * (Nt * (dl[i] + 2 * L) - 2 * N * T)))
        assert de_rec[i] == float(S) / (float(N) * float(N) * float(Nt)), i
    ch.close()


@pytest.mark.parametrize("method", ["recount", "records"])
def test_reconstruction_cell_128_c32(ctx, method):
    # the reconstruction workload's shapes: 128 x 128 cell, phase-1 LPF with cutoff 32 of a
    # 1024 x 1024 disk image (phi 0.35, r 6), 4096 candidates per step.  Drift guard: the
    # incrementally updated counts equal a fresh lpf_full of the cell; the running energy equals
    # eq. (LSE) recomputed by the oracle; the first step agrees with the oracle's chain.
    import torch
    from paper_1601_04359_amd import step_records
    print(f"[gpu] anneal 128x128 c=32 K=4096 {method}", flush=True)
    tgt = wl.anneal_target()
    bt = torch.from_numpy(tgt).cuda()
    target = ctx.full(ctx.pack(bt), 1024, 1024, 32, 32, 2)
    cell = wl.random_cell(128, 128, int(round(0.35 * 128 * 128)), 1)
    ch = _gpu_chain(ctx, cell, 32, 2, target.cpu().numpy(), 1024 * 1024, 1, method=METHODS[method])
    Ts = 1e-3 * (0.01 ** (1 / 20000)) ** np.arange(12)
    recs = step_records(ch.run(4096, Ts))
    torch.cuda.synchronize()
    fresh = ctx.full(ch.bits, 128, 128, 32, 32, 2)
    assert torch.equal(fresh, ch.counts)
    img = _unpack(ch.bits, 128, 128)
    assert int(img.sum()) == int(cell.sum())
    e = oracle.lse(ch.counts.cpu().numpy(), target.cpu().numpy(), 128 * 128, 1024 * 1024)
    assert abs(float(ch.e.cpu()[0]) - e) <= 1e-12 * e
    assert (recs["k"] >= 0).sum() > 0
    # all 12 steps against the oracle's chain with the same K = 4096 draws per step (the oracle
    # evaluates each step's draws in order up to the first accepted one), its target counts its own
    ref = oracle.AnnealState(cell, 32, 32, 2, oracle.lpf(tgt, 32, 32, 2), 1024 * 1024, 1)
    r = ref.run(12, 4096, Ts)
    for f in ("k", "a", "b"):
        assert np.array_equal(r[f], recs[f]), f
    assert np.array_equal(r["de"], recs["de"]) and np.array_equal(r["e"], recs["e"])
    ch.close()
