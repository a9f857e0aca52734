"""lpf_batch (persistent launch over uneven images, hipGraph replay) and the autotuner."""
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


def _pack(ctx, img):
    import torch
    return ctx.pack(torch.from_numpy(np.ascontiguousarray(img)).cuda())


def test_batch_uneven_small(ctx):
    import torch
    from paper_1601_04359_amd import counts_shape
    print("[gpu] batch uneven small", flush=True)
    sizes = [(16, 16), (37, 23), (64, 64), (1, 5), (100, 40), (33, 70), (128, 128), (8, 8)]
    imgs = [wl.boolean_disks(W, H, 3.0, 0.45, 50 + i) if W > 4 else wl.random_binary(W, H, 0.5, i)
            for i, (W, H) in enumerate(sizes)]
    items = [(_pack(ctx, im), W, H, W // 2, H // 2) for im, (W, H) in zip(imgs, sizes)]
    for layout in (0, 1):
        counts, offs, pool, descs = ctx.batch(items, 3, layout)
        torch.cuda.synchronize()
        c = counts.cpu().numpy().astype(np.uint32)
        for i, (im, (W, H)) in enumerate(zip(imgs, sizes)):
            shp = counts_shape(W // 2, H // 2, 3, layout)
            n = int(np.prod(shp))
            got = c[offs[i]: offs[i] + n].reshape(shp)
            assert np.array_equal(got, oracle.lpf(im, W // 2, H // 2, 3, layout=layout)), (i, layout)


def test_batch_replay_sees_new_contents(ctx):
    # the captured graph is replayed on the same pool; new image contents give new counts
    import torch
    sizes = [(48, 48), (96, 64), (200, 30)]
    imgs = [wl.random_binary(W, H, 0.5, 7 + i) for i, (W, H) in enumerate(sizes)]
    items = [(_pack(ctx, im), W, H, W // 2, H // 2) for im, (W, H) in zip(imgs, sizes)]
    counts, offs, pool, descs = ctx.batch(items, 3, 0)
    from paper_1601_04359_amd import _abi
    for rep in range(3):
        new = [wl.random_binary(W, H, 0.4 + 0.1 * rep, 100 * rep + i) for i, (W, H) in enumerate(sizes)]
        pool.copy_(torch.cat([_pack(ctx, im).reshape(-1) for im in new]))
        _abi.lpf_batch(ctx.handle, pool, descs, 3, 0, counts)
        torch.cuda.synchronize()
        c = counts.cpu().numpy().astype(np.uint32)
        for i, (im, (W, H)) in enumerate(zip(new, sizes)):
            nv = oracle.num_vectors(W // 2, H // 2)
            got = c[offs[i]: offs[i] + 2 * nv].reshape(2, nv)
            assert np.array_equal(got, oracle.lpf(im, W // 2, H // 2, 3)), (rep, i)


def test_batch_large_mixed_against_full(ctx):
    # uneven sizes up to 1024 with cutoff side/2 (several row tiles for the largest): every image
    # against lpf_full (pinned at 1024^2, cutoff 512 by the tiling test), sampled vectors against
    # the oracle
    import torch
    print("[gpu] batch large mixed", flush=True)
    spec = wl.batch_spec(12, seed=77, sides=(64, 128, 256, 512))
    spec.append(wl.batch_spec(1, seed=78, sides=(1024,))[0])  # one 1024 x 1024, cutoff 512
    imgs = [wl.batch_image(b) for b in spec]
    items = [(_pack(ctx, im), b.side, b.side, b.side // 2, b.side // 2) for im, b in zip(imgs, spec)]
    counts, offs, pool, descs = ctx.batch(items, 3, 0)
    torch.cuda.synchronize()
    g = np.random.default_rng(3)
    for i, (im, b) in enumerate(zip(imgs, spec)):
        c = b.side // 2
        nv = oracle.num_vectors(c, c)
        got = counts[offs[i]: offs[i] + 2 * nv].reshape(2, nv)
        ref = ctx.full(items[i][0], b.side, b.side, c, c)
        assert torch.equal(got, ref), i
        v = oracle.vectors(c, c)
        idx = g.choice(nv, 6, replace=False)
        assert np.array_equal(got.cpu().numpy()[:, idx].astype(np.uint32),
                              oracle.lpf_vectors(im, v[idx], 3))


def test_autotune_keeps_counts(ctx):
    import torch
    img = wl.boolean_disks(256, 256, 6.0, 0.4, 5)
    bits = _pack(ctx, img)
    before = ctx.full(bits, 256, 256, 64, 64)
    ms = ctx.autotune(bits, 256, 256, 64, 64)
    R, wpg, lds = ctx.tuned_shape(256, 256, 64, 64)
    assert ms > 0 and R in (2, 4, 8, 16) and wpg in (4, 8, 16) and lds > 0
    after = ctx.full(bits, 256, 256, 64, 64)
    torch.cuda.synchronize()
    assert torch.equal(before, after)


def test_batch_graph_replayed_with_new_buffers(ctx):
    # the captured launch is keyed by the descriptors: new pool and counts tensors (new
    # addresses) replay it, and each call's counts are those of its own images
    import torch
    from paper_1601_04359_amd import _abi
    print("[gpu] batch replay with new buffers", flush=True)
    sizes = [(40, 40), (72, 50), (130, 17)]
    base = [wl.random_binary(W, H, 0.5, 300 + i) for i, (W, H) in enumerate(sizes)]
    items = [(_pack(ctx, im), W, H, W // 3, H // 3) for im, (W, H) in zip(base, sizes)]
    counts0, offs, pool0, descs = ctx.batch(items, 3, 0)
    keep = []
    for rep in range(3):
        new = [wl.random_binary(W, H, 0.35 + 0.1 * rep, 400 + 10 * rep + i)
               for i, (W, H) in enumerate(sizes)]
        pool = torch.cat([_pack(ctx, im).reshape(-1) for im in new]).contiguous()
        counts = torch.full_like(counts0, -1)
        keep.append((pool, counts))  # distinct live allocations, so the addresses differ
        _abi.lpf_batch(ctx.handle, pool, descs, 3, 0, counts)
        torch.cuda.synchronize()
        c = counts.cpu().numpy().astype(np.uint32)
        for i, (im, (W, H)) in enumerate(zip(new, sizes)):
            nv = oracle.num_vectors(W // 3, H // 3)
            got = c[offs[i]: offs[i] + 2 * nv].reshape(2, nv)
            assert np.array_equal(got, oracle.lpf(im, W // 3, H // 3, 3)), (rep, i)


def test_batch_graph_cache_is_bounded(ctx):
    # more distinct descriptor sets than the context keeps: the oldest graphs are released and
    # captured again when their set returns, with the same counts
    import torch
    print("[gpu] batch graph cache bound", flush=True)
    first = None
    for k in range(20):
        W, H = 20 + k, 12
        im = wl.random_binary(W, H, 0.5, 500 + k)
        counts, offs, pool, descs = ctx.batch([(_pack(ctx, im), W, H, 5, 4)], 3, 0)
        torch.cuda.synchronize()
        got = counts.cpu().numpy().astype(np.uint32).reshape(2, -1)
        assert np.array_equal(got, oracle.lpf(im, 5, 4, 3)), k
        if k == 0:
            first = im
    counts, offs, pool, descs = ctx.batch([(_pack(ctx, first), 20, 12, 5, 4)], 3, 0)
    torch.cuda.synchronize()
    assert np.array_equal(counts.cpu().numpy().astype(np.uint32).reshape(2, -1),
                          oracle.lpf(first, 5, 4, 3))


def test_batch_rows_from_device_memory(ctx):
    # every image of the batch reads its rows from device memory (forced staging budget)
    import torch
    print("[gpu] batch with rows from device memory", flush=True)
    sizes = [(64, 64), (100, 40), (37, 23)]
    imgs = [wl.random_binary(W, H, 0.5, 600 + i) for i, (W, H) in enumerate(sizes)]
    items = [(_pack(ctx, im), W, H, W // 2, H // 2) for im, (W, H) in zip(imgs, sizes)]
    try:
        ctx.set_full_shape(0, 0, 0, 1)
        counts, offs, pool, descs = ctx.batch(items, 3, 0)
        torch.cuda.synchronize()
    finally:
        ctx.set_full_shape(0, 0, 0, 0)
    c = counts.cpu().numpy().astype(np.uint32)
    for i, (im, (W, H)) in enumerate(zip(imgs, sizes)):
        nv = oracle.num_vectors(W // 2, H // 2)
        got = c[offs[i]: offs[i] + 2 * nv].reshape(2, nv)
        assert np.array_equal(got, oracle.lpf(im, W // 2, H // 2, 3)), i
