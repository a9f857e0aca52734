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
    # uneven sizes up to 512 with cutoff side/2 (several row tiles for the largest): every image
    # against lpf_full (itself oracle-checked), and sampled vectors against the oracle
    import torch
    print("[gpu] batch large mixed", flush=True)
    spec = wl.batch_spec(12, seed=77, sides=(64, 128, 256, 512))
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
