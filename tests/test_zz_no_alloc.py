"""lpf_full_noalloc (the entry point that allocates nothing) against lpf_full through the C ABI:
bit-equal counts on two calls in a row, the second on a smaller image, so the second call runs
on a fixed scratch array that still holds the first call's extended image."""
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


def _both(ctx, img, cx, cy, mask, layout):
    import torch
    from paper_1601_04359_amd import _abi
    H, W = img.shape
    bits = ctx.pack(torch.from_numpy(np.ascontiguousarray(img)).cuda())
    shp = _abi.counts_shape(cx, cy, mask, layout)
    ref = torch.full(shp, -1, dtype=torch.int32, device="cuda")
    got = torch.full(shp, -7, dtype=torch.int32, device="cuda")
    _abi.lpf_full(ctx.handle, bits, W, H, cx, cy, mask, layout, ref)
    _abi.lpf_full_noalloc(ctx.handle, bits, W, H, cx, cy, mask, layout, got)
    torch.cuda.synchronize()
    return got.cpu().numpy().astype(np.uint32), ref.cpu().numpy().astype(np.uint32)


def test_noalloc_equals_full_two_calls_second_smaller(ctx):
    print("[gpu] no-alloc: 512x512 RSA cutoff 128 both phases, then 37x29 cutoff (9, 11) grid",
          flush=True)
    big = wl.rsa_512()
    got, ref = _both(ctx, big, 128, 128, 3, 0)
    assert np.array_equal(got, ref)
    # sampled oracle vectors of the large call (every 97th canonical vector)
    v = oracle.vectors(128, 128)
    idx = np.arange(0, len(v), 97)
    exp = oracle.lpf_vectors(big, v[idx], 3)
    assert np.array_equal(got[:, idx], exp)
    small = wl.random_binary(37, 29, 0.45, 4242)
    got, ref = _both(ctx, small, 9, 11, 3, 1)
    assert np.array_equal(got, ref)
    assert np.array_equal(got, oracle.lpf(small, 9, 11, 3, layout=1))


def test_noalloc_row_tiles_and_single_phase(ctx):
    print("[gpu] no-alloc: 1024x400 cutoff (20, 200) phase 1 (4 row tiles), then 8x8",
          flush=True)
    img = wl.random_binary(1024, 400, 0.6, 77)
    got, ref = _both(ctx, img, 20, 200, 2, 0)
    assert np.array_equal(got, ref)
    tiny = wl.random_binary(8, 8, 0.5, 5)
    got, ref = _both(ctx, tiny, 7, 7, 1, 0)
    assert np.array_equal(got, ref)
    assert np.array_equal(got, oracle.lpf(tiny, 7, 7, 1))


def test_noalloc_rejects_image_beyond_scratch(ctx):
    import torch
    from paper_1601_04359_amd import _abi
    print("[gpu] no-alloc: 8192x8192 rejected before any launch", flush=True)
    W = H = 8192
    bits = torch.zeros(((W + 63) // 64) * H, dtype=torch.int64, device="cuda")
    counts = torch.zeros(_abi.counts_shape(8, 8, 3, 0), dtype=torch.int32, device="cuda")
    with pytest.raises(_abi.LpfError) as ei:
        _abi.lpf_full_noalloc(ctx.handle, bits, W, H, 8, 8, 3, 0, counts)
    assert ei.value.status == _abi.LPF_E_UNSUPPORTED
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert int(counts.abs().sum()) == 0
