"""GPU parity of lpf_pack / lpf_full against the CPU oracle (bit-exact integer counts)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import brute
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


def _gpu_counts(ctx, img, cx, cy, mask=3, layout=0):
    import torch
    H, W = img.shape
    t = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    bits = ctx.pack(t)
    out = ctx.full(bits, W, H, cx, cy, mask, layout)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.uint32)


def _announce(name):
    print(f"[gpu] {name}", flush=True)


def test_pack_layout(ctx):
    import torch
    _announce("pack layout")
    for (H, W) in [(1, 1), (3, 64), (5, 65), (7, 130), (64, 64), (9, 200)]:
        img = wl.random_binary(W, H, 0.5, W * 31 + H)
        bits = ctx.pack(torch.from_numpy(img).cuda()).cpu().numpy().view(np.uint64)
        wpr = (W + 63) // 64
        ref = np.zeros((H, wpr), np.uint64)
        for y in range(H):
            for x in range(W):
                if img[y, x]:
                    ref[y, x // 64] |= np.uint64(1) << np.uint64(x % 64)
        assert np.array_equal(bits, ref), (H, W)


def test_small_boolean_64_grid(ctx):
    _announce("64x64 boolean, cutoff 16, grid layout")
    img = wl.small_boolean_64()
    got = _gpu_counts(ctx, img, 16, 16, 3, 1)
    ref = oracle.lpf(img, 16, 16, 3, layout=1)
    assert np.array_equal(got, ref)
    got_h = _gpu_counts(ctx, img, 16, 16, 3, 0)
    assert np.array_equal(got_h, oracle.lpf(img, 16, 16, 3, layout=0))


@pytest.mark.parametrize("seed", range(1, 4))
def test_small_boolean_64_more_seeds(ctx, seed):
    img = wl.small_boolean_64(1601 + seed)
    assert np.array_equal(_gpu_counts(ctx, img, 16, 16), oracle.lpf(img, 16, 16, 3))


@pytest.mark.parametrize("H,W,cx,cy", [
    (1, 1, 0, 0), (1, 7, 6, 0), (9, 1, 0, 8), (5, 7, 6, 4), (23, 37, 36, 22), (31, 33, 32, 30),
    (50, 50, 49, 49), (64, 96, 95, 63), (70, 130, 40, 30), (40, 200, 199, 39), (100, 100, 99, 99),
])
def test_ragged_full_domain(ctx, H, W, cx, cy):
    _announce(f"ragged {H}x{W} c=({cx},{cy})")
    img = wl.random_binary(W, H, 0.62, 1000 * H + W)
    got = _gpu_counts(ctx, img, cx, cy)
    ref = oracle.lpf(img, cx, cy, 3)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("mask", [1, 2])
def test_single_phase(ctx, mask):
    img = wl.boolean_disks(96, 80, 5.0, 0.4, 7)
    assert np.array_equal(_gpu_counts(ctx, img, 30, 25, mask), oracle.lpf(img, 30, 25, mask))


def test_brute_tiny(ctx):
    # the independent brute force, directly against the GPU
    for s in range(4):
        img = wl.random_binary(8, 8, 0.3 + 0.1 * s, 500 + s)
        assert np.array_equal(_gpu_counts(ctx, img, 7, 7), brute.lpf(img, 7, 7, 3))


@pytest.mark.parametrize("shape", [(1, 8, 0, 0), (2, 4, 0, 0), (4, 2, 2, 8192), (8, 1, 0, 0),
                                   (16, 1, 8, 16384), (2, 0, 4, 0), (1, 0, 1, 0), (8, 4, 3, 0)])
def test_forced_tile_shapes(ctx, shape):
    # every lane layout and the multi-tile path (small LDS budget) give the same counts
    R, S, wpg, lds = shape  # the image is 200 px wide: 7 words per row
    _announce(f"tile shape R={R} S={S} wpg={wpg} lds={lds}")
    img = wl.boolean_disks(200, 150, 6.0, 0.45, 99)
    ref = oracle.lpf(img, 40, 37, 3)
    try:
        ctx.set_full_shape(R, S, wpg, lds)
        got = _gpu_counts(ctx, img, 40, 37)
    finally:
        ctx.set_full_shape(0, 0, 0, 0)
    assert np.array_equal(got, ref)


def test_forced_shape_too_narrow(ctx):
    from paper_1601_04359_amd import LpfError
    img = wl.boolean_disks(200, 150, 6.0, 0.45, 99)
    try:
        ctx.set_full_shape(1, 1, 0, 0)
        with pytest.raises(LpfError):
            _gpu_counts(ctx, img, 40, 37)
    finally:
        ctx.set_full_shape(0, 0, 0, 0)


def test_multi_tile_grid(ctx):
    img = wl.boolean_disks(160, 300, 4.0, 0.5, 5)
    try:
        ctx.set_full_shape(0, 0, 0, 8192)
        got = _gpu_counts(ctx, img, 20, 60, 3, 1)
    finally:
        ctx.set_full_shape(0, 0, 0, 0)
    assert np.array_equal(got, oracle.lpf(img, 20, 60, 3, layout=1))


def test_deterministic(ctx):
    img = wl.boolean_disks(128, 128, 5.0, 0.5, 3)
    a = _gpu_counts(ctx, img, 32, 32)
    b = _gpu_counts(ctx, img, 32, 32)
    assert np.array_equal(a, b)


def _property_checks(img, got, cx, cy):
    H, W = img.shape
    v = oracle.vectors(cx, cy)
    unit = np.max(np.abs(v), axis=1) <= 1
    for ph in (0, 1):
        s2 = brute.s2_fft(img, ph)
        ref = s2[v[:, 1] % H, v[:, 0] % W]
        assert got[ph, 0] == int((img == ph).sum())           # eq. (l2zero)
        assert np.array_equal(got[ph, unit], ref[unit])        # unit steps = N S2
        assert np.all(got[ph].astype(np.int64) <= ref)         # L <= N S2


def test_rsa_512_cutoff_128(ctx):
    # the 512 x 512, cutoff 128 workload at full size, in the benchmark's launch configuration:
    # every one of the 33 025 x 2 counts against the oracle (about a minute on 16 host threads)
    _announce("512x512 rsa disks, cutoff 128, all vectors against the oracle")
    img = wl.rsa_512()
    got = _gpu_counts(ctx, img, 128, 128)
    ref = oracle.lpf(img, 128, 128, 3)
    assert np.array_equal(got, ref), int((got != ref).sum())
    _property_checks(img, got, 128, 128)


def test_tiled_large_image(ctx):
    # 1024 x 1024 images with cutoff 255 and 512 (several row tiles): tiling pins of every vector
    # and sampled oracle vectors of a disk image
    _announce("1024x1024 cutoff 512 (row tiles)")
    small = wl.boolean_disks(256, 256, 9.0, 0.4, 17)
    img = np.tile(small, (4, 4))
    got = _gpu_counts(ctx, img, 255, 255)
    v = oracle.vectors(255, 255)
    g = np.random.default_rng(5)
    idx = np.unique(np.concatenate([g.choice(len(v), 60, replace=False), [0, len(v) - 1]]))
    sub = oracle.lpf_vectors(small, v[idx], 3).astype(np.int64)
    assert np.array_equal(got[:, idx].astype(np.int64), 16 * sub)
    # 1024 x 1024 at cutoff 512 = a 256 (wide) x 64 (tall) tile repeated 4 x 16 times: every one
    # of the 525 313 x 2 counts is 64 times the tile's (periodicity), the tile's from the oracle
    tile = wl.boolean_disks(256, 64, 6.0, 0.4, 29)
    got = _gpu_counts(ctx, np.tile(tile, (16, 4)), 512, 512)
    sub = oracle.lpf_vectors(tile, oracle.vectors(512, 512), 3).astype(np.int64)
    assert np.array_equal(got.astype(np.int64), 64 * sub)
    big = wl.boolean_disks(1024, 1024, 7.0, 0.35, 23)
    got = _gpu_counts(ctx, big, 512, 512)
    v = oracle.vectors(512, 512)
    idx = np.unique(np.concatenate([g.choice(len(v), 40, replace=False), [0, 1, len(v) - 1]]))
    assert np.array_equal(got[:, idx], oracle.lpf_vectors(big, v[idx], 3))
    _property_checks(big, got, 512, 512)


def _both(ctx, img, cx, cy, mask=3, layout=0):
    import torch
    H, W = img.shape
    bits = ctx.pack(torch.from_numpy(np.ascontiguousarray(img)).cuda())
    std = ctx.full(bits, W, H, cx, cy, mask, layout)
    enh = ctx.full_enhanced(bits, W, H, cx, cy, mask, layout)
    torch.cuda.synchronize()
    return std.cpu().numpy(), enh.cpu().numpy()


@pytest.mark.parametrize("mask", [1, 2, 3])
def test_enhanced_equals_standard_rsa_512(ctx, mask):
    # the enhanced evaluation (segments abandoned per wave once nothing can still count) gives
    # the standard counts bit for bit on the benchmark image, for every phase mask
    _announce(f"enhanced 512x512 cutoff 128 mask {mask}")
    std, enh = _both(ctx, wl.rsa_512(), 128, 128, mask)
    assert np.array_equal(std, enh)


@pytest.mark.parametrize("name", ["checker", "stripes", "random", "boolean_ragged", "grid"])
def test_enhanced_equals_standard_shapes(ctx, name):
    _announce(f"enhanced {name}")
    if name == "checker":
        img, c = wl.checkerboard(200, 160, 10), (60, 60)
    elif name == "stripes":
        img, c = wl.stripes(192, 96, 24, 7), (90, 40)
    elif name == "random":
        img, c = wl.random_binary(150, 90, 0.5, 4), (40, 30)
    elif name == "boolean_ragged":
        img, c = wl.boolean_disks(333, 257, 5.0, 0.45, 9), (100, 80)
    else:
        img, c = wl.small_boolean_64(), (16, 16)
    layout = 1 if name == "grid" else 0
    std, enh = _both(ctx, img, c[0], c[1], 3, layout)
    assert np.array_equal(std, enh)
    if name in ("grid", "random"):
        assert np.array_equal(enh.astype(np.uint32), oracle.lpf(img, c[0], c[1], 3, layout=layout))


def test_enhanced_tiled(ctx):
    # several row tiles (forced small staging budget) and a large cutoff
    _announce("enhanced tiled 1024x512 cutoff 300")
    img = wl.boolean_disks(1024, 512, 6.0, 0.3, 31)
    try:
        ctx.set_full_shape(0, 0, 0, 65536)
        std, enh = _both(ctx, img, 300, 300)
    finally:
        ctx.set_full_shape(0, 0, 0, 0)
    assert np.array_equal(std, enh)


def test_rows_from_device_memory_forced(ctx):
    # a staging budget that cannot hold a row tile and its halo makes the kernel read rows of the
    # extended image from device memory: same counts, standard, enhanced and sampled
    _announce("rows from device memory (forced), 200x150 cutoff (40, 37)")
    import torch
    img = wl.boolean_disks(200, 150, 6.0, 0.45, 99)
    ref = oracle.lpf(img, 40, 37, 3)
    sample = wl.sample_positions(200, 150, 3000, 8)
    bits = ctx.pack(torch.from_numpy(img).cuda())
    sbits = ctx.pack(torch.from_numpy(sample).cuda())
    try:
        ctx.set_full_shape(0, 0, 0, 1)
        std, enh = _both(ctx, img, 40, 37)
        smp = ctx.full_sampled(bits, 200, 150, 40, 37, sbits, 3)
        torch.cuda.synchronize()
    finally:
        ctx.set_full_shape(0, 0, 0, 0)
    assert np.array_equal(std.astype(np.uint32), ref)
    assert np.array_equal(enh.astype(np.uint32), ref)
    assert np.array_equal(smp.cpu().numpy().astype(np.uint32),
                          oracle.lpf_sampled(img, 40, 37, sample, 3))


def test_full_domain_1024(ctx):
    # the paper's whole domain (cutoff W - 1) at 1024 x 1024: the halo rows exceed LDS, so rows
    # come from device memory.  The image is a 512 x 512 disk image tiled 2 x 2: every vector
    # within the 512 image's own domain has 4 times that image's count (the 512 run stages its
    # rows in LDS); longer vectors are checked on samples against the oracle, all by properties
    _announce("1024x1024 full domain (cutoff 1023), rows from device memory")
    small = wl.boolean_disks(512, 512, 8.0, 0.4, 41)
    img = np.tile(small, (2, 2))
    got = _gpu_counts(ctx, img, 1023, 1023)
    sub = _gpu_counts(ctx, small, 511, 511)
    v = oracle.vectors(1023, 1023)
    inner = (np.abs(v[:, 0]) <= 511) & (v[:, 1] <= 511)
    vi = v[inner].astype(np.int64)
    pos = np.where(vi[:, 0] >= 0, vi[:, 1] * 512 + vi[:, 0],
                   512 * 512 + (vi[:, 1] - 1) * 511 + vi[:, 0] + 511)
    assert np.array_equal(got[:, inner].astype(np.int64), 4 * sub[:, pos].astype(np.int64))
    g = np.random.default_rng(12)
    far = np.flatnonzero(~inner)
    idx = np.unique(np.concatenate([g.choice(far, 40, replace=False), [len(v) - 1], far[:3]]))
    assert np.array_equal(got[:, idx], oracle.lpf_vectors(img, v[idx], 3))
    sv = oracle.vectors(511, 511)
    sidx = g.choice(len(sv), 30, replace=False)
    assert np.array_equal(sub[:, sidx], oracle.lpf_vectors(small, sv[sidx], 3))
    _property_checks(img, got, 1023, 1023)


def test_cutoff_beyond_int16_is_refused(ctx):
    # vectors are int16: a cutoff above 32767 must fail before any launch, not wrap
    import torch
    from paper_1601_04359_amd import LpfError
    W = 40000
    bits = ctx.pack(torch.zeros((1, W), dtype=torch.uint8, device="cuda"))
    with pytest.raises(LpfError) as e:
        ctx.full(bits, W, 1, 32768, 0, 3)
    assert e.value.status == -95
    with pytest.raises(LpfError):
        ctx.s2(bits, W, 1, 32768, 0, 3)
