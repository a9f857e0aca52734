"""GPU parity of lpf_delta_swap against the CPU oracle (bit-exact integer deltas)."""
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


def _gpu_delta(ctx, img, cx, cy, swaps, mask=3):
    import torch
    H, W = img.shape
    bits = ctx.pack(torch.from_numpy(np.ascontiguousarray(img)).cuda())
    sw = torch.from_numpy(np.ascontiguousarray(swaps, dtype=np.int32).reshape(-1, 2)).cuda()
    out = ctx.delta_swap(bits, W, H, cx, cy, sw, mask)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _swaps(img, n, seed, near=0):
    g = np.random.default_rng(seed)
    H, W = img.shape
    ones = np.flatnonzero(img.ravel() == 1)
    zeros = np.flatnonzero(img.ravel() == 0)
    a = g.choice(ones, n)
    b = g.choice(zeros, n)
    sw = np.stack([a, b], 1)
    # pairs of nearby pixels (their segments overlap)
    for i in range(min(near, n)):
        ax, ay = a[i] % W, a[i] // W
        for d in range(1, 6):
            q = ((ay + (d % 3)) % H) * W + (ax + d) % W
            if img.flat[q] == 0:
                sw[i, 1] = q
                break
    return sw.astype(np.int32)


@pytest.mark.parametrize("H,W,cx,cy,mask", [
    (7, 9, 8, 6, 3), (12, 12, 11, 11, 3), (17, 33, 20, 16, 3), (30, 20, 19, 12, 2),
    (16, 64, 40, 15, 1), (70, 100, 30, 25, 3), (64, 65, 64, 63, 3), (5, 130, 60, 4, 3),
])
def test_delta_random_and_near(ctx, H, W, cx, cy, mask):
    print(f"[gpu] delta {H}x{W} c=({cx},{cy}) mask={mask}", flush=True)
    img = wl.random_binary(W, H, 0.45, 7 * H + W)
    sw = _swaps(img, 80, H + W, near=30)
    got = _gpu_delta(ctx, img, cx, cy, sw, mask)
    ref = oracle.delta_swap(img, cx, cy, sw, mask)
    assert np.array_equal(got, ref)


def test_delta_edge_cases(ctx):
    img = wl.boolean_disks(40, 36, 4.0, 0.4, 3)
    H, W = img.shape
    ones = np.flatnonzero(img.ravel() == 1)
    zeros = np.flatnonzero(img.ravel() == 0)
    sw = np.array([
        [ones[0], ones[0]],      # a == b
        [ones[0], ones[1]],      # same phase
        [zeros[0], zeros[5]],    # same phase
        [zeros[3], ones[7]],     # reversed order (phase 0 first)
        [-1, ones[2]],           # out of range
        [ones[2], W * H],        # out of range
        [ones[9], zeros[11]],
    ], np.int32)
    got = _gpu_delta(ctx, img, 20, 17, sw, 3)
    ref = oracle.delta_swap(img, 20, 17, np.clip(sw, 0, W * H - 1), 3)
    ref[4:6] = 0
    assert np.array_equal(got, ref)
    assert not got[:3].any()


def test_delta_matches_two_full_evaluations(ctx):
    # the interchange applied to the image and both images evaluated by lpf_full on the GPU
    import torch
    img = wl.boolean_disks(96, 96, 6.0, 0.35, 8)
    sw = _swaps(img, 6, 1)
    d = _gpu_delta(ctx, img, 24, 24, sw, 3).astype(np.int64)
    bits0 = ctx.pack(torch.from_numpy(img).cuda())
    L0 = ctx.full(bits0, 96, 96, 24, 24).cpu().numpy().astype(np.int64)
    for s, (a, b) in enumerate(sw):
        im2 = img.copy().ravel()
        im2[a], im2[b] = im2[b], im2[a]
        bits = ctx.pack(torch.from_numpy(im2.reshape(96, 96)).cuda())
        L1 = ctx.full(bits, 96, 96, 24, 24).cpu().numpy().astype(np.int64)
        assert np.array_equal(L1 - L0, d[s])


def test_delta_anneal_cell_128_c32(ctx):
    # the 128 x 128 cell with cutoff 32 of the reconstruction workload, phase 1 and both phases
    print("[gpu] delta 128x128 c=32", flush=True)
    img = wl.random_cell(128, 128, int(round(0.35 * 128 * 128)), 5)
    sw = _swaps(img, 96, 2, near=16)
    for mask in (2, 3):
        got = _gpu_delta(ctx, img, 32, 32, sw, mask)
        assert np.array_equal(got, oracle.delta_swap(img, 32, 32, sw, mask))


def test_delta_cell_256_c48(ctx):
    print("[gpu] delta 256x256 c=48", flush=True)
    img = wl.boolean_disks(256, 256, 6.0, 0.35, 11)
    sw = _swaps(img, 24, 3, near=6)
    got = _gpu_delta(ctx, img, 48, 48, sw, 3)
    assert np.array_equal(got, oracle.delta_swap(img, 48, 48, sw, 3))


def test_delta_many_candidates(ctx):
    # a 4096-candidate batch (one annealing step's worth) at 128 x 128, cutoff 32, both phases:
    # every row against the oracle, and dL(0,0) = 0 (an interchange keeps the phase counts)
    print("[gpu] delta 128x128 c=32, 4096 candidates, all rows", flush=True)
    img = wl.random_cell(128, 128, 5734, 6)
    sw = _swaps(img, 4096, 9)
    got = _gpu_delta(ctx, img, 32, 32, sw, 3)
    assert not got[:, :, 0].any()
    assert np.array_equal(got, oracle.delta_swap(img, 32, 32, sw, 3))


@pytest.mark.parametrize("H,W,cx,cy,mask,n", [
    (9, 7, 6, 8, 3, 40), (65, 64, 63, 64, 3, 40), (128, 128, 32, 32, 2, 256), (20, 300, 260, 3, 3, 12),
])
def test_delta_runs_method_equal(ctx, H, W, cx, cy, mask, n):
    # the run-based recount (the only one for cutoffs above 255) against the offset rows and the
    # oracle on the same interchanges
    from paper_1601_04359_amd import _abi
    print(f"[gpu] delta runs vs offset rows {H}x{W} c=({cx},{cy}) mask={mask}", flush=True)
    img = wl.random_binary(W, H, 0.5, 3 * H + W)
    sw = _swaps(img, n, W + 5, near=n // 3)
    rows = _gpu_delta(ctx, img, cx, cy, sw, mask)
    _abi.lpf_set_delta_method(ctx.handle, _abi.LPF_SWAP_RUNS)
    try:
        runs = _gpu_delta(ctx, img, cx, cy, sw, mask)
    finally:
        _abi.lpf_set_delta_method(ctx.handle, _abi.LPF_SWAP_AUTO)
    ref = oracle.delta_swap(img, cx, cy, sw, mask)
    assert np.array_equal(runs, ref)
    assert np.array_equal(rows, ref)


def test_delta_frames_in_device_memory(ctx):
    # 512 x 512, cutoff 40: the two extended frames (about 95 KB) exceed the LDS budget and are
    # read from device memory
    print("[gpu] delta 512x512 c=40, frames in device memory", flush=True)
    img = wl.boolean_disks(512, 512, 6.0, 0.35, 12)
    sw = _swaps(img, 24, 4, near=8)
    got = _gpu_delta(ctx, img, 40, 40, sw, 3)
    assert np.array_equal(got, oracle.delta_swap(img, 40, 40, sw, 3))
