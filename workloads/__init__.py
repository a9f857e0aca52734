"""Seeded synthetic microstructures shared by the tests, the benchmark and smoke().

This module holds input generation only -- none of the lineal-path arithmetic.  Both the CPU
oracle's callers and the GPU path's callers draw their images here, so that both sides see the
same pixels.  The paper times its kernels on its own chess, particulate and metal-foam images
(Sec. 3.2); those images are not available, so seeded disk models of the same kind stand in.

Disk digitisation: pixel (x, y) belongs to a disk of radius r centred at c when the periodic
minimum-image distance from the pixel centre (x + 1/2, y + 1/2) to c is <= r.
Images are uint8 arrays of shape (H, W) holding 0/1; phase 1 is the disk (inclusion) phase.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _stamp(img: np.ndarray, cx: float, cy: float, r: float) -> None:
    H, W = img.shape
    x0, x1 = int(math.floor(cx - r - 1)), int(math.ceil(cx + r + 1))
    y0, y1 = int(math.floor(cy - r - 1)), int(math.ceil(cy + r + 1))
    xs = np.arange(x0, x1 + 1)
    ys = np.arange(y0, y1 + 1)
    ddx = (xs + 0.5) - cx
    ddy = (ys + 0.5) - cy
    inside = (ddy[:, None] ** 2 + ddx[None, :] ** 2) <= r * r
    yy, xx = np.nonzero(inside)
    img[(ys[yy] % H), (xs[xx] % W)] = 1


def _stamp_many(img: np.ndarray, cs: np.ndarray, r: float, chunk: int = 4096) -> None:
    """Union of equal disks (same digitisation as _stamp), vectorised over chunks of centres."""
    H, W = img.shape
    b = int(math.ceil(r)) + 2
    off = np.arange(-b, b + 1)
    for s in range(0, len(cs), chunk):
        c = cs[s:s + chunk]
        bx = np.floor(c[:, 0]).astype(np.int64)
        by = np.floor(c[:, 1]).astype(np.int64)
        xs = bx[:, None] + off[None, :]                      # (k, B)
        ys = by[:, None] + off[None, :]
        ddx = (xs + 0.5) - c[:, 0:1]
        ddy = (ys + 0.5) - c[:, 1:2]
        inside = (ddy[:, :, None] ** 2 + ddx[:, None, :] ** 2) <= r * r   # (k, By, Bx)
        kk, iy, ix = np.nonzero(inside)
        img[ys[kk, iy] % H, xs[kk, ix] % W] = 1


def boolean_disks(W: int, H: int, r: float, phi: float, seed: int) -> np.ndarray:
    """Boolean model: N_d = round(-ln(1 - phi) W H / (pi r^2)) overlapping disks of radius r
    with centres uniform in [0,W) x [0,H)."""
    g = rng(seed)
    nd = int(round(-math.log(1.0 - phi) * W * H / (math.pi * r * r)))
    img = np.zeros((H, W), np.uint8)
    cs = g.random((nd, 2)) * np.array([W, H])
    _stamp_many(img, cs, r)
    return img


def boolean_disks_random_radius(W: int, H: int, rmin: float, rmax: float, phi: float,
                                seed: int) -> np.ndarray:
    """Boolean model with one radius r ~ U[rmin, rmax] drawn for the whole image."""
    g = rng(seed)
    r = float(g.uniform(rmin, rmax))
    return boolean_disks(W, H, r, phi, int(g.integers(0, 2**62)))


def rsa_disks(W: int, H: int, rmin: float, rmax: float, phi: float, seed: int,
              max_tries: int = 1_000_000) -> np.ndarray:
    """Random sequential addition of non-overlapping disks, radius ~ U[rmin, rmax], centre
    uniform; a disk is rejected when its periodic centre distance to an accepted disk j is
    below r + r_j.  Stops once the digitised phase-1 fraction reaches phi."""
    g = rng(seed)
    img = np.zeros((H, W), np.uint8)
    cs: list[tuple[float, float, float]] = []
    target = phi * W * H
    tries = 0
    while img.sum() < target:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("RSA jammed before reaching the volume fraction")
        r = float(g.uniform(rmin, rmax))
        cx, cy = float(g.random() * W), float(g.random() * H)
        ok = True
        if cs:
            a = np.asarray(cs)
            ddx = np.abs(a[:, 0] - cx)
            ddx = np.minimum(ddx, W - ddx)
            ddy = np.abs(a[:, 1] - cy)
            ddy = np.minimum(ddy, H - ddy)
            ok = bool(np.all(ddx * ddx + ddy * ddy >= (a[:, 2] + r) ** 2))
        if ok:
            cs.append((cx, cy, r))
            _stamp(img, cx, cy, r)
    return img


def stripes(W: int, H: int, period: int, width: int, vertical: bool = True) -> np.ndarray:
    """Phase-1 stripes of the given width repeating with the given period."""
    if vertical:
        row = ((np.arange(W) % period) < width).astype(np.uint8)
        return np.tile(row, (H, 1))
    col = ((np.arange(H) % period) < width).astype(np.uint8)
    return np.tile(col[:, None], (1, W))


def checkerboard(W: int, H: int, s: int) -> np.ndarray:
    """Chess-type morphology with s x s squares (the paper's first timing workload uses s=10)."""
    x = (np.arange(W) // s)[None, :]
    y = (np.arange(H) // s)[:, None]
    return ((x + y) % 2).astype(np.uint8)


def square_particles(W: int, H: int, size: int, n: int, seed: int, tries: int = 100000) -> np.ndarray:
    """Particulate suspension of Sec. 6.1: n equal size x size phase-1 squares placed one by one
    at uniform random positions of the periodic W x H cell, a placement rejected when it would
    overlap or touch (share an edge with) a square already placed."""
    g = rng(seed)
    occ = np.zeros((H, W), bool)
    img = np.zeros((H, W), np.uint8)
    placed = 0
    for _ in range(tries):
        if placed == n:
            break
        x0, y0 = int(g.integers(W)), int(g.integers(H))
        ys = np.arange(y0 - 1, y0 + size + 1) % H
        xs = np.arange(x0 - 1, x0 + size + 1) % W
        if occ[np.ix_(ys, xs)].any():
            continue
        occ[np.ix_(ys[1:-1], xs[1:-1])] = True
        img[np.ix_(ys[1:-1], xs[1:-1])] = 1
        placed += 1
    if placed != n:
        raise ValueError("could not place every square")
    return img


def sample_positions(W: int, H: int, n: int, seed: int) -> np.ndarray:
    """Monte-Carlo position set (Sec. 3): a uniformly random n-combination, without repetition,
    of the W x H start pixels, as a uint8 mask (1 = sampled)."""
    g = rng(seed)
    flat = np.zeros(W * H, np.uint8)
    flat[g.permutation(W * H)[:n]] = 1
    return flat.reshape(H, W)


def gaussian_field_3d(W: int, H: int, D: int, corr: float, phi: float, seed: int) -> np.ndarray:
    """Periodic level-cut Gaussian random field, uint8 (D, H, W): white noise smoothed by a
    periodic Gaussian of standard deviation `corr` voxels (FFT), phase 1 where the field exceeds
    its (1 - phi) quantile.  At phi ~ 0.5 both phases form continuous irregular branches, the
    morphology of the trabecular-bone specimen of Sec. 6.3."""
    g = rng(seed)
    noise = g.standard_normal((D, H, W))
    kz = np.fft.fftfreq(D)[:, None, None]
    ky = np.fft.fftfreq(H)[None, :, None]
    kx = np.fft.fftfreq(W)[None, None, :]
    filt = np.exp(-2.0 * (np.pi * corr) ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    field = np.fft.ifftn(np.fft.fftn(noise) * filt).real
    thr = np.quantile(field, 1.0 - phi)
    return (field > thr).astype(np.uint8)


def random_binary(W: int, H: int, p: float, seed: int) -> np.ndarray:
    return (rng(seed).random((H, W)) < p).astype(np.uint8)


def random_cell(W: int, H: int, n_ones: int, seed: int) -> np.ndarray:
    """Random image with exactly n_ones phase-1 pixels (annealing start, Sec. 4)."""
    g = rng(seed)
    flat = np.zeros(W * H, np.uint8)
    flat[g.permutation(W * H)[:n_ones]] = 1
    return flat.reshape(H, W)


# ------------------------------------------------------------------------------------------
# Named workloads (sizes, seeds and distributions of the benchmark configurations)
# ------------------------------------------------------------------------------------------

def small_boolean_64(seed: int = 1601) -> np.ndarray:
    """64 x 64 Boolean model, r = 4, volume fraction ~0.5 (cutoff 16, both phases)."""
    return boolean_disks(64, 64, 4.0, 0.5, seed)


def rsa_512(seed: int = 1602) -> np.ndarray:
    """512 x 512 non-overlapping disks, r ~ U[5, 20], volume fraction 0.3 (cutoff 128)."""
    return rsa_disks(512, 512, 5.0, 20.0, 0.3, seed)


@dataclass
class BatchImage:
    side: int
    phi: float
    r: float
    seed: int
    img: np.ndarray | None = None


def batch_spec(n_images: int = 256, seed: int = 1603,
               sides=(64, 128, 256, 512, 1024)) -> list[BatchImage]:
    """Uneven batch: side ~ U{sides}, phi ~ U[0.2, 0.6], r ~ U[3, 15]; cutoff = side / 2."""
    g = rng(seed)
    out = []
    for j in range(n_images):
        side = int(g.choice(np.asarray(sides)))
        phi = float(g.uniform(0.2, 0.6))
        r = float(g.uniform(3.0, 15.0))
        out.append(BatchImage(side, phi, r, seed * 1000 + j))
    return out


def batch_image(b: BatchImage) -> np.ndarray:
    if b.img is None:
        b.img = boolean_disks(b.side, b.side, b.r, b.phi, b.seed)
    return b.img


def anneal_target(side: int = 1024, phi: float = 0.35, r: float = 6.0,
                  seed: int = 1604) -> np.ndarray:
    """Target microstructure for the reconstruction workload (Boolean disks)."""
    return boolean_disks(side, side, r, phi, seed)
