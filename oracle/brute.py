"""Independent brute force for tiny images -- TEST INFRASTRUCTURE ONLY.

A second route to the lineal path function that shares nothing with ``lpf_oracle.c``: the
digitisation uses exact rational rounding (``fractions.Fraction``) of the ideal segment
instead of an error term, the half domain is obtained by filtering the full grid with the
point-symmetry rule (eq. (symmetry)) instead of by two nested rectangles, and the count is a
product of periodically rolled indicator images instead of a walk with early break.

Reading R1 (round half up in magnitude, from the segment origin) is stated here as
``round_half_up(|m| k / n)``.  ``tie_rule='down'`` gives the opposite convention, used only to
show which results depend on the convention.
"""
from __future__ import annotations

from fractions import Fraction
from math import floor, ceil

import numpy as np


def path(dx: int, dy: int, tie_rule: str = "up") -> list[tuple[int, int]]:
    n = max(abs(dx), abs(dy))
    if n == 0:
        return [(0, 0)]
    sx = -1 if dx < 0 else 1
    sy = -1 if dy < 0 else 1
    out = []
    for k in range(n + 1):
        if abs(dx) >= abs(dy):
            exact = Fraction(abs(dy) * k, n)
            q = floor(exact + Fraction(1, 2)) if tie_rule == "up" else ceil(exact - Fraction(1, 2))
            out.append((sx * k, sy * q))
        else:
            exact = Fraction(abs(dx) * k, n)
            q = floor(exact + Fraction(1, 2)) if tie_rule == "up" else ceil(exact - Fraction(1, 2))
            out.append((sx * q, sy * k))
    return out


def half_domain(cx: int, cy: int) -> list[tuple[int, int]]:
    """Vectors v of the cutoff grid such that v is the canonical one of the pair {v, -v}:
    dy > 0, or dy == 0 and dx >= 0; ordered dx >= 0 part first (by dy, then dx), then dx < 0."""
    pos, neg = [], []
    for dy in range(0, cy + 1):
        for dx in range(-cx, cx + 1):
            if dy == 0 and dx < 0:
                continue
            (pos if dx >= 0 else neg).append((dx, dy))
    return pos + neg


def lpf_vector(img: np.ndarray, dx: int, dy: int, phase: int, tie_rule: str = "up") -> int:
    ind = (np.asarray(img) == phase)
    acc = np.ones_like(ind, dtype=bool)
    for (px, py) in set(path(dx, dy, tie_rule)):
        # acc[y, x] &= ind[(y + py) % H, (x + px) % W]
        acc &= np.roll(ind, shift=(-py, -px), axis=(0, 1))
    return int(acc.sum())


def lpf(img: np.ndarray, cx: int, cy: int, phase_mask: int = 3, tie_rule: str = "up") -> np.ndarray:
    vs = half_domain(cx, cy)
    rows = []
    for ph in (0, 1):
        if phase_mask & (1 << ph):
            rows.append([lpf_vector(img, dx, dy, ph, tie_rule) for (dx, dy) in vs])
    return np.array(rows, dtype=np.uint32)


def s2_fft(img: np.ndarray, phase: int) -> np.ndarray:
    """Periodic two-point probability S2[y, x] by the FFT route (Sec. 2.1), as counts N*S2."""
    chi = (np.asarray(img) == phase).astype(np.float64)
    F = np.fft.fft2(chi)
    corr = np.fft.ifft2(np.conj(F) * F).real
    return np.rint(corr).astype(np.int64)


def _round_r1(num: int, n: int, tie_rule: str) -> int:
    exact = Fraction(num, n)
    return floor(exact + Fraction(1, 2)) if tie_rule == "up" else ceil(exact - Fraction(1, 2))


def path3(dx: int, dy: int, dz: int, tie_rule: str = "up") -> list[tuple[int, int, int]]:
    """3-D digitised segment by exact rational rounding of every minor coordinate; the major
    axis is the first of x, y, z with the largest extent."""
    d = (dx, dy, dz)
    a = [abs(t) for t in d]
    n = max(a)
    if n == 0:
        return [(0, 0, 0)]
    major = a.index(n)
    out = []
    for k in range(n + 1):
        c = [k if ax == major else _round_r1(a[ax] * k, n, tie_rule) for ax in range(3)]
        out.append(tuple(-c[ax] if d[ax] < 0 else c[ax] for ax in range(3)))
    return out


def half_domain3(cx: int, cy: int, cz: int) -> set[tuple[int, int, int]]:
    """The set of canonical vectors: of each pair {v, -v} of the cutoff box, the one whose last
    nonzero coordinate among (dz, dy) is positive, or (dx >= 0, 0, 0)."""
    out = set()
    for dz in range(-cz, cz + 1):
        for dy in range(-cy, cy + 1):
            for dx in range(-cx, cx + 1):
                if dz > 0 or (dz == 0 and dy > 0) or (dz == 0 and dy == 0 and dx >= 0):
                    out.add((dx, dy, dz))
    return out


def lpf3_vector(vol: np.ndarray, dx: int, dy: int, dz: int, phase: int) -> int:
    ind = (np.asarray(vol) == phase)
    acc = np.ones_like(ind, dtype=bool)
    for (px, py, pz) in set(path3(dx, dy, dz)):
        acc &= np.roll(ind, shift=(-pz, -py, -px), axis=(0, 1, 2))
    return int(acc.sum())
