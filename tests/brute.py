"""Pure-Python brute force of the completion steps for tiny maps.

An independent second statement of each step (Sec. III of the paper, with
the oracle's readings), written with explicit loops over pixels and window
offsets and no NumPy arithmetic, used to pin the oracle.  The Gaussian sum is
evaluated exactly with rational arithmetic and rounded to float32 with
round-half-even, so it also pins the oracle's claim that its float64 sum
rounds to the correctly rounded float32 value.
"""
from __future__ import annotations

import math
import struct
from fractions import Fraction

import numpy as np


def f32(x: float) -> float:
    """Round a Python float (float64) to the nearest float32, as a float."""
    return struct.unpack("f", struct.pack("f", x))[0]


def in_kernel(shape: int, size: int, dy: int, dx: int) -> bool:
    r = size // 2
    if abs(dy) > r or abs(dx) > r:
        return False
    if shape == 0:       # full
        return True
    if shape == 1:       # cross
        return dy == 0 or dx == 0
    if shape == 2:       # diamond
        return abs(dy) + abs(dx) <= r
    if shape == 3:       # circle
        return 4 * (dy * dy + dx * dx) <= size * size
    raise ValueError(shape)


def to_lists(a):
    return [[float(a[y][x]) for x in range(len(a[0]))] for y in range(len(a))]


def window_reduce(v, shape, size, op):
    H, W = len(v), len(v[0])
    r = size // 2
    out = [[0.0] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            best = None
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    if not in_kernel(shape, size, dy, dx):
                        continue
                    yy, xx = y + dy, x + dx
                    if 0 <= yy < H and 0 <= xx < W:
                        val = v[yy][xx]
                        best = val if best is None else op(best, val)
            out[y][x] = best
    return out


def invert(d, off, thr):
    out = []
    for row in d:
        o = []
        for x in row:
            x = float(x)
            if x != x or not (x > thr):
                o.append(0.0)
                continue
            if math.isinf(x):
                o.append(0.0)
                continue
            v = f32(off - x)
            o.append(v if v > thr else 0.0)
        out.append(o)
    return out


def fill(v, size, thr):
    grown = window_reduce(v, 0, size, max)
    return [[grown[y][x] if v[y][x] <= thr else v[y][x] for x in range(len(v[0]))]
            for y in range(len(v))]


def extend(v, thr, limit=0):
    """Copy each column's topmost non-empty value upward (at most `limit`
    rows when limit > 0)."""
    H, W = len(v), len(v[0])
    out = [row[:] for row in v]
    for x in range(W):
        top = None
        for y in range(H):
            if v[y][x] > thr:
                top = y
                break
        if top is not None:
            for y in range(top):
                if limit <= 0 or top - y <= limit:
                    out[y][x] = v[top][x]
    return out


def bilateral(v, size, sigma_space, sigma_color):
    """Bilateral weighted mean per pixel, float64, reflect-101 borders."""
    H, W = len(v), len(v[0])
    r = size // 2
    out = [[0.0] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            c = v[y][x]
            num = den = 0.0
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    q = v[refl(y + dy, H)][refl(x + dx, W)]
                    w = math.exp(-(dy * dy + dx * dx) / (2.0 * sigma_space ** 2)) * \
                        math.exp(-((q - c) ** 2) / (2.0 * sigma_color ** 2))
                    num += w * q
                    den += w
            out[y][x] = num / den
    return out


def median(v, size):
    H, W = len(v), len(v[0])
    r = size // 2
    out = [[0.0] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            s = []
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    yy = min(max(y + dy, 0), H - 1)
                    xx = min(max(x + dx, 0), W - 1)
                    s.append(v[yy][xx])
            s.sort()
            out[y][x] = s[len(s) // 2]
    return out


def refl(q, n):
    if n == 1:
        return 0
    while q < 0 or q >= n:
        q = -q if q < 0 else 2 * (n - 1) - q
    return q


def round_f32_exact(q: Fraction) -> float:
    """Correctly rounded (half-even) float32 of an exact rational."""
    c = f32(float(q))
    cands = {c, float(np.nextafter(np.float32(c), np.float32(np.inf))),
             float(np.nextafter(np.float32(c), np.float32(-np.inf)))}
    best = None
    for c in sorted(cands):
        err = abs(Fraction(c) - q)
        if best is None or err < best[0]:
            best = (err, c)
        elif err == best[0]:
            # tie: even mantissa
            bits = struct.unpack("I", struct.pack("f", c))[0]
            if bits % 2 == 0:
                best = (err, c)
    return best[1]


def binomial_taps(size):
    n = size - 1
    return [Fraction(math.comb(n, i), 2 ** n) for i in range(size)]


def gauss_exact(v, size):
    """Exact binomial-tap blur with reflect-101 borders, as Fractions."""
    H, W = len(v), len(v[0])
    r = size // 2
    w = binomial_taps(size)
    out = [[Fraction(0)] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            acc = Fraction(0)
            for i in range(-r, r + 1):
                for j in range(-r, r + 1):
                    acc += w[i + r] * w[j + r] * Fraction(v[refl(y + i, H)][refl(x + j, W)])
            out[y][x] = acc
    return out


def complete(d, *, shape=2, dsize=5, csize=5, fsize=7, lsize=31, msize=5, gsize=5,
             off=100.0, thr=None, extrapolate=True):
    """All nine stage maps as lists of lists (binomial blur only)."""
    thr = f32(0.1) if thr is None else thr
    off = f32(off)
    st = []
    v = invert(d, off, thr); st.append(v)
    v = window_reduce(v, shape, dsize, max); st.append(v)
    v = window_reduce(window_reduce(v, 0, csize, max), 0, csize, min); st.append(v)
    v = fill(v, fsize, thr); st.append(v)
    v5 = extend(v, thr) if extrapolate else v; st.append(v5)
    v = fill(v5, lsize, thr) if extrapolate else v5; st.append(v)
    v7 = median(v, msize) if msize else v; st.append(v7)
    H, W = len(v7), len(v7[0])
    if gsize:
        g = gauss_exact(v7, gsize)
        v8 = [[round_f32_exact(g[y][x]) if v7[y][x] > thr else 0.0 for x in range(W)] for y in range(H)]
    else:
        v8 = [[v7[y][x] if v7[y][x] > thr else 0.0 for x in range(W)] for y in range(H)]
    st.append(v8)
    out = [[f32(off - v8[y][x]) if v7[y][x] > thr else 0.0 for x in range(W)] for y in range(H)]
    st.append(out)
    return st
