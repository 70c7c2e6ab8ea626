"""Plain CPU oracle for IP-Basic depth completion.

Ku, Harakeh & Waslander, "In Defense of Classical Image Processing: Fast
Depth Completion on the CPU" (2018), Sec. III "Proposed Algorithm": eight
image-processing steps turn a sparse depth map into a dense one.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares no code with
the GPU library and imports nothing from it.

Written for a reader to check against the paper by eye: each step is the
plain definition over whole arrays, with no blocking, fusion or reordering.

Precision.  Maps are float32 images (the type of the depth maps the library
takes and returns).  The selection steps (dilation, erosion, fills,
extension, median) pick input values and round nothing.  The two arithmetic
steps (the inversions and the Gaussian blur) are carried in float64 and
rounded once to float32 when the step writes its map.  With the default
binomial blur taps every product and partial sum is exact in float64 for
inverted values in (0.1, 100], so the blurred map is the correctly rounded
exact weighted sum.

Readings where the paper is silent (each listed with its reason in the
design notes):
  * empty means value <= thr (thr = 0.1 by default); an input depth d is
    valid iff d > thr and fl32(off - d) > thr, so NaN, +-Inf, negatives and
    depths within thr of the offset become empty (+0.0);
  * morphology ignores taps outside the image (max and min over the in-image
    part of the window);
  * kernel shapes: FULL = all k x k; CROSS = centre row and column;
    DIAMOND = |dx| + |dy| <= k // 2; CIRCLE = dx^2 + dy^2 <= (k / 2)^2;
  * the step-2 dilation and the closing are unmasked; the fills write empty
    pixels only, with mask and dilation both taken from the step's input;
  * the extension copies, per column, the topmost non-empty value into every
    row above it; columns without one are unchanged;
  * the median is unmasked (zeros count) with a replicated border and picks
    the middle of the size^2 sorted samples;
  * the Gaussian uses reflect-101 borders; sigma <= 0 means binomial taps
    (1 4 6 4 1)/16 for size 5; it is computed over the whole map and written
    only where the median output is non-empty (mask taken before the blur);
  * the output inversion is masked by that same mask; empties stay +0.0;
  * the bilateral blur (the alternative of Sec. IV, Table 3) weighs each
    tap by exp(-(dy^2 + dx^2) / (2 s_space^2)) exp(-(v_q - v_p)^2 /
    (2 s_color^2)), divides by the sum of the weights, uses reflect-101
    borders and the Gaussian's mask; the paper gives no sigmas, so they are
    parameters (defaults 2 px and 1.5 in depth units);
  * a limited extension (the point-cloud advice of Sec. IV) copies the top
    value into at most extend_rows rows above it (0: no limit).

Parity pins: brute force on tiny maps, SciPy's ndimage routines, closed
forms and invariants (tests/test_oracle_*.py).  Parity unpinned: the readings
above themselves, which no code or data of the authors is available to check.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

F32 = np.float32
F64 = np.float64

SE_FULL, SE_CROSS, SE_DIAMOND, SE_CIRCLE = 0, 1, 2, 3
BLUR_GAUSSIAN, BLUR_BILATERAL = 0, 1


@dataclasses.dataclass
class Params:
    """Defaults are the paper's final design (Sec. III, Table 2, Table 3)."""
    dilate_shape: int = SE_DIAMOND   # 5x5 diamond, "Custom Kernel Dilation"
    dilate_size: int = 5
    close_size: int = 5              # 5x5 full, "Small Hole Closure"
    fill_size: int = 7               # 7x7 full, "Small Hole Fill"
    extrapolate: int = 1             # run "Extension to Top of Frame" and "Large Hole Fill"
    large_fill_size: int = 31        # 31x31 full, "Large Hole Fill"
    median_size: int = 5             # 5x5 median, "Median and Gaussian Blur"; 0 = off
    gauss_size: int = 5              # 5x5 Gaussian; 0 = off
    gauss_sigma: float = 0.0         # <= 0: binomial taps
    max_depth: float = 100.0         # the inversion offset, "Depth Inversion"
    valid_thresh: float = 0.1        # empty iff value <= this
    blur: int = BLUR_GAUSSIAN        # step 8: Gaussian or bilateral (Sec. IV, Table 3)
    bilateral_sigma_space: float = 2.0
    bilateral_sigma_color: float = 1.5
    extend_rows: int = 0             # rows the extension reaches above the top; 0 = all (Sec. IV)


# ---------------------------------------------------------------- kernels --

def structuring_element(shape: int, size: int) -> np.ndarray:
    """Boolean size x size kernel, anchored at its centre (Sec. III, the
    four shapes compared in Sec. IV "Custom Kernel Design")."""
    if size < 1 or size % 2 == 0:
        raise ValueError("kernel size must be odd and positive")
    r = size // 2
    dy, dx = np.mgrid[-r:r + 1, -r:r + 1]
    if shape == SE_FULL:
        return np.ones((size, size), bool)
    if shape == SE_CROSS:
        return (dx == 0) | (dy == 0)
    if shape == SE_DIAMOND:
        return (np.abs(dx) + np.abs(dy)) <= r
    if shape == SE_CIRCLE:
        return (dx * dx + dy * dy) * 4 <= size * size
    raise ValueError(f"unknown kernel shape {shape}")


def _offsets(se: np.ndarray):
    r = se.shape[0] // 2
    for i in range(se.shape[0]):
        for j in range(se.shape[1]):
            if se[i, j]:
                yield i - r, j - r


def dilate(v: np.ndarray, se: np.ndarray) -> np.ndarray:
    """Grey dilation: each pixel becomes the largest value under the kernel;
    taps outside the image are ignored."""
    H, W = v.shape
    r = se.shape[0] // 2
    pad = np.full((H + 2 * r, W + 2 * r), -np.inf, F32)
    pad[r:r + H, r:r + W] = v
    out = np.full((H, W), -np.inf, F32)
    for dy, dx in _offsets(se):
        np.maximum(out, pad[r + dy:r + dy + H, r + dx:r + dx + W], out=out)
    return out


def erode(v: np.ndarray, se: np.ndarray) -> np.ndarray:
    """Grey erosion: the smallest value under the kernel; taps outside the
    image are ignored."""
    H, W = v.shape
    r = se.shape[0] // 2
    pad = np.full((H + 2 * r, W + 2 * r), np.inf, F32)
    pad[r:r + H, r:r + W] = v
    out = np.full((H, W), np.inf, F32)
    for dy, dx in _offsets(se):
        np.minimum(out, pad[r + dy:r + dy + H, r + dx:r + dx + W], out=out)
    return out


# ------------------------------------------------------------------ steps --

def step1_invert(d: np.ndarray, p: Params) -> np.ndarray:
    """Depth inversion (Sec. III): valid depths become off - d, empties 0."""
    d = np.asarray(d, F32)
    off = F64(F32(p.max_depth))
    thr = F32(p.valid_thresh)
    with np.errstate(invalid="ignore", over="ignore"):
        v = (off - d.astype(F64)).astype(F32)     # exact in float64, one rounding
        valid = (d > thr) & (v > thr)
    return np.where(valid, v, F32(0.0)).astype(F32)


def step2_dilate(v: np.ndarray, p: Params) -> np.ndarray:
    """Custom kernel dilation (Sec. III): unmasked grey dilation with the
    chosen shape and size."""
    return dilate(v, structuring_element(p.dilate_shape, p.dilate_size))


def step3_close(v: np.ndarray, p: Params) -> np.ndarray:
    """Small hole closure (Sec. III): dilation then erosion, full kernel."""
    k = structuring_element(SE_FULL, p.close_size)
    return erode(dilate(v, k), k)


def fill_empty(v: np.ndarray, size: int, thr: float) -> np.ndarray:
    """Dilate with a full kernel and write the result at empty pixels only
    (Sec. III "Small Hole Fill" and "Large Hole Fill")."""
    empty = v <= F32(thr)
    grown = dilate(v, structuring_element(SE_FULL, size))
    return np.where(empty, grown, v).astype(F32)


def step4_small_fill(v: np.ndarray, p: Params) -> np.ndarray:
    return fill_empty(v, p.fill_size, p.valid_thresh)


def step5_extend(v: np.ndarray, p: Params) -> np.ndarray:
    """Extension to top of frame (Sec. III): in each column, the topmost
    non-empty value is copied into all rows above it (into at most
    extend_rows of them when that is positive, Sec. IV)."""
    thr = F32(p.valid_thresh)
    out = v.copy()
    for x in range(v.shape[1]):
        rows = np.flatnonzero(v[:, x] > thr)
        if rows.size:
            top = rows[0]
            first = max(0, top - p.extend_rows) if p.extend_rows > 0 else 0
            out[first:top, x] = v[top, x]
    return out


def step6_large_fill(v: np.ndarray, p: Params) -> np.ndarray:
    return fill_empty(v, p.large_fill_size, p.valid_thresh)


def step7_median(v: np.ndarray, p: Params) -> np.ndarray:
    """Median blur (Sec. III): the middle of the size^2 samples of each
    window, the border replicated."""
    k = p.median_size
    if k == 0:
        return v.copy()
    H, W = v.shape
    r = k // 2
    ry = np.clip(np.arange(-r, H + r), 0, H - 1)
    rx = np.clip(np.arange(-r, W + r), 0, W - 1)
    pad = v[np.ix_(ry, rx)]
    stack = np.stack([pad[i:i + H, j:j + W] for i in range(k) for j in range(k)])
    return np.sort(stack, axis=0)[(k * k) // 2].astype(F32)


def gaussian_taps(size: int, sigma: float) -> np.ndarray:
    """1-D taps, float64.  sigma <= 0: binomial row C(size-1, i) / 2^(size-1)
    (1 4 6 4 1 / 16 for size 5).  sigma > 0: exp(-i^2 / (2 sigma^2)),
    normalised to sum 1."""
    r = size // 2
    if sigma <= 0:
        n = size - 1
        return np.array([math.comb(n, i) for i in range(size)], F64) / F64(2 ** n)
    i = np.arange(-r, r + 1, dtype=F64)
    w = np.exp(-(i * i) / (2.0 * F64(F32(sigma)) ** 2))
    return w / w.sum()


def reflect101(q: np.ndarray, n: int) -> np.ndarray:
    """Reflect about the edge pixel: -1 -> 1, n -> n - 2 (n = 1: always 0)."""
    if n == 1:
        return np.zeros_like(q)
    period = 2 * n - 2
    m = np.mod(q, period)
    return np.where(m < n, m, period - m)


def gaussian_sum(v: np.ndarray, size: int, sigma: float) -> np.ndarray:
    """Unmasked 2-D Gaussian-weighted sum, float64 (before rounding)."""
    H, W = v.shape
    r = size // 2
    w = gaussian_taps(size, sigma)
    pad = v.astype(F64)[np.ix_(reflect101(np.arange(-r, H + r), H),
                                reflect101(np.arange(-r, W + r), W))]
    g = np.zeros((H, W), F64)
    for i in range(size):
        for j in range(size):
            g += (w[i] * w[j]) * pad[i:i + H, j:j + W]
    return g


def bilateral_sum(v: np.ndarray, size: int, sigma_space: float, sigma_color: float) -> np.ndarray:
    """Bilateral blur (Sec. IV, Table 3), float64 before rounding: the
    weighted mean of the window, each tap weighted by its distance and by
    its value's difference from the centre value."""
    H, W = v.shape
    r = size // 2
    ss = F64(F32(sigma_space))
    sc = F64(F32(sigma_color))
    c = v.astype(F64)
    pad = c[np.ix_(reflect101(np.arange(-r, H + r), H), reflect101(np.arange(-r, W + r), W))]
    num = np.zeros((H, W), F64)
    den = np.zeros((H, W), F64)
    for i in range(size):
        for j in range(size):
            dy, dx = i - r, j - r
            q = pad[i:i + H, j:j + W]
            w = math.exp(-(dy * dy + dx * dx) / (2.0 * ss * ss)) * np.exp(-((q - c) ** 2) / (2.0 * sc * sc))
            num += w * q
            den += w
    return num / den


def step8_gaussian(v7: np.ndarray, p: Params) -> np.ndarray:
    """Gaussian blur (Sec. III), or the bilateral blur (Sec. IV), written
    where the median output is non-empty."""
    mask = v7 > F32(p.valid_thresh)
    if p.gauss_size == 0:
        return np.where(mask, v7, F32(0.0)).astype(F32)
    if p.blur == BLUR_BILATERAL:
        g = bilateral_sum(v7, p.gauss_size, p.bilateral_sigma_space, p.bilateral_sigma_color).astype(F32)
    else:
        g = gaussian_sum(v7, p.gauss_size, p.gauss_sigma).astype(F32)
    return np.where(mask, g, F32(0.0)).astype(F32)


def step9_reinvert(v8: np.ndarray, v7: np.ndarray, p: Params) -> np.ndarray:
    """Output depth inversion (Sec. III): off - v where the map is
    non-empty, 0 elsewhere."""
    mask = v7 > F32(p.valid_thresh)
    off = F64(F32(p.max_depth))
    out = (off - v8.astype(F64)).astype(F32)
    return np.where(mask, out, F32(0.0)).astype(F32)


# --------------------------------------------------------------- pipeline --

N_STAGES = 9


def complete(d: np.ndarray, p: Optional[Params] = None, stop_after: int = N_STAGES) -> List[np.ndarray]:
    """Run the chain on one H x W float32 map.  Returns the map after each
    step, 1..stop_after (stage k is element k-1).  With extrapolate = 0
    steps 5 and 6 are skipped (the point-cloud use of Sec. IV) and their
    stage maps equal their inputs."""
    p = p or Params()
    d = np.asarray(d, F32)
    if d.ndim != 2 or d.shape[0] < 1 or d.shape[1] < 1:
        raise ValueError("depth map must be a non-empty 2-D array")
    out: List[np.ndarray] = []
    v1 = step1_invert(d, p); out.append(v1)
    if stop_after == 1: return out
    v2 = step2_dilate(v1, p); out.append(v2)
    if stop_after == 2: return out
    v3 = step3_close(v2, p); out.append(v3)
    if stop_after == 3: return out
    v4 = step4_small_fill(v3, p); out.append(v4)
    if stop_after == 4: return out
    v5 = step5_extend(v4, p) if p.extrapolate else v4.copy(); out.append(v5)
    if stop_after == 5: return out
    v6 = step6_large_fill(v5, p) if p.extrapolate else v5.copy(); out.append(v6)
    if stop_after == 6: return out
    v7 = step7_median(v6, p); out.append(v7)
    if stop_after == 7: return out
    v8 = step8_gaussian(v7, p); out.append(v8)
    if stop_after == 8: return out
    out.append(step9_reinvert(v8, v7, p))
    return out


def complete_map(d: np.ndarray, p: Optional[Params] = None) -> np.ndarray:
    """The dense output map alone."""
    return complete(d, p)[-1]
