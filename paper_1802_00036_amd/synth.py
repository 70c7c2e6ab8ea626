"""Seeded synthetic LIDAR-shaped sparse depth maps.

The KITTI depth-completion maps the paper evaluates on (Sec. IV, "Experiments
and Results") are not available, so every input here is synthetic with the
statistics the paper states for them:

* points come from LIDAR scan lines and lie only in the bottom two thirds of
  the frame (Sec. IV);
* 5-7 % of the pixels in that region hold a depth (Sec. IV);
* depths lie in 0-80 m and empty pixels hold 0 (Sec. III, "Depth Inversion").

The scene is a ground plane seen from a forward camera plus a few
axis-aligned boxes standing on it (piecewise-planar surfaces; the nearer
surface wins per pixel), with 1 % of the points replaced by uniform outliers.

This module draws inputs only. It holds none of the completion arithmetic and
is the one module shared by the oracle-side tests and the GPU path.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Frame:
    sparse: np.ndarray      # float32 H x W, 0 = empty
    dense_gt: np.ndarray    # float32 H x W, the surface the points were sampled from
    density: float          # achieved fraction of non-zero pixels (whole frame)
    max_depth: float        # largest depth the generator may emit


def _rng(seed_words: Sequence[int]) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed_words))))


def _scene(rng: np.random.Generator, H: int, W: int, d_max: float) -> np.ndarray:
    """Dense depth of a ground plane with boxes, float64 H x W (inf = sky)."""
    yh = H / 3.0
    z_near = rng.uniform(4.0, 6.0)
    ys = np.arange(H, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        ground_row = z_near * (H - 1 - yh) / (ys - yh)
    ground_row = np.where(ys > yh, ground_row, np.inf)
    ground_row = np.where(np.isfinite(ground_row), np.clip(ground_row, 1.0, d_max), np.inf)
    depth = np.repeat(ground_row[:, None], W, axis=1)

    n_boxes = int(rng.integers(4, 13))
    for _ in range(n_boxes):
        # foot of the box on the ground, somewhere in the lower two thirds
        y_foot = int(rng.integers(int(yh) + 2, H)) if H - (int(yh) + 2) > 0 else H - 1
        z_foot = ground_row[y_foot] if np.isfinite(ground_row[y_foot]) else d_max
        bw = int(rng.integers(max(2, W // 40), max(3, W // 6)))
        bh = int(rng.integers(max(2, H // 20), max(3, H // 3)))
        x0 = int(rng.integers(0, max(1, W - bw)))
        y0 = max(0, y_foot - bh)
        gx = rng.uniform(-0.02, 0.02)
        gy = rng.uniform(-0.01, 0.01)
        x1 = min(W, x0 + bw)                          # narrow frames clip the box
        yy, xx = np.mgrid[y0:y_foot + 1, x0:x1]
        face = z_foot + gx * (xx - x0) + gy * (yy - y0)
        face = np.clip(face, 1.0, d_max)
        region = depth[y0:y_foot + 1, x0:x1]
        np.minimum(region, face, out=region)          # nearer surface wins
    return depth


def lidar_frame(H: int, W: int, *, seed: Sequence[int], n_rows: int = 64,
                density: float = 0.05, d_max: float = 80.0,
                outlier_frac: float = 0.01,
                occlusions: Tuple[int, int] = (0, 0)) -> Frame:
    """One sparse LIDAR-shaped frame.

    Scan row k sits at round(H/3 + k (H-1-H/3)/(n_rows-1)); each point is
    jittered by -1, 0 or +1 row.  A column keeps a point on a scan row with
    probability p = density * H / n_rows; for p > 1 it gets floor(p) or
    ceil(p) points on distinct jitter rows.  ``occlusions=(lo, hi)`` removes
    every point inside lo..hi random rectangles (64-512 px wide, 32-256 px
    tall, clipped to the frame).
    """
    rng = _rng(seed)
    dense = _scene(rng, H, W, d_max)
    sparse = np.zeros((H, W), np.float32)
    n_rows = max(1, min(n_rows, H))
    yh = H / 3.0
    if n_rows == 1:
        rows = np.array([int(round(yh))])
    else:
        rows = np.round(yh + np.arange(n_rows) * (H - 1 - yh) / (n_rows - 1)).astype(np.int64)
    p = density * H / n_rows
    cols = np.arange(W)
    for y in rows:
        if p <= 1.0:
            keep = rng.random(W) < p
            jit = rng.integers(-1, 2, W)
            ys = np.clip(y + jit[keep], 0, H - 1)
            xs = cols[keep]
        else:
            base = int(np.floor(p))
            extra = rng.random(W) < (p - base)
            counts = np.minimum(base + extra.astype(np.int64), 3)
            ys_l, xs_l = [], []
            for c in (1, 2, 3):
                sel = cols[counts >= c]
                if sel.size == 0:
                    continue
                # distinct jitter rows: the c-th point of a column uses offset (c-1) - 1 permuted
                perm = rng.permuted(np.tile(np.array([-1, 0, 1]), (sel.size, 1)), axis=1)
                ys_l.append(np.clip(y + perm[:, c - 1], 0, H - 1))
                xs_l.append(sel)
            ys = np.concatenate(ys_l) if ys_l else np.zeros(0, np.int64)
            xs = np.concatenate(xs_l) if xs_l else np.zeros(0, np.int64)
        z = dense[ys, xs]
        ok = np.isfinite(z)
        ys, xs, z = ys[ok], xs[ok], z[ok]
        cur = sparse[ys, xs]
        # duplicate hits on one pixel keep the nearer one
        z32 = z.astype(np.float32)
        take = (cur == 0) | (z32 < cur)
        sparse[ys[take], xs[take]] = z32[take]

    lo, hi = occlusions
    if hi > 0:
        n_occ = int(rng.integers(lo, hi + 1))
        for _ in range(n_occ):
            ow = int(rng.integers(64, 513))
            oh = int(rng.integers(32, 257))
            ox = int(rng.integers(0, max(1, W - 1)))
            oy = int(rng.integers(int(yh), max(int(yh) + 1, H - 1)))
            sparse[oy:oy + oh, ox:ox + ow] = 0.0

    valid = np.nonzero(sparse)
    n_valid = valid[0].size
    n_out = int(round(outlier_frac * n_valid))
    if n_out > 0:
        pick = rng.choice(n_valid, size=n_out, replace=False)
        sparse[valid[0][pick], valid[1][pick]] = rng.uniform(1.0, d_max, n_out).astype(np.float32)

    gt = np.where(np.isfinite(dense), dense, 0.0).astype(np.float32)
    return Frame(sparse=sparse, dense_gt=gt, density=float(np.count_nonzero(sparse)) / (H * W),
                 max_depth=d_max)


# --------------------------------------------------------------------------
# The five workloads (frames x size, scan rows, density, depth range).

def config_frame(cfg: int, i: int, base: int = 0) -> Frame:
    """Frame i of workload ``cfg`` (the same frame config_frames returns at i)."""
    if cfg == 1:
        return lidar_frame(352, 1216, seed=[1, 0, base], n_rows=64, density=0.05)
    if cfg == 2:
        dens = _rng([2, i, base, 99]).uniform(0.04, 0.06)
        return lidar_frame(375, 1242, seed=[2, i, base], n_rows=64, density=dens)
    if cfg == 3:
        r = _rng([3, i, base, 99])
        H = int(r.integers(256, 513))
        W = int(r.integers(768, 2049))
        rows = int(r.choice([32, 64, 128]))
        dens = r.uniform(0.02, 0.10)
        return lidar_frame(H, W, seed=[3, i, base], n_rows=rows, density=dens)
    if cfg == 4:
        return lidar_frame(1024, 4096, seed=[4, i, base], n_rows=128, density=0.03,
                           d_max=120.0, occlusions=(4, 8))
    raise ValueError(f"unknown workload {cfg}")


CONFIG_SIZES = {1: 1, 2: 64, 3: 128, 4: 16}


def config_frames(cfg: int, base: int = 0, limit: Optional[int] = None) -> List[Frame]:
    """Seeded frames of workload ``cfg``:

    1: one 352x1216 frame, 64 scan rows, 5 % dense, 1-80 m.
    2: 64 frames of 375x1242, 64 scan rows, density U[4 %, 6 %], 1-80 m.
    3: 128 frames, H ~ U{256..512}, W ~ U{768..2048}, 32/64/128 scan rows,
       density U[2 %, 10 %], 1-80 m.
    4: 16 frames of 1024x4096, 128 scan rows, 3 % dense, 1-120 m, with 4-8
       occlusion rectangles and the empty sky above the top scan row.
    """
    if cfg not in CONFIG_SIZES:
        raise ValueError(f"unknown workload {cfg}")
    n = CONFIG_SIZES[cfg] if limit is None else min(CONFIG_SIZES[cfg], limit)
    return [config_frame(cfg, i, base) for i in range(n)]


SERVE_SIZES = ((352, 1216), (375, 1242), (512, 2048), (1024, 4096))
SERVE_WEIGHTS = (0.4, 0.3, 0.2, 0.1)


def serve_frame(size_idx: int, i: int, base: int = 0) -> Frame:
    """A frame of the serving mix: sizes 352x1216 / 375x1242 / 512x2048 /
    1024x4096, density U[2 %, 10 %], 1-80 m (1-120 m for the 1024-row size)."""
    H, W = SERVE_SIZES[size_idx]
    r = _rng([5, size_idx, i, base])
    dens = r.uniform(0.02, 0.10)
    big = H >= 1024
    return lidar_frame(H, W, seed=[5, size_idx, i, base, 1], n_rows=128 if big else 64,
                       density=dens, d_max=120.0 if big else 80.0)


def poisson_arrivals(rate: float, n: int, base: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Arrival times (s, from 0) and size indices for a Poisson trace."""
    r = _rng([6, int(rate), base])
    gaps = r.exponential(1.0 / rate, n)
    sizes = r.choice(len(SERVE_SIZES), size=n, p=np.array(SERVE_WEIGHTS))
    return np.cumsum(gaps), sizes


def random_map(rng: np.random.Generator, H: int, W: int, density: float,
               lo: float = 1.0, hi: float = 80.0) -> np.ndarray:
    """Uniformly scattered points (no scan structure): small fuzz inputs."""
    m = np.zeros((H, W), np.float32)
    keep = rng.random((H, W)) < density
    m[keep] = rng.uniform(lo, hi, int(keep.sum())).astype(np.float32)
    return m
