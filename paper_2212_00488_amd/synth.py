"""Seeded synthetic stereo pairs shaped like the paper's workloads.

This module is the only code shared by the CPU oracle's tests and the GPU
path's tests and benchmark.  It holds none of the stereo method's
arithmetic: it only draws a piecewise-planar ground-truth disparity map,
paints colour regions on the left image and forward-warps it into the right
image.  The Middlebury v3 'H' pairs the paper evaluates on (Section V) are
not available here; these pairs stand in for them at the same shapes.

Recipe (all draws from ``numpy.random.default_rng(seed)``, in this order):

1. K disparity segments are the Voronoi cells of K uniform seed points.
   Even-indexed segments are fronto-parallel, d = c0; odd-indexed ones are
   slanted, d = c0 + a (x - sx) + b (y - sy), with c0 ~ U[0, Dmax-1] and
   a, b ~ U(-0.15, 0.15).  GT = clip(round(d), 0, Dmax-1).
2. Colour regions are the Voronoi cells of 4K further seeds intersected with
   the segments, so that every depth edge is also a colour edge.
3. Each region gets an RGB mean ~ U[0,255]^3, a per-channel gradient
   ~ U(-0.5, 0.5) per pixel in x and in y around its colour seed, and i.i.d.
   Gaussian noise of sigma 2.  A fraction ``textureless`` of the regions has
   zero gradient and sigma 0.5 instead.  Values are rounded and clipped to
   uint8.
4. The right image is a forward warp R(x - GT(x,y), y) = L(x, y); where two
   left pixels land on the same right pixel the larger disparity wins (ties:
   the larger source x).  Right pixels nobody lands on get uniform noise.
   A left pixel is non-occluded iff x - GT >= 0 and it won its target.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.spatial import cKDTree


@dataclass
class StereoPair:
    left: np.ndarray      # uint8 [H][W][3]
    right: np.ndarray     # uint8 [H][W][3]
    gt: np.ndarray        # int16 [H][W], left-based disparity in [0, Dmax-1]
    nonocc: np.ndarray    # bool  [H][W]
    dmax: int


def _voronoi_labels(points: np.ndarray, W: int, H: int) -> np.ndarray:
    ys, xs = np.mgrid[0:H, 0:W]
    q = np.stack([xs.ravel() + 0.5, ys.ravel() + 0.5], axis=1)
    _, idx = cKDTree(points).query(q, k=1)
    return idx.reshape(H, W).astype(np.int64)


def make_pair(W: int, H: int, dmax: int, segments: int = 6,
              textureless: float = 0.0, seed: int = 0) -> StereoPair:
    """Draw one seeded synthetic pair of W x H uint8 RGB images."""
    if W < 2 or H < 2 or dmax < 1:
        raise ValueError("need W, H >= 2 and dmax >= 1")
    rng = np.random.default_rng(seed)
    K = int(segments)

    # 1. planar disparity segments
    seg_pts = rng.uniform([0.0, 0.0], [W, H], size=(K, 2))
    c0 = rng.uniform(0.0, dmax - 1, size=K)
    slope = rng.uniform(-0.15, 0.15, size=(K, 2))
    slope[0::2] = 0.0
    seg = _voronoi_labels(seg_pts, W, H)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    d = (c0[seg] + slope[seg, 0] * (xs - seg_pts[seg, 0])
         + slope[seg, 1] * (ys - seg_pts[seg, 1]))
    gt = np.clip(np.rint(d), 0, dmax - 1).astype(np.int64)

    # 2. colour regions = colour cells intersected with segments
    col_pts = rng.uniform([0.0, 0.0], [W, H], size=(4 * K, 2))
    cell = _voronoi_labels(col_pts, W, H)
    _, region = np.unique(seg * (4 * K) + cell, return_inverse=True)
    region = region.reshape(H, W)
    nreg = int(region.max()) + 1

    # 3. per-region colour model
    mean = rng.uniform(0.0, 255.0, size=(nreg, 3))
    grad = rng.uniform(-0.5, 0.5, size=(nreg, 2, 3))
    flat = rng.random(nreg) < textureless
    grad[flat] = 0.0
    sigma = np.where(flat, 0.5, 2.0)
    # reference point of each region: the colour seed of its cell
    ref_cell = np.zeros(nreg, dtype=np.int64)
    ref_cell[region.ravel()] = cell.ravel()
    ref = col_pts[ref_cell]
    r = region
    img = (mean[r]
           + grad[r, 0, :] * (xs - ref[r, 0])[..., None]
           + grad[r, 1, :] * (ys - ref[r, 1])[..., None])
    img = img + rng.standard_normal((H, W, 3)) * sigma[r][..., None]
    left = np.clip(np.rint(img), 0, 255).astype(np.uint8)

    # 4. forward warp with a z-buffer (larger disparity, then larger x, wins)
    xi = np.arange(W)[None, :].repeat(H, 0)
    yi = np.arange(H)[:, None].repeat(W, 1)
    tx = xi - gt
    ok = tx >= 0
    key = np.full((H, W), -1, dtype=np.int64)
    src_key = gt * W + xi
    np.maximum.at(key, (yi[ok], tx[ok]), src_key[ok])
    right = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
    hit = key >= 0
    win_x = np.where(hit, key % W, 0)
    right[hit] = left[yi[hit], win_x[hit]]
    nonocc = np.zeros((H, W), dtype=bool)
    tgt_key = key[yi[ok], tx[ok]]
    nonocc[yi[ok], xi[ok]] = tgt_key == src_key[ok]
    return StereoPair(left=left, right=right, gt=gt.astype(np.int16),
                      nonocc=nonocc, dmax=int(dmax))


def textured_shift_pair(W: int, H: int, shift: int, seed: int = 0):
    """Uniform-noise left image and its copy shifted by ``shift`` pixels.

    R(x, y) = L(x + shift, y) for x + shift < W; the right-most ``shift``
    columns of R are fresh noise.  Every left pixel with x >= shift has true
    disparity ``shift``.
    """
    rng = np.random.default_rng(seed)
    left = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
    right = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
    if shift > 0:
        right[:, : W - shift] = left[:, shift:]
    else:
        right[:] = left
    return left, right


def extremes_pair(W: int, H: int, block: int = 8, seed: int = 0):
    """Two independent images of ``block`` x ``block`` squares, each square
    black (0) or white (255) with probability 1/2.

    After the 2x downscale most half-resolution pixels are exactly 0 or 255,
    so matches with brightness differences of -255, 0 and +255 are all
    frequent: the ends of the absolute-difference table.
    """
    rng = np.random.default_rng(seed)
    by, bx = (H + block - 1) // block, (W + block - 1) // block

    def one():
        cells = rng.integers(0, 2, size=(by, bx), dtype=np.uint8) * np.uint8(255)
        img = np.repeat(np.repeat(cells, block, 0), block, 1)[:H, :W]
        return np.ascontiguousarray(np.repeat(img[..., None], 3, 2))

    left = one()
    return left, one()


# Workloads of the benchmark and parity suites (sizes and generator knobs).
WORKLOADS = {
    "small_320x240_d32": dict(W=320, H=240, dmax=32, segments=6,
                              textureless=0.0, seeds=[1]),
    "paper_1436x992_d145": dict(W=1436, H=992, dmax=145, segments=40,
                                textureless=0.1, seeds=[2]),
    "batch8_1920x1080_d256": dict(W=1920, H=1080, dmax=256, segments=60,
                                  textureless=0.1,
                                  seeds=list(range(300, 308))),
}


def workload_pairs(name: str, limit: int | None = None):
    """Generate the seeded pairs of a named workload."""
    w = WORKLOADS[name]
    seeds = w["seeds"] if limit is None else w["seeds"][:limit]
    return [make_pair(w["W"], w["H"], w["dmax"], w["segments"],
                      w["textureless"], s) for s in seeds]
