"""Seeded synthetic stereo pairs with ground-truth plane labels.

This module only *makes inputs*: textures, a piecewise planar / quadric
disparity field and the right view rendered from it.  It holds none of the
stereo method's arithmetic (no matching cost, filter, energy or move), so both
the FP64 oracle and the HIP library can be fed from it without sharing code.

Scene recipe (the paper evaluates on Middlebury pairs, which are not available
here; these scenes stand in for them with the same kind of structure):

* texture: per-channel uniform noise in [0, 255] smoothed by a 3x3 box filter
  with replicated borders;
* segments: a Voronoi partition of seeded sites;
* each segment carries a disparity surface centred at its site
  ``d = c + a*(u-us) + b*(v-vs) [+ k*((u-us)^2 + (v-vs)^2)]`` with
  ``a, b ~ U[-0.3, 0.3]``, ``c ~ U[c_lo, c_hi]`` and, for quadric segments,
  ``k ~ U[-1e-4, 1e-4]``; the non-constant part is shrunk by the smallest
  factor that keeps ``d`` inside ``[0, disp_max]`` on the segment;
* the right view is rendered by inverse warping: for every right pixel
  ``(x, v)`` each segment's equation ``u - d_s(u, v) = x`` is solved (closed
  form for planes, Newton steps for quadrics); a solution counts when the
  Voronoi owner of ``round(u)`` is that segment, the largest disparity wins
  (z-buffer), and the left image is sampled there by linear interpolation;
  disoccluded pixels take fresh noise;
* occlusion holes: seeded discs of radius 3..8 px in the right view filled
  with fresh noise until the requested fraction of pixels is covered.

Images are float32, HxWx3 (HWC), values in [0, 255]; u is the column and v the
row, both 0-based.  The ground-truth label of a pixel is the tangent plane
(a, b, c) of its segment's surface there, so ``d = a*u + b*v + c``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class StereoPair:
    left: np.ndarray        # (H, W, 3) float32
    right: np.ndarray       # (H, W, 3) float32
    gt_labels: np.ndarray   # (H, W, 3) float32, (a, b, c) per pixel
    gt_disp: np.ndarray     # (H, W) float32
    owner: np.ndarray       # (H, W) int32 segment index
    disp_max: float


def _box3(img: np.ndarray) -> np.ndarray:
    """3x3 mean with replicated borders, per channel."""
    p = np.pad(img, ((1, 1), (1, 1), (0, 0)), mode="edge")
    h, w = img.shape[:2]
    acc = np.zeros_like(img, dtype=np.float64)
    for dy in range(3):
        for dx in range(3):
            acc += p[dy:dy + h, dx:dx + w]
    return acc / 9.0


def _texture(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    return _box3(rng.uniform(0.0, 255.0, size=(h, w, 3)))


def _lerp_rows(img: np.ndarray, v: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Sample img[v, u] for float u (0 <= u <= W-1) by linear interpolation."""
    w = img.shape[1]
    i0 = np.floor(u).astype(np.int64)
    i0 = np.clip(i0, 0, w - 1)
    t = u - i0
    i1 = np.minimum(i0 + 1, w - 1)
    return (1.0 - t)[..., None] * img[v, i0] + t[..., None] * img[v, i1]


def make_pair(width: int, height: int, n_planar: int, n_quadric: int,
              disp_max: float, c_range: tuple, hole_frac: float,
              seed: int) -> StereoPair:
    rng = np.random.default_rng(seed)
    h, w = int(height), int(width)
    left = _texture(rng, h, w)
    fresh = _texture(rng, h, w)

    n = n_planar + n_quadric
    su = rng.uniform(0.0, w, n)
    sv = rng.uniform(0.0, h, n)
    a = rng.uniform(-0.3, 0.3, n)
    b = rng.uniform(-0.3, 0.3, n)
    c = rng.uniform(c_range[0], c_range[1], n)
    k = np.zeros(n)
    if n_quadric:
        k[n_planar:] = rng.uniform(-1e-4, 1e-4, n_quadric)

    vv, uu = np.mgrid[0:h, 0:w].astype(np.float64)
    d2 = (uu[None] - su[:, None, None]) ** 2 + (vv[None] - sv[:, None, None]) ** 2
    owner = np.argmin(d2, axis=0).astype(np.int32)
    del d2

    # Shrink each segment's non-constant part so that d stays in [0, disp_max].
    for s in range(n):
        m = owner == s
        if not m.any():
            continue
        du = uu[m] - su[s]
        dv = vv[m] - sv[s]
        g = a[s] * du + b[s] * dv + k[s] * (du * du + dv * dv)
        t = 1.0
        pos = g > 0
        neg = g < 0
        if pos.any():
            t = min(t, float(np.min((disp_max - c[s]) / g[pos])))
        if neg.any():
            t = min(t, float(np.min(c[s] / (-g[neg]))))
        t = max(t, 0.0)
        a[s] *= t
        b[s] *= t
        k[s] *= t

    # Ground truth: disparity and tangent plane per pixel.
    du = uu - su[owner]
    dv = vv - sv[owner]
    ks = k[owner]
    gt_disp = c[owner] + a[owner] * du + b[owner] * dv + ks * (du * du + dv * dv)
    ga = a[owner] + 2.0 * ks * du
    gb = b[owner] + 2.0 * ks * dv
    gc = gt_disp - ga * uu - gb * vv
    gt_labels = np.stack([ga, gb, gc], axis=-1)

    # Right view by inverse warping with a z-buffer on disparity.
    best_d = np.full((h, w), -np.inf)
    best_u = np.zeros((h, w))
    x = uu  # right-image column of each right pixel
    for s in range(n):
        denom = 1.0 - a[s]
        u = (x + c[s] - a[s] * su[s] + b[s] * (vv - sv[s])) / denom
        if k[s] != 0.0:
            for _ in range(3):
                ddu = u - su[s]
                ddv = vv - sv[s]
                g = u - (c[s] + a[s] * ddu + b[s] * ddv + k[s] * (ddu * ddu + ddv * ddv)) - x
                gp = 1.0 - (a[s] + 2.0 * k[s] * ddu)
                u = u - g / gp
        inside = (u >= 0.0) & (u <= w - 1)
        ur = np.clip(np.rint(u), 0, w - 1).astype(np.int64)
        ok = inside & (owner[vv.astype(np.int64), ur] == s)
        ddu = u - su[s]
        ddv = vv - sv[s]
        d = c[s] + a[s] * ddu + b[s] * ddv + k[s] * (ddu * ddu + ddv * ddv)
        take = ok & (d > best_d)
        best_d = np.where(take, d, best_d)
        best_u = np.where(take, u, best_u)
    vis = np.isfinite(best_d)
    vi = vv.astype(np.int64)
    right = np.where(vis[..., None], _lerp_rows(left, vi, np.clip(best_u, 0, w - 1)), fresh)

    # Occlusion holes.
    if hole_frac > 0.0:
        covered = np.zeros((h, w), dtype=bool)
        target = hole_frac * h * w
        while covered.sum() < target:
            cx = rng.uniform(0, w)
            cy = rng.uniform(0, h)
            rad = rng.uniform(3.0, 8.0)
            disc = (uu - cx) ** 2 + (vv - cy) ** 2 <= rad * rad
            covered |= disc
        right = np.where(covered[..., None], fresh, right)

    return StereoPair(left=left.astype(np.float32), right=right.astype(np.float32),
                      gt_labels=gt_labels.astype(np.float32),
                      gt_disp=gt_disp.astype(np.float32), owner=owner,
                      disp_max=float(disp_max))


def random_labels(rng: np.random.Generator, h: int, w: int, disp_max: float,
                  max_slope: float = 0.5) -> np.ndarray:
    """Arbitrary (a, b, c) label field for tests: planes through a random
    disparity in [0, disp_max] at each pixel with slopes in [-max_slope, max_slope]."""
    a = rng.uniform(-max_slope, max_slope, (h, w))
    b = rng.uniform(-max_slope, max_slope, (h, w))
    z = rng.uniform(0.0, disp_max, (h, w))
    vv, uu = np.mgrid[0:h, 0:w].astype(np.float64)
    c = z - a * uu - b * vv
    return np.stack([a, b, c], axis=-1).astype(np.float32)
