"""Named workloads: scene recipe plus the method settings each is run with.

Method settings follow the paper's experimental section (data term
e = 0.01^2, tau_col = 10, tau_grad = 2, alpha = 0.9; smoothness lambda = 1,
tau_dis = 1, epsilon = 0.01, gamma = 10; eight neighbours; 5/15/25-pixel grid
cells).  ``gf_radius`` is the radius r of the guided filter's local regression
window W'_k, which is (2r+1)^2 pixels, so the matching window W_p is
(4r+1)^2.  ``grids`` lists (cell size, K_prop, K_rand) per grid level.
"""
from __future__ import annotations

import numpy as np

from .scenes import make_pair, StereoPair

PAPER_PARAMS = dict(alpha=0.9, tau_col=10.0, tau_grad=2.0, gf_eps=1e-4,
                    lam=1.0, tau_dis=1.0, w_floor=0.01, gamma=10.0, neighbours=8)

WORKLOADS = {
    # 64x48, 4 planar segments, disparity [0,16], r=5 (11x11 W'_k).
    "tiny-64x48": dict(
        scene=dict(width=64, height=48, n_planar=4, n_quadric=0, disp_max=16.0,
                   c_range=(2.0, 14.0), hole_frac=0.0, seed=0),
        gf_radius=5, grids=[(5, 1, 3)], iterations=2, solver_seed=0),
    # 450x375, 12 planar + 2 quadric segments, 2% holes, disparity [0,60], r=20.
    "lowres-450x375": dict(
        scene=dict(width=450, height=375, n_planar=12, n_quadric=2, disp_max=60.0,
                   c_range=(7.5, 52.5), hole_frac=0.02, seed=1),
        gf_radius=20, grids=[(5, 1, 7), (15, 1, 7), (25, 1, 7)], iterations=10,
        solver_seed=0),
    # 1500x1000, 40 planar + 6 quadric segments, 2% holes, disparity [0,200], r=20.
    "highres-1500x1000": dict(
        scene=dict(width=1500, height=1000, n_planar=40, n_quadric=6, disp_max=200.0,
                   c_range=(25.0, 175.0), hole_frac=0.02, seed=2),
        gf_radius=20, grids=[(5, 1, 7), (15, 1, 7), (25, 1, 7)], iterations=10,
        solver_seed=0),
}


def workload(name: str) -> dict:
    return WORKLOADS[name]


def make_workload_pair(name: str) -> StereoPair:
    return make_pair(**WORKLOADS[name]["scene"])


def params_for(name: str) -> dict:
    """Flat parameter dict (image size, disparity range, filter radius, paper settings)."""
    wl = WORKLOADS[name]
    sc = wl["scene"]
    p = dict(PAPER_PARAMS)
    p.update(width=sc["width"], height=sc["height"], disp_max=sc["disp_max"],
             gf_radius=wl["gf_radius"])
    return p


def many_pair_scenes(n_pairs: int = 64, seed0: int = 3000):
    """Scene recipes of the uneven-size many-pair batch: width ~ U[320,1500],
    height = 0.67*width rounded to a multiple of 8, disparity range 0.13*width,
    otherwise generated like the 450x375 scene."""
    out = []
    for i in range(n_pairs):
        rng = np.random.default_rng(seed0 + i)
        w = int(rng.integers(320, 1501))
        h = int(round(0.67 * w / 8.0)) * 8
        dmax = float(round(0.13 * w))
        out.append(dict(width=w, height=h, n_planar=12, n_quadric=2, disp_max=dmax,
                        c_range=(dmax / 8.0, 7.0 * dmax / 8.0), hole_frac=0.02,
                        seed=seed0 + i))
    return out
