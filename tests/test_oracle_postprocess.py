"""Pins of the right-view data term and of the post-processing in the oracle.

Right view: the paper defines it by swapping I_L and I_R in Eqs. (7) and (9)
and adding the disparity in the warp; the oracle evaluates it as the left-view
term of the mirrored pair, which is checked here against the swapped formula
evaluated directly and against a perfect shift.  Post-processing (left-right
check, row filling, weighted median): closed forms on constant maps, a step
edge with its occlusion, equal-weight medians and colour edges."""
import numpy as np
import pytest

from oracle import Oracle
from _util import base_params, texture

ALPHA, TAU_C, TAU_G = 0.9, 10.0, 2.0


def _gray(img):
    return 0.299 * img[..., 0] + 0.587 * img[..., 1] + 0.114 * img[..., 2]


def _gradx(img):
    g = _gray(img.astype(np.float64))
    p = np.pad(g, ((0, 0), (1, 1)), mode="edge")
    return 0.5 * (p[:, 2:] - p[:, :-2])


def _mirror_label(f, W):
    a, b, c = (float(x) for x in f)
    return np.array([-a, b, c + a * (W - 1)], np.float32)


def test_right_view_raw_cost_is_eq9_with_images_swapped_and_disparity_added():
    rng = np.random.default_rng(4)
    W, H = 50, 20
    L, R = texture(rng, H, W), texture(rng, H, W)
    o = Oracle.right_view(base_params(W, H), L, R)
    gL, gR = _gradx(L), _gradx(R)
    n = 0
    for _ in range(400):
        x, v = int(rng.integers(0, W)), int(rng.integers(0, H))
        a, b = rng.uniform(-0.3, 0.3, 2)
        c = rng.uniform(-5, 20)
        f = np.array([a, b, c], np.float32)
        fm = _mirror_label(f, W)
        d = float(fm[0]) * (W - 1 - x) + float(fm[1]) * v + float(fm[2])  # the same plane, mirrored
        s = x + d  # the paper's warp for the right view: add the disparity
        if abs(s - round(s)) < 1e-4 or abs(s) < 1e-4 or abs(s - (W - 1)) < 1e-4:
            continue  # the tap choice is made in FP32; skip positions where that decides
        if s < 0 or s > W - 1:
            expect = (1 - ALPHA) * TAU_C + ALPHA * TAU_G
        else:
            i0 = int(np.floor(s))
            t = s - i0
            i1 = min(i0 + 1, W - 1)
            J = (1 - t) * L[v, i0].astype(np.float64) + t * L[v, i1]
            K = (1 - t) * gL[v, i0] + t * gL[v, i1]
            expect = (1 - ALPHA) * min(np.abs(R[v, x].astype(np.float64) - J).sum(), TAU_C) + \
                ALPHA * min(abs(gR[v, x] - K), TAU_G)
        got = o.raw_cost(W - 1 - x, v, fm)
        # the sample position is formed in FP32 (as in the left view): a few
        # 1e-6 px of position, times the image slope, separate the two
        assert abs(got - expect) < 1e-3, (x, v, s, got, expect)
        n += 1
    assert n > 300


def test_right_view_perfect_shift_costs_zero():
    """If the right image is the left one shifted by k (I_R(x) = I_L(x + k)),
    the right view's fronto-parallel label d = k costs zero wherever x + k lies
    inside the image (away from the replicated-gradient border)."""
    rng = np.random.default_rng(5)
    W, H, k = 48, 12, 6
    L = texture(rng, H, W)
    R = np.zeros_like(L)
    R[:, :W - k] = L[:, k:]
    R[:, W - k:] = texture(rng, H, k)
    o = Oracle.right_view(base_params(W, H), L, R)
    for v in range(H):
        for x in range(1, W - k - 1):
            assert o.raw_cost(W - 1 - x, v, np.array([0, 0, k], np.float32)) < 1e-9


def _fronto(d):
    lab = np.zeros(d.shape + (3,), np.float32)
    lab[..., 2] = d
    return lab


def _mirror_field(lab):
    """Right-view labels in the mirrored frame of a right-image label field."""
    W = lab.shape[1]
    out = lab[:, ::-1].copy()
    out[..., 2] = lab[:, ::-1, 2] + lab[:, ::-1, 0] * (W - 1)
    out[..., 0] = -lab[:, ::-1, 0]
    return out


def test_postprocess_constant_maps():
    rng = np.random.default_rng(6)
    W, H, k = 40, 10, 5
    o = Oracle(base_params(W, H), texture(rng, H, W), texture(rng, H, W))
    left = _fronto(np.full((H, W), float(k)))
    right = _mirror_field(_fronto(np.full((H, W), float(k))))
    disp, inv = o.postprocess(left, right)
    expect_inv = np.zeros((H, W), np.uint8)
    expect_inv[:, :k] = 1  # u - k < 0: no match in the right image
    assert np.array_equal(inv, expect_inv)
    assert np.all(disp == k)


def test_postprocess_step_edge_invalidates_the_occlusion_and_fills_with_background():
    """Background d=4 left of u=20, foreground d=10 from u=20.  In the right
    image the foreground covers x >= 10, so left pixels 14..19 (background,
    matching x = 10..15) and 0..3 (matching x < 0) are inconsistent; they are
    filled with the background plane (the lower disparity)."""
    rng = np.random.default_rng(7)
    W, H = 40, 8
    img = np.full((H, W, 3), 100.0, np.float32)  # uniform colour: equal median weights
    o = Oracle(base_params(W, H), img, texture(rng, H, W))
    dl = np.where(np.arange(W)[None, :] < 20, 4.0, 10.0) * np.ones((H, 1))
    # right map by forward warping the left one with a z-buffer (larger disparity wins)
    dr = np.full((H, W), np.nan)
    for u in range(W):
        x = u - int(dl[0, u])
        if 0 <= x < W and not (dr[0, x] >= dl[0, u]):
            dr[:, x] = dl[0, u]
    dr = np.where(np.isnan(dr), 10.0, dr)  # right-border pixels seen by nothing: any value
    disp, inv = o.postprocess(_fronto(dl), _mirror_field(_fronto(dr)))
    expect = np.zeros(W, np.uint8)
    expect[:4] = 1
    expect[14:20] = 1
    assert np.array_equal(inv, np.tile(expect, (H, 1)))
    assert np.all(disp[:, 14:20] == 4.0)
    assert np.all(disp[:, :4] == 4.0)
    assert np.all(disp[inv == 0] == dl[inv == 0])


def test_weighted_median_with_equal_weights_is_the_lower_median():
    """A uniform image gives every window pixel the same weight, so the
    weighted median is the ceil(n/2)-th smallest value of the window.  All
    pixels are made inconsistent (right map offset by 50) and no row has a
    consistent pixel, so the filled values are the pixels' own disparities."""
    rng = np.random.default_rng(8)
    W, H, R = 45, 40, 17
    img = np.full((H, W, 3), 50.0, np.float32)
    o = Oracle(base_params(W, H), img, img)
    dl = rng.uniform(0, 12, (H, W))
    disp, inv = o.postprocess(_fronto(dl), _mirror_field(_fronto(dl + 50.0)))
    assert inv.all()
    dl32 = _fronto(dl)[..., 2].astype(np.float64)
    for (v, u) in [(0, 0), (20, 22), (39, 44), (5, 30), (33, 3)]:
        win = np.sort(dl32[max(v - R, 0):v + R + 1, max(u - R, 0):u + R + 1].ravel())
        assert disp[v, u] == win[(win.size + 1) // 2 - 1]


def test_weighted_median_keeps_to_its_colour_region():
    """Two colour regions whose L1 colour distance (3 x 200) makes the cross
    weights quantise to zero: every pixel takes the median of its own region,
    whatever share of the window the other region covers."""
    W, H = 40, 30
    img = np.zeros((H, W, 3), np.float32)
    img[:, 25:] = 200.0
    o = Oracle(base_params(W, H), img, img)
    dl = np.where(np.arange(W)[None, :] < 25, 3.0, 7.0) * np.ones((H, 1))
    disp, inv = o.postprocess(_fronto(dl), _mirror_field(_fronto(dl + 50.0)))
    assert inv.all()
    assert np.all(disp[:, :25] == 3.0) and np.all(disp[:, 25:] == 7.0)
