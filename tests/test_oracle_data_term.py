"""Pins of the oracle's data term against closed forms and brute force.

Matching cost: Eqs.(8),(9); guided-filter weights: Eq.(7); subregion
filtering: Eqs.(18)-(20).  Each pin is chosen so that a plausible mistake
(wrong warp sign, swapped interpolation weights, a swapped slope, a missing
border normalisation, a transposed covariance) fails at least one of them.
"""
import numpy as np
import pytest

from oracle import Oracle
from _util import base_params, texture

# The C library's fmaf (correctly rounded single-precision fused multiply-add),
# used only to reproduce the FP32 position the contract forms.
import ctypes as _C
import ctypes.util as _CU
_libm = _C.CDLL(_CU.find_library("m"))
_libm.fmaf.restype = _C.c_float
_libm.fmaf.argtypes = [_C.c_float, _C.c_float, _C.c_float]


def _FMA(p, q, s):
    return _libm.fmaf(float(p), float(q), float(s))


def _u(h, w):
    return np.broadcast_to(np.arange(w, dtype=np.float64)[None, :], (h, w))


@pytest.mark.parametrize("ch,coef", [(0, 0.299), (1, 0.587), (2, 0.114)])
def test_gray_coefficient_and_central_difference(ch, coef):
    # A ramp of slope 5 in one channel: gray slope 5*coef; the kernel
    # [-0.5 0 0.5] returns the slope inside and half of it at replicated borders.
    h, w = 3, 12
    img = np.zeros((h, w, 3), np.float32)
    img[:, :, ch] = 5.0 * _u(h, w)
    o = Oracle(base_params(w, h), img, img)
    gl, gr = o.grads()
    assert np.allclose(gl[:, 1:-1], 5.0 * coef, atol=1e-12)
    assert np.allclose(gl[:, [0, -1]], 2.5 * coef, atol=1e-12)
    assert np.array_equal(gl, gr)


def test_perfect_integer_shift_costs_zero_and_outside_costs_rho_max(rng):
    # Right view = left view shifted by c: the fronto-parallel label c matches
    # exactly, so rho = 0 where both gradients are interior; samples left of
    # the image cost the fully truncated value.
    h, w, c = 6, 30, 4
    left = texture(rng, h, w)
    right = np.array(texture(rng, h, w))
    right[:, : w - c] = left[:, c:]
    o = Oracle(base_params(w, h), left, right)
    f = np.array([0, 0, c], np.float32)
    rho = o.rho_map(f)
    assert np.allclose(rho[:, c + 1: w - 2], 0.0, atol=1e-12)
    assert np.all(rho[:, :c] == o.rho_max)
    assert o.rho_max == pytest.approx(0.1 * 10 + 0.9 * 2, abs=1e-15)
    wrong = o.rho_map(np.array([0, 0, c + 1], np.float32))
    assert wrong[:, c + 2: w - 2].mean() > 1.0


@pytest.mark.parametrize("delta,expect", [(1.0, 0.3), (2.0, 0.6), (3.0, 0.9), (5.0, 1.0)])
def test_colour_term_l1_and_truncation(rng, delta, expect):
    # Right = left + delta in every channel: the gray gradient is unchanged and
    # the L1 colour difference is 3*delta, truncated at tau_col = 10.
    h, w = 4, 16
    left = texture(rng, h, w)
    o = Oracle(base_params(w, h), left, left + np.float32(delta))
    rho = o.rho_map(np.zeros(3, np.float32))
    assert np.allclose(rho, expect, atol=1e-9)


@pytest.mark.parametrize("s", [0.5, 1.5, 3.0])
def test_gradient_term_and_truncation(rng, s):
    # Right = left + s*u in every channel: colour difference 3*s*u, gray
    # gradient difference s inside (s/2 at the replicated borders), truncated at 2.
    h, w = 4, 20
    left = texture(rng, h, w)
    right = left + np.float32(s) * _u(h, w)[..., None].astype(np.float32)
    o = Oracle(base_params(w, h), left, right)
    rho = o.rho_map(np.zeros(3, np.float32))
    u = np.arange(1, w - 1)
    expect = 0.1 * np.minimum(3 * s * u, 10.0) + 0.9 * min(s, 2.0)
    assert np.allclose(rho[:, 1:-1], expect[None, :], atol=1e-4)


def test_linear_interpolation_and_slanted_warp_exact_on_linear_images():
    # Right view linear in x: interpolation is exact, so a left view built as
    # the right view warped by a slanted plane is matched with zero cost by that
    # plane, and a fronto-parallel label off by 0.25 px costs 0.1*sum|m|*0.25.
    h, w = 10, 40
    m = np.array([1.0, 2.0, 3.0])
    q = np.array([10.0, 20.0, 30.0])
    x = np.arange(w, dtype=np.float64)
    right = (m[None, None, :] * x[None, :, None] + q).repeat(h, axis=0).astype(np.float32)
    a, b, c = 0.1, -0.05, 3.3
    vv, uu = np.mgrid[0:h, 0:w].astype(np.float64)
    d = a * uu + b * vv + c
    left = (m[None, None, :] * (uu - d)[..., None] + q).astype(np.float32)
    o = Oracle(base_params(w, h), left, right)
    rho = o.rho_map(np.array([a, b, c], np.float32))
    xs = uu - d
    ok = (xs >= 1.0) & (xs <= w - 2) & (uu >= 1) & (uu <= w - 2)
    assert ok.sum() > 200
    # left gradient is (1-a)*gray slope, right gradient is the gray slope.
    gslope = float(0.299 * m[0] + 0.587 * m[1] + 0.114 * m[2])
    expect = 0.9 * min(abs(a * gslope), 2.0)
    assert np.allclose(rho[ok], expect, atol=2e-4)
    # fronto-parallel pair, fractional shift 2.25 vs 2.0
    left2 = (m[None, None, :] * (uu - 2.25)[..., None] + q).astype(np.float32)
    o2 = Oracle(base_params(w, h), left2, right)
    r_ok = o2.rho_map(np.array([0, 0, 2.25], np.float32))[:, 4:-2]
    r_off = o2.rho_map(np.array([0, 0, 2.0], np.float32))[:, 4:-2]
    assert np.allclose(r_ok, 0.0, atol=2e-5)
    assert np.allclose(r_off, 0.1 * m.sum() * 0.25, atol=2e-5)


def test_cost_continuous_across_integer_positions(rng):
    h, w = 5, 30
    o = Oracle(base_params(w, h), texture(rng, h, w), texture(rng, h, w))
    lo = o.rho_map(np.array([0, 0, 3.0 - 1e-3], np.float32))
    hi = o.rho_map(np.array([0, 0, 3.0 + 1e-3], np.float32))
    assert np.max(np.abs(lo - hi)[:, 5:]) < 0.2


# ---------------------------------------------------------------------------
# Guided filter, Eq.(7) and its box form.
# ---------------------------------------------------------------------------

def _box_mean(x, r):
    """Count-normalised mean over the clipped (2r+1)^2 window, by brute force."""
    h, w = x.shape
    out = np.zeros_like(x)
    for v in range(h):
        for u in range(w):
            out[v, u] = x[max(v - r, 0): v + r + 1, max(u - r, 0): u + r + 1].mean()
    return out


def test_filter_of_constant_is_constant_everywhere(rng):
    h, w, r = 14, 20, 3
    o = Oracle(base_params(w, h, r), texture(rng, h, w), texture(rng, h, w))
    out = o.filter_map(np.full((h, w), 1.7))
    assert np.allclose(out, 1.7, atol=1e-11)


def test_constant_guide_reduces_to_box_of_box(rng):
    # With a constant guide Sigma_k = 0 and the covariance term vanishes, so
    # a_k = 0, b_k = mean(rho) and phi = box(box(rho)), count-normalised.
    h, w, r = 13, 17, 2
    left = np.zeros((h, w, 3), np.float32) + np.array([100, 50, 200], np.float32)
    o = Oracle(base_params(w, h, r), left, texture(rng, h, w))
    rho = rng.uniform(0, 3, (h, w))
    assert np.allclose(o.filter_map(rho), _box_mean(_box_mean(rho, r), r), atol=1e-9)


def test_linear_model_of_the_guide_is_reproduced(rng):
    # Guided-filter exactness: rho = c^T I + d0 with I = I_L/255 and e -> 0
    # gives a_k = c, b_k = d0, hence phi = rho.
    h, w, r = 16, 18, 2
    left = texture(rng, h, w)
    I = left.astype(np.float64) / 255.0
    rho = I @ np.array([0.5, -0.3, 0.8]) + 1.2
    o = Oracle(base_params(w, h, r, gf_eps=1e-12), left, left)
    assert np.allclose(o.filter_map(rho), rho, atol=1e-6)


def test_direct_eq7_equals_box_form_at_every_pixel(rng):
    h, w, r = 12, 15, 2
    o = Oracle(base_params(w, h, r), texture(rng, h, w), texture(rng, h, w))
    for f in ([0, 0, 1.5], [0.2, -0.1, 3.0]):
        f = np.array(f, np.float32)
        full = o.unary_region((0, 0, w, h), f)
        direct = np.array([[o.unary_direct(u, v, f) for u in range(w)] for v in range(h)])
        assert np.allclose(direct, full, atol=1e-10)


def test_weights_sum_to_one_and_are_symmetric_inside(rng):
    h, w, r = 24, 24, 2
    o = Oracle(base_params(w, h, r), texture(rng, h, w), texture(rng, h, w))
    side = 4 * r + 1
    for (pu, pv) in [(0, 0), (3, 11), (23, 5), (12, 12)]:
        assert o.gf_weights(pu, pv).sum() == pytest.approx(1.0, abs=1e-12)
    # interior pair p, s with every window involved unclipped
    p, s = (11, 12), (13, 10)
    wp = o.gf_weights(*p)
    ws = o.gf_weights(*s)
    w_ps = wp[s[1] - p[1] + 2 * r, s[0] - p[0] + 2 * r]
    w_sp = ws[p[1] - s[1] + 2 * r, p[0] - s[0] + 2 * r]
    assert w_ps == pytest.approx(w_sp, abs=1e-14)
    assert side == wp.shape[0]


@pytest.mark.parametrize("rect", [(0, 0, 5, 5), (6, 3, 13, 9), (12, 8, 40, 40), (7, 7, 8, 8),
                                  (-3, -3, 2, 30), (0, 0, 19, 14)])
def test_subregion_filter_equals_whole_image_filter(rng, rect):
    # Region independence: M = R dilated by 2r carries every sample that
    # reaches phi over R, so the subregion result equals filtering rho over
    # the whole image and reading it at R.
    h, w, r = 14, 19, 2
    o = Oracle(base_params(w, h, r), texture(rng, h, w), texture(rng, h, w))
    f = np.array([0.15, 0.05, 2.5], np.float32)
    full = o.filter_map(o.rho_map(f))
    u0, v0, u1, v1 = rect
    u0, v0, u1, v1 = max(u0, 0), max(v0, 0), min(u1, w), min(v1, h)
    assert np.allclose(o.unary_region(rect, f), full[v0:v1, u0:u1], atol=1e-11)


def test_coefficients_match_whole_image_definition(rng):
    # a_k, b_k exported over R+ agree with the plain per-k regression solved
    # here with numpy's least squares on the window samples (ridge e).
    h, w, r = 12, 14, 2
    left = texture(rng, h, w)
    o = Oracle(base_params(w, h, r), left, texture(rng, h, w))
    f = np.array([0.0, 0.1, 2.0], np.float32)
    rho = o.rho_map(f)
    ab = o.coeffs_region((4, 3, 9, 8), f)
    I = left.astype(np.float64) / 255.0
    e = 1e-4
    for (ku, kv) in [(2, 1), (5, 5), (10, 9)]:
        win = (slice(max(kv - r, 0), kv + r + 1), slice(max(ku - r, 0), ku + r + 1))
        X = I[win].reshape(-1, 3)
        y = rho[win].reshape(-1)
        n = len(y)
        Xc = X - X.mean(0)
        # ridge regression y ~ a^T I + b with penalty n*e*|a|^2 (He et al.)
        a = np.linalg.solve(Xc.T @ Xc / n + e * np.eye(3), Xc.T @ (y - y.mean()) / n)
        b = y.mean() - a @ X.mean(0)
        got = ab[kv - 1, ku - 2]
        assert np.allclose(got[:3], a, atol=1e-8) and got[3] == pytest.approx(b, abs=1e-8)


# ---------------------------------------------------------------------------
# The warp of Eq. (8) in single precision (the position that selects the
# interpolation taps and the in-view test is formed in FP32 on both sides)
# against the same warp in FP64.
# ---------------------------------------------------------------------------
def _ulp32(x):
    """Spacing of float32 at |x| (rounded up to the next binade edge)."""
    a = np.abs(np.asarray(x, np.float64)) * (1.0 + 2.0 ** -20) + 1e-30
    return 2.0 ** (np.floor(np.log2(a)) - 23.0)


def _rho_fp64_warp(o, left, right, f, alpha=0.9, tau_col=10.0, tau_grad=2.0):
    """Eqs. (8), (9) with x = u - (a u + b v + c) in FP64 from the FP32 label:
    the raw cost per pixel, the taps' floor, the in-view flag and the local
    slope |d rho / d x| bound at the taps."""
    h, w = left.shape[:2]
    gl, gr = o.grads()
    a, b, c = (float(t) for t in np.asarray(f, np.float32))
    v, u = np.mgrid[0:h, 0:w].astype(np.float64)
    x = u - (a * u + b * v + c)
    inview = (x >= 0.0) & (x <= w - 1)
    xc = np.where(inview, x, 0.0)
    i0 = np.floor(xc).astype(np.int64)
    t = xc - i0
    i1 = np.minimum(i0 + 1, w - 1)
    t = np.where(i0 >= w - 1, 0.0, t)
    rows = v.astype(np.int64)
    R0, R1 = right[rows, i0].astype(np.float64), right[rows, i1].astype(np.float64)
    J = (1.0 - t)[..., None] * R0 + t[..., None] * R1
    col = np.abs(left.astype(np.float64) - J).sum(-1)
    K = (1.0 - t) * gr[rows, i0] + t * gr[rows, i1]
    grd = np.abs(gl - K)
    rho = (1.0 - alpha) * np.minimum(col, tau_col) + alpha * np.minimum(grd, tau_grad)
    rho = np.where(inview, rho, (1.0 - alpha) * tau_col + alpha * tau_grad)
    slope = (1.0 - alpha) * np.abs(R1 - R0).sum(-1) + alpha * np.abs(gr[rows, i1] - gr[rows, i0])
    # error of the FP32 contract: the inner and the outer fused multiply-add
    # and the subtraction each round once to float32
    eps = 0.5 * (_ulp32(b * v + c) + _ulp32(a * u + b * v + c) + _ulp32(x)) + 1e-12
    return rho, x, inview, i0, slope, eps


def test_fp32_warp_contract_against_fp64_warp(rng):
    """The oracle forms the sample position in FP32 (the same contract as the
    device).  Against the warp in FP64: wherever the in-view test and the taps
    agree, rho differs by at most the local slope times the FP32 rounding of
    the position; wherever they disagree, the FP64 position lies within that
    rounding of an integer, of 0 or of W-1.  The change this makes to phi is
    bounded through the direct weights of Eq. (7)."""
    h, w, r = 12, 450, 5
    left, right = texture(rng, h, w), texture(rng, h, w)
    o = Oracle(base_params(w, h, r, disp_max=60.0), left, right)
    labels = [rng.uniform([-0.3, -0.3, 0.0], [0.3, 0.3, 60.0]) for _ in range(12)]
    labels += [rng.uniform([-3.0, -3.0, -100.0], [3.0, 3.0, 100.0]) for _ in range(6)]
    # fronto-parallel labels one ulp away from an integer shift (positions a
    # rounding away from the taps' edges) and labels whose warp ends near the
    # image's last column
    for k in (3.0, 17.0, 41.0):
        labels += [[0.0, 0.0, np.nextafter(np.float32(k), np.float32(0))],
                   [0.0, 0.0, np.nextafter(np.float32(k), np.float32(100))]]
    labels += [[1.0 - 2.0 ** -12, 0.0, -(w - 1) * 2.0 ** -12], [2.0 ** -13, 1e-4, 0.0]]
    n_diff = n_all = 0
    worst_rel = 0.0
    dphi_max = 0.0
    for f in labels:
        f = np.asarray(f, np.float32)
        rho32 = o.rho_map(f)
        rho64, x64, in64, i0_64, slope, eps = _rho_fp64_warp(o, left, right, f)
        # the oracle's own decision at each pixel, recovered from its rho: a
        # sample it takes in view costs what FP64 computes at the taps floor(x32)
        a, b, c = (np.float32(t) for t in f)
        fmaf = np.frompyfunc(lambda p, q, s: float(np.float32(_FMA(np.float32(p), np.float32(q), np.float32(s)))),
                             3, 1)
        v, u = np.mgrid[0:h, 0:w].astype(np.float32)
        d32 = fmaf(a, u, fmaf(b, v, c)).astype(np.float32)
        x32 = (u - d32).astype(np.float32).astype(np.float64)
        assert np.all(np.abs(x32 - x64) <= eps), "FP32 position beyond its rounding bound"
        in32 = (x32 >= 0.0) & (x32 <= w - 1)
        i0_32 = np.floor(np.where(in32, x32, 0.0))
        agree = (in32 == in64) & (~in64 | (i0_32 == i0_64))
        n_all += agree.size
        n_diff += int((~agree).sum())
        # same decisions: rho differs by the slope times the position's rounding
        err = np.abs(rho32 - rho64)
        assert np.all(err[agree] <= slope[agree] * np.abs(x32 - x64)[agree] + 1e-9)
        worst_rel = max(worst_rel, float(np.max(np.abs(x32 - x64) / np.maximum(eps, 1e-30))))
        # different decisions: only within the rounding of an edge
        dist = np.minimum(np.abs(x64 - np.round(x64)), np.minimum(np.abs(x64), np.abs(x64 - (w - 1))))
        assert np.all(dist[~agree] <= eps[~agree]), "a decision differs away from a tap or image edge"
        # phi at sampled pixels: |phi32 - phi64| <= sum_s |w_ps| |rho32 - rho64|
        for pu, pv in [(5, 3), (200, 6), (w - 3, 9), (37, 0)]:
            wts = o.gf_weights(pu, pv)
            s0u, s0v = pu - 2 * r, pv - 2 * r
            vs, us = np.mgrid[0:wts.shape[0], 0:wts.shape[1]]
            su, sv = us + s0u, vs + s0v
            ok = (su >= 0) & (su < w) & (sv >= 0) & (sv < h)
            d32p = float(np.sum(wts[ok] * rho32[sv[ok], su[ok]]))
            d64p = float(np.sum(wts[ok] * rho64[sv[ok], su[ok]]))
            bound = float(np.sum(np.abs(wts[ok]) * err[sv[ok], su[ok]]))
            assert abs(d32p - d64p) <= bound + 1e-12
            assert d32p == pytest.approx(o.unary_direct(pu, pv, f), abs=1e-10)
            dphi_max = max(dphi_max, abs(d32p - d64p))
    assert n_diff > 0, "no sample near a tap edge: the classification above was never exercised"
    print(f"\nFP32 warp vs FP64: {n_diff} of {n_all} samples decided differently (all within rounding of an "
          f"edge); largest |x32 - x64| / bound {worst_rel:.2f}; largest |phi32 - phi64| {dphi_max:.2e}")
