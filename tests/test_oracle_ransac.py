"""Pins of the oracle's RANSAC proposer (Alg. 1: a plane fitted to the current
disparity map over the centre cell by LO-RANSAC) against exact planes, gross
outliers, an independent least-squares solver (numpy) and the degenerate
cells where no plane is defined."""
import numpy as np
import pytest

from oracle import Oracle
from _util import base_params, texture

TAU = 1.0  # inlier threshold in disparity (a reading: the paper names LO-RANSAC only)


def _oracle(w, h, seed=3):
    rng = np.random.default_rng(seed)
    return Oracle(base_params(w, h), texture(rng, h, w), texture(rng, h, w))


def _ransac(o, lab, cell, ci, cj, seed=5, iteration=0):
    # Alg. 1 order: step 0 propagation (k_prop = 1), step 1 RANSAC (k_rans = 1)
    return o.propose(lab, seed, iteration, 0, cell, ci, cj, 1, 1, 8.0, 1.0, k_rans=1)


def _set_disparities(lab, cell, ci, cj, fn):
    """Fronto-parallel labels whose disparity at each pixel of the cell is fn(u, v)."""
    h, w = lab.shape[:2]
    for v in range(cj * cell, min((cj + 1) * cell, h)):
        for u in range(ci * cell, min((ci + 1) * cell, w)):
            lab[v, u] = (0.0, 0.0, fn(u, v))


@pytest.mark.parametrize("cell,ci,cj", [(5, 3, 2), (15, 1, 1), (25, 1, 0)])
def test_ransac_recovers_an_exact_plane(cell, ci, cj):
    o = _oracle(60, 40)
    lab = o.init_labels(1)
    a, b, c = 0.25, -0.125, 10.5  # exact in binary: every disparity of the cell is exact
    for v in range(40):
        for u in range(60):
            lab[v, u] = (a, b, c)
    out = _ransac(o, lab, cell, ci, cj)
    assert np.array_equal(out, np.array([a, b, c], np.float32))


@pytest.mark.parametrize("cell,ci,cj,frac", [(15, 1, 1, 0.3), (25, 1, 0, 0.45), (5, 4, 3, 0.2)])
def test_ransac_ignores_gross_outliers(cell, ci, cj, frac):
    rng = np.random.default_rng(cell)
    o = _oracle(60, 40)
    lab = o.init_labels(1)
    a, b, c = 0.1234, -0.2345, 17.0
    _set_disparities(lab, cell, ci, cj, lambda u, v: a * u + b * v + c)
    pix = [(u, v) for v in range(cj * cell, min((cj + 1) * cell, 40)) for u in range(ci * cell, min((ci + 1) * cell, 60))]
    bad = rng.choice(len(pix), int(frac * len(pix)), replace=False)
    for q in bad:
        u, v = pix[q]
        lab[v, u] = (0.0, 0.0, a * u + b * v + c + rng.choice([-1, 1]) * rng.uniform(5, 30))
    out = _ransac(o, lab, cell, ci, cj).astype(np.float64)
    for u, v in pix:
        assert abs(out[0] * u + out[1] * v + out[2] - (a * u + b * v + c)) < 1e-4


def test_ransac_result_is_the_least_squares_plane_of_its_inliers():
    """Noisy inliers (|noise| <= 0.4) and outliers off by 3 or more: the
    inlier set is unambiguous and the result must equal numpy's least-squares
    plane of it (an independent solver for the local-optimisation step)."""
    rng = np.random.default_rng(7)
    o = _oracle(60, 40)
    cell, ci, cj = 25, 1, 0
    lab = o.init_labels(2)
    a, b, c = -0.17, 0.08, 23.0
    truth = {}
    for v in range(cj * cell, (cj + 1) * cell):
        for u in range(ci * cell, (ci + 1) * cell):
            if rng.random() < 0.25:
                d = a * u + b * v + c + rng.choice([-1, 1]) * rng.uniform(3, 20)
                inl = False
            else:
                d = a * u + b * v + c + rng.uniform(-0.4, 0.4)
                inl = True
            lab[v, u] = (0.0, 0.0, d)
            truth[(u, v)] = (float(np.float32(d)), inl)
    out = _ransac(o, lab, cell, ci, cj).astype(np.float64)
    pts = [(u, v, d) for (u, v), (d, inl) in truth.items() if inl]
    A = np.array([[u, v, 1.0] for u, v, _ in pts])
    y = np.array([d for _, _, d in pts])
    ls = np.linalg.lstsq(A, y, rcond=None)[0]
    assert np.allclose(out, ls, rtol=1e-6, atol=1e-5), (out, ls)
    # and the inlier set of the result is exactly the true inlier set
    got = {(u, v) for (u, v), (d, _) in truth.items() if abs(d - (out[0] * u + out[1] * v + out[2])) <= TAU}
    assert got == {(u, v) for (u, v), (_, inl) in truth.items() if inl}


@pytest.mark.parametrize("w,h,ci,cj", [(61, 40, 12, 3), (60, 41, 5, 8), (61, 41, 12, 8)])
def test_ransac_on_degenerate_cells_falls_back_to_propagation(w, h, ci, cj):
    """Clipped edge cells one pixel wide or high (collinear pixels) or of a
    single pixel define no plane: the candidate is the label of the pixel the
    propagation proposer draws for the same step."""
    o = _oracle(w, h)
    lab = o.init_labels(4)
    for seed in range(5):
        out = _ransac(o, lab, 5, ci, cj, seed=seed)
        prop = o.propose(lab, seed, 0, 0, 5, ci, cj, 1, 2, 8.0, 1.0)  # step 1 < k_prop = 2: propagation
        assert np.array_equal(out, prop)


def test_ransac_steps_in_the_optimisation_lower_the_energy():
    """Alg. 1 with one RANSAC step between propagation and refinement: the
    energy never rises, and every step is one expansion of its region."""
    o = _oracle(40, 30, seed=9)
    lab, cost, e, ev = o.optimize(0, [(5, 1, 2, 1)], 2)
    assert np.all(np.diff(e) <= 1e-9)
    regions = 0
    for cj in range(6):
        for ci in range(8):
            u0, v0, u1, v1 = max((ci - 1) * 5, 0), max((cj - 1) * 5, 0), min((ci + 2) * 5, 40), min((cj + 2) * 5, 30)
            regions += (u1 - u0) * (v1 - v0)
    assert ev == 40 * 30 + 2 * 4 * regions
