"""Pins of the oracle's smoothness term, energy, expansion move, random
numbers and scheduler.

Smoothness term: Eqs.(10)-(12) and its properties stated in Sec. 3.2 (zero
for equal labels, 2|c_p-c_q| for fronto-parallel labels, Lemma 1).  Energy:
Eq.(5) with eight neighbours.  Expansion: Eq.(13) restricted to R, solved
exactly (checked against exhaustive enumeration).  Scheduler: Eq.(15) and
Lemma 3; random initialisation and perturbation of Sec. 3.4.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import Oracle
from _util import base_params, texture

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _oracle(rng, w=12, h=10, r=2, **kw):
    return Oracle(base_params(w, h, r, **kw), texture(rng, h, w), texture(rng, h, w))


def test_pairwise_zero_for_equal_labels_and_coplanar(rng):
    o = _oracle(rng)
    f = np.array([0.1, 0.2, 3.0], np.float32)
    assert o.pairwise((5, 5), (6, 5), f, f) == 0.0
    # two planes that agree along row 5 give zero on a horizontal pair of that row
    g = np.array([0.1, 0.7, 3.0 - 0.5 * 5], np.float32)
    assert o.pairwise((5, 5), (6, 5), f, g) == pytest.approx(0.0, abs=1e-6)
    assert o.pairwise((5, 5), (5, 6), f, g) > 0.0


def test_pairwise_symmetric_bitwise(rng):
    o = _oracle(rng)
    for _ in range(200):
        fp = rng.uniform(-1, 1, 3).astype(np.float32)
        fq = rng.uniform(-1, 1, 3).astype(np.float32)
        p = (int(rng.integers(1, 10)), int(rng.integers(1, 9)))
        d = [(1, 0), (0, 1), (1, 1), (-1, 1)][rng.integers(4)]
        q = (p[0] + d[0], p[1] + d[1])
        assert o.pairwise(p, q, fp, fq) == o.pairwise(q, p, fq, fp)


def test_pairwise_fronto_parallel_and_weight_closed_form():
    h, w = 3, 4
    left = np.zeros((h, w, 3), np.float32) + 100
    left[0, 1] = [110, 100, 100]        # L1 distance 10 to (0,0): w = exp(-1)
    left[2, 3] = [200, 255, 0]          # far: w < eps
    o = Oracle(base_params(w, h), left, left)
    assert o.weight((0, 0), (1, 0)) == pytest.approx(math.exp(-1.0), rel=1e-15)
    assert o.weight((0, 1), (1, 1)) == 1.0
    assert o.weight((2, 2), (3, 2)) < 0.01
    for c1, c2 in [(3.0, 3.2), (3.0, 3.4), (3.0, 9.0)]:
        fp = np.array([0, 0, c1], np.float32)
        fq = np.array([0, 0, c2], np.float32)
        # psi-bar = 2|c_p - c_q|, truncated at tau_dis = 1
        bar = 2 * abs(float(np.float32(c1)) - float(np.float32(c2)))
        assert o.pairwise((0, 0), (1, 0), fp, fq) == pytest.approx(math.exp(-1.0) * min(bar, 1.0), rel=1e-12)
        assert o.pairwise((2, 2), (3, 2), fp, fq) == pytest.approx(0.01 * min(bar, 1.0), rel=1e-12)


def test_lemma1_expansion_submodularity_real_and_quantised(rng):
    # psi(a,a) + psi(b,g) <= psi(b,a) + psi(a,g), and with every term rounded
    # up to 2^-20 the integer inequality still holds (ceil is subadditive).
    o = _oracle(rng)
    Q = 2.0 ** 20
    viol_real = 0
    for _ in range(5000):
        a, b, g = (rng.uniform([-0.5, -0.5, 0], [0.5, 0.5, 8]).astype(np.float32) for _ in range(3))
        if rng.random() < 0.3:
            a = b.copy() if rng.random() < 0.5 else g.copy()
        p = (int(rng.integers(1, 10)), int(rng.integers(0, 9)))
        d = [(1, 0), (0, 1), (1, 1), (-1, 1)][rng.integers(4)]
        q = (p[0] + d[0], p[1] + d[1])
        A = o.pairwise(p, q, b, g)
        B = o.pairwise(p, q, b, a)
        C = o.pairwise(p, q, a, g)
        D = o.pairwise(p, q, a, a)
        assert D == 0.0
        viol_real += (D + A > B + C + 1e-12)
        assert math.ceil(B * Q) + math.ceil(C * Q) >= math.ceil(A * Q)
    assert viol_real == 0


def test_energy_counts_each_neighbour_pair_once_with_equal_diagonal_weight():
    # Constant colour (w = 1), two fronto-parallel halves 10 px apart: every
    # crossing pair costs lambda * tau_dis = 1.  Eight neighbours: H horizontal
    # plus 2(H-1) diagonal crossings; four neighbours: H.
    h, w = 7, 10
    left = np.zeros((h, w, 3), np.float32) + 80
    lab = np.zeros((h, w, 3), np.float32)
    lab[:, 5:, 2] = 10.0
    zero = np.zeros((h, w))
    o8 = Oracle(base_params(w, h), left, left)
    o4 = Oracle(base_params(w, h, neighbours=4), left, left)
    assert o8.energy(lab, zero)[0] == pytest.approx(3 * h - 2, abs=1e-12)
    assert o4.energy(lab, zero)[0] == pytest.approx(h, abs=1e-12)
    costs = np.arange(h * w, dtype=np.float64).reshape(h, w)
    e, eu, ep = o8.energy(lab, costs)
    assert eu == costs.sum() and ep == pytest.approx(3 * h - 2)


# ---------------------------------------------------------------------------
# Exact binary minimisation
# ---------------------------------------------------------------------------

def _random_problem(rng, h, w, lo, hi, wmax):
    U = rng.integers(lo, hi + 1, (h, w)).astype(np.int64)
    w4 = rng.integers(0, wmax + 1, (h, w, 4)).astype(np.int64)
    return U, w4


@pytest.mark.parametrize("shape", [(4, 4), (3, 5), (1, 1), (1, 7), (5, 3), (2, 2)])
@pytest.mark.parametrize("kind", ["generic", "ties"])
def test_maxflow_equals_bruteforce_minimal_alpha_set(rng, shape, kind):
    o = _oracle(rng)
    for _ in range(25):
        if kind == "generic":
            U, w4 = _random_problem(rng, *shape, -60, 60, 40)
        else:
            U, w4 = _random_problem(rng, *shape, -2, 2, 2)
        xb, eb = o.solve_bruteforce(U, w4)
        xm = o.solve_maxflow(U, w4)
        assert o.binary_energy(U, w4, xm) == eb
        assert np.array_equal(xb, xm)


def test_canonical_cut_is_subset_of_every_minimiser(rng):
    o = _oracle(rng)
    h, w = 3, 4
    n = h * w
    for _ in range(10):
        U, w4 = _random_problem(rng, h, w, -2, 2, 2)
        xm = o.solve_maxflow(U, w4).reshape(-1)
        emin = o.binary_energy(U, w4, xm)
        for m in range(1 << n):
            y = np.array([(m >> i) & 1 for i in range(n)], np.uint8)
            e = o.binary_energy(U, w4, y)
            assert e >= emin
            if e == emin:
                assert np.all(xm <= y)


def test_expansion_maxflow_equals_bruteforce_on_image(tiny_oracle, tiny_pair):
    o = tiny_oracle
    pair, prm = tiny_pair
    rng = np.random.default_rng(7)
    base = o.init_labels(3)
    costs0 = o.pixel_costs(base)
    for k in range(12):
        u0, v0 = int(rng.integers(0, 60)), int(rng.integers(0, 44))
        rect = (u0, v0, u0 + 4, v0 + 4)
        alpha = pair.gt_labels[v0 + 1, u0 + 1] if k % 2 else base[v0 + 2, u0 + 2]
        la, ca = base.copy(), costs0.copy()
        lb, cb = base.copy(), costs0.copy()
        da, na = o.expand(la, ca, rect, alpha, bruteforce=True)
        db, nb = o.expand(lb, cb, rect, alpha, bruteforce=False)
        assert da == db and na == nb and da <= 0
        assert np.array_equal(la, lb) and np.array_equal(ca, cb)


def test_expansion_never_increases_energy(tiny_oracle, tiny_pair):
    o = tiny_oracle
    pair, prm = tiny_pair
    labels = o.init_labels(11)
    costs = o.pixel_costs(labels)
    e_prev = o.energy(labels, costs)[0]
    rng = np.random.default_rng(3)
    for k in range(20):
        u0, v0 = int(rng.integers(-5, 55)), int(rng.integers(-5, 40))
        rect = (u0, v0, u0 + 15, v0 + 15)
        alpha = pair.gt_labels[min(max(v0 + 7, 0), 47), min(max(u0 + 7, 0), 63)]
        de, nc = o.expand(labels, costs, rect, alpha)
        e = o.energy(labels, costs)[0]
        # quantised decrease is exact; the real energy may differ by rounding of
        # each term to 2^-20 (at most |R| * 12 terms per pixel)
        assert de <= 0
        assert e <= e_prev + 15 * 15 * 12 * 2.0 ** -20
        assert e == pytest.approx(e_prev + de / 2.0 ** 20, abs=15 * 15 * 12 * 2.0 ** -20)
        e_prev = e
    # the stored per-pixel costs equal phi_p(f_p) recomputed from scratch
    assert np.allclose(costs, o.pixel_costs(labels), atol=1e-10)


def test_pixel_with_candidate_label_is_isolated(tiny_oracle):
    o = tiny_oracle
    labels = o.init_labels(5)
    costs = o.pixel_costs(labels)
    rect = (10, 10, 15, 15)
    alpha = labels[12, 12].copy()
    phi = o.unary_region(rect, alpha)
    U, w4 = o.expand_problem(labels, costs, phi, rect, alpha)
    assert U[2, 2] == 0 and np.all(w4[2, 2] == 0)
    # the edges into (12,12) from its backward neighbours carry no weight either
    assert w4[2, 1, 0] == 0 and w4[1, 2, 1] == 0 and w4[1, 1, 2] == 0 and w4[1, 3, 3] == 0


# ---------------------------------------------------------------------------
# Random numbers, initialisation, proposals, grouping
# ---------------------------------------------------------------------------

def _golden_splitmix():
    vals = []
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                vals.append(int(line, 16))
    return vals


def test_splitmix64_published_sequence(tiny_oracle):
    gold = _golden_splitmix()
    inc = 0x9E3779B97F4A7C15
    for k, g in enumerate(gold):
        assert tiny_oracle.rng_key((k * inc) & (2 ** 64 - 1), []) == g


def test_init_plane_passes_through_random_disparity(tiny_oracle):
    o = tiny_oracle
    lab = o.init_labels(42).astype(np.float64)
    h, w = lab.shape[:2]
    vv, uu = np.mgrid[0:h, 0:w]
    d = lab[..., 0] * uu + lab[..., 1] * vv + lab[..., 2]
    scale = np.abs(lab[..., 0] * uu) + np.abs(lab[..., 1] * vv) + np.abs(lab[..., 2]) + 1
    assert np.all(d >= -1e-6 * scale) and np.all(d <= 16.0 + 1e-6 * scale)
    # normal n = (-a, -b, 1)/|.| is uniform on the upper hemisphere:
    # n_z uniform on (0, 1], azimuth uniform.
    nz = 1.0 / np.sqrt(1.0 + lab[..., 0] ** 2 + lab[..., 1] ** 2)
    az = np.arctan2(-lab[..., 1], -lab[..., 0])
    assert stats.kstest(nz.ravel(), "uniform").pvalue > 1e-3
    assert stats.kstest((az.ravel() + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3
    assert stats.kstest((d.ravel() / 16.0), "uniform").pvalue > 1e-3
    assert np.array_equal(o.init_labels(42), o.init_labels(42))
    assert not np.array_equal(o.init_labels(42), o.init_labels(43))


def test_propagation_takes_a_label_of_the_centre_cell(tiny_oracle):
    o = tiny_oracle
    lab = o.init_labels(1)
    cell = 5
    for (ci, cj) in [(0, 0), (3, 2), (12, 9)]:
        cellpix = lab[cj * cell:(cj + 1) * cell, ci * cell:(ci + 1) * cell].reshape(-1, 3)
        for step in range(3):
            a = o.propose(lab, 9, 0, 0, cell, ci, cj, step, 3, 8.0, 1.0)
            assert any(np.array_equal(a, p) for p in cellpix)


def test_perturbation_zero_size_round_trips_and_size_bounds_disparity(tiny_oracle):
    o = tiny_oracle
    lab = o.init_labels(2)
    cell = 5
    for (ci, cj) in [(1, 1), (7, 4)]:
        cellpix = lab[cj * cell:(cj + 1) * cell, ci * cell:(ci + 1) * cell]
        a0 = o.propose(lab, 9, 0, 0, cell, ci, cj, 1, 1, 0.0, 0.0)
        # some label of the cell is reproduced up to float rounding
        diffs = np.abs(cellpix.reshape(-1, 3) - a0).max(axis=1) / (1 + np.abs(a0).max())
        assert diffs.min() < 1e-5
        # with r_n = 0 the disparity at r moves by at most r_d; it moves by
        # at most r_d/2 on the next refinement step (sizes halve)
        for step, bound in [(1, 4.0), (2, 2.0)]:
            a = o.propose(lab, 9, 0, 0, cell, ci, cj, step, 1, 4.0, 0.0)
            src = o.propose(lab, 9, 0, 0, cell, ci, cj, 0, 1, 4.0, 0.0)  # noqa: F841
            # locate r: the label of the cell that the same draw picked
            best = None
            for v in range(cj * cell, (cj + 1) * cell):
                for u in range(ci * cell, (ci + 1) * cell):
                    f = lab[v, u].astype(np.float64)
                    da = a[0] * u + a[1] * v + a[2] - (f[0] * u + f[1] * v + f[2])
                    slope = np.abs(a[:2] - f[:2]).max()
                    if slope < 1e-5 and (best is None or abs(da) < abs(best)):
                        best = da
            assert best is not None and abs(best) <= bound * (1 + 1e-5) + 1e-3


def test_groups_are_separated_by_a_cell(rng):
    # Eq.(15): cells of one group are 4 cells apart in both directions, so their
    # 3x3-cell regions never touch (not even diagonally).
    for cell, w, h in [(5, 64, 48), (15, 450, 375), (25, 450, 375), (7, 30, 22)]:
        nci, ncj = -(-w // cell), -(-h // cell)
        for k in range(16):
            cells = [(i, j) for j in range(ncj) for i in range(nci) if 4 * (j % 4) + (i % 4) == k]
            rects = [(max((i - 1) * cell, 0), max((j - 1) * cell, 0), min((i + 2) * cell, w),
                      min((j + 2) * cell, h)) for i, j in cells]
            for a in range(len(rects)):
                for b in range(a + 1, len(rects)):
                    ra, rb = rects[a], rects[b]
                    gap_u = max(rb[0] - ra[2], ra[0] - rb[2])
                    gap_v = max(rb[1] - ra[3], ra[1] - rb[3])
                    assert max(gap_u, gap_v) >= cell


def test_group_result_independent_of_cell_order(tiny_oracle):
    # Lemma 3: the expansions of one group do not interact, so running them in
    # parallel (OpenMP, any order) equals running them one by one in reverse.
    o = tiny_oracle
    seed, cell, kp, kr = 17, 5, 1, 3
    lab = o.init_labels(seed)
    cost = o.pixel_costs(lab)
    for group in (0, 5, 15):
        la, ca = lab.copy(), cost.copy()
        o.run_group(la, ca, seed, 0, 0, cell, kp, kr, 8.0, 1.0, group)
        lb, cb = lab.copy(), cost.copy()
        gi, gj = group % 4, group // 4
        cells = [(i, j) for j in range(gj, 10, 4) for i in range(gi, 13, 4)]
        for (i, j) in reversed(cells):
            rect = ((i - 1) * cell, (j - 1) * cell, (i + 2) * cell, (j + 2) * cell)
            for t in range(kp + kr):
                a = o.propose(lb, seed, 0, 0, cell, i, j, t, kp, 8.0, 1.0)
                o.expand(lb, cb, rect, a)
        assert np.array_equal(la, lb) and np.array_equal(ca, cb)
        # only pixels of the group's regions changed
        changed = np.any(la != lab, axis=-1)
        inside = np.zeros_like(changed)
        for (i, j) in cells:
            inside[max((j - 1) * cell, 0):(j + 2) * cell, max((i - 1) * cell, 0):(i + 2) * cell] = True
        assert not np.any(changed & ~inside)


def test_plain_method_tiny_energy_decreases_and_counts(tiny_oracle, tiny_pair):
    o = tiny_oracle
    pair, prm = tiny_pair
    labels, costs, energy, evals = o.optimize(0, [(5, 1, 3)], 2)
    assert evals == 199104 + 64 * 48
    assert np.all(np.diff(energy) < 0)
    assert np.allclose(costs, o.pixel_costs(labels), atol=1e-10)
    e_check = o.energy(labels, costs)[0]
    assert e_check == pytest.approx(energy[-1], rel=1e-12)


def test_expand_step_equals_one_by_one_and_returns_phi(tiny_oracle):
    # One step of a group in parallel (Lemma 3) equals the same expansions one
    # by one in reverse order, and the phi it returns is the region's data
    # term of Eq. (6) as unary_region computes it.
    o = tiny_oracle
    seed, cell = 5, 5
    lab = o.init_labels(seed)
    cost = o.pixel_costs(lab)
    for group in (0, 6, 15):
        gi, gj = group % 4, group // 4
        cells = [(i, j) for j in range(gj, 10, 4) for i in range(gi, 13, 4)]
        rects = [((i - 1) * cell, (j - 1) * cell, (i + 2) * cell, (j + 2) * cell) for i, j in cells]
        alphas = np.array([o.propose(lab, seed, 0, 0, cell, i, j, 1, 1, 8.0, 1.0) for i, j in cells], np.float32)
        la, ca = lab.copy(), cost.copy()
        de, nc, phi = o.expand_step(la, ca, rects, alphas, want_phi=True)
        lb, cb = lab.copy(), cost.copy()
        for q in reversed(range(len(rects))):
            d1, n1 = o.expand(lb, cb, rects[q], alphas[q])
            assert d1 == de[q] and n1 == nc[q]
        assert np.array_equal(la, lb) and np.array_equal(ca, cb)
        at = 0
        for rc, a in zip(rects, alphas):
            ref = o.unary_region(rc, a).reshape(-1)
            assert np.array_equal(phi[at:at + len(ref)], ref)
            at += len(ref)
        assert at == len(phi)
        assert nc.sum() > 0 and np.all(de <= 0)


def test_batch_cycle_draws_every_candidate_before_the_cells_first_move(tiny_oracle):
    # With one candidate per cell the batch cycle is the plain method; with
    # more, its candidates are those the proposer draws from the labels at the
    # group's start (each move still exact: the energy never rises), so it
    # differs from the plain method, whose later candidates see earlier moves.
    o = tiny_oracle
    l1, c1, e1, _ = o.optimize(4, [(5, 1, 0)], 2)
    l2, c2, e2, _ = o.optimize(4, [(5, 1, 0)], 2, batch_cycle=True)
    assert np.array_equal(l1, l2) and np.array_equal(e1, e2)
    lb, cb, eb, _ = o.optimize(4, [(5, 1, 3)], 2, batch_cycle=True)
    lp, cp, ep, _ = o.optimize(4, [(5, 1, 3)], 2)
    assert np.all(np.diff(eb) < 0) and not np.array_equal(lb, lp)
    assert np.allclose(cb, o.pixel_costs(lb), atol=1e-10)
    # group 0 by hand: candidates from the start labels, moves in order
    lab = o.init_labels(4)
    cost = o.pixel_costs(lab)
    la, ca = lab.copy(), cost.copy()
    o.run_group(la, ca, 4, 0, 0, 5, 1, 3, 8.0, 1.0, 0)  # plain, for contrast
    lbat, cbat = lab.copy(), cost.copy()
    cells = [(i, j) for j in range(0, 10, 4) for i in range(0, 13, 4)]
    cand = {q: [o.propose(lab, 4, 0, 0, 5, i, j, t, 1, 8.0, 1.0) for t in range(4)] for q, (i, j) in enumerate(cells)}
    for q, (i, j) in enumerate(cells):
        rect = ((i - 1) * 5, (j - 1) * 5, (i + 2) * 5, (j + 2) * 5)
        for t in range(4):
            o.expand(lbat, cbat, rect, cand[q][t])
    lg, cg = lab.copy(), cost.copy()
    o.run_group(lg, cg, 4, 0, 0, 5, 1, 3, 8.0, 1.0, 0, batch_cycle=True)
    assert np.array_equal(lg, lbat) and np.array_equal(cg, cbat)
    assert np.any(la != lbat)
