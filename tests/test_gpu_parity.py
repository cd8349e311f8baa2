"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Costs: |phi_gpu - phi_oracle| <= 1e-4 * max(|phi_oracle|, rho_max) (FP32
device arithmetic against FP64 direct sums).  Integer outputs (binary-problem
weights, labels after moves) are compared exactly; where the two sides'
unary values straddle a decision, the FP64 margin of that decision is
reported instead (near ties only).
"""
import numpy as np
import pytest

from oracle import Oracle
from synth import make_workload_pair, params_for, random_labels
from _util import base_params, texture

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_1603_08328_amd.lexp")

REL = 1e-4


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _label4(lab3):
    h, w = lab3.shape[:2]
    out = np.zeros((h, w, 4), np.float32)
    out[..., :3] = lab3
    return out


def assert_cost_close(gpu, ora, rho_max, what=""):
    gpu = np.asarray(gpu, np.float64)
    ora = np.asarray(ora, np.float64)
    assert gpu.shape == ora.shape
    err = np.abs(gpu - ora)
    bound = REL * np.maximum(np.abs(ora), rho_max)
    bad = err > bound
    assert not bad.any(), f"{what}: {bad.sum()} of {bad.size} beyond tolerance, max err {err.max():.3e}"


class Pair:
    def __init__(self, name=None, params=None, left=None, right=None):
        if name is not None:
            pair = make_workload_pair(name)
            params = params_for(name)
            left, right = pair.left, pair.right
            self.gt = pair.gt_labels
        self.p = dict(params)
        self.left, self.right = left, right
        self.ora = Oracle(self.p, left, right)
        self.ctx = L.lexp_create(self.p, _cuda(left), _cuda(right))
        self.W, self.H, self.r = int(self.p["width"]), int(self.p["height"]), int(self.p["gf_radius"])
        self.rho_max = self.ora.rho_max


@pytest.fixture(scope="module")
def tiny():
    assert torch.cuda.is_available()
    return Pair("tiny-64x48")


@pytest.fixture(scope="module")
def lowres():
    return Pair("lowres-450x375")


def _unary(P, rects, labels):
    rects = np.asarray(rects, np.int32).reshape(-1, 4)
    labels = np.asarray(labels, np.float32).reshape(-1, 3)
    sizes = []
    for u0, v0, u1, v1 in rects:
        w = max(min(u1, P.W) - max(u0, 0), 0)
        h = max(min(v1, P.H) - max(v0, 0), 0)
        sizes.append(w * h)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    out = torch.full((max(int(np.sum(sizes)), 1),), float("nan"), dtype=torch.float32, device="cuda")
    L.lexp_unary_cost(P.ctx, rects, labels, offs, out)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    return [out[o:o + s] for o, s in zip(offs, sizes)]


def _label_mix(P, rng, n):
    """GT planes, random slanted planes, fronto-parallel, steep, out-of-view."""
    labs = []
    for k in range(n):
        kind = k % 5
        if kind == 0:
            labs.append(P.gt[rng.integers(P.H), rng.integers(P.W)])
        elif kind == 1:
            labs.append(random_labels(rng, 1, 1, float(P.p["disp_max"]))[0, 0])
        elif kind == 2:
            labs.append([0.0, 0.0, rng.uniform(0, P.p["disp_max"])])
        elif kind == 3:
            labs.append([rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(-100, 100)])
        else:
            labs.append([0.0, 0.0, 1e4])
    return np.array(labs, np.float32)


# ---------------------------------------------------------------------------
def test_setup_buffers(tiny):
    P = tiny
    l4, r4, g, wt = (t.cpu().numpy() for t in L.lexp_debug_guide(P.ctx))
    assert np.array_equal(l4[..., :3], P.left) and np.array_equal(r4[..., :3], P.right)
    gl, gr = P.ora.grads()
    assert np.allclose(l4[..., 3], gl, atol=2e-4) and np.allclose(r4[..., 3], gr, atol=2e-4)
    mu, sg = P.ora.guide()
    assert np.allclose(np.moveaxis(g[:3], 0, -1), mu, atol=1e-6)
    e = P.p["gf_eps"]
    S = np.zeros((P.H, P.W, 3, 3))
    idx = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for k, (i, j) in enumerate(idx):
        S[..., i, j] = sg[..., k]
        S[..., j, i] = sg[..., k]
    inv = np.linalg.inv(S + e * np.eye(3))
    got = np.moveaxis(g[3:], 0, -1)
    for k, (i, j) in enumerate(idx):
        assert np.allclose(got[..., k], inv[..., i, j], rtol=1e-4, atol=1e-3 * np.abs(inv).max())
    for v in range(0, P.H, 7):
        for u in range(0, P.W, 5):
            for d, (du, dv) in enumerate([(1, 0), (0, 1), (1, 1), (-1, 1)]):
                q = (u + du, v + dv)
                if 0 <= q[0] < P.W and q[1] < P.H:
                    assert wt[v, u, d] == pytest.approx(P.ora.weight((u, v), q), rel=4e-16)
                else:
                    assert wt[v, u, d] == 0.0


def test_unary_tiny_every_region_of_the_grid(tiny):
    P = tiny
    rng = np.random.default_rng(0)
    rects, labels = [], []
    for j in range(-(-P.H // 5)):
        for i in range(-(-P.W // 5)):
            for lab in _label_mix(P, rng, 4):
                rects.append(((i - 1) * 5, (j - 1) * 5, (i + 2) * 5, (j + 2) * 5))
                labels.append(lab)
    got = _unary(P, rects, labels)
    for rc, lab, g in zip(rects, labels, got):
        ref = P.ora.unary_region(rc, lab).reshape(-1)
        assert_cost_close(g, ref, P.rho_max, f"rect {rc} label {lab}")


@pytest.mark.parametrize("size", [(1, 1), (15, 15), (45, 45), (75, 75), (130, 100), (17, 140)])
def test_unary_lowres_random_rects(lowres, size):
    P = lowres
    rng = np.random.default_rng(size[0] * 1000 + size[1])
    rects = []
    for k in range(6):
        u0 = int(rng.integers(-size[0] // 2, P.W - size[0] // 2))
        v0 = int(rng.integers(-size[1] // 2, P.H - size[1] // 2))
        rects.append((u0, v0, u0 + size[0], v0 + size[1]))
    rects.append((P.W - size[0], P.H - size[1], P.W, P.H))  # bottom-right corner
    labels = _label_mix(P, rng, len(rects))
    got = _unary(P, rects, labels)
    for rc, lab, g in zip(rects, labels, got):
        assert_cost_close(g, P.ora.unary_region(rc, lab).reshape(-1), P.rho_max, f"rect {rc} label {lab}")


def test_unary_highres_group_launches_sampled():
    """1500x1000 workload: every region of one cell group per level in one
    launch, as the optimisation's launches at that size (hundreds to
    thousands of tiles, several rounds per CU), and a sample of the regions
    against the oracle."""
    P = Pair("highres-1500x1000")
    rng = np.random.default_rng(77)
    for cell in (5, 15, 25):
        nci, ncj = -(-P.W // cell), -(-P.H // cell)
        cells = [(i, j) for j in range(1, ncj, 4) for i in range(2, nci, 4)]
        rects = [((i - 1) * cell, (j - 1) * cell, (i + 2) * cell, (j + 2) * cell) for i, j in cells]
        labs = _label_mix(P, rng, len(rects))
        got = _unary(P, rects, labs)
        for q in rng.choice(len(rects), 8, replace=False):
            ref = P.ora.unary_region(rects[q], labs[q]).reshape(-1)
            assert_cost_close(got[q], ref, P.rho_max, f"cell {cell} rect {rects[q]} label {labs[q]}")
    P.ctx.close()


def test_unary_whole_image_one_item(lowres):
    P = lowres
    lab = P.gt[200, 220]
    g = _unary(P, [(0, 0, P.W, P.H)], [lab])[0]
    assert_cost_close(g, P.ora.unary_region((0, 0, P.W, P.H), lab).reshape(-1), P.rho_max, "whole image")


def test_fully_truncated_patch_costs_rho_max_exactly(tiny):
    P = tiny
    got = _unary(P, [(0, 0, 64, 48), (10, 10, 25, 25)], [[0, 0, 1e4], [0.0, 0.0, -500.0]])
    rho_f32 = np.float32((1 - 0.9) * 10 + 0.9 * 2)
    assert np.all(got[0] == rho_f32) and np.all(got[1] == rho_f32)
    # wherever the oracle's phi is rho_max up to FP64 rounding, the device value is exactly rho_max
    rng = np.random.default_rng(3)
    labels = random_labels(rng, 1, 30, 16.0, max_slope=2.0)[0]
    rects = [(0, 0, 64, 48)] * len(labels)
    got = _unary(P, rects, labels)
    n_plateau = 0
    for lab, g in zip(labels, got):
        ref = P.ora.unary_region((0, 0, 64, 48), lab).reshape(-1)
        flat = np.abs(ref - P.rho_max) < 1e-12
        n_plateau += flat.sum()
        assert np.all(g[flat] == rho_f32)
    assert n_plateau > 100


def test_empty_and_outside_items_are_noops(tiny):
    P = tiny
    out = torch.full((10,), 7.0, device="cuda")
    rects = np.array([(5, 5, 5, 9), (70, 0, 80, 5), (-9, -9, -1, -1)], np.int32)
    L.lexp_unary_cost(P.ctx, rects, np.zeros((3, 3), np.float32), np.zeros(3, np.int64), out)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
    L.lexp_unary_cost(P.ctx, np.zeros((0, 4), np.int32), np.zeros((0, 3), np.float32), np.zeros(0, np.int64), out)


def test_invalid_arguments_raise(tiny):
    P = tiny
    out = torch.zeros(300, device="cuda")
    with pytest.raises(L.LexpError):
        L.lexp_unary_cost(P.ctx, [(0, 0, 4, 4)], [[np.nan, 0, 0]], [0], out)
    with pytest.raises(L.LexpError):
        L.lexp_unary_cost(P.ctx, [(0, 0, 4, 4)], [[0, 0, 0]], [-1], out)
    with pytest.raises(ValueError):
        L.lexp_unary_cost(P.ctx, [(0, 0, 40, 40)], [[0, 0, 0]], [0], out)  # output too small
    bad = dict(P.p, gf_radius=0)
    with pytest.raises(L.LexpError):
        L.lexp_create(bad, _cuda(P.left), _cuda(P.right))
    # every parameter range the header states
    for change in (dict(gf_radius=33), dict(neighbours=6), dict(gf_eps=0.0), dict(gamma=0.0), dict(alpha=1.5),
                   dict(lam=-1.0), dict(tau_dis=65.0, lam=1.0), dict(tau_col=2e4), dict(disp_max=float("inf")),
                   dict(host_threads=65), dict(device_cut=2), dict(view=2), dict(graph=2)):
        with pytest.raises(L.LexpError):
            L.lexp_create(dict(P.p, **change), _cuda(P.left), _cuda(P.right))


@pytest.mark.parametrize("r", [1, 2, 5, 9])
def test_unary_small_image_windows_larger_than_image(r):
    rng = np.random.default_rng(r)
    h, w = 5, 7
    p = base_params(w, h, r)
    P = Pair(params=p, left=texture(rng, h, w), right=texture(rng, h, w))
    labs = [[0, 0, 1.5], [0.2, -0.1, 2.0], [0, 0, 0]]
    got = _unary(P, [(0, 0, w, h), (2, 1, 4, 4), (6, 4, 7, 5)], labs)
    for rc, lab, g in zip([(0, 0, w, h), (2, 1, 4, 4), (6, 4, 7, 5)], labs, got):
        assert_cost_close(g, P.ora.unary_region(rc, lab).reshape(-1), P.rho_max, f"r={r} {rc}")


def test_unary_maximum_radius():
    """r = 28, the largest window the fused kernel takes on MI355X (57 x 57
    windows, M = R dilated by 56; a tile's rings and M rows in one workgroup's
    160 KB of LDS leave strips of two columns): costs of interior,
    border-clipped, ragged and 1x1 regions against the oracle, and r = 29
    rejected when the context is created.  The right image is the left one
    shifted by 5 px, so the label d = 5 matches (low costs) and the others mix
    matched, partly out-of-view and fully out-of-view samples."""
    rng = np.random.default_rng(28)
    h, w = 150, 190
    left = texture(rng, h, w)
    right = texture(rng, h, w)
    right[:, :w - 5] = left[:, 5:]
    with pytest.raises(L.LexpError):
        L.lexp_create(base_params(w, h, 29), _cuda(left), _cuda(right))
    P = Pair(params=base_params(w, h, 28), left=left, right=right)
    rects = [(60, 50, 105, 95), (0, 0, 45, 45), (150, 110, 190, 150), (95, 70, 96, 71), (20, 100, 95, 150),
             (0, 0, w, h)]
    labs = [[0, 0, 5.0], [0.02, -0.01, 5.5], [0, 0, 5.0], [0.1, 0.05, 3.0], [0, 0, 1e4], [-0.05, 0.02, 8.0]]
    got = _unary(P, rects, labs)
    for rc, lab, g in zip(rects, labs, got):
        ref = P.ora.unary_region(rc, lab).reshape(-1)
        assert_cost_close(g, ref, P.rho_max, f"r=28 {rc}")
    # the matching label costs well below rho_max inside the view
    assert float(np.median(got[0])) < 0.5 * P.rho_max


def test_guided_coeffs(lowres):
    """Coefficients (a_k, b_k) of Eq. (7) over R+, against the oracle's.

    The device forms the covariance vector cov(I, rho)_k = mean(I rho) -
    mu_k mean(rho) from FP32 window sums of values bounded by rho_max (|I| <= 1),
    so its error is a few FP32 units of rho_max; the solve multiplies that
    error by at most kappa_k = ||(Sigma_k + eU)^-1||_2 = 1 / (lambda_min(Sigma_k)
    + e), up to 1/e = 1e4 where the guide is flat.  Tolerance: |a_gpu - a_ora|
    <= kappa_k * 64 * 2^-24 * rho_max + 1e-4 |a_ora| per entry.  The window
    mean of rho, b_k + a_k . mu_k, is well conditioned: <= 64 * 2^-24 * rho_max
    plus the rounding of mu_k to FP32 in the kernel (2^-23 |a_k| |mu_k|_1)."""
    P = lowres
    rng = np.random.default_rng(9)
    rects = [(100, 100, 115, 115), (0, 0, 45, 45), (400, 300, 475, 375), (10, 200, 90, 230)]
    labels = [P.gt[107, 107], P.gt[20, 20], P.gt[340, 430], random_labels(rng, 1, 1, 60.0)[0, 0]]
    sizes = []
    for u0, v0, u1, v1 in rects:
        sizes.append((min(u1 + P.r, P.W) - max(u0 - P.r, 0)) * (min(v1 + P.r, P.H) - max(v0 - P.r, 0)))
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    out = torch.full((int(np.sum(sizes)) * 4,), float("nan"), device="cuda")
    L.lexp_guided_coeffs(P.ctx, rects, labels, offs, out)
    out = out.cpu().numpy().reshape(-1, 4)
    mu, sg = P.ora.guide()
    eps = P.p["gf_eps"]
    tau = 64 * 2.0 ** -24 * P.rho_max
    worst = [0.0, 0.0]
    for rc, lab, o, s in zip(rects, labels, offs, sizes):
        ref = P.ora.coeffs_region(rc, lab).reshape(-1, 4)
        got = out[o:o + s].astype(np.float64)
        u0, v0, u1, v1 = rc
        pu0, pv0, pu1, pv1 = max(u0 - P.r, 0), max(v0 - P.r, 0), min(u1 + P.r, P.W), min(v1 + P.r, P.H)
        m = mu[pv0:pv1, pu0:pu1].reshape(-1, 3)
        s6 = sg[pv0:pv1, pu0:pu1].reshape(-1, 6)
        S = np.stack([s6[:, [0, 1, 2]], s6[:, [1, 3, 4]], s6[:, [2, 4, 5]]], axis=1)
        kappa = 1.0 / (np.linalg.eigvalsh(S)[:, 0] + eps)
        da = np.abs(got[:, :3] - ref[:, :3])
        assert np.all(da <= kappa[:, None] * tau + 1e-4 * np.abs(ref[:, :3])), np.max(da / kappa[:, None])
        rbar_g = got[:, 3] + (got[:, :3] * m).sum(1)
        rbar_o = ref[:, 3] + (ref[:, :3] * m).sum(1)
        lim = tau + 2.0 ** -23 * (np.abs(got[:, :3]) * np.abs(m)).sum(1)
        assert np.all(np.abs(rbar_g - rbar_o) <= lim), np.abs(rbar_g - rbar_o).max()
        worst[0] = max(worst[0], float(np.max(da.max(1) / kappa)))
        worst[1] = max(worst[1], float(np.max(np.abs(rbar_g - rbar_o))))
    print(f"\n[coeffs] max |da| / kappa = {worst[0]:.3e} (bound {tau:.3e}); "
          f"max |(b + a.mu) error| = {worst[1]:.3e}", flush=True)


def test_pixel_costs_tiny_all_pixels(tiny):
    P = tiny
    lab = P.ora.init_labels(21)
    out = torch.zeros((P.H, P.W), device="cuda")
    L.lexp_pixel_costs(P.ctx, _cuda(_label4(lab)), out)
    assert_cost_close(out.cpu().numpy(), P.ora.pixel_costs(lab), P.rho_max, "pixel costs")


def test_pixel_costs_lowres_sampled(lowres):
    P = lowres
    lab = P.ora.init_labels(4)
    lab[100:200, 100:300] = P.gt[100:200, 100:300]
    out = torch.zeros((P.H, P.W), device="cuda")
    L.lexp_pixel_costs(P.ctx, _cuda(_label4(lab)), out)
    rng = np.random.default_rng(1)
    mask = np.zeros((P.H, P.W), np.uint8)
    mask.reshape(-1)[rng.choice(P.H * P.W, 600, replace=False)] = 1
    mask[0, :] = 1
    mask[:, -1] = 1
    ref = P.ora.pixel_costs(lab, mask)
    m = mask.astype(bool)
    assert_cost_close(out.cpu().numpy()[m], ref[m], P.rho_max, "sampled pixel costs")


def test_pairwise_device_path(tiny):
    P = tiny
    rng = np.random.default_rng(2)
    for _ in range(300):
        p = (int(rng.integers(1, P.W - 1)), int(rng.integers(0, P.H - 1)))
        d = [(1, 0), (0, 1), (1, 1), (-1, 1)][rng.integers(4)]
        q = (p[0] + d[0], p[1] + d[1])
        fp = rng.uniform([-0.5, -0.5, 0], [0.5, 0.5, 16]).astype(np.float32)
        fq = fp.copy() if rng.random() < 0.2 else rng.uniform([-0.5, -0.5, 0], [0.5, 0.5, 16]).astype(np.float32)
        a = L.lexp_pairwise(P.ctx, p, q, fp, fq)
        b = P.ora.pairwise(p, q, fp, fq)
        assert a == pytest.approx(b, rel=1e-15, abs=0)
        assert L.lexp_pairwise(P.ctx, q, p, fq, fp) == a


def test_energy_matches_oracle(tiny):
    P = tiny
    lab = P.ora.init_labels(8)
    lab[10:30, 10:40] = P.gt[10:30, 10:40]
    costs = np.random.default_rng(0).uniform(0, 3, (P.H, P.W)).astype(np.float32)
    t, u, pw = L.lexp_energy(P.ctx, _cuda(_label4(lab)), _cuda(costs))
    e, eu, ep = P.ora.energy(lab, costs.astype(np.float64))
    assert u == pytest.approx(eu, rel=1e-12) and pw == pytest.approx(ep, rel=1e-12)
    assert t == pytest.approx(e, rel=1e-12)


def _gpu_state(P, seed):
    lab = torch.zeros((P.H, P.W, 4), device="cuda")
    L.lexp_init_labels(P.ctx, seed, lab)
    cost = torch.zeros((P.H, P.W), device="cuda")
    L.lexp_pixel_costs(P.ctx, lab, cost)
    torch.cuda.synchronize()
    return lab, cost


def test_graph_terms_pairwise_part_exact(tiny):
    P = tiny
    lab, cost = _gpu_state(P, 13)
    lab3 = lab.cpu().numpy()[..., :3]
    assert np.array_equal(lab3, P.ora.init_labels(13))
    ocost = P.ora.pixel_costs(lab3)
    rects = [(0, 0, 10, 10), (15, 0, 30, 10), (35, 20, 50, 35), (0, 38, 64, 48)]
    rng = np.random.default_rng(4)
    alphas = np.array([lab3[3, 3], P.gt[5, 20], P.gt[25, 40], lab3[40, 30]], np.float32)
    alphas[1] = rng.uniform([-0.2, -0.2, 2], [0.2, 0.2, 14])
    sizes = [(u1 - u0) * (v1 - v0) for u0, v0, u1, v1 in rects]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    phi = torch.zeros(int(np.sum(sizes)), device="cuda")
    L.lexp_unary_cost(P.ctx, rects, alphas, offs, phi)
    terms = torch.zeros(int(np.sum(sizes)) * 5, dtype=torch.int32, device="cuda")
    L.lexp_graph_terms(P.ctx, rects, alphas, phi, offs, lab, cost, terms)
    terms = terms.cpu().numpy().reshape(-1, 5)
    for rc, a, o, s in zip(rects, alphas, offs, sizes):
        phi_o = P.ora.unary_region(rc, a)
        U, w4 = P.ora.expand_problem(lab3, ocost, phi_o, rc, a)
        t = terms[o:o + s]
        assert np.array_equal(t[:, 1:], w4.reshape(-1, 4)), "pairwise weights differ"
        # unary part: both sides round phi differences of < 1e-4 * 2.8 each
        assert np.all(np.abs(t[:, 0] - U.reshape(-1)) <= 2 * 2.8e-4 * 2 ** 20 + 2)


def _margin(P, lab3, cost, rect, alpha, x_gpu, x_ora):
    """FP64 energy difference between the two binary labellings."""
    phi = P.ora.unary_region(rect, alpha)
    U, w4 = P.ora.expand_problem(lab3, cost, phi, rect, alpha)
    return abs(P.ora.binary_energy(U, w4, x_gpu) - P.ora.binary_energy(U, w4, x_ora)) * 2.0 ** -20


def test_expansion_steps_match_oracle_in_lockstep(tiny):
    """Both sides start from the same labels and apply the same sequence of
    group steps (candidates drawn by the oracle's proposer from its state);
    labels are compared after every step.  A differing pixel is accepted only
    as a near tie of the FP64 binary energy."""
    P = tiny
    seed = 0
    lab, cost = _gpu_state(P, seed)
    olab = P.ora.init_labels(seed)
    ocost = P.ora.pixel_costs(olab)
    cell, kp, kr = 5, 1, 3
    nci, ncj = -(-P.W // cell), -(-P.H // cell)
    near_ties = 0
    for k in range(16):
        cells = [(i, j) for j in range(k // 4, ncj, 4) for i in range(k % 4, nci, 4)]
        rects = [((i - 1) * cell, (j - 1) * cell, (i + 2) * cell, (j + 2) * cell) for i, j in cells]
        for step in range(kp + kr):
            alphas = np.array([P.ora.propose(olab, seed, 0, 0, cell, i, j, step, kp, 8.0, 1.0)
                               for i, j in cells], np.float32)
            got = _unary(P, rects, alphas)
            offs = np.concatenate([[0], np.cumsum([len(g) for g in got])[:-1]]).astype(np.int64)
            phi = _cuda(np.concatenate(got).astype(np.float32))
            before = olab.copy()
            for rc, a in zip(rects, alphas):
                P.ora.expand(olab, ocost, rc, a)
            L.lexp_expand_region(P.ctx, rects, alphas, phi, offs, lab, cost)
            g3 = lab.cpu().numpy()[..., :3]
            diff = np.any(g3 != olab, axis=-1)
            if diff.any():
                for rc, a in zip(rects, alphas):
                    u0, v0, u1, v1 = max(rc[0], 0), max(rc[1], 0), min(rc[2], P.W), min(rc[3], P.H)
                    if not diff[v0:v1, u0:u1].any():
                        continue
                    xg = np.all(g3[v0:v1, u0:u1] == a, axis=-1) & np.any(before[v0:v1, u0:u1] != a, axis=-1)
                    xo = np.all(olab[v0:v1, u0:u1] == a, axis=-1) & np.any(before[v0:v1, u0:u1] != a, axis=-1)
                    m = _margin(P, before, P.ora.pixel_costs(before), rc, a, xg.astype(np.uint8),
                                xo.astype(np.uint8))
                    assert m < 1e-3, f"group {k} step {step} rect {rc}: margin {m}"
                    near_ties += 1
                # continue from the oracle's state on both sides
                lab = _cuda(_label4(olab))
                cost = torch.zeros((P.H, P.W), device="cuda")
                L.lexp_pixel_costs(P.ctx, lab, cost)
    assert near_ties <= 2


def test_expand_rejects_touching_regions_and_leaves_state(tiny):
    P = tiny
    lab, cost = _gpu_state(P, 1)
    before = lab.clone()
    rects = [(0, 0, 10, 10), (10, 10, 20, 20)]  # diagonal contact
    phi = torch.zeros(200, device="cuda")
    with pytest.raises(L.LexpError):
        L.lexp_expand_region(P.ctx, rects, [[0, 0, 1]] * 2, phi, [0, 100], lab, cost)
    assert torch.equal(lab, before)


def test_optimize_tiny_bit_identical_to_oracle(tiny):
    P = tiny
    lab = torch.zeros((P.H, P.W, 4), device="cuda")
    cost = torch.zeros((P.H, P.W), device="cuda")
    e, t = L.lexp_optimize(P.ctx, [(5, 1, 3)], 2, 0, lab, cost)
    olab, ocost, oe, _ = P.ora.optimize(0, [(5, 1, 3)], 2)
    g3 = lab.cpu().numpy()[..., :3]
    assert np.array_equal(g3.view(np.uint32), olab.view(np.uint32)), \
        f"{np.any(g3 != olab, axis=-1).sum()} pixels differ"
    assert np.allclose(e, oe, rtol=1e-5)
    assert_cost_close(cost.cpu().numpy(), ocost, P.rho_max, "final costs")
    # determinism
    lab2 = torch.zeros_like(lab)
    cost2 = torch.zeros_like(cost)
    L.lexp_optimize(P.ctx, [(5, 1, 3)], 2, 0, lab2, cost2)
    assert torch.equal(lab, lab2) and torch.equal(cost, cost2)


@pytest.mark.parametrize("device_cut", [0, 1])
def test_optimize_four_neighbourhood_bit_identical_to_oracle(device_cut):
    """The 4-neighbourhood (forward neighbours (1,0) and (0,1) only): a whole
    run at 64x48, every cut on the host or part of them on the device, gives
    the oracle's labels bit for bit."""
    pair = make_workload_pair("tiny-64x48")
    P = Pair(params=dict(params_for("tiny-64x48"), neighbours=4, device_cut=device_cut), left=pair.left,
             right=pair.right)
    lab = torch.zeros((P.H, P.W, 4), device="cuda")
    cost = torch.zeros((P.H, P.W), device="cuda")
    e, _ = L.lexp_optimize(P.ctx, [(5, 1, 3)], 2, 0, lab, cost)
    olab, ocost, oe, _ = P.ora.optimize(0, [(5, 1, 3)], 2)
    g3 = lab.cpu().numpy()[..., :3]
    assert np.array_equal(g3.view(np.uint32), olab.view(np.uint32)), \
        f"{np.any(g3 != olab, axis=-1).sum()} pixels differ"
    assert np.allclose(e, oe, rtol=1e-5)
    assert_cost_close(cost.cpu().numpy(), ocost, P.rho_max, "final costs")


@pytest.mark.parametrize("device_cut", [0, 1])
def test_optimize_paper_radius_two_levels_bit_identical_to_oracle(device_cut):
    """The paper's filter radius r = 20 (41 x 41 windows) with two grid levels
    (5- and 15-px cells, the second with 45 x 45 regions split into strips),
    a whole 2-iteration run on a 120x90 scene: the oracle's labels bit for
    bit, every cut on the host or part of them on the device."""
    from synth.scenes import make_pair
    from synth import PAPER_PARAMS
    pair = make_pair(width=120, height=90, n_planar=5, n_quadric=1, disp_max=24.0, c_range=(3.0, 21.0),
                     hole_frac=0.02, seed=5)
    prm = dict(PAPER_PARAMS, width=120, height=90, disp_max=24.0, gf_radius=20, device_cut=device_cut)
    P = Pair(params=prm, left=pair.left, right=pair.right)
    grids = [(5, 1, 3), (15, 1, 3)]
    lab = torch.zeros((P.H, P.W, 4), device="cuda")
    cost = torch.zeros((P.H, P.W), device="cuda")
    e, _ = L.lexp_optimize(P.ctx, grids, 2, 0, lab, cost)
    olab, ocost, oe, _ = P.ora.optimize(0, grids, 2)
    g3 = lab.cpu().numpy()[..., :3]
    assert np.array_equal(g3.view(np.uint32), olab.view(np.uint32)), \
        f"{np.any(g3 != olab, axis=-1).sum()} pixels differ"
    assert np.allclose(e, oe, rtol=1e-5)
    assert_cost_close(cost.cpu().numpy(), ocost, P.rho_max, "final costs")


@pytest.mark.parametrize("device_cut", [0, 1])
def test_optimize_three_levels_bit_identical_to_oracle(device_cut):
    """The 450x375 workload's three grid levels (5-, 15- and 25-px cells, r =
    20) on a 200x150 scene, one iteration from the random labels: the oracle's
    labels bit for bit, every cut on the host or (one host thread, so that the
    larger groups are split) part of them on the device."""
    from synth.scenes import make_pair
    from synth import PAPER_PARAMS
    pair = make_pair(width=200, height=150, n_planar=6, n_quadric=1, disp_max=30.0, c_range=(4.0, 26.0),
                     hole_frac=0.02, seed=6)
    prm = dict(PAPER_PARAMS, width=200, height=150, disp_max=30.0, gf_radius=20, device_cut=device_cut,
               host_threads=1 if device_cut else 0)
    P = Pair(params=prm, left=pair.left, right=pair.right)
    grids = [(5, 1, 3), (15, 1, 3), (25, 1, 3)]
    lab = torch.zeros((P.H, P.W, 4), device="cuda")
    cost = torch.zeros((P.H, P.W), device="cuda")
    e, _ = L.lexp_optimize(P.ctx, grids, 1, 0, lab, cost)
    olab, ocost, oe, _ = P.ora.optimize(0, grids, 1)
    g3 = lab.cpu().numpy()[..., :3]
    assert np.array_equal(g3.view(np.uint32), olab.view(np.uint32)), \
        f"{np.any(g3 != olab, axis=-1).sum()} pixels differ"
    assert np.allclose(e, oe, rtol=1e-5)
    assert_cost_close(cost.cpu().numpy(), ocost, P.rho_max, "final costs")


def test_optimize_three_levels_right_view_bit_identical_to_oracle():
    """As above (three grid levels, r = 20, 200x150, one iteration) for the
    right view (the mirrored pair's left-view run): the oracle's labels bit
    for bit.  (With RANSAC steps the candidates often come close to labels
    already there and a few regions' cuts differ within the costs' rounding,
    so that run is checked step by step instead:
    test_ransac_three_levels_lockstep_with_oracle.)"""
    from synth.scenes import make_pair
    from synth import PAPER_PARAMS
    pair = make_pair(width=200, height=150, n_planar=6, n_quadric=1, disp_max=30.0, c_range=(4.0, 26.0),
                     hole_frac=0.02, seed=6)
    prm = dict(PAPER_PARAMS, width=200, height=150, disp_max=30.0, gf_radius=20)
    ctx = L.lexp_create(dict(prm, view=1), _cuda(pair.left), _cuda(pair.right))
    ora = Oracle.right_view(prm, pair.left, pair.right)
    grids = [(5, 1, 3), (15, 1, 3), (25, 1, 3)]
    lab = torch.zeros((150, 200, 4), device="cuda")
    cost = torch.zeros((150, 200), device="cuda")
    e, _ = L.lexp_optimize(ctx, grids, 1, 4, lab, cost)
    ctx.close()
    olab, ocost, oe, _ = ora.optimize(4, grids, 1)
    g3 = lab.cpu().numpy()[..., :3]
    assert np.array_equal(g3.view(np.uint32), olab.view(np.uint32)), \
        f"{np.any(g3 != olab, axis=-1).sum()} pixels differ"
    assert np.allclose(e, oe, rtol=1e-5)
    assert_cost_close(cost.cpu().numpy(), ocost, ora.rho_max, "final costs")


def test_optimize_rejects_bad_schedules_and_leaves_state(tiny):
    """Schedules outside the ranges the header states are refused before any
    work is queued: the labels and costs keep their values."""
    import ctypes
    P = tiny
    lab = torch.full((P.H, P.W, 4), 7.0, device="cuda")
    cost = torch.full((P.H, P.W), 3.0, device="cuda")
    lib = L.load_library()
    e, t = np.zeros(3), np.zeros(3)

    def run(field, value, index=None):
        s = L.make_schedule([(5, 1, 3)], 2)
        if index is None:
            setattr(s, field, value)
        else:
            getattr(s, field)[index] = value
        return lib.lexp_optimize(P.ctx.handle, ctypes.byref(s), ctypes.c_uint64(0), ctypes.c_void_p(lab.data_ptr()),
                                 ctypes.c_void_p(cost.data_ptr()), e.ctypes.data, t.ctypes.data, None)

    bad = [("n_levels", 0, None), ("n_levels", 5, None), ("iterations", -1, None), ("cell", 0, 0),
           ("k_prop", -1, 0), ("k_rand", 64, 0), ("k_rans", -1, 0), ("tile_cols", 129, 0), ("tile_fill", -1, 0),
           ("speculate", 2, None), ("batch_cycle", 2, None), ("learned", 2, None)]
    for field, value, index in bad:
        assert run(field, value, index) == L.LEXP_EINVAL, (field, value)
    assert run("learned", 1, None) == L.LEXP_ESTATE  # no network set on the context
    torch.cuda.synchronize()
    assert bool(torch.all(lab == 7.0)) and bool(torch.all(cost == 3.0))


def test_optimize_tiny_with_ransac_bit_identical_to_oracle(tiny):
    """Alg. 1 with the RANSAC proposer enabled (one propagation, one RANSAC
    and two refinement steps per cell): labels bit-identical to the oracle's
    run, energies to 1e-5."""
    P = tiny
    grids = [(5, 1, 2, 1)]
    lab = torch.zeros((P.H, P.W, 4), device="cuda")
    cost = torch.zeros((P.H, P.W), device="cuda")
    e, _ = L.lexp_optimize(P.ctx, grids, 2, 3, lab, cost)
    olab, ocost, oe, _ = P.ora.optimize(3, grids, 2)
    g3 = lab.cpu().numpy()[..., :3]
    assert np.array_equal(g3.view(np.uint32), olab.view(np.uint32)), \
        f"{np.any(g3 != olab, axis=-1).sum()} pixels differ"
    assert np.allclose(e, oe, rtol=1e-5)
    assert_cost_close(cost.cpu().numpy(), ocost, P.rho_max, "final costs")


# ---------------------------------------------------------------------------
# Device max-flow (push-relabel kernel) against the host max-flow and the
# oracle: the cut of the fewest ones is unique, so the comparison is bitwise.
def _binary_problems(rng, shapes, kind, reps):
    probs = []
    for h, w in shapes:
        for _ in range(reps):
            if kind == "generic":
                U = rng.integers(-60, 61, (h, w))
                w4 = rng.integers(0, 41, (h, w, 4))
            elif kind == "ties":
                U = rng.integers(-2, 3, (h, w))
                w4 = rng.integers(0, 3, (h, w, 4))
            elif kind == "sparse":
                U = rng.integers(-5, 6, (h, w)) * (rng.random((h, w)) < 0.3)
                w4 = rng.integers(0, 9, (h, w, 4)) * (rng.random((h, w, 4)) < 0.5)
            else:  # large values near the documented limit
                U = rng.integers(-(2 ** 30), 2 ** 30 + 1, (h, w))
                w4 = rng.integers(0, 2 ** 30 + 1, (h, w, 4))
            # no weight towards neighbours outside the grid
            w4[:, -1, 0] = 0
            w4[-1, :, 1:] = 0
            w4[:, -1, 2] = 0
            w4[:, 0, 3] = 0
            probs.append((U.astype(np.int64), w4.astype(np.int64)))
    return probs


@pytest.mark.parametrize("kind", ["generic", "ties", "sparse", "huge"])
def test_device_cut_equals_host_cut(tiny, kind):
    rng = np.random.default_rng({"generic": 1, "ties": 2, "sparse": 3, "huge": 4}[kind])
    shapes = [(1, 1), (1, 7), (6, 1), (3, 5), (15, 15), (9, 23), (22, 22)]
    probs = _binary_problems(rng, shapes, kind, 6)
    xs, status = L.lexp_solve_binary_device(tiny.ctx, probs)
    assert status.all()
    for (U, w4), x in zip(probs, xs):
        assert np.array_equal(x, L.lexp_solve_binary(U, w4)), (U.shape, kind)


@pytest.mark.parametrize("shape", [(45, 45), (31, 64), (60, 60), (75, 75), (40, 120), (76, 77), (80, 80)])
def test_device_cut_large_regions(tiny, shape):
    """Regions up to about 3,100 nodes keep all residuals in LDS, larger ones
    up to about 5,850 nodes the compact layout (forward residuals, 32-bit
    excess, 16-bit heights); still larger ones are not run (status 0, left to
    the host max-flow)."""
    rng = np.random.default_rng(sum(shape))
    probs = _binary_problems(rng, [shape], "generic", 2) + _binary_problems(rng, [shape], "sparse", 2) + \
        _binary_problems(rng, [shape], "ties", 1)
    xs, status = L.lexp_solve_binary_device(tiny.ctx, probs)
    fits = shape[0] * shape[1] * 28 <= 160 * 1024 - 64
    assert (status == (1 if fits else 0)).all()
    if fits:
        for (U, w4), x in zip(probs, xs):
            assert np.array_equal(x, L.lexp_solve_binary(U, w4))


def test_device_cut_compact_layout_mixed_sizes_and_large_values(tiny):
    """One launch with a 75x75 problem runs every problem in the compact
    layout, small ones included.  Values near the 2^30 limit either solve
    exactly or stop on excess overflow (status 0), never give a wrong cut."""
    rng = np.random.default_rng(21)
    probs = _binary_problems(rng, [(75, 75), (1, 1), (3, 5), (15, 15), (45, 45)], "generic", 1) + \
        _binary_problems(rng, [(60, 70)], "huge", 3)
    xs, status = L.lexp_solve_binary_device(tiny.ctx, probs)
    assert status[:5].all()
    for (U, w4), x, st in zip(probs, xs, status):
        if st:
            assert np.array_equal(x, L.lexp_solve_binary(U, w4))


def test_device_cut_compact_layout_excess_overflow_is_left_to_host(tiny):
    """Four arcs of capacity 2^30 into one node in the same round give it an
    excess of 2^32, past the compact layout's 32-bit excess: the region must
    stop with status 0 (it is then cut on the host)."""
    h, w = 60, 60
    U = np.zeros((h, w), np.int64)
    w4 = np.zeros((h, w, 4), np.int64)
    cu, cv = 30, 30
    U[cv, cu] = -(2 ** 30)
    for d, (du, dv) in enumerate([(1, 0), (0, 1), (1, 1), (-1, 1)]):
        pu, pv = cu - du, cv - dv
        U[pv, pu] = 2 ** 30
        w4[pv, pu, d] = 2 ** 30
    xs, status = L.lexp_solve_binary_device(tiny.ctx, [(U, w4)])
    assert status[0] == 0
    assert L.lexp_solve_binary(U, w4).sum() >= 0  # the host solves it


def test_device_cut_of_real_expansion_problems(tiny):
    """Binary problems of actual expansions (oracle terms) against the
    oracle's own max-flow."""
    P = tiny
    rng = np.random.default_rng(11)
    lab = P.ora.init_labels(5)
    costs = P.ora.pixel_costs(lab, np.ones((P.H, P.W), np.uint8))
    probs = []
    for _ in range(12):
        ci, cj = int(rng.integers(0, 13)), int(rng.integers(0, 10))
        rect = ((ci - 1) * 5, (cj - 1) * 5, (ci + 2) * 5, (cj + 2) * 5)
        a = P.ora.propose(lab, 3, 0, 0, 5, ci, cj, int(rng.integers(0, 4)), 1, 8.0, 1.0)
        phi = P.ora.unary_region(rect, a)
        probs.append(P.ora.expand_problem(lab, costs, phi, rect, a))
    xs, status = L.lexp_solve_binary_device(P.ctx, probs)
    assert status.all()
    for (U, w4), x in zip(probs, xs):
        assert np.array_equal(x, P.ora.solve_maxflow(U, w4))


def test_device_cut_rejects_bad_terms(tiny):
    U = np.zeros((2, 2), np.int64)
    w4 = np.zeros((2, 2, 4), np.int64)
    w4[0, 0, 0] = -1
    with pytest.raises(L.LexpError):
        L.lexp_solve_binary_device(tiny.ctx, [(U, w4)])
    U[0, 0] = 2 ** 30 + 1
    w4[0, 0, 0] = 0
    with pytest.raises(L.LexpError):
        L.lexp_solve_binary_device(tiny.ctx, [(U, w4)])


def test_device_cut_four_neighbourhood():
    rng = np.random.default_rng(9)
    p = base_params(20, 16, neighbours=4)
    left, right = texture(rng, 16, 20), texture(rng, 16, 20)
    ctx = L.lexp_create(p, _cuda(left), _cuda(right))
    probs = _binary_problems(rng, [(16, 20), (7, 9)], "generic", 4)
    for U, w4 in probs:
        w4[..., 2:] = 0
    xs, status = L.lexp_solve_binary_device(ctx, probs)
    assert status.all()
    for (U, w4), x in zip(probs, xs):
        assert np.array_equal(x, L.lexp_solve_binary(U, w4, neighbours=4))


def test_optimize_device_and_host_cuts_identical(lowres):
    """One iteration of the plain method at 450x375 with the device max-flow
    enabled (5 px cells: one part of each group cut on the device) and with
    every cut on the host: identical labels and costs, bit for bit."""
    P = lowres
    out = []
    for dc in (1, 0):
        p = dict(P.p, device_cut=dc)
        ctx = L.lexp_create(p, _cuda(P.left), _cuda(P.right))
        L.lexp_set_timing(ctx, True)
        lab = torch.zeros((P.H, P.W, 4), device="cuda")
        cost = torch.zeros((P.H, P.W), device="cuda")
        e, _ = L.lexp_optimize(ctx, [(5, 1, 7), (15, 1, 7), (25, 1, 7)], 1, 0, lab, cost)
        if dc:
            assert L.lexp_get_stats(ctx)["expand_calls"] > 0
        out.append((lab.cpu().numpy(), cost.cpu().numpy(), e))
        ctx.close()
    assert np.array_equal(out[0][0].view(np.uint32), out[1][0].view(np.uint32))
    assert np.array_equal(out[0][1].view(np.uint32), out[1][1].view(np.uint32))
    assert out[0][2][-1] == out[1][2][-1]


# ---------------------------------------------------------------------------
# Many pairs in one run: every group step of every pair in shared launches.
def _scene(width, height, disp_max, seed, r, n_planar=4, n_quadric=0, holes=0.0):
    from synth import make_pair, PAPER_PARAMS
    sc = dict(width=width, height=height, n_planar=n_planar, n_quadric=n_quadric, disp_max=disp_max,
              c_range=(disp_max / 8.0, 7.0 * disp_max / 8.0), hole_frac=holes, seed=seed)
    pair = make_pair(**sc)
    p = dict(PAPER_PARAMS, width=width, height=height, disp_max=disp_max, gf_radius=r)
    return p, pair


def _alone_and_batched(scenes, grids, iterations, seeds, **ctx_kw):
    ctxs, alone = [], []
    for (p, pair), sd in zip(scenes, seeds):
        ctx = L.lexp_create(dict(p, **ctx_kw), _cuda(pair.left), _cuda(pair.right))
        lab = torch.zeros((p["height"], p["width"], 4), device="cuda")
        cost = torch.zeros((p["height"], p["width"]), device="cuda")
        e, _ = L.lexp_optimize(ctx, grids, iterations, sd, lab, cost)
        alone.append((lab.cpu().numpy(), cost.cpu().numpy(), e))
        ctxs.append(ctx)
    labs = [torch.full((p["height"], p["width"], 4), float("nan"), device="cuda") for p, _ in scenes]
    costs = [torch.full((p["height"], p["width"]), float("nan"), device="cuda") for p, _ in scenes]
    L.lexp_set_timing(ctxs[0], True)
    L.lexp_reset_stats(ctxs[0])
    es, ts = L.lexp_optimize_batch(ctxs, grids, iterations, seeds, labs, costs)
    stats = L.lexp_get_stats(ctxs[0])
    batched = [(l.cpu().numpy(), c.cpu().numpy(), e) for l, c, e in zip(labs, costs, es)]
    for c in ctxs:
        c.close()
    assert np.all(np.diff(ts) >= 0)
    return alone, batched, stats


def _assert_same_runs(alone, batched):
    for i, (a, b) in enumerate(zip(alone, batched)):
        assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32)), \
            f"pair {i}: {np.any(a[0] != b[0], axis=-1).sum()} labels differ"
        assert np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32)), f"pair {i}: costs differ"
        assert np.array_equal(a[2], b[2]), f"pair {i}: energy traces differ"


@pytest.mark.parametrize("device_cut", [0, 1])
def test_optimize_batch_equals_per_pair_runs_small_pairs(device_cut):
    """Three pairs of uneven sizes (ragged cells, different disparity ranges),
    r = 5, the tiny schedule, every cut on the host or part of them on the
    device: each pair's labels, costs and energies in the batched run equal
    its run alone, bit for bit; the 64x48 pair also equals the oracle's run."""
    scenes = [_scene(64, 48, 16.0, 0, 5), _scene(97, 61, 20.0, 11, 5), _scene(37, 29, 9.0, 12, 5)]
    tiny_p = params_for("tiny-64x48")
    tiny_pair = make_workload_pair("tiny-64x48")
    scenes[0] = (tiny_p, tiny_pair)
    seeds = [0, 7, 2 ** 40 + 3]
    # one host thread: groups of more than four regions are split and the
    # device max-flow takes a tuned share of them
    alone, batched, stats = _alone_and_batched(scenes, [(5, 1, 3)], 2, seeds, device_cut=device_cut,
                                               host_threads=1 if device_cut else 0)
    _assert_same_runs(alone, batched)
    # one cost launch per group step and part, for all three pairs
    if device_cut:
        assert 16 * 4 * 2 <= stats["unary_launches"] <= 2 * 16 * 4 * 2
        assert stats["device_cut_share"][0] > 0
    else:
        assert stats["unary_launches"] == 16 * 4 * 2
    olab, _, oe, _ = Oracle(tiny_p, tiny_pair.left, tiny_pair.right).optimize(0, [(5, 1, 3)], 2)
    assert np.array_equal(batched[0][0][..., :3].view(np.uint32), olab.view(np.uint32))
    assert np.allclose(batched[0][2], oe, rtol=1e-5)
    for e in (b[2] for b in batched):
        assert np.all(np.diff(e) <= 0)


def test_optimize_batch_with_device_cuts_equals_per_pair_runs(lowres):
    """The 450x375 pair together with two smaller pairs of the many-pair
    recipe (r = 20, three grid levels, one iteration): the level-1 groups are
    split and cut partly on the device, the small pairs' groups are not; every
    pair equals its run alone."""
    from synth.workloads import many_pair_scenes
    scenes = [(lowres.p, make_workload_pair("lowres-450x375"))]
    for sc in many_pair_scenes(2, seed0=3000):
        w = 320 + (sc["width"] - 320) // 8   # a smaller member of the same recipe
        h = int(round(0.67 * w / 8.0)) * 8
        scenes.append(_scene(w, h, float(round(0.13 * w)), sc["seed"], 20, 12, 2, 0.02))
    alone, batched, stats = _alone_and_batched(scenes, [(5, 1, 7), (15, 1, 7), (25, 1, 7)], 1, [0, 1, 2])
    _assert_same_runs(alone, batched)
    assert stats["unary_launches"] > 0


def test_optimize_batch_rejects_mixed_radius_and_shared_buffers(tiny):
    p2, pair2 = _scene(40, 32, 10.0, 3, 4)
    ctx2 = L.lexp_create(p2, _cuda(pair2.left), _cuda(pair2.right))
    lab = [torch.zeros((tiny.H, tiny.W, 4), device="cuda"), torch.zeros((32, 40, 4), device="cuda")]
    cost = [torch.zeros((tiny.H, tiny.W), device="cuda"), torch.zeros((32, 40), device="cuda")]
    with pytest.raises(L.LexpError):
        L.lexp_optimize_batch([tiny.ctx, ctx2], [(5, 1, 3)], 1, [0, 0], lab, cost)
    with pytest.raises(L.LexpError):
        L.lexp_optimize_batch([tiny.ctx, tiny.ctx], [(5, 1, 3)], 1, [0, 0], [lab[0], lab[0]], [cost[0], cost[0]])
    ctx2.close()


def test_sampled_timing_counts_every_launch_and_times_every_nth(tiny):
    """lexp_set_timing(ctx, N): every fused launch is counted, every N-th is
    timed (events at the kernel's own start and end), with its bytes and
    evaluations, also per grid level; N = 1 times them all; negative periods
    are refused."""
    P = tiny
    lab = torch.zeros((P.H, P.W, 4), device="cuda")
    cost = torch.zeros((P.H, P.W), device="cuda")
    for every in (1, 3):
        L.lexp_set_timing(P.ctx, every)
        L.lexp_reset_stats(P.ctx)
        L.lexp_optimize(P.ctx, [(5, 1, 3), (10, 1, 3)], 1, 0, lab, cost)
        st = L.lexp_get_stats(P.ctx)
        n = st["unary_launches"]
        assert n > 0 and st["unary_timed_launches"] == (n + every - 1) // every
        assert st["unary_kernel_ms"] > 0
        # the timed launches split by grid level (two levels here)
        assert sum(st["unary_level_launches"]) == st["unary_timed_launches"]
        assert all(x > 0 for x in st["unary_level_launches"][:2]) and st["unary_level_launches"][2:] == [0, 0]
        assert sum(st["unary_level_ms"]) == pytest.approx(st["unary_kernel_ms"], rel=1e-9)
        assert sum(st["unary_level_alg_bytes"]) == pytest.approx(st["unary_timed_alg_bytes"], rel=1e-12)
        if every == 1:
            assert st["unary_timed_alg_bytes"] == st["unary_alg_bytes"]
            assert st["unary_timed_evals"] == st["unary_evals"]
        else:
            assert 0 < st["unary_timed_alg_bytes"] < st["unary_alg_bytes"]
            assert 0 < st["unary_timed_evals"] < st["unary_evals"]
    with pytest.raises(L.LexpError):
        L.lexp_set_timing(P.ctx, -1)
    L.lexp_set_timing(P.ctx, 0)


def test_create_rejects_images_past_the_offset_limit(tiny):
    """The fused kernel addresses packed images with 32-bit byte offsets, so a
    context takes at most 2^27 - 1 pixels; larger sizes are refused before any
    allocation (the image pointers are not read)."""
    lib = L.load_library()
    p = tiny.p
    buf = torch.zeros(3, device="cuda")
    for w, h in [(16384, 8192), (1 << 27, 1)]:
        P = L.lexp_params(w, h, float(p["disp_max"]), float(p["alpha"]), float(p["tau_col"]), float(p["tau_grad"]),
                          int(p["gf_radius"]), float(p["gf_eps"]), float(p["lam"]), float(p["tau_dis"]),
                          float(p["w_floor"]), float(p["gamma"]), int(p["neighbours"]), 0, 1, 0, 0)
        out = L.C.c_void_p()
        st = lib.lexp_create(L.C.byref(P), L.C.c_void_p(buf.data_ptr()), L.C.c_void_p(buf.data_ptr()), None,
                             L.C.byref(out))
        assert st == L.LEXP_EINVAL and not out.value, (w, h, st)
        assert b"2^27" in lib.lexp_last_error()


# ---------------------------------------------------------------------------
# Right view and post-processing.
def _right_view(P):
    """Right-view context of a Pair and its oracle (both in the mirrored frame)."""
    ctx = L.lexp_create(dict(P.p, view=1), _cuda(P.left), _cuda(P.right))
    ora = Oracle.right_view(P.p, P.left, P.right)
    return ctx, ora


def test_right_view_unary_matches_oracle(lowres):
    P = lowres
    ctx, ora = _right_view(P)
    rng = np.random.default_rng(31)
    for size in [(15, 15), (45, 45), (75, 75), (1, 1)]:
        rects, labs = [], []
        for k in range(6):
            u0, v0 = int(rng.integers(-10, P.W - 5)), int(rng.integers(-10, P.H - 5))
            rects.append((u0, v0, u0 + size[0], v0 + size[1]))
            labs.append(random_labels(rng, 1, 1, float(P.p["disp_max"]))[0, 0] if k % 2 else
                        [0.0, 0.0, rng.uniform(0, P.p["disp_max"])])
        rects = np.array(rects, np.int32)
        labs = np.array(labs, np.float32)
        sizes = [max(min(u1, P.W) - max(u0, 0), 0) * max(min(v1, P.H) - max(v0, 0), 0) for u0, v0, u1, v1 in rects]
        offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        out = torch.full((int(sum(sizes)),), float("nan"), device="cuda")
        L.lexp_unary_cost(ctx, rects, labs, offs, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        for r, f, o, n in zip(rects, labs, offs, sizes):
            if n:
                assert_cost_close(got[o:o + n], ora.unary_region(tuple(r), f).ravel(), P.rho_max, "right view")
    ctx.close()


def test_right_view_optimize_bit_identical_to_oracle_and_batched_with_left(tiny):
    """The tiny pair's right view alone equals the oracle's right-view run; run
    together with the left view in one batch, both views equal their runs
    alone."""
    P = tiny
    ctx, ora = _right_view(P)
    lab = torch.zeros((P.H, P.W, 4), device="cuda")
    cost = torch.zeros((P.H, P.W), device="cuda")
    e, _ = L.lexp_optimize(ctx, [(5, 1, 3)], 2, 0, lab, cost)
    olab, _, oe, _ = ora.optimize(0, [(5, 1, 3)], 2)
    g3 = lab.cpu().numpy()[..., :3]
    assert np.array_equal(g3.view(np.uint32), olab.view(np.uint32)), f"{np.any(g3 != olab, axis=-1).sum()} differ"
    assert np.allclose(e, oe, rtol=1e-5)
    labl = torch.zeros_like(lab)
    costl = torch.zeros_like(cost)
    el, _ = L.lexp_optimize(P.ctx, [(5, 1, 3)], 2, 0, labl, costl)
    labs = [torch.zeros_like(lab), torch.zeros_like(lab)]
    costs = [torch.zeros_like(cost), torch.zeros_like(cost)]
    es, _ = L.lexp_optimize_batch([P.ctx, ctx], [(5, 1, 3)], 2, [0, 0], labs, costs)
    assert torch.equal(labs[0], labl) and torch.equal(labs[1], lab)
    assert np.array_equal(es[0], el) and np.array_equal(es[1], e)
    ctx.close()


def test_view_labels_conversion(tiny):
    P = tiny
    ctx, _ = _right_view(P)
    rng = np.random.default_rng(2)
    lab = np.zeros((P.H, P.W, 4), np.float32)
    lab[..., :3] = random_labels(rng, P.H, P.W, 16.0)
    got = L.lexp_view_labels(ctx, _cuda(lab)).cpu().numpy()
    m = lab[:, ::-1]
    expect = np.zeros_like(lab)
    expect[..., 0] = -m[..., 0]
    expect[..., 1] = m[..., 1]
    expect[..., 2] = (m[..., 2].astype(np.float64) + m[..., 0].astype(np.float64) * (P.W - 1)).astype(np.float32)
    assert np.array_equal(got.view(np.uint32), expect.view(np.uint32))
    same = L.lexp_view_labels(P.ctx, _cuda(lab)).cpu().numpy()
    assert np.array_equal(same, lab)
    # the converted labels give the same disparity at mirrored pixels
    u = np.arange(P.W)[None, :]
    v = np.arange(P.H)[:, None]
    d_ctx = lab[..., 0] * u + lab[..., 1] * v + lab[..., 2]  # disparity at context-frame pixel u
    d_img = got[..., 0] * u + got[..., 1] * v + got[..., 2]
    assert np.allclose(d_img, d_ctx[:, ::-1], atol=1e-3)
    ctx.close()


@pytest.mark.parametrize("which", ["tiny", "lowres"])
def test_postprocess_matches_oracle(tiny, lowres, which):
    """Both views optimised on the device, then post-processed on the device
    and by the oracle from the same labels: the disparity maps agree bit for
    bit (FP64 arithmetic rounded once to FP32) and so do the masks of the
    inconsistent pixels."""
    P = tiny if which == "tiny" else lowres
    grids = [(5, 1, 3)] if which == "tiny" else [(5, 1, 7), (15, 1, 7), (25, 1, 7)]
    ctx_r, _ = _right_view(P)
    labs = [torch.zeros((P.H, P.W, 4), device="cuda") for _ in range(2)]
    costs = [torch.zeros((P.H, P.W), device="cuda") for _ in range(2)]
    L.lexp_optimize_batch([P.ctx, ctx_r], grids, 2, [1, 2], labs, costs)
    disp, inv = L.lexp_postprocess(P.ctx, labs[0], ctx_r, labs[1])
    torch.cuda.synchronize()
    ll = labs[0].cpu().numpy()[..., :3]
    lr = labs[1].cpu().numpy()[..., :3]
    odisp, oinv = P.ora.postprocess(ll, lr)
    inv = inv.cpu().numpy()
    assert np.array_equal(inv, oinv), f"{(inv != oinv).sum()} flags differ"
    assert 0 < inv.sum() < inv.size
    got = disp.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), odisp.astype(np.float32).view(np.uint32)), \
        f"{(got != odisp.astype(np.float32)).sum()} of {got.size} differ"
    ctx_r.close()


def test_postprocess_rejects_wrong_views(tiny):
    lab = torch.zeros((tiny.H, tiny.W, 4), device="cuda")
    with pytest.raises(L.LexpError):
        L.lexp_postprocess(tiny.ctx, lab, tiny.ctx, lab)


@pytest.mark.parametrize("which", ["tiny", "lowres"])
def test_graph_mode_gives_identical_runs(tiny, lowres, which):
    """Each part step's device work captured in a HIP graph and replayed:
    labels, costs and energies equal the eager run's bit for bit (single
    pair, and a batch of two pairs)."""
    P = tiny if which == "tiny" else lowres
    grids = [(5, 1, 3)] if which == "tiny" else [(5, 1, 7), (15, 1, 7), (25, 1, 7)]
    runs = []
    for graph in (0, 1):
        ctx = L.lexp_create(dict(P.p, graph=graph), _cuda(P.left), _cuda(P.right))
        ctx2 = L.lexp_create(dict(P.p, graph=graph, view=1), _cuda(P.left), _cuda(P.right))
        lab = torch.zeros((P.H, P.W, 4), device="cuda")
        cost = torch.zeros((P.H, P.W), device="cuda")
        e, _ = L.lexp_optimize(ctx, grids, 1, 4, lab, cost)
        labs = [torch.zeros_like(lab), torch.zeros_like(lab)]
        costs = [torch.zeros_like(cost), torch.zeros_like(cost)]
        es, _ = L.lexp_optimize_batch([ctx, ctx2], grids, 1, [4, 9], labs, costs)
        st = L.lexp_get_stats(ctx)
        runs.append((lab.cpu().numpy(), cost.cpu().numpy(), e, [x.cpu().numpy() for x in labs], es))
        assert (st["graphs_captured"] > 0) == bool(graph)
        ctx.close()
        ctx2.close()
    a, b = runs
    assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))
    assert np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32))
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[4], b[4])
    for x, y in zip(a[3], b[3]):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
