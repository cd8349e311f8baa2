"""The 450x375 workload (r = 20; cells of 5, 15 and 25 px; one propagation
and seven refinement candidates per cell and level) on the HIP path, checked
step by step.

- Against the FP64 oracle: the first iteration of Alg. 2 (every level, every
  group of Eq. (15), every step of Alg. 1), both sides from the same labels.
  After every group step the costs phi(alpha) of every region are compared
  within the cost tolerance and the labels bit for bit.  A region whose cut
  differs is accepted only when the difference is explained by the costs'
  rounding: its FP64 energy margin (oracle energy of the library's cut minus
  that of the oracle's cut) must not exceed the sum, over the pixels where
  the cuts differ, of the difference between the two sides' unary terms.
- lexp_optimize against the same steps issued one by one through the C ABI
  (lexp_propose, lexp_unary_cost, lexp_expand_region): bit-identical labels,
  costs and energy, so the library's own loop (tiles, parts, pipelining,
  device and host cuts) is the method written out in this file.
- Device max-flow at every level (one host thread, so every level is split
  and a tuned share is cut on the device) against every cut on the host.
- A region's costs do not depend on the regions it shares a launch with.
"""
import time

import numpy as np
import pytest

from synth import make_workload_pair, params_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_1603_08328_amd.lexp")

GRIDS = [(5, 1, 7), (15, 1, 7), (25, 1, 7)]
REL = 1e-4
Q = 2.0 ** 20


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _label4(lab3):
    out = np.zeros(lab3.shape[:2] + (4,), np.float32)
    out[..., :3] = lab3
    return out


def _group(W, H, cell, k):
    """Cells (i = column, j = row) of group k = 4 (j mod 4) + (i mod 4), Eq. (15),
    and their 3x3-cell regions, clipped to the image."""
    nci, ncj = -(-W // cell), -(-H // cell)
    cells = [(i, j) for j in range(k // 4, ncj, 4) for i in range(k % 4, nci, 4)]
    rects = []
    for i, j in cells:
        u0, v0 = max((i - 1) * cell, 0), max((j - 1) * cell, 0)
        rects.append((u0, v0, min((i + 2) * cell, W), min((j + 2) * cell, H)))
    sizes = np.array([(u1 - u0) * (v1 - v0) for u0, v0, u1, v1 in rects], np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    return cells, np.array(rects, np.int32), sizes, offs


@pytest.fixture(scope="module")
def lowres():
    from oracle import Oracle
    pair = make_workload_pair("lowres-450x375")
    prm = params_for("lowres-450x375")
    return pair, prm, Oracle(prm, pair.left, pair.right)


def _lockstep_first_iteration(prm, pair, ora, grids, seed, tag):
    """The first iteration of Alg. 2 issued group step by group step on the
    library (lexp_propose, lexp_unary_cost, lexp_expand_region) and the oracle
    from the same labels; grids hold (cell, K_prop, K_rand[, K_RANS]).  Costs
    are compared within the tolerance after every step, labels bit for bit; a
    region whose cut differs must be explained by the costs' rounding (its FP64
    margin at most the summed unary-term differences where the cuts differ),
    and both sides then continue from the oracle's labels.  Returns (group
    steps, regions, near ties, largest margin)."""
    W, H = prm["width"], prm["height"]
    rho_max = ora.rho_max
    t0 = time.time()
    ctx = L.lexp_create(prm, _cuda(pair.left), _cuda(pair.right))
    lab = torch.zeros((H, W, 4), device="cuda")
    cost = torch.zeros((H, W), device="cuda")
    L.lexp_init_labels(ctx, seed, lab)
    L.lexp_pixel_costs(ctx, lab, cost)
    olab = ora.init_labels(seed)
    assert np.array_equal(lab.cpu().numpy()[..., :3].view(np.uint32), olab.view(np.uint32))
    ocost = ora.pixel_costs(olab)
    # the initial per-pixel costs (1x1 regions), every pixel
    gc = cost.cpu().numpy().astype(np.float64)
    err = np.abs(gc - ocost)
    assert np.all(err <= REL * np.maximum(np.abs(ocost), rho_max)), f"initial costs: max err {err.max():.3e}"
    print(f"\n[{tag}] set-up and initial costs {time.time() - t0:.1f} s", flush=True)

    r_d, r_n = prm["disp_max"] / 2.0, 1.0
    near_ties, worst_margin, n_phi, n_regions, n_steps = 0, 0.0, 0, 0, 0
    max_rel = 0.0
    for h, g in enumerate(grids):
        cell, kp, kr = g[:3]
        krans = g[3] if len(g) > 3 else 0
        for k in range(16):
            cells, rects, sizes, offs = _group(W, H, cell, k)
            total = int(sizes.sum())
            for step in range(kp + krans + kr):
                alphas = np.array([ora.propose(olab, seed, 0, h, cell, i, j, step, kp, r_d, r_n, k_rans=krans)
                                   for i, j in cells], np.float32)
                # the library's proposer on the same labels: the same candidates
                for q in range(0, len(cells), 5):
                    i, j = cells[q]
                    a = L.lexp_propose(olab, seed, 0, h, cell, i, j, step, kp, r_d, r_n, k_rans=krans)
                    assert np.array_equal(a.view(np.uint32), alphas[q].view(np.uint32))
                phi = torch.empty(total, device="cuda")
                L.lexp_unary_cost(ctx, rects, alphas, offs, phi)
                lab_before, cost_before = lab.clone(), cost.clone()
                before, ocost_before = olab.copy(), ocost.copy()
                _, _, ophi = ora.expand_step(olab, ocost, rects, alphas, want_phi=True)
                gphi = phi.cpu().numpy().astype(np.float64)
                e = np.abs(gphi - ophi)
                tol = REL * np.maximum(np.abs(ophi), rho_max)
                assert np.all(e <= tol), \
                    f"level {cell} group {k} step {step}: {(e > tol).sum()} costs beyond tolerance, max {e.max():.3e}"
                max_rel = max(max_rel, float(np.max(e / np.maximum(np.abs(ophi), rho_max))))
                n_phi += total
                n_regions += len(cells)
                n_steps += 1
                L.lexp_expand_region(ctx, rects, alphas, phi, offs, lab, cost)
                g3 = lab.cpu().numpy()[..., :3]
                diff = np.any(g3.view(np.uint32) != olab.view(np.uint32), axis=-1)
                if not diff.any():
                    continue
                for q, (rc, a) in enumerate(zip(rects, alphas)):
                    u0, v0, u1, v1 = (int(x) for x in rc)
                    if not diff[v0:v1, u0:u1].any():
                        continue
                    # only pixels of the regions can change, and only to alpha
                    took = np.any(before[v0:v1, u0:u1] != a, axis=-1)
                    xg = (np.all(g3[v0:v1, u0:u1] == a, axis=-1) & took).astype(np.uint8)
                    xo = (np.all(olab[v0:v1, u0:u1] == a, axis=-1) & took).astype(np.uint8)
                    phi_o = ophi[offs[q]:offs[q] + sizes[q]].reshape(v1 - v0, u1 - u0)
                    Uo, w4o = ora.expand_problem(before, ocost_before, phi_o, (u0, v0, u1, v1), a)
                    terms = torch.zeros(int(sizes[q]) * 5, dtype=torch.int32, device="cuda")
                    L.lexp_graph_terms(ctx, [rc], [a], phi[offs[q]:offs[q] + sizes[q]].contiguous(), [0],
                                       lab_before, cost_before, terms)
                    tg = terms.cpu().numpy().reshape(v1 - v0, u1 - u0, 5).astype(np.int64)
                    assert np.array_equal(tg[..., 1:], w4o), "pairwise terms differ"
                    dU = np.abs(tg[..., 0] - Uo)
                    # each unary term differs by the rounding of two costs, within tolerance
                    cb = cost_before.cpu().numpy()[v0:v1, u0:u1].astype(np.float64)
                    lim = (REL * np.maximum(np.abs(phi_o), rho_max) +
                           REL * np.maximum(np.abs(ocost_before[v0:v1, u0:u1]), rho_max)) * Q + 2
                    assert np.all(dU <= lim), f"unary terms differ beyond the cost tolerance ({dU.max()})"
                    assert np.all(np.abs(cb - ocost_before[v0:v1, u0:u1]) <=
                                  REL * np.maximum(np.abs(ocost_before[v0:v1, u0:u1]), rho_max))
                    margin = ora.binary_energy(Uo, w4o, xg) - ora.binary_energy(Uo, w4o, xo)
                    bound = int(np.sum(dU[xg != xo]))
                    assert 0 <= margin <= bound, \
                        f"level {cell} group {k} step {step} rect {tuple(rc)}: margin {margin} > bound {bound}"
                    near_ties += 1
                    worst_margin = max(worst_margin, margin / Q)
                # continue both sides from the oracle's labels
                lab = _cuda(_label4(olab))
                cost = torch.zeros((H, W), device="cuda")
                L.lexp_pixel_costs(ctx, lab, cost)
            print(f"[{tag}] level {cell} group {k}: {time.time() - t0:.1f} s, near ties {near_ties}", flush=True)
    ctx.close()
    print(f"[{tag}] {n_steps} group steps, {n_regions} regions, {n_phi} costs compared (max relative error "
          f"{max_rel:.2e}); {near_ties} regions decided differently within the cost rounding "
          f"(largest FP64 margin {worst_margin:.3e})", flush=True)
    return n_steps, n_regions, near_ties, worst_margin


def test_lowres_first_iteration_lockstep_with_oracle(lowres):
    pair, prm, ora = lowres
    n_steps, _, near_ties, _ = _lockstep_first_iteration(prm, pair, ora, GRIDS, 0, "lockstep")
    assert n_steps == 3 * 16 * 8
    assert near_ties <= 20


def test_ransac_three_levels_lockstep_with_oracle():
    """Alg. 1 with the RANSAC proposer (one propagation, one RANSAC and two
    refinement steps per cell) at the 450x375 workload's three grid levels
    and r = 20, on a 200x150 scene, step by step against the oracle: RANSAC
    candidates fit planes to the current disparities, so they often come
    close to labels already there, and a region's cut may then differ only
    within the costs' rounding (checked as above)."""
    from oracle import Oracle
    from synth import PAPER_PARAMS
    from synth.scenes import make_pair
    pair = make_pair(width=200, height=150, n_planar=6, n_quadric=1, disp_max=30.0, c_range=(4.0, 26.0),
                     hole_frac=0.02, seed=6)
    prm = dict(PAPER_PARAMS, width=200, height=150, disp_max=30.0, gf_radius=20)
    grids = [(5, 1, 2, 1), (15, 1, 2, 1), (25, 1, 2, 1)]
    n_steps, n_regions, near_ties, _ = _lockstep_first_iteration(prm, pair, Oracle(prm, pair.left, pair.right),
                                                                 grids, 4, "ransac lockstep")
    assert n_steps == 3 * 16 * 4
    # every differing region is checked against the rounding bound above; a
    # systematic error would show in far more than 1% of the regions (16 of
    # 5,552 were decided differently when this test was written)
    assert near_ties <= n_regions // 100


def _abi_first_iteration(prm, pair, seed):
    """Alg. 2 (first iteration) with Alg. 1 per cell, issued step by step
    through the C ABI on the library's own labels."""
    W, H = prm["width"], prm["height"]
    ctx = L.lexp_create(prm, _cuda(pair.left), _cuda(pair.right))
    lab = torch.zeros((H, W, 4), device="cuda")
    cost = torch.zeros((H, W), device="cuda")
    L.lexp_init_labels(ctx, seed, lab)
    L.lexp_pixel_costs(ctx, lab, cost)
    e0 = L.lexp_energy(ctx, lab, cost)[0]
    r_d, r_n = prm["disp_max"] / 2.0, 1.0
    mirror = lab.cpu().numpy()[..., :3].copy()
    for h, (cell, kp, kr) in enumerate(GRIDS):
        for k in range(16):
            cells, rects, sizes, offs = _group(W, H, cell, k)
            for step in range(kp + kr):
                alphas = np.array([L.lexp_propose(mirror, seed, 0, h, cell, i, j, step, kp, r_d, r_n)
                                   for i, j in cells], np.float32)
                phi = torch.empty(int(sizes.sum()), device="cuda")
                L.lexp_unary_cost(ctx, rects, alphas, offs, phi)
                L.lexp_expand_region(ctx, rects, alphas, phi, offs, lab, cost)
                mirror = lab.cpu().numpy()[..., :3].copy()
    e1 = L.lexp_energy(ctx, lab, cost)[0]
    ctx.close()
    return lab.cpu().numpy(), cost.cpu().numpy(), (e0, e1)


def test_lowres_optimize_equals_group_steps_through_the_abi(lowres):
    pair, prm, _ = lowres
    W, H = prm["width"], prm["height"]
    seed = 0
    ref_lab, ref_cost, ref_e = _abi_first_iteration(prm, pair, seed)
    for threads, dc in ((0, 1), (1, 1)):
        ctx = L.lexp_create(dict(prm, host_threads=threads, device_cut=dc), _cuda(pair.left), _cuda(pair.right))
        lab = torch.zeros((H, W, 4), device="cuda")
        cost = torch.zeros((H, W), device="cuda")
        e, _ = L.lexp_optimize(ctx, GRIDS, 1, seed, lab, cost)
        ctx.close()
        g = lab.cpu().numpy()
        assert np.array_equal(g.view(np.uint32), ref_lab.view(np.uint32)), \
            f"threads {threads}: {np.any(g != ref_lab, axis=-1).sum()} labels differ"
        assert np.array_equal(cost.cpu().numpy().view(np.uint32), ref_cost.view(np.uint32))
        assert e[0] == ref_e[0] and e[1] == ref_e[1]
    assert ref_e[1] < ref_e[0]


def test_lowres_device_cuts_at_every_level_equal_host_cuts(lowres):
    """One host thread: every level's groups hold more than four regions per
    thread, so every level is split and the device max-flow cuts a tuned
    share of its 15x15, 45x45 and 75x75 regions.  Labels, costs and energy
    equal those with every cut on the host, bit for bit."""
    pair, prm, _ = lowres
    W, H = prm["width"], prm["height"]
    out = []
    for threads, dc in ((1, 1), (0, 0)):
        ctx = L.lexp_create(dict(prm, host_threads=threads, device_cut=dc), _cuda(pair.left), _cuda(pair.right))
        L.lexp_set_timing(ctx, 1)
        lab = torch.zeros((H, W, 4), device="cuda")
        cost = torch.zeros((H, W), device="cuda")
        e, _ = L.lexp_optimize(ctx, GRIDS, 1, 0, lab, cost)
        st = L.lexp_get_stats(ctx)
        ctx.close()
        if dc:
            share = st["device_cut_share"][:3]
            print(f"\n[device cut] shares per level {share}, regions left to the host "
                  f"{st['device_cut_fallbacks']}", flush=True)
            assert all(s > 0 for s in share), share
        out.append((lab.cpu().numpy(), cost.cpu().numpy(), e))
    assert np.array_equal(out[0][0].view(np.uint32), out[1][0].view(np.uint32)), \
        f"{np.any(out[0][0] != out[1][0], axis=-1).sum()} labels differ"
    assert np.array_equal(out[0][1].view(np.uint32), out[1][1].view(np.uint32))
    assert np.array_equal(out[0][2], out[1][2])


def test_region_costs_do_not_depend_on_the_launch(lowres):
    """A narrow pair (64x48, r = 20) batched with the 450x375 pair: its tiles
    are narrower than the large pair's, so a shared launch uses the kernel
    instance of the wider tiles.  With one host thread the 450x375 pair's
    groups are split and their share tuned by time.  Every pair's labels,
    costs and energies equal its run alone, bit for bit."""
    from synth import make_pair, PAPER_PARAMS
    pair, prm, _ = lowres
    small = make_pair(width=64, height=48, n_planar=4, n_quadric=0, disp_max=12.0, c_range=(1.5, 10.5),
                      hole_frac=0.0, seed=21)
    sp = dict(PAPER_PARAMS, width=64, height=48, disp_max=12.0, gf_radius=20)
    scenes = [(dict(prm, host_threads=1), pair), (dict(sp, host_threads=1), small)]
    seeds = [0, 5]
    ctxs, alone = [], []
    for (p, pr), sd in zip(scenes, seeds):
        ctx = L.lexp_create(p, _cuda(pr.left), _cuda(pr.right))
        lab = torch.zeros((p["height"], p["width"], 4), device="cuda")
        cost = torch.zeros((p["height"], p["width"]), device="cuda")
        e, _ = L.lexp_optimize(ctx, GRIDS, 1, sd, lab, cost)
        alone.append((lab.cpu().numpy(), cost.cpu().numpy(), e))
        ctxs.append(ctx)
    labs = [torch.zeros((p["height"], p["width"], 4), device="cuda") for p, _ in scenes]
    costs = [torch.zeros((p["height"], p["width"]), device="cuda") for p, _ in scenes]
    es, _ = L.lexp_optimize_batch(ctxs, GRIDS, 1, seeds, labs, costs)
    for c in ctxs:
        c.close()
    for i, (a, l, c, e) in enumerate(zip(alone, labs, costs, es)):
        assert np.array_equal(a[0].view(np.uint32), l.cpu().numpy().view(np.uint32)), f"pair {i}: labels differ"
        assert np.array_equal(a[1].view(np.uint32), c.cpu().numpy().view(np.uint32)), f"pair {i}: costs differ"
        assert np.array_equal(a[2], e), f"pair {i}: energies differ"
