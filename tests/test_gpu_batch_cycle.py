"""The batch cycle of Alg. 1 (Sec. 3.4: every candidate of a cell drawn from
the labels at its group step's start, all candidates of all regions evaluated
in one launch, the moves then made in order) and explicit tile plans of the
fused cost kernel, through the C ABI."""
import numpy as np
import pytest

from synth import make_workload_pair, params_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_1603_08328_amd.lexp")


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(ctx, prm, grids, iters, seed, **kw):
    lab = torch.zeros((prm["height"], prm["width"], 4), device="cuda")
    cost = torch.zeros((prm["height"], prm["width"]), device="cuda")
    e, t = L.lexp_optimize(ctx, grids, iters, seed, lab, cost, **kw)
    return lab.cpu().numpy(), cost.cpu().numpy(), e


@pytest.fixture(scope="module")
def tiny():
    from oracle import Oracle
    pair = make_workload_pair("tiny-64x48")
    prm = params_for("tiny-64x48")
    return pair, prm, Oracle(prm, pair.left, pair.right)


def test_batch_cycle_tiny_bit_identical_to_oracle(tiny):
    pair, prm, ora = tiny
    ctx = L.lexp_create(prm, _cuda(pair.left), _cuda(pair.right))
    L.lexp_set_timing(ctx, 1)
    lab, cost, e = _run(ctx, prm, [(5, 1, 3)], 2, 0, batch_cycle=True)
    st = L.lexp_get_stats(ctx)
    ctx.close()
    olab, ocost, oe, _ = ora.optimize(0, [(5, 1, 3)], 2, batch_cycle=True)
    g3 = lab[..., :3]
    assert np.array_equal(g3.view(np.uint32), olab.view(np.uint32)), f"{np.any(g3 != olab, axis=-1).sum()} differ"
    assert np.allclose(e, oe, rtol=1e-5)
    err = np.abs(cost - ocost)
    assert np.all(err <= 1e-4 * np.maximum(np.abs(ocost), ora.rho_max))
    # one fused launch per group step, covering every candidate of every region
    assert st["unary_launches"] == 2 * 16
    plain = ora.optimize(0, [(5, 1, 3)], 2)[0]
    assert not np.array_equal(plain, olab)


def test_batch_cycle_three_levels_bit_identical_to_oracle():
    """The batch cycle with the 450x375 workload's three grid levels (5-, 15-
    and 25-px cells, r = 20; the regions of the larger cells cut into strips in
    the one launch per group step) on a 200x150 scene, one iteration from the
    random labels: the oracle's batch cycle, bit for bit."""
    from oracle import Oracle
    from synth import PAPER_PARAMS
    from synth.scenes import make_pair
    pair = make_pair(width=200, height=150, n_planar=6, n_quadric=1, disp_max=30.0, c_range=(4.0, 26.0),
                     hole_frac=0.02, seed=6)
    prm = dict(PAPER_PARAMS, width=200, height=150, disp_max=30.0, gf_radius=20)
    grids = [(5, 1, 3), (15, 1, 3), (25, 1, 3)]
    ctx = L.lexp_create(prm, _cuda(pair.left), _cuda(pair.right))
    lab, cost, e = _run(ctx, prm, grids, 1, 0, batch_cycle=True)
    ctx.close()
    ora = Oracle(prm, pair.left, pair.right)
    olab, ocost, oe, _ = ora.optimize(0, grids, 1, batch_cycle=True)
    g3 = lab[..., :3]
    assert np.array_equal(g3.view(np.uint32), olab.view(np.uint32)), f"{np.any(g3 != olab, axis=-1).sum()} differ"
    assert np.allclose(e, oe, rtol=1e-5)
    assert np.all(np.abs(cost - ocost) <= 1e-4 * np.maximum(np.abs(ocost), ora.rho_max))


def test_batch_cycle_lowres_device_and_host_cuts_and_pairs_identical():
    """450x375, one iteration of the batch cycle: every cut on the host, the
    device max-flow at every level (one host thread), and the pair batched
    with a smaller pair of the many-pair recipe: identical runs."""
    from synth import make_pair, PAPER_PARAMS
    pair = make_workload_pair("lowres-450x375")
    prm = params_for("lowres-450x375")
    grids = [(5, 1, 7), (15, 1, 7), (25, 1, 7)]
    out = []
    for threads, dc in ((0, 0), (1, 1)):
        ctx = L.lexp_create(dict(prm, host_threads=threads, device_cut=dc), _cuda(pair.left), _cuda(pair.right))
        out.append(_run(ctx, prm, grids, 1, 0, batch_cycle=True))
        ctx.close()
    assert np.array_equal(out[0][0].view(np.uint32), out[1][0].view(np.uint32))
    assert np.array_equal(out[0][1].view(np.uint32), out[1][1].view(np.uint32))
    assert out[0][2][1] < out[0][2][0]
    small = make_pair(width=200, height=136, n_planar=6, n_quadric=1, disp_max=26.0, c_range=(3.25, 22.75),
                      hole_frac=0.02, seed=3001)
    sp = dict(PAPER_PARAMS, width=200, height=136, disp_max=26.0, gf_radius=20)
    ctxs = [L.lexp_create(prm, _cuda(pair.left), _cuda(pair.right)),
            L.lexp_create(sp, _cuda(small.left), _cuda(small.right))]
    alone_small = _run(ctxs[1], sp, grids, 1, 9, batch_cycle=True)
    labs = [torch.zeros((p["height"], p["width"], 4), device="cuda") for p in (prm, sp)]
    costs = [torch.zeros((p["height"], p["width"]), device="cuda") for p in (prm, sp)]
    L.lexp_set_timing(ctxs[0], 1)
    es, _ = L.lexp_optimize_batch(ctxs, grids, 1, [0, 9], labs, costs, batch_cycle=True)
    st = L.lexp_get_stats(ctxs[0])
    for c in ctxs:
        c.close()
    assert np.array_equal(labs[0].cpu().numpy().view(np.uint32), out[0][0].view(np.uint32))
    assert np.array_equal(labs[1].cpu().numpy().view(np.uint32), alone_small[0].view(np.uint32))
    assert np.array_equal(es[1], alone_small[2])
    # one launch per group step for both pairs and all eight candidates
    assert st["unary_launches"] == 3 * 16


def test_tile_plans(tiny):
    """An explicit plan equal to the default rule gives the default run bit for
    bit; another plan (narrower strips, more row strips) still gives the
    oracle's labels on the 64x48 workload and is deterministic; plans out of
    range are refused."""
    pair, prm, ora = tiny
    ctx = L.lexp_create(prm, _cuda(pair.left), _cuda(pair.right))
    grids = [(5, 1, 3)]
    base = _run(ctx, prm, grids, 2, 0)
    same = _run(ctx, prm, grids, 2, 0, tiles=[(0, 256)])
    assert np.array_equal(base[0], same[0]) and np.array_equal(base[1], same[1])
    other = [_run(ctx, prm, grids, 2, 0, tiles=[(4, 1024)]) for _ in range(2)]
    assert np.array_equal(other[0][0], other[1][0]) and np.array_equal(other[0][1], other[1][1])
    olab, ocost, oe, _ = ora.optimize(0, grids, 2)
    assert np.array_equal(other[0][0][..., :3].view(np.uint32), olab.view(np.uint32))
    err = np.abs(other[0][1] - ocost)
    assert np.all(err <= 1e-4 * np.maximum(np.abs(ocost), ora.rho_max))
    assert not np.array_equal(other[0][1], base[1])  # a different plan rounds differently
    for bad in ([(-1, 0)], [(129, 0)], [(0, -5)]):
        with pytest.raises(L.LexpError):
            _run(ctx, prm, grids, 1, 0, tiles=bad)
    ctx.close()
