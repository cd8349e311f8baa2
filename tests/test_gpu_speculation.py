"""Speculative costs in lexp_optimize: while the host cuts a step of a
single-part group, the device evaluates the next step's two possible
candidates of every region (Alg. 1 propagation and refinement steps read one
label, which the cut keeps or sets to the current candidate).  The runs must
equal the ones without speculation bit for bit, through the C ABI."""
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
    L.lexp_set_timing(ctx, 1)
    L.lexp_reset_stats(ctx)
    e, _ = L.lexp_optimize(ctx, grids, iters, seed, lab, cost, **kw)
    return lab.cpu().numpy(), cost.cpu().numpy(), e, L.lexp_get_stats(ctx)


def _same(a, b):
    assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))
    assert np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32))
    assert np.array_equal(a[2], b[2])


@pytest.mark.parametrize("grids", [[(5, 1, 7), (15, 1, 7), (25, 1, 7)], [(15, 1, 6, 1), (25, 1, 6, 1)]],
                         ids=["plain", "ransac"])
def test_speculation_gives_identical_runs(grids):
    """450x375, one iteration, every cut on 16 host threads: the 15- and
    25-px groups (47 and 17 regions, at most four per thread: one part) take
    speculative costs for every step after their first (RANSAC steps
    excepted), the 5-px groups (two parts, staggered) none; none is missed,
    and labels, costs, energies and the count of useful evaluations equal
    the run without speculation."""
    pair = make_workload_pair("lowres-450x375")
    prm = dict(params_for("lowres-450x375"), device_cut=0, host_threads=16)
    ctx = L.lexp_create(prm, _cuda(pair.left), _cuda(pair.right))
    on = _run(ctx, prm, grids, 1, 0, speculate=True)
    off = _run(ctx, prm, grids, 1, 0)
    ctx.close()
    _same(on, off)
    st, st0 = on[3], off[3]
    assert st0["spec_steps"] == 0 and st0["spec_misses"] == 0
    assert st["spec_misses"] == 0
    kr = [g[3] if len(g) > 3 else 0 for g in grids]
    expect = sum(16 * (g[1] + g[2] + r - 1 - r) for g, r in zip(grids, kr) if g[0] >= 15)
    assert st["spec_steps"] == expect
    assert st["unary_evals"] == st0["unary_evals"]
    assert st["unary_launches"] == st0["unary_launches"]  # a speculative launch replaces the step's own


def test_speculation_with_device_cuts_and_split_groups():
    """The default set-up (device max-flow on, the 5-px groups split in two
    parts, which are not speculated): identical to the run without."""
    pair = make_workload_pair("lowres-450x375")
    prm = params_for("lowres-450x375")
    grids = [(5, 1, 7), (15, 1, 7), (25, 1, 7)]
    ctx = L.lexp_create(prm, _cuda(pair.left), _cuda(pair.right))
    on = _run(ctx, prm, grids, 1, 3, speculate=True)
    off = _run(ctx, prm, grids, 1, 3)
    ctx.close()
    _same(on, off)
    assert on[3]["spec_misses"] == 0 and on[3]["spec_steps"] > 0
