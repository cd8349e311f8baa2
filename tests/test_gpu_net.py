"""The learned proposal network on the device (BF16 MFMA implicit GEMMs)
against its PyTorch CPU reference, and learned proposals in the optimiser.

Both sides round the same values to BF16 at the same points and sum in FP32;
they differ in the order of FP32 sums, which now and then moves a BF16
rounding by one unit.  The tolerances below are a few BF16 units of the
values' scale."""
import numpy as np
import pytest

from oracle import net as N
from synth import make_workload_pair, params_for, random_labels

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_1603_08328_amd.lexp")


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _split(w, b):
    """Flat weight/bias arrays -> oracle parameters [(W[tap][out][in], b)]."""
    ps, wi, bi = [], 0, 0
    for l in range(N.N_LAYERS):
        ci, co = N.CH[l], N.CH[l + 1]
        ps.append((torch.from_numpy(w[wi:wi + 9 * co * ci].reshape(9, co, ci).astype(np.float32)),
                   torch.from_numpy(b[bi:bi + co].astype(np.float32))))
        wi += 9 * co * ci
        bi += co
    return ps


@pytest.fixture(scope="module")
def setup():
    pair = make_workload_pair("tiny-64x48")
    prm = params_for("tiny-64x48")
    ctx = L.lexp_create(prm, _cuda(pair.left), _cuda(pair.right))
    rng = np.random.default_rng(0)
    lab = np.zeros((48, 64, 4), np.float32)
    lab[..., :3] = np.where(rng.random((48, 64, 1)) < 0.5, random_labels(rng, 48, 64, 16.0), pair.gt_labels)
    net = L.lexp_net_create(64, 48, seed=7)
    w, b = L.lexp_net_get_weights(net)
    b = np.random.default_rng(1).normal(0, 0.05, b.shape).astype(np.float32)  # nonzero biases too
    L.lexp_net_set_weights(net, w, b)
    return pair, prm, ctx, lab, net, w, b


def test_net_sizes_and_init():
    nw, nb = L.lexp_net_sizes()
    assert nw == sum(9 * N.CH[l] * N.CH[l + 1] for l in range(5)) and nb == sum(N.CH[1:])
    net = L.lexp_net_create(32, 16, seed=3)
    w, b = L.lexp_net_get_weights(net)
    assert np.all(b == 0)
    off = 0
    for l in range(5):
        n = 9 * N.CH[l] * N.CH[l + 1]
        lim = np.sqrt(6.0 / (9 * N.CH[l]))
        assert np.all(np.abs(w[off:off + n]) <= lim) and np.abs(w[off:off + n]).max() > 0.9 * lim
        off += n
    w2, _ = L.lexp_net_get_weights(L.lexp_net_create(32, 16, seed=3))
    assert np.array_equal(w, w2)


def test_net_forward_matches_reference(setup):
    pair, prm, ctx, lab, net, w, b = setup
    y = L.lexp_net_forward(net, ctx, _cuda(lab)).cpu().numpy()
    x0 = N.net_input(pair.left, pair.right, lab[..., :3], prm["disp_max"])
    _, yo = N.forward(_split(w, b), x0)
    yo = yo[0].permute(1, 2, 0).numpy()
    err = np.abs(y - yo)
    scale = np.abs(yo).max()
    assert err.max() <= 2e-2 * scale, (err.max(), scale)
    assert np.median(err) <= 1e-3 * scale


def test_net_train_step_gradients_and_loss_match_reference(setup):
    pair, prm, ctx, lab, _, w, b = setup
    net = L.lexp_net_create(64, 48, seed=7)
    L.lexp_net_set_weights(net, w, b)
    target = np.zeros_like(lab)
    target[..., :3] = pair.gt_labels
    loss = L.lexp_net_train_step(net, ctx, _cuda(lab), _cuda(target), lr=1e-3)
    gw, gb = L.lexp_net_get_grads(net)
    ps = _split(w, b)
    x0 = N.net_input(pair.left, pair.right, lab[..., :3], prm["disp_max"])
    acts, yo = N.forward(ps, x0)
    tgt = pair.gt_labels.astype(np.float64)
    u = np.arange(64)[None, :]
    v = np.arange(48)[:, None]
    td = tgt[..., 0] * u + tgt[..., 1] * v + tgt[..., 2]
    oloss, gy = N.loss_and_grad(yo, td, prm["disp_max"])
    assert abs(loss - oloss) <= 1e-3 * oloss
    grads = N.backward(ps, acts, gy)
    ow = np.concatenate([g[0].numpy().ravel() for g in grads])
    ob = np.concatenate([g[1].numpy().ravel() for g in grads])
    for got, ref in ((gw, ow), (gb, ob)):
        off = 0
        for l in range(5):
            n = (9 * N.CH[l] * N.CH[l + 1]) if got is gw else N.CH[l + 1]
            g, r = got[off:off + n], ref[off:off + n]
            assert np.abs(g - r).max() <= 3e-2 * np.abs(r).max() + 1e-12, (l, np.abs(g - r).max(), np.abs(r).max())
            assert np.corrcoef(g, r)[0, 1] > 0.999 or np.abs(r).max() < 1e-9
            off += n
    # Adam's first step moves each weight by lr * g / (|g| + eps)
    w1, _ = L.lexp_net_get_weights(net)
    assert np.allclose(w1 - w, -1e-3 * gw / (np.abs(gw) + 1e-8), atol=2e-7)


def test_training_lowers_the_loss(setup):
    pair, prm, ctx, lab, _, w, b = setup
    net = L.lexp_net_create(64, 48, seed=7)
    target = np.zeros_like(lab)
    target[..., :3] = pair.gt_labels
    losses = [L.lexp_net_train_step(net, ctx, _cuda(lab), _cuda(target), lr=1e-3) for _ in range(60)]
    assert losses[-1] < 0.7 * losses[0], losses[::10]


def test_optimize_with_learned_proposals(setup):
    """Learned proposals in half the refinement steps: the energy never
    rises, runs are deterministic, and a batch of two pairs equals the pairs
    run alone."""
    pair, prm, ctx, lab, net, w, b = setup
    L.lexp_set_net(ctx, net)
    out = []
    for _ in range(2):
        labs = torch.zeros((48, 64, 4), device="cuda")
        cost = torch.zeros((48, 64), device="cuda")
        e, _ = L.lexp_optimize(ctx, [(5, 1, 3)], 2, 0, labs, cost, learned=True)
        assert np.all(np.diff(e) <= 1e-9)
        out.append((labs.cpu().numpy(), e))
    assert np.array_equal(out[0][0], out[1][0])
    plain = torch.zeros((48, 64, 4), device="cuda")
    L.lexp_optimize(ctx, [(5, 1, 3)], 2, 0, plain, torch.zeros((48, 64), device="cuda"))
    assert not np.array_equal(plain.cpu().numpy(), out[0][0])  # the learned steps change the search
    ctx2 = L.lexp_create(prm, _cuda(pair.right), _cuda(pair.left))
    L.lexp_set_net(ctx2, net)
    alone2 = torch.zeros((48, 64, 4), device="cuda")
    L.lexp_optimize(ctx2, [(5, 1, 3)], 2, 5, alone2, torch.zeros((48, 64), device="cuda"), learned=True)
    labs = [torch.zeros((48, 64, 4), device="cuda") for _ in range(2)]
    costs = [torch.zeros((48, 64), device="cuda") for _ in range(2)]
    L.lexp_optimize_batch([ctx, ctx2], [(5, 1, 3)], 2, [0, 5], labs, costs, learned=True)
    assert np.array_equal(labs[0].cpu().numpy(), out[0][0])
    assert torch.equal(labs[1], alone2)
    with pytest.raises(L.LexpError):
        L.lexp_set_net(ctx, None)
        L.lexp_optimize(ctx, [(5, 1, 3)], 1, 0, labs[0], costs[0], learned=True)


def test_optimize_learned_equals_oracle_driven_by_the_networks_output(setup):
    """lexp_optimize with learned proposals against Alg. 2 run by the oracle
    with the same proposer rule (odd refinement steps from the second
    iteration on take the network's plane at the step's pixel).  The oracle is
    given the device network's output on the oracle's own labels at the start
    of each level pass: that output is an input of the proposer, like its
    random numbers (the network itself is checked against its CPU reference
    above).  Labels bit-identical, energy to 1e-5."""
    from oracle import Oracle
    pair, prm, ctx, _, net, _, _ = setup
    ora = Oracle(prm, pair.left, pair.right)
    L.lexp_set_net(ctx, net)
    H, W = 48, 64
    seed, grids, iters = 0, [(5, 1, 3)], 3
    labs = torch.zeros((H, W, 4), device="cuda")
    cost = torch.zeros((H, W), device="cuda")
    e, _ = L.lexp_optimize(ctx, grids, iters, seed, labs, cost, learned=True)
    olab = ora.init_labels(seed)
    ocost = ora.pixel_costs(olab)
    r_d, r_n = prm["disp_max"] / 2.0, 1.0
    n_learned = 0
    for it in range(iters):
        for h, (cell, kp, kr) in enumerate(grids):
            planes = None
            if it >= 1:
                l4 = np.zeros((H, W, 4), np.float32)
                l4[..., :3] = olab
                y = L.lexp_net_forward(net, ctx, _cuda(l4))
                planes = ora.planes_from_net_output(y.cpu().numpy())
            nci, ncj = -(-W // cell), -(-H // cell)
            for k in range(16):
                cells = [(i, j) for j in range(k // 4, ncj, 4) for i in range(k % 4, nci, 4)]
                rects = [((i - 1) * cell, (j - 1) * cell, (i + 2) * cell, (j + 2) * cell) for i, j in cells]
                for step in range(kp + kr):
                    alphas = [ora.propose_learned(olab, planes, seed, it, h, cell, i, j, step, kp, r_d, r_n)
                              for i, j in cells]
                    if planes is not None and step >= kp and (step - kp) % 2 == 1:
                        n_learned += len(cells)
                    ora.expand_step(olab, ocost, rects, alphas)
        r_d *= 0.5
        r_n *= 0.5
    g3 = labs.cpu().numpy()[..., :3]
    assert n_learned > 0
    assert np.array_equal(g3.view(np.uint32), olab.view(np.uint32)), f"{np.any(g3 != olab, axis=-1).sum()} differ"
    assert ora.energy(olab, ocost)[0] == pytest.approx(e[-1], rel=1e-5)
