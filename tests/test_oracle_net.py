"""Pins of the proposal network's reference (oracle/net.py): the convolution
against direct loops, the backward pass against finite differences (FP64,
no rounding), the loss against closed forms and the first Adam step."""
import numpy as np
import pytest
import torch

from oracle import net as N


def _params(rng, scale=0.3):
    ps = []
    for l in range(N.N_LAYERS):
        ci, co = N.CH[l], N.CH[l + 1]
        w = torch.from_numpy(rng.normal(0, scale / np.sqrt(9 * ci), (9, co, ci)))
        b = torch.from_numpy(rng.normal(0, 0.05, co))
        ps.append((w, b))
    return ps


def test_first_layer_equals_direct_loops():
    rng = np.random.default_rng(1)
    ps = _params(rng)
    x0 = torch.from_numpy(rng.normal(0, 1, (1, 16, 5, 6)))
    acts, _ = N.forward(ps, x0, round=False)
    w, b = ps[0]
    x = x0[0].numpy()
    h, wd = 5, 6
    for o in range(32):
        for v in range(h):
            for u in range(wd):
                s = float(b[o])
                for ky in range(3):
                    for kx in range(3):
                        yy, xx = v + ky - 1, u + kx - 1
                        if 0 <= yy < h and 0 <= xx < wd:
                            s += float(np.dot(w[3 * ky + kx, o].numpy(), x[:, yy, xx]))
                assert abs(acts[1][0, o, v, u].item() - max(s, 0.0)) < 1e-12


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    ps = _params(rng, scale=1.0)
    h, w, dmax = 7, 9, 20.0
    x0 = torch.from_numpy(rng.normal(0, 1, (1, 16, h, w)))
    target = rng.uniform(0, dmax, (h, w))

    def loss_of(params):
        _, y = N.forward(params, x0, round=False)
        return N.loss_and_grad(y, target, dmax)[0]

    acts, y = N.forward(ps, x0, round=False)
    _, gy = N.loss_and_grad(y, target, dmax)
    grads = N.backward(ps, acts, gy, round=False)
    eps = 1e-6
    for l in range(N.N_LAYERS):
        w, b = ps[l]
        for _ in range(4):
            idx = tuple(int(rng.integers(0, s)) for s in w.shape)
            if l == N.N_LAYERS - 1:
                idx = (idx[0], int(rng.integers(0, N.OUT_USED)), idx[2])
            old = w[idx].item()
            w[idx] = old + eps
            lp = loss_of(ps)
            w[idx] = old - eps
            lm = loss_of(ps)
            w[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - grads[l][0][idx].item()) < 1e-6 + 1e-4 * abs(fd), (l, idx, fd, grads[l][0][idx].item())
        o = int(rng.integers(0, N.OUT_USED if l == N.N_LAYERS - 1 else b.shape[0]))
        old = b[o].item()
        b[o] = old + eps
        lp = loss_of(ps)
        b[o] = old - eps
        lm = loss_of(ps)
        b[o] = old
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grads[l][1][o].item()) < 1e-6 + 1e-4 * abs(fd)


@pytest.mark.parametrize("delta", [0.0, 0.75, -3.5])
def test_loss_of_a_shifted_fronto_parallel_plane(delta):
    h, w, dmax, T = 6, 8, 40.0, 12.0
    y = torch.zeros((1, 16, h, w), dtype=torch.float64)
    y[0, 2] = (T + delta) / dmax
    loss, g = N.loss_and_grad(y, np.full((h, w), T), dmax)
    assert abs(loss - abs(delta)) < 1e-12
    if delta:
        # every residual has the sign of delta: d loss / d(d_p) = sign / n per pixel
        assert np.allclose(g[0, 2].numpy(), np.sign(delta) * dmax / (h * w))


def test_first_adam_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(3)
    ps = _params(rng)
    before = [(w.clone(), b.clone()) for w, b in ps]
    grads = [(torch.from_numpy(rng.normal(0, 1, w.shape)), torch.from_numpy(rng.normal(0, 1, b.shape)))
             for w, b in ps]
    N.adam_step(ps, grads, {}, lr=1e-3)
    for (w0, b0), (w1, b1), (gw, gb) in zip(before, ps, grads):
        assert torch.allclose(w1 - w0, -1e-3 * gw / (gw.abs() + 1e-8), atol=1e-12)
        assert torch.allclose(b1 - b0, -1e-3 * gb / (gb.abs() + 1e-8), atol=1e-12)


def test_learned_step_takes_the_plane_at_the_steps_own_pixel(tiny_oracle):
    """Every pixel carries its own fronto-parallel label, so a label names its
    pixel.  With zero perturbation sizes a refinement step returns f_r of its
    drawn pixel r (the perturbation round-trips); a learned refinement step
    (odd refinement index) returns planes[r] of the same pixel; every other
    step is the plain proposer's."""
    o = tiny_oracle
    H, W = o.H, o.W
    lab = np.zeros((H, W, 3), np.float32)
    lab[..., 2] = np.arange(H * W, dtype=np.float32).reshape(H, W)
    planes = np.zeros((H, W, 3), np.float32)
    planes[..., 0] = 1.0
    planes[..., 2] = lab[..., 2] + 0.5
    for (ci, cj) in [(0, 0), (3, 2), (12, 9)]:
        for step in range(6):
            plain = o.propose(lab, 3, 1, 0, 5, ci, cj, step, 1, 0.0, 0.0)
            learned = o.propose_learned(lab, planes, 3, 1, 0, 5, ci, cj, step, 1, 0.0, 0.0)
            assert np.array_equal(o.propose_learned(lab, None, 3, 1, 0, 5, ci, cj, step, 1, 0.0, 0.0), plain)
            px = int(plain[2])
            u, v = px % W, px // W
            assert ci * 5 <= u < ci * 5 + 5 and cj * 5 <= v < cj * 5 + 5
            if step >= 1 and (step - 1) % 2 == 1:
                assert np.array_equal(learned, planes[v, u])
            else:
                assert np.array_equal(learned, plain)


def test_planes_from_net_output_pass_through_the_predicted_disparity(tiny_oracle):
    o = tiny_oracle
    rng = np.random.default_rng(3)
    y = np.zeros((o.H, o.W, 16), np.float32)
    y[..., 0] = rng.uniform(-0.5, 0.5, (o.H, o.W))
    y[..., 1] = rng.uniform(-0.5, 0.5, (o.H, o.W))
    y[..., 2] = rng.uniform(0.0, 1.0, (o.H, o.W))
    pl = o.planes_from_net_output(y)
    v, u = np.mgrid[0:o.H, 0:o.W]
    d = pl[..., 0].astype(np.float64) * u + pl[..., 1].astype(np.float64) * v + pl[..., 2].astype(np.float64)
    d_pred = y[..., 2].astype(np.float64) * o.p["disp_max"]
    # c is rounded once to FP32 (|c| < 64 here)
    assert np.all(np.abs(d - d_pred) <= 2.0 ** -24 * 64)
    assert np.array_equal(pl[..., :2], y[..., :2])
