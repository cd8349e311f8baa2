"""Training and evaluation of the learned proposal network (orchestration
only: every arithmetic step runs in the library's kernels).

Training data: synthetic pairs made like the 450x375 workload with scene
seeds from 1000; for each, the plain method's labels after 1 and after 3
iterations are inputs and its labels after 10 iterations the target.
Evaluation: held-out scene seeds from 1200, the plain method against the
method with learned proposals in half of its refinement steps, compared by
the wall time each needs to come within 0.5% of the plain method's final
energy.
"""
from __future__ import annotations

import time

import numpy as np

from . import lexp as L


def _scene(seed: int):
    from synth import make_pair, params_for, workload
    sc = dict(workload("lowres-450x375")["scene"], seed=int(seed))
    return make_pair(**sc), params_for("lowres-450x375")


def _run(ctx, grids, iterations, seed, learned=False):
    import torch
    h, w = ctx.height, ctx.width
    lab = torch.zeros((h, w, 4), device="cuda")
    cost = torch.zeros((h, w), device="cuda")
    e, t = L.lexp_optimize(ctx, grids, iterations, seed, lab, cost, learned=learned)
    return lab, e, t


def make_training_set(seeds, input_iterations=(1, 3), target_iterations=10, solver_seed=0, log=None):
    """[(ctx, input labels, target labels)] (device tensors), one entry per
    seed and input iteration count.  log (optional) is called with a line of
    progress every ten scenes."""
    import torch
    from synth import workload
    grids = workload("lowres-450x375")["grids"]
    out = []
    t0 = time.perf_counter()
    for k, sd in enumerate(seeds):
        if log and k % 10 == 0:
            log(f"training set: scene {k} of {len(seeds)}, {time.perf_counter() - t0:.0f} s")
        pair, prm = _scene(sd)
        ctx = L.lexp_create(prm, torch.from_numpy(pair.left).cuda(), torch.from_numpy(pair.right).cuda())
        target, _, _ = _run(ctx, grids, target_iterations, solver_seed)
        for it in input_iterations:
            inp, _, _ = _run(ctx, grids, it, solver_seed)
            out.append((ctx, inp, target))
    return out


def train(net, samples, epochs=20, lr=1e-3, seed=0):
    """Adam over the samples in a seeded order each epoch; returns the mean
    loss of every epoch."""
    rng = np.random.default_rng(seed)
    hist = []
    for _ in range(epochs):
        order = rng.permutation(len(samples))
        losses = [L.lexp_net_train_step(net, samples[i][0], samples[i][1], samples[i][2], lr=lr) for i in order]
        hist.append(float(np.mean(losses)))
    return hist


def _time_to(e, t, level):
    for ei, ti in zip(e, t):
        if ei <= level:
            return float(ti)
    return None


def evaluate(net, seeds, iterations=10, solver_seed=0, tol=0.005, log=None):
    """Plain against learned proposals on held-out scenes: per scene, the
    final energies, the energy and time traces, and the wall time each run
    needs to come within tol of the plain run's final energy."""
    import torch
    from synth import workload
    grids = workload("lowres-450x375")["grids"]
    res = []
    for sd in seeds:
        pair, prm = _scene(sd)
        ctx = L.lexp_create(prm, torch.from_numpy(pair.left).cuda(), torch.from_numpy(pair.right).cuda())
        L.lexp_set_net(ctx, net)
        _run(ctx, grids, 1, solver_seed)  # warm-up
        _, ep, tp = _run(ctx, grids, iterations, solver_seed)
        _, el, tl = _run(ctx, grids, iterations, solver_seed, learned=True)
        level = ep[-1] * (1 + tol)
        if log:
            log(f"held-out scene {sd}: plain {ep[-1]:.1f}, learned {el[-1]:.1f}")
        res.append(dict(seed=int(sd), plain_final=float(ep[-1]), learned_final=float(el[-1]),
                        plain_time_to=_time_to(ep, tp, level), learned_time_to=_time_to(el, tl, level),
                        plain_total_s=float(tp[-1]), learned_total_s=float(tl[-1]),
                        plain_energy=[round(float(x), 2) for x in ep], learned_energy=[round(float(x), 2) for x in el],
                        plain_time=[round(float(x), 4) for x in tp], learned_time=[round(float(x), 4) for x in tl]))
        ctx.close()
    return res


def conv_throughput(net, ctx, labels, reps=20):
    """(forward ms, train-step ms, forward TFLOP/s, train-step TFLOP/s) on one
    image: 2 * pixels * sum over layers of 9 * in * out FLOPs per forward,
    three times that per training step (forward, input and weight
    gradients)."""
    import torch
    h, w = ctx.height, ctx.width
    macs = sum(9 * a * b for a, b in zip((16, 32, 32, 32, 32), (32, 32, 32, 32, 16)))
    fl = 2.0 * h * w * macs
    L.lexp_net_forward(net, ctx, labels)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        L.lexp_net_forward(net, ctx, labels)
    e.record()
    torch.cuda.synchronize()
    f_ms = s.elapsed_time(e) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        L.lexp_net_train_step(net, ctx, labels, labels, lr=1e-12)
    t_ms = (time.perf_counter() - t0) / reps * 1e3
    return f_ms, t_ms, fl / (f_ms * 1e-3) / 1e12, 3 * fl / (t_ms * 1e-3) / 1e12
