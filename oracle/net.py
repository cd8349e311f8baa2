"""Reference of the learned proposal network (test infrastructure only).

Plain PyTorch CPU operations.  Only the tests and the benchmark's CPU leg use
this module; the library never does.  It shares no code with the HIP path.

The network proposes a plane label per pixel from the two images and the
current label field: five 3x3 convolutions (zero padding), ReLU after the
first four, 32 channels inside.  Readings (the paper's method admits any
proposer of alpha_ij; this one is not in the paper):
  * input, 16 channels per pixel: left RGB / 255; right RGB / 255 at the
    pixel's match x = u - d (linear interpolation, zero outside the right
    image); a, b, d / disp_max with d = a u + b v + c; 1 where the match is
    inside the right image; then six zeros (the context's own frame);
  * output, 16 channels of which the first three are used: (a, b, d / disp_max)
    of a plane; the candidate of a pixel is that plane, c = d - a u - b v;
  * layer channels 16 -> 32 -> 32 -> 32 -> 32 -> 16; weights indexed
    [tap][out][in] with tap = 3 ky + kx, offset (kx - 1, ky - 1);
  * BF16 operands with FP32 sums: weights, activations and the gradients fed
    to the products are rounded to BF16 (nearest even); the last layer's
    output and every sum stay FP32;
  * loss: the mean over pixels p of the mean over the 5x5 neighbourhood q of
    p (clipped) of |d_p + a_p (u_q - u_p) + b_p (v_q - v_p) - d*_q| in pixels
    (d*: the target label field's disparity), i.e. the L1 disparity error of
    the plane proposed at p over a 5x5 cell around it;
  * Adam (beta 0.9 / 0.999, eps 1e-8, bias-corrected) on FP32 master weights.
With round=False every step is plain FP64, for the gradient pins.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

CH = [16, 32, 32, 32, 32, 16]
N_LAYERS = 5
OUT_USED = 3
LOSS_R = 2


def _bf16(t: torch.Tensor, on: bool) -> torch.Tensor:
    return t.to(torch.bfloat16).to(torch.float32) if on else t


def _w_torch(w: torch.Tensor) -> torch.Tensor:
    """[tap][out][in] -> conv2d's [out][in][ky][kx]."""
    taps, co, ci = w.shape
    return w.reshape(3, 3, co, ci).permute(2, 3, 0, 1)


def net_input(left: np.ndarray, right: np.ndarray, labels: np.ndarray, disp_max: float) -> torch.Tensor:
    """(1, 16, H, W) input of the network (FP64, unrounded)."""
    h, w = labels.shape[:2]
    lab = labels.astype(np.float64)
    u = np.arange(w)[None, :]
    v = np.arange(h)[:, None]
    d = lab[..., 0] * u + lab[..., 1] * v + lab[..., 2]
    xm = u - d
    inside = (xm >= 0) & (xm <= w - 1)
    i0 = np.where(inside, np.floor(np.where(inside, xm, 0)), 0).astype(np.int64)
    i1 = np.minimum(i0 + 1, w - 1)
    t = np.where(inside, xm - i0, 0.0)
    rows = np.broadcast_to(v, (h, w))
    r = right.astype(np.float64)
    warped = (1 - t)[..., None] * r[rows, i0] + t[..., None] * r[rows, i1]
    warped[~inside] = 0.0
    x = np.zeros((16, h, w))
    x[0:3] = np.moveaxis(left.astype(np.float64) / 255.0, -1, 0)
    x[3:6] = np.moveaxis(warped / 255.0, -1, 0)
    x[6] = lab[..., 0]
    x[7] = lab[..., 1]
    x[8] = d / disp_max
    x[9] = inside
    return torch.from_numpy(x)[None]


def forward(params, x0: torch.Tensor, round: bool = True):
    """Returns the activations [x0 .. x4] (as fed to the products) and the
    FP32 output y (1, 16, H, W)."""
    dt = torch.float32 if round else torch.float64
    acts = [_bf16(x0.to(dt), round)]
    for l in range(N_LAYERS):
        w, b = params[l]
        z = F.conv2d(acts[-1], _bf16(_w_torch(w.to(dt)), round), b.to(dt), padding=1)
        if l < N_LAYERS - 1:
            acts.append(_bf16(torch.relu(z), round))
        else:
            return acts, z


def loss_and_grad(y: torch.Tensor, target_disp: np.ndarray, disp_max: float):
    """Loss and dLoss/dy (same shape as y, zero beyond the used channels)."""
    yy = y[0].to(torch.float64)
    h, w = target_disp.shape
    a, b, dn = yy[0], yy[1], yy[2]
    d = dn * disp_max
    t = torch.from_numpy(target_disp.astype(np.float64))
    ga = torch.zeros(h, w, dtype=torch.float64)
    gb = torch.zeros_like(ga)
    gd = torch.zeros_like(ga)
    cnt = torch.zeros_like(ga)
    total = torch.zeros(h, w, dtype=torch.float64)
    for dy in range(-LOSS_R, LOSS_R + 1):
        for dx in range(-LOSS_R, LOSS_R + 1):
            # neighbour q = p + (dx, dy) when inside the image
            ok = torch.zeros(h, w, dtype=torch.bool)
            ok[max(-dy, 0):h - max(dy, 0), max(-dx, 0):w - max(dx, 0)] = True
            tq = torch.zeros_like(t)
            tq[max(-dy, 0):h - max(dy, 0), max(-dx, 0):w - max(dx, 0)] = \
                t[max(dy, 0):h - max(-dy, 0), max(dx, 0):w - max(-dx, 0)]
            r = d + a * dx + b * dy - tq
            s = torch.sign(r) * ok
            total += torch.abs(r) * ok
            gd += s
            ga += s * dx
            gb += s * dy
            cnt += ok
    n = h * w
    loss = float((total / cnt).sum() / n)
    g = torch.zeros_like(y, dtype=torch.float64)
    g[0, 0] = ga / cnt / n
    g[0, 1] = gb / cnt / n
    g[0, 2] = gd / cnt / n * disp_max
    return loss, g


def backward(params, acts, g_y: torch.Tensor, round: bool = True):
    """Gradients [(dW, db)] per layer ([tap][out][in], [out]), the incoming
    gradient of each layer rounded to BF16 before its products."""
    dt = torch.float32 if round else torch.float64
    grads = [None] * N_LAYERS
    g = _bf16(g_y.to(dt), round)
    for l in range(N_LAYERS - 1, -1, -1):
        w, _ = params[l]
        x = acts[l]
        # dW[tap][o][i] = sum_p g[o](p) x[i](p + off(tap))
        co, ci = w.shape[1], w.shape[2]
        h, wd = x.shape[2], x.shape[3]
        xp = F.pad(x, (1, 1, 1, 1))
        dw = torch.zeros((9, co, ci), dtype=dt)
        for ky in range(3):
            for kx in range(3):
                xs = xp[0, :, ky:ky + h, kx:kx + wd].reshape(ci, -1)
                dw[3 * ky + kx] = g[0].reshape(co, -1) @ xs.T
        db = g[0].sum(dim=(1, 2))
        grads[l] = (dw, db)
        if l > 0:
            dx = F.conv_transpose2d(g, _bf16(_w_torch(w.to(dt)), round), padding=1)
            g = _bf16(dx * (x > 0), round)
    return grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on the FP32 master weights (in place); state: dict with
    't' and per-parameter moments."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for l in range(N_LAYERS):
        for k in range(2):
            p = params[l][k]
            gk = grads[l][k].to(p.dtype)
            key = (l, k)
            m, v = state.get(key, (torch.zeros_like(p), torch.zeros_like(p)))
            m = b1 * m + (1 - b1) * gk
            v = b2 * v + (1 - b2) * gk * gk
            state[key] = (m, v)
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            p -= lr * mh / (torch.sqrt(vh) + eps)


def planes_from_output(y: torch.Tensor, disp_max: float) -> np.ndarray:
    """(H, W, 3) candidate planes (a, b, c) of the output, FP32."""
    yy = y[0].to(torch.float64).numpy()
    h, w = yy.shape[1:]
    u = np.arange(w)[None, :]
    v = np.arange(h)[:, None]
    a, b = yy[0], yy[1]
    c = yy[2] * disp_max - a * u - b * v
    return np.stack([a, b, c], axis=-1).astype(np.float32)
