"""Python binding of the C ABI in include/lexp.h (ctypes).

Argument marshalling only: every step of the method runs in liblexp.so (HIP
kernels on the device, max-flow and proposers on the host).  Device buffers
are PyTorch tensors on a ROCm device; host arrays are numpy arrays.  The
functions carry the C names.  Importing works without a GPU; calling a
device function without the built library or without a GPU raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; LEXP_LIBRARY names another build of the same library (comparisons of builds)
LIB_PATH = os.environ.get("LEXP_LIBRARY") or os.path.join(_HERE, "liblexp.so")

LEXP_OK, LEXP_EINVAL, LEXP_ENOMEM, LEXP_EDEVICE, LEXP_ESTATE = 0, -1, -2, -3, -4
LEXP_QUANTUM = 2.0 ** -20


class LexpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lexp status {status}: {msg}")
        self.status = status


class lexp_params(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("disp_max", C.c_double),
                ("alpha", C.c_double), ("tau_col", C.c_double), ("tau_grad", C.c_double),
                ("gf_radius", C.c_int32), ("gf_eps", C.c_double),
                ("lam", C.c_double), ("tau_dis", C.c_double), ("w_floor", C.c_double),
                ("gamma", C.c_double), ("neighbours", C.c_int32), ("host_threads", C.c_int32),
                ("device_cut", C.c_int32), ("view", C.c_int32), ("graph", C.c_int32)]


class lexp_plane(C.Structure):
    _fields_ = [("a", C.c_float), ("b", C.c_float), ("c", C.c_float)]


class lexp_rect(C.Structure):
    _fields_ = [("u0", C.c_int32), ("v0", C.c_int32), ("u1", C.c_int32), ("v1", C.c_int32)]


class lexp_schedule(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("cell", C.c_int32 * 4), ("k_prop", C.c_int32 * 4),
                ("k_rand", C.c_int32 * 4), ("iterations", C.c_int32), ("k_rans", C.c_int32 * 4),
                ("learned", C.c_int32), ("batch_cycle", C.c_int32), ("tile_cols", C.c_int32 * 4),
                ("tile_fill", C.c_int32 * 4), ("speculate", C.c_int32)]


class lexp_stats(C.Structure):
    _fields_ = [("unary_launches", C.c_int64), ("unary_items", C.c_int64), ("unary_evals", C.c_int64),
                ("unary_kernel_ms", C.c_double), ("unary_alg_bytes", C.c_double),
                ("expand_calls", C.c_int64), ("host_cut_ms", C.c_double), ("host_wait_ms", C.c_double),
                ("host_enqueue_ms", C.c_double), ("host_update_ms", C.c_double),
                ("host_cut_level_ms", C.c_double * 4), ("device_cut_fallbacks", C.c_int64),
                ("device_cut_share", C.c_double * 4), ("graphs_captured", C.c_int64),
                ("device_cut_block", C.c_int32 * 4), ("device_cut_relabel", C.c_int32 * 4),
                ("unary_timed_launches", C.c_int64), ("unary_timed_alg_bytes", C.c_double),
                ("unary_timed_evals", C.c_int64), ("host_solve_level_ms", C.c_double * 4),
                ("host_solves", C.c_int64 * 4), ("unary_level_ms", C.c_double * 4),
                ("unary_level_alg_bytes", C.c_double * 4), ("unary_level_launches", C.c_int64 * 4),
                ("spec_steps", C.c_int64), ("spec_misses", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["host_cut_level_ms"] = list(d["host_cut_level_ms"])
        d["device_cut_share"] = list(d["device_cut_share"])
        d["device_cut_block"] = list(d["device_cut_block"])
        d["device_cut_relabel"] = list(d["device_cut_relabel"])
        d["host_solve_level_ms"] = list(d["host_solve_level_ms"])
        d["host_solves"] = list(d["host_solves"])
        for k in ("unary_level_ms", "unary_level_alg_bytes", "unary_level_launches"):
            d[k] = list(d[k])
        return d


# Every symbol the header declares, with (restype, argtypes).
_vp, _i32, _i64, _u64, _f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
_SIGS = {
    "lexp_create": (_i32, [C.POINTER(lexp_params), _vp, _vp, _vp, C.POINTER(_vp)]),
    "lexp_destroy": (_i32, [_vp]),
    "lexp_last_error": (C.c_char_p, []),
    "lexp_unary_cost": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "lexp_guided_coeffs": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "lexp_pixel_costs": (_i32, [_vp, _vp, _vp, _vp]),
    "lexp_expand_region": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "lexp_graph_terms": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "lexp_pairwise": (_i32, [_vp, _i32, _i32, _i32, _i32, lexp_plane, lexp_plane, C.POINTER(_f64)]),
    "lexp_energy": (_i32, [_vp, _vp, _vp, C.POINTER(_f64), C.POINTER(_f64), C.POINTER(_f64), _vp]),
    "lexp_energy_noalloc": (_i32, [_vp, _vp, _vp, C.POINTER(_f64), C.POINTER(_f64), C.POINTER(_f64), _vp]),
    "lexp_init_labels": (_i32, [_vp, _u64, _vp, _vp]),
    "lexp_optimize": (_i32, [_vp, C.POINTER(lexp_schedule), _u64, _vp, _vp, _vp, _vp, _vp]),
    "lexp_view_labels": (_i32, [_vp, _vp, _vp, _vp]),
    "lexp_net_sizes": (_i32, [_vp, _vp]),
    "lexp_net_create": (_i32, [_i32, _i32, _u64, C.POINTER(_vp)]),
    "lexp_net_destroy": (_i32, [_vp]),
    "lexp_net_set_weights": (_i32, [_vp, _vp, _vp]),
    "lexp_net_get_weights": (_i32, [_vp, _vp, _vp]),
    "lexp_net_get_grads": (_i32, [_vp, _vp, _vp]),
    "lexp_net_forward": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "lexp_net_train_step": (_i32, [_vp, _vp, _vp, _vp, C.c_float, C.POINTER(_f64), _vp]),
    "lexp_set_net": (_i32, [_vp, _vp]),
    "lexp_postprocess": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "lexp_optimize_batch": (_i32, [_i32, _vp, C.POINTER(lexp_schedule), _vp, _vp, _vp, _vp, _vp, _vp]),
    "lexp_set_timing": (_i32, [_vp, _i32]),
    "lexp_get_stats": (_i32, [_vp, C.POINTER(lexp_stats)]),
    "lexp_reset_stats": (_i32, [_vp]),
    "lexp_debug_guide": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "lexp_solve_binary": (_i32, [_i32, _i32, _i32, _vp, _vp, _vp]),
    "lexp_solve_binary_device": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "lexp_rng_key": (_u64, [_u64, _vp, _i32]),
    "lexp_init_labels_host": (_i32, [_i32, _i32, _f64, _u64, _vp]),
    "lexp_propose": (_i32, [_i32, _i32, _vp, _u64, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _f64, _f64,
                            C.POINTER(lexp_plane)]),
}

_lib = None


def load_library():
    """Loads liblexp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1603_08328_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != LEXP_OK:
        msg = load_library().lexp_last_error()
        raise LexpError(status, msg.decode() if msg else "")


def lexp_last_error() -> str:
    m = load_library().lexp_last_error()
    return m.decode() if m else ""


# ---- marshalling helpers ------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t, dtype, shape=None, min_numel=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name} holds {t.numel()} values, needs {min_numel}")
    return C.c_void_p(t.data_ptr())


def _host(a, dtype, cols=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    if cols is not None:
        a = a.reshape(-1, cols)
    return a


def _clipped_sizes(ctx, rects, dilate=0):
    r = rects.astype(np.int64)
    u0 = np.maximum(r[:, 0] - dilate, 0)
    v0 = np.maximum(r[:, 1] - dilate, 0)
    u1 = np.minimum(r[:, 2] + dilate, ctx.width)
    v1 = np.minimum(r[:, 3] + dilate, ctx.height)
    # R+ of an empty rectangle is empty too
    w0 = np.minimum(r[:, 2], ctx.width) - np.maximum(r[:, 0], 0)
    h0 = np.minimum(r[:, 3], ctx.height) - np.maximum(r[:, 1], 0)
    empty = (w0 <= 0) | (h0 <= 0)
    sz = np.maximum(u1 - u0, 0) * np.maximum(v1 - v0, 0)
    sz[empty] = 0
    return sz


class LexpContext:
    """Owns one lexp_ctx (one stereo pair)."""

    def __init__(self, handle, params: dict):
        self.handle = handle
        self.params = dict(params)
        self.width = int(params["width"])
        self.height = int(params["height"])
        self.radius = int(params["gf_radius"])

    def close(self):
        if self.handle:
            load_library().lexp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lexp_create(params: dict, left, right, stream=None) -> LexpContext:
    lib = load_library()
    torch = _torch()
    h, w = int(params["height"]), int(params["width"])
    P = lexp_params(w, h, float(params["disp_max"]), float(params["alpha"]), float(params["tau_col"]),
                    float(params["tau_grad"]), int(params["gf_radius"]), float(params["gf_eps"]),
                    float(params["lam"]), float(params["tau_dis"]), float(params["w_floor"]),
                    float(params["gamma"]), int(params["neighbours"]), int(params.get("host_threads", 0)),
                    int(params.get("device_cut", 1)), int(params.get("view", 0)), int(params.get("graph", 0)))
    lp = _dev(left, torch.float32, (h, w, 3), name="left")
    rp = _dev(right, torch.float32, (h, w, 3), name="right")
    out = C.c_void_p()
    _check(lib.lexp_create(C.byref(P), lp, rp, _stream_ptr(stream), C.byref(out)))
    return LexpContext(out, params)


def lexp_destroy(ctx: LexpContext):
    ctx.close()


def _items(ctx, rects, labels, offsets):
    rects = _host(rects, np.int32, 4)
    labels = _host(labels, np.float32, 3)
    offsets = _host(offsets, np.int64).reshape(-1)
    n = rects.shape[0]
    if labels.shape[0] != n or offsets.shape[0] != n:
        raise ValueError("rects, labels and offsets must have the same length")
    return n, rects, labels, offsets


def lexp_unary_cost(ctx, rects, labels, offsets, out_cost, stream=None):
    torch = _torch()
    n, rects, labels, offsets = _items(ctx, rects, labels, offsets)
    need = int(np.max(offsets + _clipped_sizes(ctx, rects))) if n else 0
    op = _dev(out_cost, torch.float32, min_numel=need, name="out_cost")
    _check(load_library().lexp_unary_cost(ctx.handle, n, rects.ctypes.data, labels.ctypes.data,
                                          offsets.ctypes.data, op, _stream_ptr(stream)))


def lexp_guided_coeffs(ctx, rects, labels, offsets, out_ab, stream=None):
    torch = _torch()
    n, rects, labels, offsets = _items(ctx, rects, labels, offsets)
    need = int(np.max(offsets + _clipped_sizes(ctx, rects, ctx.radius))) * 4 if n else 0
    op = _dev(out_ab, torch.float32, min_numel=need, name="out_ab")
    _check(load_library().lexp_guided_coeffs(ctx.handle, n, rects.ctypes.data, labels.ctypes.data,
                                             offsets.ctypes.data, op, _stream_ptr(stream)))


def lexp_pixel_costs(ctx, labels, out_cost, stream=None):
    torch = _torch()
    lp = _dev(labels, torch.float32, (ctx.height, ctx.width, 4), name="labels")
    op = _dev(out_cost, torch.float32, (ctx.height, ctx.width), name="out_cost")
    _check(load_library().lexp_pixel_costs(ctx.handle, lp, op, _stream_ptr(stream)))


def lexp_expand_region(ctx, rects, alpha, alpha_cost, offsets, labels, cur_cost, stream=None):
    """Returns (delta_Eq int64[n], n_changed int32[n])."""
    torch = _torch()
    n, rects, alpha, offsets = _items(ctx, rects, alpha, offsets)
    need = int(np.max(offsets + _clipped_sizes(ctx, rects))) if n else 0
    ap = _dev(alpha_cost, torch.float32, min_numel=need, name="alpha_cost")
    lp = _dev(labels, torch.float32, (ctx.height, ctx.width, 4), name="labels")
    cp = _dev(cur_cost, torch.float32, (ctx.height, ctx.width), name="cur_cost")
    de = np.zeros(n, np.int64)
    nc = np.zeros(n, np.int32)
    _check(load_library().lexp_expand_region(ctx.handle, n, rects.ctypes.data, alpha.ctypes.data, ap,
                                             offsets.ctypes.data, lp, cp, de.ctypes.data, nc.ctypes.data,
                                             _stream_ptr(stream)))
    return de, nc


def lexp_graph_terms(ctx, rects, alpha, alpha_cost, offsets, labels, cur_cost, out_terms, stream=None):
    torch = _torch()
    n, rects, alpha, offsets = _items(ctx, rects, alpha, offsets)
    need = int(np.max(offsets + _clipped_sizes(ctx, rects))) if n else 0
    ap = _dev(alpha_cost, torch.float32, min_numel=need, name="alpha_cost")
    lp = _dev(labels, torch.float32, (ctx.height, ctx.width, 4), name="labels")
    cp = _dev(cur_cost, torch.float32, (ctx.height, ctx.width), name="cur_cost")
    tp = _dev(out_terms, torch.int32, min_numel=need * 5, name="out_terms")
    _check(load_library().lexp_graph_terms(ctx.handle, n, rects.ctypes.data, alpha.ctypes.data, ap,
                                           offsets.ctypes.data, lp, cp, tp, _stream_ptr(stream)))


def lexp_pairwise(ctx, p, q, fp, fq) -> float:
    out = C.c_double()
    fp = [float(x) for x in fp]
    fq = [float(x) for x in fq]
    _check(load_library().lexp_pairwise(ctx.handle, int(p[0]), int(p[1]), int(q[0]), int(q[1]),
                                        lexp_plane(*fp), lexp_plane(*fq), C.byref(out)))
    return out.value


def lexp_energy(ctx, labels, cur_cost, stream=None):
    """Returns (total, unary, pairwise)."""
    torch = _torch()
    lp = _dev(labels, torch.float32, (ctx.height, ctx.width, 4), name="labels")
    cp = _dev(cur_cost, torch.float32, (ctx.height, ctx.width), name="cur_cost")
    t, u, p = C.c_double(), C.c_double(), C.c_double()
    _check(load_library().lexp_energy(ctx.handle, lp, cp, C.byref(t), C.byref(u), C.byref(p),
                                      _stream_ptr(stream)))
    return t.value, u.value, p.value


def lexp_energy_noalloc(ctx, labels, cur_cost, stream=None):
    """lexp_energy without allocation (the library's fixed per-GPU array).
    Returns (total, unary, pairwise)."""
    torch = _torch()
    lp = _dev(labels, torch.float32, (ctx.height, ctx.width, 4), name="labels")
    cp = _dev(cur_cost, torch.float32, (ctx.height, ctx.width), name="cur_cost")
    t, u, p = C.c_double(), C.c_double(), C.c_double()
    _check(load_library().lexp_energy_noalloc(ctx.handle, lp, cp, C.byref(t), C.byref(u), C.byref(p),
                                              _stream_ptr(stream)))
    return t.value, u.value, p.value


def lexp_init_labels(ctx, seed, labels, stream=None):
    torch = _torch()
    lp = _dev(labels, torch.float32, (ctx.height, ctx.width, 4), name="labels")
    _check(load_library().lexp_init_labels(ctx.handle, C.c_uint64(seed), lp, _stream_ptr(stream)))


def make_schedule(grids, iterations, learned=False, batch_cycle=False, tiles=None, speculate=False) -> lexp_schedule:
    """grids: (cell, K_prop, K_rand) or (cell, K_prop, K_rand, K_RANS) per level;
    tiles: None or one (widest column strip, fill) per level (0: default);
    speculate: evaluate each step's two possible successors while the host
    cuts it (single-part groups; the same results either way)."""
    s = lexp_schedule()
    if not 1 <= len(grids) <= 4:
        raise ValueError("1 to 4 grid levels")
    s.n_levels = len(grids)
    for i, g in enumerate(grids):
        s.cell[i], s.k_prop[i], s.k_rand[i] = int(g[0]), int(g[1]), int(g[2])
        s.k_rans[i] = int(g[3]) if len(g) > 3 else 0
    s.iterations = int(iterations)
    s.learned = 1 if learned else 0
    s.batch_cycle = 1 if batch_cycle else 0
    s.speculate = 1 if speculate and not batch_cycle else 0
    if tiles is not None:
        if len(tiles) != len(grids):
            raise ValueError("one tile plan per grid level")
        for i, (cols, fill) in enumerate(tiles):
            s.tile_cols[i], s.tile_fill[i] = int(cols), int(fill)
    return s


def lexp_optimize(ctx, grids, iterations, seed, labels, cur_cost, stream=None, learned=False, batch_cycle=False,
                  tiles=None, speculate=False):
    """Alg. 2 on the device + host; returns (energy_trace, time_trace)."""
    torch = _torch()
    lp = _dev(labels, torch.float32, (ctx.height, ctx.width, 4), name="labels")
    cp = _dev(cur_cost, torch.float32, (ctx.height, ctx.width), name="cur_cost")
    sch = make_schedule(grids, iterations, learned, batch_cycle, tiles, speculate)
    e = np.zeros(iterations + 1)
    t = np.zeros(iterations + 1)
    _check(load_library().lexp_optimize(ctx.handle, C.byref(sch), C.c_uint64(seed), lp, cp, e.ctypes.data,
                                        t.ctypes.data, _stream_ptr(stream)))
    return e, t


def lexp_optimize_batch(ctxs, grids, iterations, seeds, labels, cur_costs, stream=None, learned=False,
                        batch_cycle=False, tiles=None, speculate=False):
    """Alg. 2 for several pairs at once (one launch per group step for all of
    them); returns (energy traces [n_pairs, iterations+1], time_trace)."""
    torch = _torch()
    n = len(ctxs)
    if not (len(seeds) == len(labels) == len(cur_costs) == n):
        raise ValueError("ctxs, seeds, labels and cur_costs need one entry per pair")
    hs = (C.c_void_p * n)(*[c.handle for c in ctxs])
    lp = (C.c_void_p * n)(*[_dev(l, torch.float32, (c.height, c.width, 4), name="labels")
                            for c, l in zip(ctxs, labels)])
    cp = (C.c_void_p * n)(*[_dev(q, torch.float32, (c.height, c.width), name="cur_cost")
                            for c, q in zip(ctxs, cur_costs)])
    sd = (C.c_uint64 * n)(*[int(x) for x in seeds])
    sch = make_schedule(grids, iterations, learned, batch_cycle, tiles, speculate)
    e = np.zeros((n, iterations + 1))
    ep = (C.c_void_p * n)(*[e[i].ctypes.data for i in range(n)])
    t = np.zeros(iterations + 1)
    _check(load_library().lexp_optimize_batch(n, hs, C.byref(sch), sd, lp, cp, ep, t.ctypes.data,
                                              _stream_ptr(stream)))
    return e, t


def lexp_view_labels(ctx, labels, stream=None):
    """The context's label field in its view image's own frame (a new device
    tensor HxWx4): a copy for the left view, un-mirrored for the right view."""
    torch = _torch()
    lp = _dev(labels, torch.float32, (ctx.height, ctx.width, 4), name="labels")
    out = torch.empty_like(labels)
    _check(load_library().lexp_view_labels(ctx.handle, lp, C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def lexp_postprocess(left_ctx, labels_left, right_ctx, labels_right, stream=None):
    """Left-right check, row filling and weighted median of the left view;
    returns (disparity HxW float32, inconsistent mask HxW uint8), device tensors."""
    torch = _torch()
    h, w = left_ctx.height, left_ctx.width
    lp = _dev(labels_left, torch.float32, (h, w, 4), name="labels_left")
    rp = _dev(labels_right, torch.float32, (h, w, 4), name="labels_right")
    disp = torch.empty((h, w), dtype=torch.float32, device=labels_left.device)
    inv = torch.empty((h, w), dtype=torch.uint8, device=labels_left.device)
    _check(load_library().lexp_postprocess(left_ctx.handle, lp, right_ctx.handle, rp, C.c_void_p(disp.data_ptr()),
                                           C.c_void_p(inv.data_ptr()), _stream_ptr(stream)))
    return disp, inv


class LexpNet:
    """Owns one lexp_net (the learned proposal network)."""

    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle:
            load_library().lexp_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lexp_net_sizes():
    nw, nb = C.c_int32(), C.c_int32()
    _check(load_library().lexp_net_sizes(C.byref(nw), C.byref(nb)))
    return nw.value, nb.value


def lexp_net_create(max_width, max_height, seed=0) -> LexpNet:
    out = C.c_void_p()
    _check(load_library().lexp_net_create(int(max_width), int(max_height), C.c_uint64(seed), C.byref(out)))
    return LexpNet(out)


def lexp_net_set_weights(net, weights, biases):
    nw, nb = lexp_net_sizes()
    w = np.ascontiguousarray(np.asarray(weights, np.float32).ravel())
    b = np.ascontiguousarray(np.asarray(biases, np.float32).ravel())
    if w.size != nw or b.size != nb:
        raise ValueError(f"need {nw} weights and {nb} biases")
    _check(load_library().lexp_net_set_weights(net.handle, w.ctypes.data, b.ctypes.data))


def _net_params(fn, net):
    nw, nb = lexp_net_sizes()
    w = np.zeros(nw, np.float32)
    b = np.zeros(nb, np.float32)
    _check(fn(net.handle, w.ctypes.data, b.ctypes.data))
    return w, b


def lexp_net_get_weights(net):
    return _net_params(load_library().lexp_net_get_weights, net)


def lexp_net_get_grads(net):
    return _net_params(load_library().lexp_net_get_grads, net)


def lexp_net_forward(net, ctx, labels, stream=None):
    """Network output (device tensor HxWx16, FP32) for a context's labels."""
    torch = _torch()
    lp = _dev(labels, torch.float32, (ctx.height, ctx.width, 4), name="labels")
    out = torch.empty((ctx.height, ctx.width, 16), dtype=torch.float32, device=labels.device)
    _check(load_library().lexp_net_forward(net.handle, ctx.handle, lp, C.c_void_p(out.data_ptr()),
                                           _stream_ptr(stream)))
    return out


def lexp_net_train_step(net, ctx, labels, target, lr=1e-3, stream=None) -> float:
    torch = _torch()
    lp = _dev(labels, torch.float32, (ctx.height, ctx.width, 4), name="labels")
    tp = _dev(target, torch.float32, (ctx.height, ctx.width, 4), name="target")
    loss = C.c_double()
    _check(load_library().lexp_net_train_step(net.handle, ctx.handle, lp, tp, C.c_float(lr), C.byref(loss),
                                              _stream_ptr(stream)))
    return loss.value


def lexp_set_net(ctx, net):
    _check(load_library().lexp_set_net(ctx.handle, net.handle if net is not None else None))
    ctx._net = net  # keep the network alive as long as the context uses it


def lexp_set_timing(ctx, enable):
    """enable: False/0 off; True/1 time every fused launch; N > 1 every N-th."""
    _check(load_library().lexp_set_timing(ctx.handle, int(enable)))


def lexp_get_stats(ctx) -> dict:
    s = lexp_stats()
    _check(load_library().lexp_get_stats(ctx.handle, C.byref(s)))
    return s.as_dict()


def lexp_reset_stats(ctx):
    _check(load_library().lexp_reset_stats(ctx.handle))


def lexp_debug_guide(ctx, stream=None):
    """Returns (left4 HxWx4, right4 HxWx4, guide 9xHxW, weights HxWx4 float64) device tensors."""
    torch = _torch()
    h, w = ctx.height, ctx.width
    dev = torch.device("cuda")
    l4 = torch.empty((h, w, 4), dtype=torch.float32, device=dev)
    r4 = torch.empty((h, w, 4), dtype=torch.float32, device=dev)
    g = torch.empty((9, h, w), dtype=torch.float32, device=dev)
    wt = torch.empty((h, w, 4), dtype=torch.float64, device=dev)
    _check(load_library().lexp_debug_guide(ctx.handle, C.c_void_p(l4.data_ptr()), C.c_void_p(r4.data_ptr()),
                                           C.c_void_p(g.data_ptr()), C.c_void_p(wt.data_ptr()),
                                           _stream_ptr(stream)))
    return l4, r4, g, wt


# ---- host-side pieces (no device needed) ----------------------------------------
def lexp_solve_binary(U, w4, neighbours=8):
    U = np.ascontiguousarray(np.asarray(U, dtype=np.int64))
    h, w = U.shape
    w4 = np.ascontiguousarray(np.asarray(w4, dtype=np.int64).reshape(h, w, 4))
    x = np.zeros((h, w), np.uint8)
    _check(load_library().lexp_solve_binary(w, h, int(neighbours), U.ctypes.data, w4.ctypes.data, x.ctypes.data))
    return x


def lexp_solve_binary_device(ctx, problems, stream=None):
    """problems: list of (U [h, w], w4 [h, w, 4]) integer arrays.  Returns
    (list of x [h, w] uint8, status int32 [n])."""
    n = len(problems)
    dims = np.zeros(2 * max(n, 1), np.int32)
    parts, sizes = [], []
    for i, (U, w4) in enumerate(problems):
        U = np.asarray(U, dtype=np.int64)
        h, w = U.shape
        dims[2 * i], dims[2 * i + 1] = w, h
        t = np.concatenate([U.reshape(h * w, 1), np.asarray(w4, dtype=np.int64).reshape(h * w, 4)], axis=1)
        parts.append(t.astype(np.int32).reshape(-1))
        sizes.append((h, w))
    terms = np.ascontiguousarray(np.concatenate(parts) if parts else np.zeros(5, np.int32))
    x = np.zeros(max(1, sum(h * w for h, w in sizes)), np.uint8)
    status = np.zeros(max(n, 1), np.int32)
    _check(load_library().lexp_solve_binary_device(ctx.handle, n, dims.ctypes.data, terms.ctypes.data, x.ctypes.data,
                                                   status.ctypes.data, _stream_ptr(stream)))
    out, o = [], 0
    for h, w in sizes:
        out.append(x[o:o + h * w].reshape(h, w).copy())
        o += h * w
    return out, status[:n]


def lexp_rng_key(seed, fields) -> int:
    f = np.ascontiguousarray(np.asarray(fields, dtype=np.uint64))
    return int(load_library().lexp_rng_key(C.c_uint64(seed), f.ctypes.data if f.size else None, int(f.size)))


def lexp_init_labels_host(width, height, disp_max, seed) -> np.ndarray:
    out = np.zeros((height, width, 3), np.float32)
    _check(load_library().lexp_init_labels_host(int(width), int(height), float(disp_max), C.c_uint64(seed),
                                                out.ctypes.data))
    return out


def lexp_propose(labels_hw3, seed, iteration, level, cell, ci, cj, step, k_prop, r_d, r_n,
                 k_rans=0) -> np.ndarray:
    lab = np.ascontiguousarray(np.asarray(labels_hw3, dtype=np.float32))
    h, w = lab.shape[:2]
    out = lexp_plane()
    _check(load_library().lexp_propose(w, h, lab.ctypes.data, C.c_uint64(seed), int(iteration), int(level),
                                       int(cell), int(ci), int(cj), int(step), int(k_prop), int(k_rans),
                                       float(r_d), float(r_n), C.byref(out)))
    return np.array([out.a, out.b, out.c], np.float32)
