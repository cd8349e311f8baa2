"""ctypes front end of the FP64 oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It loads ``liblexp_oracle.so`` (plain C, built by ``oracle/build.py``)
and shares nothing with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

_lib = None


class OraParams(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("disp_max", C.c_double),
                ("alpha", C.c_double), ("tau_col", C.c_double), ("tau_grad", C.c_double),
                ("gf_radius", C.c_int32), ("gf_eps", C.c_double),
                ("lam", C.c_double), ("tau_dis", C.c_double), ("w_floor", C.c_double),
                ("gamma", C.c_double), ("neighbours", C.c_int32)]


def _P(dt):
    return np.ctypeslib.ndpointer(dtype=dt, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    L = C.CDLL(LIB)
    vp = C.c_void_p
    f32, f64, i64, u8 = _P(np.float32), _P(np.float64), _P(np.int64), _P(np.uint8)
    L.ora_create.restype = vp
    L.ora_create.argtypes = [C.POINTER(OraParams), f32, f32]
    L.ora_destroy.argtypes = [vp]
    L.ora_gray_grad.argtypes = [vp, f64, f64]
    L.ora_guide.argtypes = [vp, f64, f64]
    L.ora_rho_max.restype = C.c_double
    L.ora_rho_max.argtypes = [vp]
    L.ora_raw_cost.restype = C.c_double
    L.ora_raw_cost.argtypes = [vp, C.c_int, C.c_int, f32]
    L.ora_rho_map.argtypes = [vp, f32, f64]
    L.ora_gf_weights.argtypes = [vp, C.c_int, C.c_int, f64]
    L.ora_unary_direct.restype = C.c_double
    L.ora_unary_direct.argtypes = [vp, C.c_int, C.c_int, f32]
    L.ora_unary_region.restype = C.c_int64
    L.ora_unary_region.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, f32, vp, vp]
    L.ora_filter_map.argtypes = [vp, f64, f64]
    L.ora_pixel_costs.argtypes = [vp, f32, vp, f64]
    L.ora_weight.restype = C.c_double
    L.ora_weight.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int]
    L.ora_pairwise.restype = C.c_double
    L.ora_pairwise.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, f32, f32]
    L.ora_energy.restype = C.c_double
    L.ora_energy.argtypes = [vp, f32, vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.ora_expand_problem.argtypes = [vp, f32, f64, f64, C.c_int, C.c_int, C.c_int, C.c_int, f32, i64, i64]
    L.ora_binary_energy.restype = C.c_int64
    L.ora_binary_energy.argtypes = [C.c_int, C.c_int, C.c_int, i64, i64, u8]
    L.ora_solve_maxflow.argtypes = [C.c_int, C.c_int, C.c_int, i64, i64, u8]
    L.ora_solve_bruteforce.restype = C.c_int64
    L.ora_solve_bruteforce.argtypes = [C.c_int, C.c_int, C.c_int, i64, i64, u8]
    L.ora_expand_step.restype = None
    L.ora_expand_step.argtypes = [vp, f32, f64, C.c_int, _P(np.int32), f32, vp, vp, vp]
    L.ora_expand.restype = C.c_int64
    L.ora_expand.argtypes = [vp, f32, f64, C.c_int, C.c_int, C.c_int, C.c_int, f32, C.c_int,
                             C.POINTER(C.c_int32)]
    L.ora_rng_key.restype = C.c_uint64
    L.ora_rng_key.argtypes = [C.c_uint64, _P(np.uint64), C.c_int]
    L.ora_init_labels.argtypes = [vp, C.c_uint64, f32]
    L.ora_propose.argtypes = [vp, f32, C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                              C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, f32]
    L.ora_propose_learned.argtypes = [vp, f32, vp, C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                      C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, f32]
    L.ora_run_group.restype = C.c_int64
    L.ora_run_group.argtypes = [vp, f32, f64, C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_int,
                                C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.POINTER(C.c_int64)]
    L.ora_optimize.restype = C.c_int64
    L.ora_optimize.argtypes = [vp, C.c_uint64, C.c_int, _P(np.int32), _P(np.int32), _P(np.int32),
                               _P(np.int32), C.c_int, f32, f64, vp]
    L.ora_run_group_ex.restype = C.c_int64
    L.ora_run_group_ex.argtypes = [vp, f32, f64, C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_int64)]
    L.ora_optimize_ex.restype = C.c_int64
    L.ora_optimize_ex.argtypes = [vp, C.c_uint64, C.c_int, _P(np.int32), _P(np.int32), _P(np.int32),
                                  _P(np.int32), C.c_int, C.c_int, f32, f64, vp]
    L.ora_postprocess.restype = None
    L.ora_postprocess.argtypes = [vp, f32, f32, f64, _P(np.uint8)]
    L.ora_num_threads.restype = C.c_int
    L.ora_set_threads.argtypes = [C.c_int]
    L.ora_set_threads.restype = None
    _lib = L
    return L


def _lab(f):
    return np.ascontiguousarray(np.asarray(f, dtype=np.float32).reshape(3))


class Oracle:
    """FP64 reference for one stereo pair.

    ``params`` is a dict with width, height, disp_max, alpha, tau_col,
    tau_grad, gf_radius, gf_eps, lam, tau_dis, w_floor, gamma, neighbours.
    """

    def __init__(self, params: dict, left: np.ndarray, right: np.ndarray):
        L = lib()
        self.p = dict(params)
        self.W = int(params["width"])
        self.H = int(params["height"])
        self.r = int(params["gf_radius"])
        P = OraParams(self.W, self.H, float(params["disp_max"]), float(params["alpha"]),
                      float(params["tau_col"]), float(params["tau_grad"]), self.r,
                      float(params["gf_eps"]), float(params["lam"]), float(params["tau_dis"]),
                      float(params["w_floor"]), float(params["gamma"]), int(params["neighbours"]))
        self._left = np.ascontiguousarray(left, dtype=np.float32)
        self._right = np.ascontiguousarray(right, dtype=np.float32)
        assert self._left.shape == (self.H, self.W, 3)
        self.ctx = L.ora_create(C.byref(P), self._left, self._right)
        if not self.ctx:
            raise ValueError("oracle: invalid parameters")
        self._L = L

    def close(self):
        if self.ctx:
            self._L.ora_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- inputs -----------------------------------------------------------
    def grads(self):
        gl = np.zeros((self.H, self.W))
        gr = np.zeros((self.H, self.W))
        self._L.ora_gray_grad(self.ctx, gl, gr)
        return gl, gr

    def guide(self):
        mu = np.zeros((self.H, self.W, 3))
        sg = np.zeros((self.H, self.W, 6))
        self._L.ora_guide(self.ctx, mu, sg)
        return mu, sg

    @property
    def rho_max(self) -> float:
        return self._L.ora_rho_max(self.ctx)

    # --- data term -----------------------------------------------------------
    def raw_cost(self, u, v, f) -> float:
        return self._L.ora_raw_cost(self.ctx, int(u), int(v), _lab(f))

    def rho_map(self, f) -> np.ndarray:
        out = np.zeros((self.H, self.W))
        self._L.ora_rho_map(self.ctx, _lab(f), out)
        return out

    def gf_weights(self, pu, pv) -> np.ndarray:
        side = 4 * self.r + 1
        out = np.zeros((side, side))
        self._L.ora_gf_weights(self.ctx, int(pu), int(pv), out)
        return out

    def unary_direct(self, pu, pv, f) -> float:
        return self._L.ora_unary_direct(self.ctx, int(pu), int(pv), _lab(f))

    @staticmethod
    def _clip(W, H, rect):
        u0, v0, u1, v1 = rect
        return max(u0, 0), max(v0, 0), min(u1, W), min(v1, H)

    def unary_region(self, rect, f) -> np.ndarray:
        u0, v0, u1, v1 = self._clip(self.W, self.H, rect)
        w, h = max(u1 - u0, 0), max(v1 - v0, 0)
        out = np.zeros((h, w))
        if w and h:
            self._L.ora_unary_region(self.ctx, *map(int, rect), _lab(f), out.ctypes.data, None)
        return out

    def coeffs_region(self, rect, f) -> np.ndarray:
        u0, v0, u1, v1 = self._clip(self.W, self.H, rect)
        if u1 <= u0 or v1 <= v0:
            return np.zeros((0, 0, 4))
        r = self.r
        pu0, pv0 = max(u0 - r, 0), max(v0 - r, 0)
        pu1, pv1 = min(u1 + r, self.W), min(v1 + r, self.H)
        out = np.zeros((pv1 - pv0, pu1 - pu0, 4))
        self._L.ora_unary_region(self.ctx, *map(int, rect), _lab(f), None, out.ctypes.data)
        return out

    def filter_map(self, rho: np.ndarray) -> np.ndarray:
        out = np.zeros((self.H, self.W))
        self._L.ora_filter_map(self.ctx, np.ascontiguousarray(rho, dtype=np.float64), out)
        return out

    def pixel_costs(self, labels, mask=None) -> np.ndarray:
        out = np.zeros((self.H, self.W))
        lab = np.ascontiguousarray(labels, dtype=np.float32)
        m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        self._L.ora_pixel_costs(self.ctx, lab, None if m is None else m.ctypes.data, out)
        return out

    # --- smoothness term / energy -----------------------------------------------
    def weight(self, p, q) -> float:
        return self._L.ora_weight(self.ctx, int(p[0]), int(p[1]), int(q[0]), int(q[1]))

    def pairwise(self, p, q, fp, fq) -> float:
        return self._L.ora_pairwise(self.ctx, int(p[0]), int(p[1]), int(q[0]), int(q[1]), _lab(fp), _lab(fq))

    def energy(self, labels, costs=None):
        lab = np.ascontiguousarray(labels, dtype=np.float32)
        eu, ep = C.c_double(), C.c_double()
        cc = None if costs is None else np.ascontiguousarray(costs, dtype=np.float64)
        e = self._L.ora_energy(self.ctx, lab, None if cc is None else cc.ctypes.data, C.byref(eu), C.byref(ep))
        return e, eu.value, ep.value

    # --- expansion ----------------------------------------------------------------
    def expand_problem(self, labels, costs, phi_alpha, rect, alpha):
        u0, v0, u1, v1 = self._clip(self.W, self.H, rect)
        w, h = u1 - u0, v1 - v0
        U = np.zeros(w * h, dtype=np.int64)
        w4 = np.zeros(w * h * 4, dtype=np.int64)
        self._L.ora_expand_problem(self.ctx, np.ascontiguousarray(labels, dtype=np.float32),
                                   np.ascontiguousarray(costs, dtype=np.float64),
                                   np.ascontiguousarray(phi_alpha, dtype=np.float64).reshape(-1),
                                   u0, v0, u1, v1, _lab(alpha), U, w4)
        return U.reshape(h, w), w4.reshape(h, w, 4)

    def solve_maxflow(self, U, w4):
        h, w = U.shape
        x = np.zeros(w * h, dtype=np.uint8)
        self._L.ora_solve_maxflow(w, h, int(self.p["neighbours"]), np.ascontiguousarray(U.reshape(-1), dtype=np.int64),
                                  np.ascontiguousarray(w4.reshape(-1), dtype=np.int64), x)
        return x.reshape(h, w)

    def solve_bruteforce(self, U, w4):
        h, w = U.shape
        x = np.zeros(w * h, dtype=np.uint8)
        e = self._L.ora_solve_bruteforce(w, h, int(self.p["neighbours"]),
                                         np.ascontiguousarray(U.reshape(-1), dtype=np.int64),
                                         np.ascontiguousarray(w4.reshape(-1), dtype=np.int64), x)
        return x.reshape(h, w), e

    def binary_energy(self, U, w4, x):
        h, w = U.shape
        nf = 2 if int(self.p["neighbours"]) == 4 else 4
        return self._L.ora_binary_energy(w, h, nf, np.ascontiguousarray(U.reshape(-1), dtype=np.int64),
                                         np.ascontiguousarray(w4.reshape(-1), dtype=np.int64),
                                         np.ascontiguousarray(x.reshape(-1), dtype=np.uint8))

    def expand(self, labels, costs, rect, alpha, bruteforce=False):
        """In place on labels (H,W,3 float32) and costs (H,W float64)."""
        assert labels.dtype == np.float32 and labels.flags.c_contiguous
        assert costs.dtype == np.float64 and costs.flags.c_contiguous
        nc = C.c_int32()
        de = self._L.ora_expand(self.ctx, labels, costs, *map(int, rect), _lab(alpha), int(bruteforce), C.byref(nc))
        return de, nc.value

    def expand_step(self, labels, costs, rects, alphas, want_phi=False):
        """One step of a group: ora_expand on every region (pairwise separated
        by a pixel, so independent by Lemma 3) in parallel, in place on labels
        and costs.  Returns (dEq [n], n_changed [n], phi) with phi the
        concatenated phi(alpha) of the clipped regions (row-major) or None."""
        assert labels.dtype == np.float32 and labels.flags.c_contiguous
        assert costs.dtype == np.float64 and costs.flags.c_contiguous
        rects = np.ascontiguousarray(np.asarray(rects, dtype=np.int32).reshape(-1, 4))
        alphas = np.ascontiguousarray(np.asarray(alphas, dtype=np.float32).reshape(-1, 3))
        n = len(rects)
        de = np.zeros(n, np.int64)
        nc = np.zeros(n, np.int32)
        phi = None
        if want_phi:
            tot = 0
            for u0, v0, u1, v1 in rects:
                a0, b0, a1, b1 = self._clip(self.W, self.H, (u0, v0, u1, v1))
                tot += max(a1 - a0, 0) * max(b1 - b0, 0)
            phi = np.zeros(max(tot, 1))
        self._L.ora_expand_step(self.ctx, labels, costs, n, rects, alphas,
                                None if phi is None else phi.ctypes.data, de.ctypes.data, nc.ctypes.data)
        return de, nc, phi

    # --- randomness, proposals, driver ----------------------------------------------
    def rng_key(self, seed, fields):
        f = np.ascontiguousarray(np.asarray(fields, dtype=np.uint64))
        return self._L.ora_rng_key(C.c_uint64(seed), f, len(f))

    def init_labels(self, seed) -> np.ndarray:
        out = np.zeros((self.H, self.W, 3), dtype=np.float32)
        self._L.ora_init_labels(self.ctx, C.c_uint64(seed), out)
        return out

    def propose(self, labels, seed, iteration, level, cell, ci, cj, step, k_prop, r_d, r_n, k_rans=0):
        """Candidate of step `step` of Alg. 1: propagation for step < k_prop,
        RANSAC for the next k_rans steps, refinement after."""
        out = np.zeros(3, dtype=np.float32)
        self._L.ora_propose(self.ctx, np.ascontiguousarray(labels, dtype=np.float32), C.c_uint64(seed),
                            iteration, level, cell, ci, cj, step, k_prop, k_rans, float(r_d), float(r_n), out)
        return out

    def propose_learned(self, labels, planes, seed, iteration, level, cell, ci, cj, step, k_prop, r_d, r_n,
                        k_rans=0):
        """Candidate with learned proposals: refinement steps with an odd
        refinement index take planes[r] (planes: HxWx3 float32, the plane a
        network proposes at each pixel; None: no learned step)."""
        out = np.zeros(3, dtype=np.float32)
        pl = None if planes is None else np.ascontiguousarray(planes, dtype=np.float32)
        assert pl is None or pl.shape == (self.H, self.W, 3)
        self._L.ora_propose_learned(self.ctx, np.ascontiguousarray(labels, dtype=np.float32),
                                    None if pl is None else pl.ctypes.data, C.c_uint64(seed), iteration, level,
                                    cell, ci, cj, step, k_prop, k_rans, float(r_d), float(r_n), out)
        return out

    def planes_from_net_output(self, y):
        """Planes of the proposal network's output (HxWx16; channels 0-2 are
        a, b and d / disp_max at the pixel): the plane with slopes (a, b)
        through disparity d at (u, v), c = d - a u - b v, in FP64 from the FP32
        outputs, rounded once to FP32."""
        y = np.asarray(y, dtype=np.float32)
        v, u = np.mgrid[0:self.H, 0:self.W].astype(np.float64)
        a = y[..., 0].astype(np.float64)
        b = y[..., 1].astype(np.float64)
        c = (y[..., 2].astype(np.float64) * float(self.p["disp_max"]) - a * u) - b * v
        return np.stack([a, b, c], axis=-1).astype(np.float32)

    def run_group(self, labels, costs, seed, iteration, level, cell, k_prop, k_rand, r_d, r_n, group, k_rans=0,
                  batch_cycle=False):
        de = C.c_int64(0)
        ev = self._L.ora_run_group_ex(self.ctx, labels, costs, C.c_uint64(seed), iteration, level, cell,
                                      k_prop, k_rans, k_rand, float(r_d), float(r_n), group,
                                      1 if batch_cycle else 0, C.byref(de))
        return ev, de.value

    def optimize(self, seed, grids, iterations, batch_cycle=False):
        """grids: (cell, K_prop, K_rand) or (cell, K_prop, K_rand, K_RANS) per level.
        batch_cycle: every candidate of a cell's Alg. 1 from the labels before
        the cell's first move (Sec. 3.4's batch cycle)."""
        n = len(grids)
        cells = np.array([g[0] for g in grids], dtype=np.int32)
        kp = np.array([g[1] for g in grids], dtype=np.int32)
        kr = np.array([g[2] for g in grids], dtype=np.int32)
        ks = np.array([g[3] if len(g) > 3 else 0 for g in grids], dtype=np.int32)
        labels = np.zeros((self.H, self.W, 3), dtype=np.float32)
        costs = np.zeros((self.H, self.W))
        energy = np.zeros(iterations + 1)
        ev = self._L.ora_optimize_ex(self.ctx, C.c_uint64(seed), n, cells, kp, ks, kr, iterations,
                                     1 if batch_cycle else 0, labels, costs, energy.ctypes.data)
        return labels, costs, energy, ev

    @classmethod
    def right_view(cls, params: dict, left: np.ndarray, right: np.ndarray) -> "Oracle":
        """The right image's data term: I_L and I_R swapped in Eqs. (7) and (9)
        with the disparity added in the warp (Eq. (8)), computed as the
        left-view term of the horizontally mirrored pair.  Its pixels, label
        fields and rects are in the mirrored frame of the right image: pixel
        (u, v) is right pixel (W-1-u, v), and label (a, b, c) there is the plane
        (-a, b, c + a (W-1)) of the right image."""
        return cls(params, np.ascontiguousarray(right[:, ::-1]), np.ascontiguousarray(left[:, ::-1]))

    def postprocess(self, labels_left, labels_right_mirrored):
        """Left-right check, row filling and weighted median of the left view
        (this oracle must be the left view's).  Returns (disparity FP64 HxW,
        inconsistent-pixel mask HxW uint8)."""
        out = np.zeros((self.H, self.W))
        inv = np.zeros((self.H, self.W), np.uint8)
        self._L.ora_postprocess(self.ctx, np.ascontiguousarray(labels_left, dtype=np.float32),
                                np.ascontiguousarray(labels_right_mirrored, dtype=np.float32), out, inv)
        return out, inv

    @staticmethod
    def num_threads() -> int:
        return lib().ora_num_threads()

    @staticmethod
    def set_threads(n: int) -> None:
        """Threads of the oracle's parallel loops (0: the default)."""
        lib().ora_set_threads(int(n))
