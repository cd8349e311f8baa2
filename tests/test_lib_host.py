"""Host-side parts of liblexp.so, checked against the oracle on the CPU (no
device calls): exported symbols, the Boykov-Kolmogorov max-flow, the
counter-based random numbers, random initialisation and proposals."""
import os
import re

import numpy as np
import pytest

from oracle import Oracle
import paper_1603_08328_amd.lexp as L
from _util import base_params, texture

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "lexp.h")).read()
    return sorted(set(re.findall(r"^(?:lexp_status|const char\*|uint64_t)\s+(lexp_\w+)\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = L.load_library()
    syms = _header_symbols()
    assert len(syms) >= 19
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(L._SIGS), set(syms) ^ set(L._SIGS)


def _oracle(rng, w=12, h=10, **kw):
    return Oracle(base_params(w, h, **kw), texture(rng, h, w), texture(rng, h, w))


@pytest.mark.parametrize("shape", [(4, 4), (3, 5), (1, 1), (1, 9), (6, 2), (5, 5)])
@pytest.mark.parametrize("kind", ["generic", "ties", "sparse"])
@pytest.mark.parametrize("nb", [8, 4])
def test_bk_equals_exhaustive_minimal_set(rng, shape, kind, nb):
    o = _oracle(rng, neighbours=nb)
    h, w = shape
    for _ in range(30):
        if kind == "generic":
            U = rng.integers(-60, 61, (h, w))
            w4 = rng.integers(0, 41, (h, w, 4))
        elif kind == "ties":
            U = rng.integers(-2, 3, (h, w))
            w4 = rng.integers(0, 3, (h, w, 4))
        else:
            U = rng.integers(-5, 6, (h, w)) * (rng.random((h, w)) < 0.3)
            w4 = rng.integers(0, 9, (h, w, 4)) * (rng.random((h, w, 4)) < 0.5)
        U = U.astype(np.int64)
        w4 = w4.astype(np.int64)
        if h * w <= 20:
            xb, _ = o.solve_bruteforce(U, w4)
        else:
            xb = o.solve_maxflow(U, w4)
        xk = L.lexp_solve_binary(U, w4, nb)
        assert np.array_equal(xb, xk)


@pytest.mark.parametrize("shape", [(15, 15), (45, 45), (20, 75)])
def test_bk_equals_dinic_on_region_sized_grids(rng, shape):
    o = _oracle(rng)
    h, w = shape
    for scale in (1, 1000, 2 ** 20):
        U = (rng.normal(0, 1, (h, w)) * scale).astype(np.int64)
        w4 = (np.abs(rng.normal(0, 0.7, (h, w, 4))) * scale).astype(np.int64)
        w4[rng.random((h, w, 4)) < 0.2] = 0
        xd = o.solve_maxflow(U, w4)
        xk = L.lexp_solve_binary(U, w4)
        assert np.array_equal(xd, xk)
        assert o.binary_energy(U, w4, xk) == o.binary_energy(U, w4, xd)


def test_bk_rejects_negative_weights():
    U = np.zeros((2, 2), np.int64)
    w4 = np.zeros((2, 2, 4), np.int64)
    w4[0, 0, 0] = -1
    with pytest.raises(L.LexpError):
        L.lexp_solve_binary(U, w4)


def test_rng_key_chain_matches_oracle(tiny_oracle, rng):
    for _ in range(200):
        seed = int(rng.integers(0, 2 ** 63))
        fields = [int(x) for x in rng.integers(0, 2 ** 31, int(rng.integers(0, 8)))]
        assert L.lexp_rng_key(seed, fields) == tiny_oracle.rng_key(seed, fields)


@pytest.mark.parametrize("seed", [0, 1, 12345, 2 ** 61 + 7])
def test_init_labels_bitwise_equal_to_oracle(tiny_oracle, seed):
    a = L.lexp_init_labels_host(64, 48, 16.0, seed)
    b = tiny_oracle.init_labels(seed)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_proposals_bitwise_equal_to_oracle(tiny_oracle):
    o = tiny_oracle
    rng = np.random.default_rng(5)
    lab = o.init_labels(3)
    n = 0
    for it in range(3):
        for level, cell in enumerate((5, 15, 25)):
            nci, ncj = -(-64 // cell), -(-48 // cell)
            for _ in range(20):
                ci, cj = int(rng.integers(0, nci)), int(rng.integers(0, ncj))
                for step in range(8):
                    kp = 1 if level == 0 else 2
                    args = (lab, 77, it, level, cell, ci, cj, step, kp, 8.0 / 2 ** it, 1.0 / 2 ** it)
                    a = L.lexp_propose(*args)
                    b = o.propose(*args)
                    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (args[2:], a, b)
                    n += 1
    assert n == 3 * 3 * 20 * 8


@pytest.mark.parametrize("CH", [4, 16])
def test_fused_kernel_row_pipeline_fits_its_rings(CH):
    """Replays the fused cost kernel's row pipeline on the CPU for many tile
    shapes: per step, stage A produces up to kChunk rows, C emits window rows
    from rows produced in earlier steps, E moves the previous step's rows into
    the second ring and G outputs from rows E wrote in earlier steps.  Checks
    that neither ring ever holds more than 2r+1+2*kChunk live rows and that
    the loop ends.  The kernel moves 16 rows per step."""
    for H in (1, 2, 7, 48, 120, 300):
        for r in (1, 2, 5, 20, 32):
            ring = 2 * r + 1 + 2 * CH
            for tv0 in range(0, H, max(1, H // 7)):
                for th in (1, 3, 16, 128):
                    tv1 = min(tv0 + th, H)
                    yp0, yp1 = max(tv0 - r, 0), min(tv1 + r, H)
                    ym0, ym1 = max(tv0 - 2 * r, 0), min(tv1 + 2 * r, H)
                    produced, kv, lo_c = ym0, yp0, ym0
                    e_first, e_rows, kv_e = yp0, 0, yp0
                    pv, lo2_c = tv0, yp0
                    steps = 0
                    while pv < tv1:
                        steps += 1
                        assert steps < 4 * (ym1 - ym0) + 20
                        avail1, avail3 = produced, kv_e
                        nA = min(CH, ym1 - produced)
                        assert produced + nA - lo_c <= ring          # ring1: C's rows + A's new rows
                        nC = 0
                        while nC < CH and kv + nC < yp1 and min(kv + nC + r, H - 1) < avail1:
                            nC += 1
                        first = kv
                        if nC:
                            lo_c = max(kv + nC - 1 - r, 0)
                            kv += nC
                        assert kv_e + e_rows - lo2_c <= ring         # ring3: G's rows + E's new rows
                        nG = 0
                        while pv + nG < tv1 and min(pv + nG + r, H - 1) < avail3:
                            nG += 1
                        if nG:
                            lo2_c = max(pv + nG - 1 - r, 0)
                            pv += nG
                        kv_e = e_first + e_rows
                        e_first, e_rows = first, nC
                        produced += nA


@pytest.mark.parametrize("w,h", [(64, 48), (61, 41)])
def test_ransac_proposals_bitwise_equal_to_oracle(tiny_pair, w, h):
    """The library's RANSAC proposer and the oracle's, written apart, agree
    bit for bit: on a ground-truth plane field with 30% of its labels
    replaced by random ones, on purely random labels and on the clipped
    edge cells of a ragged grid (degenerate one-pixel-wide cells included);
    the refinement steps after the RANSAC steps keep their perturbation
    schedule."""
    rng = np.random.default_rng(w + h)
    pair, _ = tiny_pair
    o = Oracle(base_params(w, h), texture(rng, h, w), texture(rng, h, w))
    rand = o.init_labels(3)
    gt = np.zeros((h, w, 3), np.float32)
    gh, gw = min(h, 48), min(w, 64)
    gt[:gh, :gw] = pair.gt_labels[:gh, :gw]
    gt[gh:, :] = gt[gh - 1:gh, :]
    gt[:, gw:] = gt[:, gw - 1:gw]
    mixed = np.where(rng.random((h, w, 1)) < 0.3, rand, gt).astype(np.float32)
    n = 0
    for lab in (mixed, rand):
        for it in range(2):
            for level, cell in enumerate((5, 15, 25)):
                nci, ncj = -(-w // cell), -(-h // cell)
                cells = [(ci, cj) for cj in range(ncj) for ci in range(nci)]
                if len(cells) > 40:
                    cells = [cells[k] for k in rng.choice(len(cells), 40, replace=False)] + [(nci - 1, ncj - 1)]
                for ci, cj in cells:
                    for step in range(1, 5):  # k_prop = 1, k_rans = 2: steps 1-2 RANSAC, 3-4 refinement
                        args = (lab, 11, it, level, cell, ci, cj, step, 1, 6.0, 0.5)
                        a = L.lexp_propose(*args, k_rans=2)
                        b = o.propose(*args, k_rans=2)
                        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (args[2:], a, b)
                        n += 1
    assert n > 500


def test_tile_plan_table_lookup():
    """The committed tile plans: one entry per (image size, radius, cell,
    mode) the tuner measured, each the default rule unless a plan beat it by
    the tuner's margin; levels the table does not hold take the default."""
    from paper_1603_08328_amd import autotune as A
    t = A.load_table()
    assert "gfx950" in t and len(t["gfx950"]) >= 12
    for k, e in t["gfx950"].items():
        default = e["default_kernel_ms_per_group_step"]
        chosen = e["tried"][f"{e['cols']},{e['fill']}"]
        assert (e["cols"], e["fill"]) == (0, 256) or chosen < (1 - A.MARGIN) * default, k
        assert min(e["tried"].values()) == e["tried"][e["fastest"]]
    grids = [(5, 1, 7), (15, 1, 7), (25, 1, 7)]
    got = A.plans_for(450, 375, 20, grids, table=t)
    assert got == [(t["gfx950"][f"450x375/r20/c{c}/plain"]["cols"], t["gfx950"][f"450x375/r20/c{c}/plain"]["fill"])
                   for c, _, _ in grids]
    assert A.plans_for(451, 375, 20, grids, table=t) == [(0, 0)] * 3
    assert A.plans_for(450, 375, 20, [(7, 1, 7)], table=t) == [(0, 0)]
