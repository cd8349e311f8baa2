"""lexp_energy_noalloc, the entry point for callers that cannot allocate,
against lexp_energy through the C ABI: the same partial sums added in the same
order, so the same values bit for bit; two calls in a row, the second on a
smaller image; a call after that on the larger image again (the array keeps
the last call's contents, and nothing in it needs clearing); images beyond the
array's size are refused before any work."""
import numpy as np
import pytest

from synth import make_workload_pair, params_for

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_1603_08328_amd.lexp")


def _state(name, seed):
    pair = make_workload_pair(name)
    prm = params_for(name)
    ctx = L.lexp_create(prm, torch.from_numpy(pair.left).cuda(), torch.from_numpy(pair.right).cuda())
    lab = torch.zeros((prm["height"], prm["width"], 4), device="cuda")
    cost = torch.zeros((prm["height"], prm["width"]), device="cuda")
    L.lexp_init_labels(ctx, seed, lab)
    L.lexp_pixel_costs(ctx, lab, cost)
    return ctx, lab, cost


def test_energy_noalloc_equals_energy_on_successive_calls():
    big = _state("lowres-450x375", 3)
    small = _state("tiny-64x48", 4)
    for ctx, lab, cost in (big, small, big):
        ref = L.lexp_energy(ctx, lab, cost)
        got = L.lexp_energy_noalloc(ctx, lab, cost)
        assert got == ref, (got, ref)
        assert got[0] == got[1] + got[2] and got[1] > 0 and got[2] > 0
    # on another stream too
    ctx, lab, cost = small
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        got = L.lexp_energy_noalloc(ctx, lab, cost, stream=st)
    assert got == L.lexp_energy(ctx, lab, cost)
    for ctx, _, _ in (big, small):
        ctx.close()


def test_energy_noalloc_refuses_images_beyond_its_array():
    from synth import PAPER_PARAMS
    w, h = 1450, 1450  # 2,102,500 pixels > LEXP_NOALLOC_MAX_PIXELS = 2,097,152
    rng = np.random.default_rng(0)
    img = torch.from_numpy(rng.uniform(0, 255, (h, w, 3)).astype(np.float32)).cuda()
    prm = dict(PAPER_PARAMS, width=w, height=h, disp_max=60.0, gf_radius=5)
    ctx = L.lexp_create(prm, img, img)
    lab = torch.zeros((h, w, 4), device="cuda")
    cost = torch.zeros((h, w), device="cuda")
    with pytest.raises(L.LexpError) as ei:
        L.lexp_energy_noalloc(ctx, lab, cost)
    assert ei.value.status == -1 and "2097152" in str(ei.value)
    assert L.lexp_energy(ctx, lab, cost)[0] == 0.0
    ctx.close()
