"""The synthetic scene generator: determinism, ranges and consistency of its
ground truth with the rendered right view."""
import numpy as np

from synth import make_pair, make_workload_pair, WORKLOADS
from synth.workloads import many_pair_scenes


def test_deterministic_and_seed_dependent():
    a = make_workload_pair("tiny-64x48")
    b = make_workload_pair("tiny-64x48")
    assert np.array_equal(a.left, b.left) and np.array_equal(a.right, b.right)
    sc = dict(WORKLOADS["tiny-64x48"]["scene"], seed=99)
    c = make_pair(**sc)
    assert not np.array_equal(a.left, c.left)


def test_ranges_and_structure():
    p = make_workload_pair("lowres-450x375")
    assert p.left.shape == (375, 450, 3) and p.left.dtype == np.float32
    assert p.left.min() >= 0 and p.left.max() <= 255
    assert p.gt_disp.min() >= -1e-6 and p.gt_disp.max() <= 60 + 1e-6
    assert len(np.unique(p.owner)) == 14
    vv, uu = np.mgrid[0:375, 0:450]
    d = p.gt_labels[..., 0] * uu + p.gt_labels[..., 1] * vv + p.gt_labels[..., 2]
    assert np.allclose(d, p.gt_disp, atol=1e-3)


def test_ground_truth_explains_right_view():
    # Sampling the right view at u - d(u,v) reproduces the left view wherever
    # the pixel is visible and the sample falls near an integer column (away
    # from integers the two linear interpolations blur the noise texture);
    # a 3 px wrong disparity does not.
    p = make_workload_pair("lowres-450x375")
    h, w = p.gt_disp.shape
    vv, uu = np.mgrid[0:h, 0:w]

    def err_at(disp):
        x = uu - disp.astype(np.float64)
        ok = (x >= 0) & (x <= w - 1)
        i0 = np.clip(np.floor(x).astype(int), 0, w - 1)
        i1 = np.minimum(i0 + 1, w - 1)
        t = x - i0
        samp = (1 - t[..., None]) * p.right[vv, i0] + t[..., None] * p.right[vv, i1]
        return np.abs(samp - p.left).sum(-1), ok, np.minimum(t, 1 - t)

    err, ok, frac = err_at(p.gt_disp)
    near = ok & (frac < 0.02)
    assert near.sum() > 3000 and np.mean(err[near] < 3.0) > 0.7
    wrong, ok2, _ = err_at(p.gt_disp + 3.0)
    assert np.median(wrong[ok2]) > 3 * np.median(err[ok])


def test_many_pair_recipes():
    sc = many_pair_scenes(64)
    assert len(sc) == 64
    for s in sc:
        assert 320 <= s["width"] <= 1500 and s["height"] % 8 == 0
        assert s["disp_max"] == round(0.13 * s["width"])
