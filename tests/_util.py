"""Small helpers shared by the tests (no method arithmetic)."""
import numpy as np


def base_params(w, h, r=2, **kw):
    from synth import PAPER_PARAMS
    p = dict(PAPER_PARAMS)
    p.update(width=w, height=h, disp_max=16.0, gf_radius=r)
    p.update(kw)
    return p


def texture(rng, h, w):
    """Box-smoothed uniform noise in [0,255] (float32, HxWx3)."""
    from synth.scenes import _texture
    return _texture(rng, h, w).astype(np.float32)
