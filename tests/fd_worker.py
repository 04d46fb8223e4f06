"""Worker of the central-difference check on the 128^3 gradient workload: each
process rebuilds the case and the unperturbed FP64 records once, then evaluates
L = sum(W * D) in FP64 for single-voxel perturbations of M or I."""
import numpy as np

import oracle
from paper_2208_00001_amd import synth

_state = {}


def init(volume):
    c = synth.config5()[volume]
    img = c["image"].astype(np.float64)
    msk = c["mask"].astype(np.float64)
    _, rec0 = oracle.ggdt(img, msk, c["spacing"], c["v"], c["lam"], c["iterations"], "f64", records=True)
    _state.update(c=c, img=img, msk=msk, W=c["weight"].astype(np.float64), rec0=rec0)


def perturbed_loss(task):
    """task = (which, idx, sign, eps) -> (L, records unchanged)."""
    which, idx, sgn, eps = task
    c, img, msk = _state["c"], _state["img"], _state["msk"]
    if which == "M":
        m2 = msk.copy()
        m2[idx] += sgn * eps
        i2 = img
    else:
        i2 = img.copy()
        i2[(0,) + idx] += sgn * eps
        m2 = msk
    D, rec = oracle.ggdt(i2, m2, c["spacing"], c["v"], c["lam"], c["iterations"], "f64", records=True)
    return float(np.sum(_state["W"] * D)), bool(np.array_equal(rec, _state["rec0"]))
