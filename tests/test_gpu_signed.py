"""GPU parity of the signed distance and the geodesic symmetric filter through the
C ABI, against the oracle's compositions (FP32, bitwise expected, 1e-5 relative
bar).  Sizes span several tiles with ragged tails; edge cases: iterations = 0,
unit dimensions, zero thresholds, the hand-worked cases.  At the 256^3 size the
composition is checked by properties that hold at any size: antisymmetry for a
binary mask, and S = D(M) - D(1 - M) with the transform's own output (whose
bitwise parity at that size is pinned separately)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from gpu_util import DEV, assert_parity, to_dev, to_host
from paper_2208_00001_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "signed_gsf_hand.json")


def gpu_signed(c, mask=None):
    from paper_2208_00001_amd import binding as B
    m = c["mask"] if mask is None else mask
    out = B.ggdt_signed(to_dev(c["image"]), to_dev(m), c["spacing"], c["v"], c["lam"], c["iterations"])
    return to_host(out)


def gpu_gsf(c, theta_d, theta_e):
    from paper_2208_00001_amd import binding as B
    ws_n = int(B.load_library().ggdt_gsf_workspace_bytes(c["mask"].ndim, B._dims(c["mask"].shape),
                                                          c["image"].shape[0]))
    import torch
    ws = torch.empty(ws_n, dtype=torch.uint8, device=DEV)
    out = B.ggdt_gsf(to_dev(c["image"]), to_dev(c["mask"]), theta_d, theta_e, c["spacing"], c["v"], c["lam"],
                     c["iterations"], workspace=ws)
    assert B.workspace_status(ws) == 0, "watchdog fired"
    return to_host(out)


CASES = [
    ((37, 300), 1, 0.5, 2, True),
    ((130, 97), 3, 1.0, 2, False),
    ((70, 260), 1, 0.0, 1, False),
    ((19, 35, 41), 1, 1.0, 2, False),
    ((23, 18, 37), 1, 0.7, 2, True),
    ((17, 20, 21), 2, 0.4, 1, False),
    ((1, 33, 40), 1, 0.5, 2, True),
    ((12, 14), 1, 0.5, 0, True),
    ((40, 50), 4, 0.6, 2, False),  # four channels: the 2D tile kernel
]


@pytest.mark.parametrize("shape,C,lam,iters,soft", CASES)
def test_signed_parity(shape, C, lam, iters, soft):
    c = synth.small_case(shape, C=C, seed=101, lam=lam, iterations=iters, soft=soft, v=4.0 if soft else 1e10)
    print(f"signed {shape} C={C} lam={lam} it={iters}", flush=True)
    got = gpu_signed(c)
    ref = oracle.signed(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], iters)
    assert assert_parity(got, ref, what="signed"), "not bitwise"


@pytest.mark.parametrize("shape,C,lam,iters,soft", CASES)
@pytest.mark.parametrize("thetas", [(1.5, 0.5), (0.0, 0.0), (0.0, 2.0)])
def test_gsf_parity(shape, C, lam, iters, soft, thetas):
    c = synth.small_case(shape, C=C, seed=103, lam=lam, iterations=iters, soft=soft, v=4.0 if soft else 1e10)
    print(f"gsf {shape} C={C} lam={lam} it={iters} thetas={thetas}", flush=True)
    got = gpu_gsf(c, *thetas)
    ref = oracle.gsf(c["image"], c["mask"], thetas[0], thetas[1], c["spacing"], c["v"], c["lam"], iters)
    assert assert_parity(got, ref, what="gsf"), "not bitwise"


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def _eval(expr):
    return float(eval(expr, {"__builtins__": {}}, {"sqrt": math.sqrt}))


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_hand_worked_on_gpu(case):
    mask = np.array(case["mask"], dtype=np.float32)
    c = dict(image=np.zeros((1,) + mask.shape, np.float32), mask=mask, spacing=case["spacing"], v=case["v"],
             lam=float(case["lam"]), iterations=case["iterations"])
    s = gpu_signed(c)
    g = gpu_gsf(c, case["theta_d"], case["theta_e"])
    exp_s = np.vectorize(_eval)(np.array(case["signed"], dtype=object)).astype(np.float64)
    exp_g = np.vectorize(_eval)(np.array(case["gsf"], dtype=object)).astype(np.float64)
    np.testing.assert_allclose(s, exp_s, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(g, exp_g, rtol=1e-6, atol=1e-6)


def test_full_size_256_properties():
    """256^3, lambda 1, 4 iterations (the transform's benchmark volume): S equals
    the difference of the two transforms, and S(1 - M) = -S(M) for its binary mask."""
    from paper_2208_00001_amd import binding as B
    c = synth.config3()
    img, m = to_dev(c["image"]), to_dev(c["mask"])
    s = B.ggdt_signed(img, m, c["spacing"], c["v"], c["lam"], c["iterations"])
    d_obj = B.ggdt3d(img, m, c["spacing"], c["v"], c["lam"], c["iterations"])
    d_bg = B.ggdt3d(img, 1.0 - m, c["spacing"], c["v"], c["lam"], c["iterations"])
    assert bool((s == d_obj - d_bg).all())
    s_c = B.ggdt_signed(img, 1.0 - m, c["spacing"], c["v"], c["lam"], c["iterations"])
    assert bool((s_c == -s).all())
    assert bool((s[m == 0] <= 0).all()) and bool((s[m == 1] >= 0).all())
