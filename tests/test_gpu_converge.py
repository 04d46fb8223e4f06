"""Convergence mode through the C ABI vs the oracle's run-to-fixed-point (FP32):
the same distances bit for bit and the same iteration count; a run stopped by
max_iterations equals the plain transform with that many iterations."""
import numpy as np
import pytest

import oracle
from gpu_util import DEV, assert_parity, to_dev, to_host
from paper_2208_00001_amd import synth

pytestmark = pytest.mark.gpu

CASES = [
    ((64, 70), 1, 1.0, False),
    ((300, 257), 3, 0.5, False),
    ((90, 41), 1, 0.0, False),
    ((33, 40, 29), 1, 1.0, False),
    ((27, 31, 44), 1, 0.7, True),
    ((20, 26, 18), 2, 0.4, False),
    ((48, 40, 36), 1, 0.0, True),
]


@pytest.mark.parametrize("shape,C,lam,soft", CASES, ids=lambda v: str(v))
def test_converge_matches_oracle(shape, C, lam, soft):
    from paper_2208_00001_amd import binding as B
    c = synth.small_case(shape, C=C, seed=31, lam=lam, iterations=1, soft=soft, v=10.0 if soft else 1e10)
    print(f"case {c['name']} lam={lam} soft={soft}", flush=True)
    ref, n_ref = oracle.until_converged(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], 100, "f32")
    out, n = B.ggdt_converge(to_dev(c["image"]), to_dev(c["mask"]), c["spacing"], c["v"], c["lam"], 100)
    assert n == n_ref, (n, n_ref)
    assert assert_parity(to_host(out), ref, what=c["name"]), "not bitwise"


def test_converge_stopped_by_max_iterations():
    from paper_2208_00001_amd import binding as B
    c = synth.small_case((61, 47, 38), C=1, seed=32, lam=1.0, iterations=1)
    _, n_ref = oracle.until_converged(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], 100, "f32")
    assert n_ref >= 2
    img, m = to_dev(c["image"]), to_dev(c["mask"])
    out, n = B.ggdt_converge(img, m, c["spacing"], c["v"], c["lam"], n_ref - 1)
    assert n == -1
    plain = B.ggdt3d(img, m, c["spacing"], c["v"], c["lam"], n_ref - 1)
    assert np.array_equal(to_host(out), to_host(plain))
    out0, n0 = B.ggdt_converge(img, m, c["spacing"], c["v"], c["lam"], 0)
    assert n0 == -1 and np.array_equal(to_host(out0), c["v"] * c["mask"])
