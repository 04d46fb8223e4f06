"""Toivanen's raster scan on the GPU (hyperplane sweeps) against the oracle's
sequential FP32 sweeps, bit for bit: 2D and 3D, 1-3 channels, lambda 0, general
and 1, soft and hard seeds, unit dimensions, iterations 0-3, one row block and
pipelines of several (ragged) row blocks (bands of 1024 image rows, slabs of
1024 / H volume planes), the LDS-ring form and the general one (more than 3
channels, or a block's rings beyond the LDS), the edge cost's fast forms and
their fallbacks on extreme image values, up to the 256^3 benchmark volume (one iteration)."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_parity, to_dev, to_host
from paper_2208_00001_amd import synth

pytestmark = pytest.mark.gpu

CASES = [
    ((37, 53), 1, 1.0, 2, False), ((64, 65), 3, 0.5, 1, True), ((1, 300), 1, 0.0, 2, False), ((300, 1), 2, 0.8, 1, True),
    ((5, 6, 7), 1, 1.0, 2, False), ((1, 1, 1), 1, 0.5, 1, False), ((9, 1, 30), 1, 0.0, 3, True),
    ((20, 33, 18), 2, 0.4, 2, True), ((80, 81, 20), 1, 1.0, 2, False),  # 7 slabs of 12 planes
    ((70, 75, 9), 3, 0.7, 1, True), ((33, 40, 12), 1, 0.3, 0, True),
    ((2100, 37), 2, 0.6, 2, True), ((1030, 5), 1, 1.0, 1, False),  # 3 and 2 bands of image rows
    ((3, 1500, 4), 1, 0.9, 2, False), ((300, 16, 3), 1, 0.5, 2, True),  # slabs of 1 plane; 5 ragged slabs
    # the general form: 4 channels; rows of a volume beyond the LDS rings (1500 > 1024 rows above, and
    # 2 channels of 700 rows)
    ((70, 41), 4, 0.7, 2, True), ((5, 700, 3), 2, 0.6, 1, True),
    ((4, 600, 3), 1, 0.8, 2, False), ((6, 300, 5), 3, 0.5, 1, True),  # slabs of one plane: 1024 and 512 threads
]


@pytest.mark.parametrize("shape,C,lam,it,soft", CASES, ids=lambda v: str(v))
def test_toivanen_matches_oracle(shape, C, lam, it, soft):
    from paper_2208_00001_amd import binding as B
    c = synth.small_case(shape, C=C, seed=600 + sum(shape), lam=lam, iterations=it, soft=soft,
                         v=8.0 if soft else 1e10)
    print(f"toivanen {shape} C={C} lam={lam} it={it} soft={soft}", flush=True)
    ref = oracle.toivanen(c["image"], c["mask"], c["spacing"], c["v"], lam, it, "f32")
    got = to_host(B.ggdt_toivanen(to_dev(c["image"]), to_dev(c["mask"]), c["spacing"], c["v"], lam, it, check=True))
    assert assert_parity(got, ref, what=str(shape)), "not bitwise"


def test_toivanen_128_both_lambdas_to_fixed_point():
    """The 128^2 image at lambda 0 and 1: after as many iterations as the
    oracle's Toivanen needs to reach its fixed point, the GPU result equals it."""
    from paper_2208_00001_amd import binding as B
    for lam in (0.0, 1.0):
        c = synth.config1(lam)
        ref, n = oracle.toivanen(c["image"], c["mask"], c["spacing"], c["v"], lam, 100, "f32", converge=True)
        print(f"config1 lam={lam}: {n} iterations", flush=True)
        got = to_host(B.ggdt_toivanen(to_dev(c["image"]), to_dev(c["mask"]), c["spacing"], c["v"], lam, n + 1,
                                      check=True))
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_toivanen_256_volume_one_iteration():
    from paper_2208_00001_amd import binding as B
    c = synth.config3()
    print("config3 toivanen, 1 iteration", flush=True)
    ref = oracle.toivanen(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], 1, "f32")
    got = to_host(B.ggdt_toivanen(to_dev(c["image"]), to_dev(c["mask"]), c["spacing"], c["v"], c["lam"], 1,
                                  check=True))
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("shape,scale,lam", [((23, 31, 19), 1e-30, 1.0), ((23, 31, 19), 1e25, 1.0),
                                             ((23, 31, 19), 1e25, 0.0), ((140, 90), 1e-30, 1.0),
                                             ((140, 90), 1e25, 1.0)])
def test_toivanen_fast_form_fallback_on_extreme_values(shape, scale, lam):
    """lambda 1 with |I| < 2^-40, or |I| > 2^60, must take the root (the image
    classification rules out w = |I(x) - I(y)|), as for the passes."""
    from paper_2208_00001_amd import binding as B
    c = synth.small_case(shape, C=1, seed=7, lam=lam, iterations=2)
    c["image"] = (c["image"] * np.float32(scale)).astype(np.float32)
    print(f"toivanen extreme {shape} scale={scale} lam={lam}", flush=True)
    ref = oracle.toivanen(c["image"], c["mask"], c["spacing"], c["v"], lam, 2, "f32")
    got = to_host(B.ggdt_toivanen(to_dev(c["image"]), to_dev(c["mask"]), c["spacing"], c["v"], lam, 2, check=True))
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("shape,C,lam,spacing", [((29, 35, 26), 1, 0.3, (1.0, 0.5, 2.0)),
                                                  ((21, 30, 17), 2, 0.9, (0.25, 1.0, 1.0)),
                                                  ((260, 190), 1, 0.6, (3.0, 0.5))])
def test_toivanen_general_root_over_wide_magnitudes(shape, C, lam, spacing):
    """The general edge cost with image magnitudes log-uniform over [2^-40, 2^59]
    (random signs), where a shortened correctly rounded root would go wrong."""
    from paper_2208_00001_amd import binding as B
    c = synth.small_case(shape, C=C, seed=11, lam=lam, iterations=2, spacing=spacing)
    rng = np.random.default_rng(11)
    e = rng.uniform(-40.0, 59.0, size=c["image"].shape)
    c["image"] = (np.sign(rng.uniform(-1, 1, size=e.shape)) * np.exp2(e)).astype(np.float32)
    print(f"toivanen wide {shape} C={C} lam={lam}", flush=True)
    ref = oracle.toivanen(c["image"], c["mask"], c["spacing"], 1e30, lam, 2, "f32")
    got = to_host(B.ggdt_toivanen(to_dev(c["image"]), to_dev(c["mask"]), c["spacing"], 1e30, lam, 2, check=True))
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("shape,C,scale", [((60, 70), 3, 1.0), ((14, 18, 16), 2, 1.0), ((14, 18, 16), 2, 2.0 ** -30)])
def test_toivanen_lam1_multichannel_root_forms(shape, C, scale):
    """lambda 1, several channels, a quantised image (zero root arguments): the
    normal-range root, and the full root for values near 2^-30."""
    from paper_2208_00001_amd import binding as B
    c = synth.small_case(shape, C=C, seed=23, lam=1.0, iterations=2)
    c["image"] = (np.round(c["image"] * 2.0) * np.float32(scale)).astype(np.float32)
    print(f"toivanen lam1 {shape} C={C} scale={scale}", flush=True)
    ref = oracle.toivanen(c["image"], c["mask"], c["spacing"], c["v"], 1.0, 2, "f32")
    got = to_host(B.ggdt_toivanen(to_dev(c["image"]), to_dev(c["mask"]), c["spacing"], c["v"], 1.0, 2, check=True))
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
