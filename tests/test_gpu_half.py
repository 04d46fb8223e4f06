"""16-bit image storage (bf16, fp16) on the GPU: the kernels widen each image
value to fp32 exactly and run the FP32 schedule unchanged, so the result must
equal the oracle's FP32 schedule on the widened image bit for bit (within the
1e-5 bar, expected bitwise): 2D images with 1-3 channels (row kernel) and
single-channel volumes (both layouts of the cell kernel, scan-contiguous and
not), every lambda regime, and the full-size 2D 2048^2 x 3 and 3D 256^3
workloads against the oracle's plane-parallel FP32 schedule (equal to the
serial one bit for bit, pinned in test_oracle.py)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_parity, to_dev, to_host
from paper_2208_00001_amd import synth

pytestmark = pytest.mark.gpu

DTYPES = {"bf16": torch.bfloat16, "f16": torch.float16}
GGDT_ERR_UNSUPPORTED = -8


def rounded(image, dtype):
    """The image rounded to the 16-bit format (host, round to nearest even) and
    its exact fp32 widening."""
    t = torch.from_numpy(np.ascontiguousarray(image)).to(dtype)
    return t, t.float().numpy()


CASES = [((70, 90), 1, 0.0, 2), ((70, 90), 1, 1.0, 2), ((131, 77), 2, 0.5, 2), ((64, 200), 3, 0.7, 1),
         ((33, 47, 29), 1, 1.0, 2), ((33, 47, 29), 1, 0.0, 1), ((40, 36, 44), 1, 0.6, 2), ((1, 20, 33), 1, 0.8, 2),
         ((17, 1, 64), 1, 1.0, 3)]


@pytest.mark.parametrize("fmt", list(DTYPES))
@pytest.mark.parametrize("shape,C,lam,it", CASES, ids=lambda v: str(v))
def test_half_image_matches_oracle_on_widened_image(fmt, shape, C, lam, it):
    from paper_2208_00001_amd import binding as B
    c = synth.small_case(shape, C=C, seed=960 + len(shape) + C, lam=lam, iterations=it)
    print(f"case {c['name']} {fmt} lam={lam} it={it}", flush=True)
    img16, widened = rounded(c["image"], DTYPES[fmt])
    got = to_host(B.ggdt_half(img16.to("cuda"), to_dev(c["mask"]), c["spacing"], c["v"], lam, it, check=True))
    ref = oracle.ggdt(widened, c["mask"], c["spacing"], c["v"], lam, it, "f32")
    assert assert_parity(got, ref, what=f"{fmt} {c['name']}"), "not bitwise"
    # the fp32 entry on the widened image gives the same bits
    f32 = to_host(B.ggdt2d(to_dev(widened), to_dev(c["mask"]), c["spacing"], c["v"], lam, it) if len(shape) == 2
                  else B.ggdt3d(to_dev(widened), to_dev(c["mask"]), c["spacing"], c["v"], lam, it))
    assert np.array_equal(got, f32)


@pytest.mark.parametrize("fmt", list(DTYPES))
def test_half_full_size_workloads(fmt):
    from paper_2208_00001_amd import binding as B
    for c in (synth.config3(), synth.config2(0.5)):
        print(f"workload {c['name']} {fmt}", flush=True)
        img16, widened = rounded(c["image"], DTYPES[fmt])
        got = to_host(B.ggdt_half(img16.to("cuda"), to_dev(c["mask"]), c["spacing"], c["v"], c["lam"],
                                  c["iterations"], check=True))
        ref, _ = oracle.ggdt_omp(widened, c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"])
        assert np.array_equal(got, ref), f"{c['name']} {fmt}: differs from the oracle on the widened image"


def test_half_unsupported_geometries_are_rejected():
    from paper_2208_00001_amd import binding as B
    img = torch.zeros((2, 8, 9, 10), dtype=torch.bfloat16, device="cuda")
    m = torch.ones((8, 9, 10), device="cuda")
    with pytest.raises(B.GGDTError) as e:
        B.ggdt_half(img, m, (1.0, 1.0, 1.0), 1e10, 1.0, 1)
    assert e.value.code == GGDT_ERR_UNSUPPORTED


@pytest.mark.parametrize("fmt", list(DTYPES))
@pytest.mark.parametrize("shape,lam,it", [((24, 16, 64), 1.0, 2), ((20, 18, 50), 0.6, 2), ((13, 11, 37), 0.0, 2),
                                          ((9, 40, 72), 0.8, 1)], ids=lambda v: str(v))
def test_half_volume_last_axis_in_place(fmt, shape, lam, it):
    """Single-channel volumes with the minimal workspace: the passes along the
    last axis stage the 16-bit image in place, by 16-byte groups of 8 positions
    (every run start 16-byte aligned), by 4-byte pairs (even offsets) or per
    lane (odd), and must still equal the oracle on the widened image."""
    from paper_2208_00001_amd import binding as B
    c = synth.small_case(shape, C=1, seed=980 + sum(shape), lam=lam, iterations=it)
    print(f"case {c['name']} {fmt} lam={lam} it={it} (minimal workspace)", flush=True)
    img16, widened = rounded(c["image"], DTYPES[fmt])
    ws = B.new_workspace(shape, 1, "cuda", minimal=True)
    got = to_host(B.ggdt_half(img16.to("cuda"), to_dev(c["mask"]), c["spacing"], c["v"], lam, it, workspace=ws,
                              check=True))
    ref = oracle.ggdt(widened, c["mask"], c["spacing"], c["v"], lam, it, "f32")
    assert assert_parity(got, ref, what=f"{fmt} {c['name']}"), "not bitwise"
