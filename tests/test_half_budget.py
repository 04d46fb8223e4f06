"""Error budget of 16-bit image storage, on the CPU with the oracle.

Rounding the image to a 16-bit format changes each value by at most u |I|
(round to nearest: u = 2^-8 for bfloat16, 2^-11 for binary16 in its normal
range).  An edge cost w = sqrt(A + lambda sum_c d_c^2) has |dw/dd| <= sqrt(lambda)
per unit of the difference vector d, so each edge changes by at most
sqrt(lambda C) 2 u max|I|, and a chain of the schedule (at most K =
iterations * 2 * sum_a (N_a - 1) edges) by K times that.  With the FP32
rounding of both runs, (K + 5) 2^-24 of each value, the transform on the
rounded image stays within that budget of the transform on the fp32 image."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2208_00001_amd import synth

U = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}
DTYPES = {"bf16": torch.bfloat16, "f16": torch.float16}


@pytest.mark.parametrize("fmt", list(U))
@pytest.mark.parametrize("shape,C,lam,it", [((40, 50), 1, 1.0, 2), ((37, 29), 3, 0.5, 2), ((12, 14, 13), 1, 1.0, 2),
                                            ((11, 9, 12), 2, 0.3, 1), ((30, 31), 2, 0.9, 3)])
def test_half_image_error_within_budget(fmt, shape, C, lam, it):
    c = synth.small_case(shape, C=C, seed=970 + C, lam=lam, iterations=it)
    widened = torch.from_numpy(c["image"]).to(DTYPES[fmt]).float().numpy()
    assert np.all(np.abs(widened - c["image"]) <= U[fmt] * np.abs(c["image"]) + 2.0 ** -24)
    d = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], lam, it, "f32").astype(np.float64)
    dh = oracle.ggdt(widened, c["mask"], c["spacing"], c["v"], lam, it, "f32").astype(np.float64)
    K = it * 2 * sum(n - 1 for n in shape)
    edge = math.sqrt(lam * C) * 2 * U[fmt] * float(np.abs(c["image"]).max())
    bound = K * edge + (K + 5) * 2.0 ** -24 * (d + dh)
    assert np.all(np.abs(dh - d) <= bound), float(np.max(np.abs(dh - d) - bound))
    # hard seeds stay 0 (other voxels may reach 0 too at lambda = 1, where rounding
    # can make neighbouring values equal and their edge cost 0)
    seeds = c["mask"] == 0
    assert np.all(d[seeds] == 0) and np.all(dh[seeds] == 0)
