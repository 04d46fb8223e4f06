"""Central finite differences on the 4 x 128^3 gradient workload (volume 0):
L = sum(W * D), lambda 0.7, 3 iterations, soft mask, v = 10.

At 200 random voxels away from argmin ties (for M and for I each), dL/dM and
dL/dI from FP64 central differences (eps = 1e-3, the oracle's FP64 schedule)
are compared with the FP64 reverse pass and
with the FP32 reverse pass, which the GPU backward equals bit for bit (checked
on all four volumes of this workload by the GPU tests).  "Away from argmin
ties" is made checkable: a voxel counts only if both perturbed FP64 runs keep
every record of the unperturbed run (then L is smooth there and the central
difference is a valid reference); the others are counted as ties, and voxels
are drawn until 200 qualify.  Bound: |g - fd| <= 1e-3 |fd| + 1e-6 max|W|.

The perturbed FP64 runs use the oracle's exact incremental re-evaluation
(PerturbedF64, equal to the full FP64 schedule bit for bit, pinned in
test_oracle.py), about 0.03 s each instead of 5 s, on a thread pool.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2208_00001_amd import synth

pytestmark = pytest.mark.slow

NVOX = 200
EPS = 1e-3


def test_config5_gradient_vs_central_differences():
    c = synth.config5()[0]
    img = c["image"].astype(np.float64)
    msk = c["mask"].astype(np.float64)
    W64 = c["weight"].astype(np.float64)
    _, rec32 = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32",
                           records=True)
    gi32, gm32 = oracle.backward(c["image"], rec32, c["weight"], c["spacing"], c["v"], c["lam"], c["iterations"],
                                 "f32")
    pert = oracle.PerturbedF64(img, msk, c["spacing"], c["v"], c["lam"], c["iterations"])
    gi64, gm64 = oracle.backward(img, pert.records, W64, c["spacing"], c["v"], c["lam"], c["iterations"], "f64")
    rng = np.random.default_rng(220800605)

    def loss(task):
        which, idx, sgn = task
        D, same = pert.run(which, idx, sgn * EPS)
        return float(np.sum(W64 * D)), same

    tol_abs = 1e-6 * float(np.abs(W64).max())
    checked = {"M": 0, "I": 0}
    ties = {"M": 0, "I": 0}
    f32_off = {"M": 0, "I": 0}
    worst64 = {"M": 0.0, "I": 0.0}
    nthreads = max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(max_workers=nthreads) as ex:
        for which in ("M", "I"):
            # draw voxels until NVOX of them are away from ties (at most 10 NVOX draws)
            drawn = 0
            while checked[which] < NVOX and drawn < 10 * NVOX:
                batch = [tuple(int(rng.integers(0, s)) for s in msk.shape) for _ in range(64)]
                drawn += len(batch)
                res = list(ex.map(loss, [(which, idx, sgn) for idx in batch for sgn in (1, -1)]))
                for b, idx in enumerate(batch):
                    if checked[which] >= NVOX:
                        break
                    (lp, same_p), (lm, same_m) = res[2 * b], res[2 * b + 1]
                    if not (same_p and same_m):
                        ties[which] += 1
                        continue
                    fd = (lp - lm) / (2 * EPS)
                    an64 = gm64[idx] if which == "M" else gi64[(0,) + idx]
                    an32 = float(gm32[idx] if which == "M" else gi32[(0,) + idx])
                    bound = 1e-3 * abs(fd) + tol_abs
                    worst64[which] = max(worst64[which], abs(an64 - fd) / bound)
                    assert abs(an64 - fd) <= bound, ("FP64 reverse pass vs central difference", which, idx, an64, fd)
                    if abs(an32 - fd) > bound:
                        f32_off[which] += 1  # the FP32 schedule took another argmin on this voxel's paths
                    checked[which] += 1
    print(f"checked {checked}, ties {ties}, FP32 gradient outside the bound {f32_off}, "
          f"worst FP64 error / bound {worst64}", flush=True)
    assert checked["M"] == NVOX and checked["I"] == NVOX, (checked, ties)
    # The FP32 reverse pass (the GPU's gradient) follows the FP32 schedule's own
    # argmins; where they differ from the FP64 schedule's, its gradient differs.
    # That may happen at a few voxels only.
    for w in ("M", "I"):
        assert f32_off[w] <= checked[w] // 20, (w, f32_off, checked)
