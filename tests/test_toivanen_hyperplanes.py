"""The hyperplane order of Toivanen's sweeps, checked on the CPU.

The GPU form of Toivanen's scan updates all voxels of a hyperplane
t = 4z + 2y + x (2D: t = 2y + x) in parallel, the hyperplanes in order (the
backward sweep in reverse).  Every neighbour a voxel reads in a sweep lies on an
earlier hyperplane, so the values must equal the sequential raster sweep's bit
for bit.  This test runs that order in plain Python (each hyperplane's voxels
in an order shuffled per hyperplane, so nothing can rely on raster order within
one) against the oracle's sequential sweep, at lambda 0 and 1 with one channel,
where every FP32 step is a single IEEE operation numpy performs exactly (the
fused multiply-adds of the edge cost reduce to plain values there)."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2208_00001_amd import synth


def causal_offsets(ndim):
    offs = []
    for o in itertools.product(*([(-1, 0, 1)] * ndim)):
        first = next((c for c in o if c != 0), 0)
        if first < 0:
            offs.append(o)
    return offs


def hyperplane_toivanen(image, mask, spacing, v, lam, iterations, seed):
    assert lam in (0.0, 1.0)
    nd = mask.ndim
    dims = mask.shape
    img = image.astype(np.float32)
    D = (np.float32(v) * mask.astype(np.float32)).astype(np.float32)
    offs = causal_offsets(nd)
    A = [np.float32((1.0 - lam) * sum((float(np.float32(spacing[b])) * abs(o[b])) ** 2 for b in range(nd)))
         for o in offs]
    weights = (4, 2, 1)[3 - nd:]
    T = sum(wt * (n - 1) for wt, n in zip(weights, dims)) + 1
    planes = {}
    for x in itertools.product(*[range(n) for n in dims]):
        planes.setdefault(sum(wt * c for wt, c in zip(weights, x)), []).append(x)
    rng = np.random.default_rng(seed)
    for _ in range(iterations):
        for sgn in (1, -1):
            for s in range(T):
                t = s if sgn > 0 else T - 1 - s
                vox = planes.get(t, [])
                for k in rng.permutation(len(vox)):
                    x = vox[k]
                    best = D[x]
                    for o, a in zip(offs, A):
                        y = tuple(c + sgn * d for c, d in zip(x, o))
                        if any(c < 0 or c >= n for c, n in zip(y, dims)):
                            continue
                        if lam == 0.0:
                            w = np.sqrt(a)
                        else:
                            d = np.float32(img[x] - img[y])
                            w = np.sqrt(np.float32(d * d))
                        cand = np.float32(D[y] + w)
                        if cand < best:
                            best = cand
                    D[x] = best
    return D


@pytest.mark.parametrize("shape,lam,it,soft", [((9, 13), 1.0, 2, False), ((7, 1), 0.0, 1, False),
                                               ((11, 8), 0.0, 2, True), ((5, 6, 7), 1.0, 2, False),
                                               ((4, 7, 3), 0.0, 1, True), ((1, 5, 9), 1.0, 3, True)])
def test_hyperplane_order_equals_sequential_sweep(shape, lam, it, soft):
    c = synth.small_case(shape, C=1, seed=sum(shape), lam=lam, iterations=it, soft=soft, v=6.0 if soft else 1e10)
    ref = oracle.toivanen(c["image"], c["mask"], c["spacing"], c["v"], lam, it, "f32")
    got = hyperplane_toivanen(c["image"][0], c["mask"], c["spacing"], c["v"], lam, it, seed=len(shape))
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
