"""Helpers shared by the GPU tests: device transfer and the parity bar."""
import numpy as np
import torch

DEV = "cuda:0"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    denom = np.abs(ref)
    err = np.abs(got - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(denom > 0, err / denom, np.where(err == 0, 0.0, np.inf))
    return rel


def assert_parity(got, ref, rtol=1e-5, what=""):
    """The bar for FP32 outputs: |g - o| <= rtol * |o| per voxel, exact where o == 0.
    Also reports whether the match is bitwise (it is expected to be)."""
    rel = rel_err(got, ref)
    bad = ~(rel <= rtol)
    assert not bad.any(), (f"{what}: {int(bad.sum())} voxels over {rtol} relative; max rel {np.nanmax(rel):.3e}; "
                           f"first at {np.argwhere(bad)[0].tolist()}")
    return bool(np.array_equal(np.asarray(got), np.asarray(ref)))
