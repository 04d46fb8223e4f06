"""The allocation-free 3D forward (ggdt3d_noalloc), called through the C ABI:
two calls in a row on one stream, the second with a smaller volume, each equal
to ggdt3d with a caller workspace (the bar of the parity tests: 1e-5 relative,
expected bitwise) and to the oracle; and a volume whose scratch would exceed
the library's fixed array is rejected before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_parity, to_dev, to_host
from paper_2208_00001_amd import synth

pytestmark = pytest.mark.gpu

GGDT_ERR_WORKSPACE_TOO_SMALL = -4


def _noalloc(lib, img, m, spacing, v, lam, iterations, out):
    sp = (ctypes.c_float * 3)(*[float(s) for s in spacing])
    C = img.shape[0] if img.dim() == 4 else 1
    D, H, W = m.shape
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib.ggdt3d_noalloc(ctypes.c_void_p(img.data_ptr()), ctypes.c_void_p(m.data_ptr()), sp, float(v),
                              float(lam), int(iterations), ctypes.c_void_p(out.data_ptr()), C, D, H, W, stream)


def test_noalloc_matches_workspace_entry_on_two_calls():
    from paper_2208_00001_amd import binding as B
    lib = B.load_library()
    cases = [synth.small_case((70, 90, 110), C=1, seed=951, lam=1.0, iterations=2),
             synth.small_case((23, 41, 37), C=1, seed=952, lam=0.6, iterations=3, soft=True, v=10.0)]
    for k, c in enumerate(cases):
        print(f"call {k}: shape {c['mask'].shape} lam {c['lam']}", flush=True)
        img, m = to_dev(c["image"]), to_dev(c["mask"])
        out = torch.full(c["mask"].shape, -1.0, device=img.device)
        rc = _noalloc(lib, img, m, c["spacing"], c["v"], c["lam"], c["iterations"], out)
        assert rc == 0, B.GGDTError(rc, "ggdt3d_noalloc")
        ref = B.ggdt3d(img, m, c["spacing"], c["v"], c["lam"], c["iterations"], check=True)
        got = to_host(out)
        assert assert_parity(got, to_host(ref), what=f"call {k} vs ggdt3d")
        assert np.array_equal(got, to_host(ref))
        orc = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32")
        assert np.array_equal(got, orc)


def test_noalloc_rejects_volumes_beyond_its_scratch():
    from paper_2208_00001_amd import binding as B
    lib = B.load_library()
    img = torch.zeros((2, 600, 600), device="cuda")
    out = torch.empty_like(img)
    rc = _noalloc(lib, img, img, (1.0, 1.0, 1.0), 1e10, 1.0, 1, out)
    assert rc == GGDT_ERR_WORKSPACE_TOO_SMALL
