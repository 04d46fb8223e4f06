"""ORACLE — test infrastructure only.

Plain CPU reference of the generalised geodesic distance transform computed by
directional raster-scan passes (FastGeodis paper, section "Implementation"), plus
the independent checkers that pin it (Dijkstra, the lambda = 0 closed form, path
enumeration, per-pass chain brute force, reverse-mode gradient).  The arithmetic
lives in ``ggdt_ref.c``; this module only marshals numpy arrays through ctypes.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library and
never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ggdt_ref.c")
_LIB = os.path.join(_HERE, "libggdt_ref.so")
_CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC"]

_lib = None


def build() -> str:
    """Compile ggdt_ref.c into libggdt_ref.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(shape):
    return (ctypes.c_int * len(shape))(*shape)


def _split(image, mask):
    """image: (C, *spatial) or (*spatial) -> (C, spatial shape)."""
    mask = np.asarray(mask)
    spatial = mask.shape
    image = np.asarray(image)
    if image.shape == spatial:
        image = image[None]
    if image.shape[1:] != spatial or len(spatial) not in (2, 3):
        raise ValueError(f"shape mismatch: image {image.shape} mask {spatial}")
    return image, spatial


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


def passes_per_iteration(ndim: int) -> int:
    return 2 * ndim


def pass_schedule(ndim: int, iterations: int):
    """(axis, sign) of every directional pass, in execution order."""
    return [(a, s) for _ in range(iterations) for a in range(ndim) for s in (1, -1)]


def ggdt(image, mask, spacing, v, lam, iterations, precision="f32", records=False):
    """Fixed-iteration raster-scan GGDT.  Returns D (and records if asked:
    uint8 array (passes, *spatial), 0 = keep, 1 + j = parent offset j)."""
    lib = _load()
    image, spatial = _split(image, mask)
    C = image.shape[0]
    nd = len(spatial)
    npass = iterations * 2 * nd
    rec = np.zeros((npass,) + spatial, dtype=np.uint8) if records else None
    if precision == "f32":
        img, m, sp = _f32(image), _f32(mask), _f32(spacing)
        out = np.empty(spatial, dtype=np.float32)
        fn, vv, ll = lib.ref_ggdt_f32, ctypes.c_float(v), ctypes.c_float(lam)
    elif precision == "f64":
        img, m, sp = _f64(image), _f64(mask), _f64(spacing)
        out = np.empty(spatial, dtype=np.float64)
        fn, vv, ll = lib.ref_ggdt_f64, ctypes.c_double(v), ctypes.c_double(lam)
    else:
        raise ValueError(precision)
    rc = fn(nd, _dims(spatial), C, _p(img), _p(m), _p(sp), vv, ll, int(iterations), _p(out),
            _p(rec) if rec is not None else None)
    _check(rc, "ref_ggdt")
    return (out, rec) if records else out


def ggdt_omp(image, mask, spacing, v, lam, iterations):
    """The FP32 schedule with each plane's voxels shared among OpenMP threads
    (OMP_NUM_THREADS); same values as ``ggdt(..., "f32")``.  Returns (D, threads)."""
    lib = _load()
    image, spatial = _split(image, mask)
    img, m, sp = _f32(image), _f32(mask), _f32(spacing)
    out = np.empty(spatial, dtype=np.float32)
    rc = lib.ref_ggdt_f32_omp(len(spatial), _dims(spatial), image.shape[0], _p(img), _p(m), _p(sp),
                              ctypes.c_float(v), ctypes.c_float(lam), int(iterations), _p(out))
    if rc < 0:
        raise RuntimeError(f"ref_ggdt_f32_omp failed with code {rc}")
    return out, rc


# ------------------------------------------------ signed distance and GSF
# The paper names a signed geodesic distance and the geodesic symmetric filter
# (GSF) of Criminisi et al. 2008 among what the software computes (sections
# "Statement of need" and "Implementation") without defining them; these are
# this project's readings, composed from the FP32 schedule with FP32 pointwise
# operations.  Object masks use the seed convention: 0 on the object, 1 elsewhere.

def signed(image, mask, spacing, v, lam, iterations):
    """S = D(I; M) - D(I; 1 - M): negative on the object, positive outside."""
    m = _f32(mask)
    d_obj = ggdt(image, m, spacing, v, lam, iterations, "f32")
    d_bg = ggdt(image, np.float32(1) - m, spacing, v, lam, iterations, "f32")
    return d_obj - d_bg


def object_mask(S, theta):
    """Mask of the object {x : S(x) < theta}: 0 on it, 1 elsewhere."""
    return np.where(_f32(S) < np.float32(theta), np.float32(0), np.float32(1))


def gsf(image, mask, theta_d, theta_e, spacing, v, lam, iterations):
    """Geodesic symmetric filter: the closing (dilate by theta_d, then erode by
    theta_e) and the opening (erode, then dilate) of the object of M, merged
    through their signed distances: returns (S_d + S_e) + (theta_e - theta_d),
    where S_d, S_e are the signed distances of the dilated and eroded objects.
    The filtered object is where the result is negative."""
    s0 = signed(image, mask, spacing, v, lam, iterations)
    s_d = signed(image, object_mask(s0, theta_d), spacing, v, lam, iterations)
    s_e = signed(image, object_mask(s0, -np.float32(theta_e)), spacing, v, lam, iterations)
    t = np.float32(theta_e) - np.float32(theta_d)
    return (s_d + s_e) + t


def single_pass(image, D, spacing, lam, axis, sign, precision="f32", records=False):
    """One directional pass applied to a copy of D."""
    lib = _load()
    image, spatial = _split(image, D)
    C = image.shape[0]
    rec = np.zeros(spatial, dtype=np.uint8) if records else None
    if precision == "f32":
        img, sp, out = _f32(image), _f32(spacing), _f32(D).copy()
        rc = lib.ref_pass_f32(len(spatial), _dims(spatial), C, _p(img), _p(sp), ctypes.c_float(lam),
                              int(axis), int(sign), _p(out), _p(rec) if rec is not None else None)
    else:
        img, sp, out = _f64(image), _f64(spacing), _f64(D).copy()
        rc = lib.ref_pass_f64(len(spatial), _dims(spatial), C, _p(img), _p(sp), ctypes.c_double(lam),
                              int(axis), int(sign), _p(out), _p(rec) if rec is not None else None)
    _check(rc, "ref_pass")
    return (out, rec) if records else out


def until_converged(image, mask, spacing, v, lam, max_iterations=10000, precision="f32"):
    """Iterate whole iterations until a fixed point; returns (D, iterations)."""
    lib = _load()
    image, spatial = _split(image, mask)
    C = image.shape[0]
    if precision == "f32":
        img, m, sp = _f32(image), _f32(mask), _f32(spacing)
        out = np.empty(spatial, dtype=np.float32)
        n = lib.ref_ggdt_until_converged_f32(len(spatial), _dims(spatial), C, _p(img), _p(m), _p(sp),
                                             ctypes.c_float(v), ctypes.c_float(lam),
                                             int(max_iterations), _p(out))
    else:
        img, m, sp = _f64(image), _f64(mask), _f64(spacing)
        out = np.empty(spatial, dtype=np.float64)
        n = lib.ref_ggdt_until_converged_f64(len(spatial), _dims(spatial), C, _p(img), _p(m), _p(sp),
                                             ctypes.c_double(v), ctypes.c_double(lam),
                                             int(max_iterations), _p(out))
    if n < 0:
        raise RuntimeError(f"did not converge within {max_iterations} iterations (code {n})")
    return out, n


def toivanen(image, mask, spacing, v, lam, iterations, precision="f32", converge=False):
    """Toivanen's sequential raster scan (forward then backward raster sweep per
    iteration, in-place updates over the preceding half of the 8/26-neighbourhood).
    converge=False: exactly `iterations` iterations, returns D.  converge=True:
    until an iteration changes nothing (at most `iterations`), returns (D, n)."""
    lib = _load()
    image, spatial = _split(image, mask)
    C = image.shape[0]
    if precision == "f32":
        img, m, sp = _f32(image), _f32(mask), _f32(spacing)
        out = np.empty(spatial, dtype=np.float32)
        n = lib.ref_toivanen_f32(len(spatial), _dims(spatial), C, _p(img), _p(m), _p(sp), ctypes.c_float(v),
                                 ctypes.c_float(lam), int(iterations), int(converge), _p(out))
    else:
        img, m, sp = _f64(image), _f64(mask), _f64(spacing)
        out = np.empty(spatial, dtype=np.float64)
        n = lib.ref_toivanen_f64(len(spatial), _dims(spatial), C, _p(img), _p(m), _p(sp), ctypes.c_double(v),
                                 ctypes.c_double(lam), int(iterations), int(converge), _p(out))
    if n < 0 and not (converge and n == -1):
        raise RuntimeError(f"ref_toivanen failed with code {n}")
    if converge:
        if n < 0:
            raise RuntimeError(f"did not converge within {iterations} iterations")
        return out, n
    return out


def dijkstra(image, mask, spacing, v, lam, precision="f64"):
    """Multi-source Dijkstra on the 8/26-connected grid with the same edge cost."""
    lib = _load()
    image, spatial = _split(image, mask)
    C = image.shape[0]
    if precision == "f32":
        img, m, sp = _f32(image), _f32(mask), _f32(spacing)
        out = np.empty(spatial, dtype=np.float32)
        rc = lib.ref_dijkstra_f32(len(spatial), _dims(spatial), C, _p(img), _p(m), _p(sp),
                                  ctypes.c_float(v), ctypes.c_float(lam), _p(out))
    else:
        img, m, sp = _f64(image), _f64(mask), _f64(spacing)
        out = np.empty(spatial, dtype=np.float64)
        rc = lib.ref_dijkstra_f64(len(spatial), _dims(spatial), C, _p(img), _p(m), _p(sp),
                                  ctypes.c_double(v), ctypes.c_double(lam), _p(out))
    _check(rc, "ref_dijkstra")
    return out


def chamfer_closed_form(mask, spacing, v):
    """lambda = 0 distances from the king-move chain formula, FP64, O(n^2)."""
    lib = _load()
    m = _f64(mask)
    sp = _f64(spacing)
    out = np.empty(m.shape, dtype=np.float64)
    rc = lib.ref_chamfer_closed_form_f64(m.ndim, _dims(m.shape), _p(m), _p(sp), ctypes.c_double(v), _p(out))
    _check(rc, "ref_chamfer_closed_form_f64")
    return out


def bruteforce_paths(image, mask, spacing, v, lam, prune=False, max_visits=2_000_000_000):
    """Minimum over all simple paths (prune=False) or bound-pruned walks, FP64."""
    lib = _load()
    image, spatial = _split(image, mask)
    img, m, sp = _f64(image), _f64(mask), _f64(spacing)
    out = np.empty(spatial, dtype=np.float64)
    lib.ref_bruteforce_paths_f64.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p]
    rc = lib.ref_bruteforce_paths_f64(len(spatial), _dims(spatial), image.shape[0], _p(img), _p(m), _p(sp),
                                      v, lam, int(bool(prune)), int(max_visits), _p(out))
    _check(rc, "ref_bruteforce_paths_f64")
    return out


def pass_bruteforce(image, D_in, spacing, lam, axis, sign):
    """One pass as a min over monotone chains, each target on its own, FP64."""
    lib = _load()
    image, spatial = _split(image, D_in)
    img, sp, din = _f64(image), _f64(spacing), _f64(D_in)
    out = np.empty(spatial, dtype=np.float64)
    rc = lib.ref_pass_bruteforce_f64(len(spatial), _dims(spatial), image.shape[0], _p(img), _p(sp),
                                     ctypes.c_double(lam), int(axis), int(sign), _p(din), _p(out))
    _check(rc, "ref_pass_bruteforce_f64")
    return out


def backward(image, records, grad_out, spacing, v, lam, iterations, precision="f32"):
    """Reverse-mode gradient of the fixed schedule; returns (dL/dI, dL/dM)."""
    lib = _load()
    g = np.asarray(grad_out)
    image, spatial = _split(image, g)
    C = image.shape[0]
    rec = np.ascontiguousarray(records, dtype=np.uint8)
    if rec.shape != (iterations * 2 * len(spatial),) + spatial:
        raise ValueError(f"records shape {rec.shape}")
    if precision == "f32":
        img, sp, go = _f32(image), _f32(spacing), _f32(g)
        gi = np.empty(image.shape, dtype=np.float32)
        gm = np.empty(spatial, dtype=np.float32)
        rc = lib.ref_ggdt_backward_f32(len(spatial), _dims(spatial), C, _p(img), _p(sp), ctypes.c_float(v),
                                       ctypes.c_float(lam), int(iterations), _p(rec), _p(go), _p(gi), _p(gm))
    else:
        img, sp, go = _f64(image), _f64(spacing), _f64(g)
        gi = np.empty(image.shape, dtype=np.float64)
        gm = np.empty(spatial, dtype=np.float64)
        rc = lib.ref_ggdt_backward_f64(len(spatial), _dims(spatial), C, _p(img), _p(sp), ctypes.c_double(v),
                                       ctypes.c_double(lam), int(iterations), _p(rec), _p(go), _p(gi), _p(gm))
    _check(rc, "ref_ggdt_backward")
    return gi, gm


class PerturbedF64:
    """Exact incremental re-evaluation of the FP64 schedule for single-voxel
    changes of the input (a checker for central differences).

    Holds the base run's state after every pass (``ref_ggdt_f64_trajectory``);
    ``run(which, index, delta)`` returns (D, records_unchanged) of the FP64
    schedule on the input with M[index] (which = "M") or I[channel][index]
    (which = "I") increased by delta, equal bit for bit to ``ggdt(...,
    "f64", records=True)`` on that input.  ``run`` may be called from several
    threads at once (the library call releases the GIL)."""

    def __init__(self, image, mask, spacing, v, lam, iterations):
        lib = _load()
        image, spatial = _split(image, mask)
        self.img, self.m, self.sp = _f64(image), _f64(mask), _f64(spacing)
        self.spatial, self.C = spatial, image.shape[0]
        self.v, self.lam, self.iterations = float(v), float(lam), int(iterations)
        n = int(np.prod(spatial))
        npass = self.iterations * 2 * len(spatial)
        self.traj = np.empty((npass + 1,) + spatial, dtype=np.float64)
        self.records = np.empty((npass,) + spatial, dtype=np.uint8)
        rc = lib.ref_ggdt_f64_trajectory(len(spatial), _dims(spatial), self.C, _p(self.img), _p(self.m),
                                         _p(self.sp), ctypes.c_double(self.v), ctypes.c_double(self.lam),
                                         self.iterations, _p(self.traj), _p(self.records))
        _check(rc, "ref_ggdt_f64_trajectory")
        self.n = n

    @property
    def base(self):
        """The base run's final D."""
        return self.traj[-1]

    def run(self, which, index, delta, channel=0):
        lib = _load()
        flat = int(np.ravel_multi_index(tuple(index), self.spatial))
        out = np.empty(self.spatial, dtype=np.float64)
        same = ctypes.c_int(0)
        rc = lib.ref_ggdt_f64_perturbed(len(self.spatial), _dims(self.spatial), self.C, _p(self.img), _p(self.m),
                                        _p(self.sp), ctypes.c_double(self.v), ctypes.c_double(self.lam),
                                        self.iterations, _p(self.traj), _p(self.records),
                                        0 if which == "M" else 1, int(channel), ctypes.c_long(flat),
                                        ctypes.c_double(delta), _p(out), ctypes.byref(same))
        _check(rc, "ref_ggdt_f64_perturbed")
        return out, bool(same.value)
