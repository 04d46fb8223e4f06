"""ctypes binding of libggdt.so: argument marshalling only.

PyTorch provides device memory and the HIP stream (torch's current stream);
every step of the transform runs in the library's HIP kernels.  There is no CPU
fallback: if the library is missing or the device is not gfx950, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libggdt.so")

GGDT_OK = 0
_c_int, _c_float, _c_size, _vp = ctypes.c_int, ctypes.c_float, ctypes.c_size_t, ctypes.c_void_p


class GGDTError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = _lib.ggdt_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} (status {code})")


class GGDTInstance(ctypes.Structure):
    _fields_ = [
        ("ndim", _c_int), ("C", _c_int), ("dims", _c_int * 3),
        ("image", _vp), ("softmask", _vp), ("out", _vp),
        ("spacing", _c_float * 3), ("v", _c_float), ("lam", _c_float), ("iterations", _c_int),
        ("records", _vp), ("grad_out", _vp), ("grad_image", _vp), ("grad_softmask", _vp),
    ]


class GGDTTuning(ctypes.Structure):
    _fields_ = [("tile_p", _c_int), ("tile_q", _c_int), ("chunk", _c_int), ("wg_per_cu", _c_int)]


_lib = None

_SIGS = {
    "ggdt_strerror": (ctypes.c_char_p, [_c_int]),
    "ggdt_workspace_bytes": (_c_size, [_c_int, _vp, _c_int]),
    "ggdt_workspace_min_bytes": (_c_size, [_c_int, _vp, _c_int]),
    "ggdt_records_bytes": (_c_size, [_c_int, _vp, _c_int]),
    "ggdt_backward_workspace_bytes": (_c_size, [_c_int, _vp, _c_int]),
    "ggdt_backward_workspace_min_bytes": (_c_size, [_c_int, _vp, _c_int]),
    "ggdt2d": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _c_int, _c_int, _c_int, _vp, _c_size, _vp]),
    "ggdt3d": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _c_int, _c_int, _c_int, _c_int, _vp, _c_size,
                        _vp]),
    "ggdt2d_forward_rec": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _vp, _c_int, _c_int, _c_int, _vp,
                                    _c_size, _vp]),
    "ggdt3d_forward_rec": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _vp, _c_int, _c_int, _c_int,
                                    _c_int, _vp, _c_size, _vp]),
    "ggdt2d_backward": (_c_int, [_vp, _vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _vp, _c_int, _c_int, _c_int,
                                 _vp, _c_size, _vp]),
    "ggdt3d_backward": (_c_int, [_vp, _vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _vp, _c_int, _c_int, _c_int,
                                 _c_int, _vp, _c_size, _vp]),
    "ggdt2d_converge": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _c_int, _c_int, _c_int, _vp,
                                 _c_size, _vp]),
    "ggdt3d_converge": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _c_int, _c_int, _c_int, _c_int,
                                 _vp, _c_size, _vp]),
    "ggdt_signed_workspace_bytes": (_c_size, [_c_int, _vp, _c_int]),
    "ggdt_gsf_workspace_bytes": (_c_size, [_c_int, _vp, _c_int]),
    "ggdt2d_signed": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _c_int, _c_int, _c_int, _vp, _c_size,
                               _vp]),
    "ggdt3d_signed": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _c_int, _c_int, _c_int, _c_int, _vp,
                               _c_size, _vp]),
    "ggdt2d_gsf": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_float, _c_float, _c_int, _vp, _c_int, _c_int,
                            _c_int, _vp, _c_size, _vp]),
    "ggdt3d_gsf": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_float, _c_float, _c_int, _vp, _c_int, _c_int,
                            _c_int, _c_int, _vp, _c_size, _vp]),
    "ggdt3d_noalloc": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _c_int, _c_int, _c_int, _c_int,
                                _vp]),
    "ggdt2d_toivanen": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _c_int, _c_int, _c_int, _vp,
                                 _c_size, _vp]),
    "ggdt3d_toivanen": (_c_int, [_vp, _vp, _vp, _c_float, _c_float, _c_int, _vp, _c_int, _c_int, _c_int, _c_int, _vp,
                                 _c_size, _vp]),
    "ggdt2d_half": (_c_int, [_vp, _c_int, _vp, _vp, _c_float, _c_float, _c_int, _vp, _c_int, _c_int, _c_int, _vp,
                             _c_size, _vp]),
    "ggdt3d_half": (_c_int, [_vp, _c_int, _vp, _vp, _c_float, _c_float, _c_int, _vp, _c_int, _c_int, _c_int, _c_int,
                             _vp, _c_size, _vp]),
    "ggdt_workspace_iterations": (_c_int, [_vp, _vp, _vp]),
    "ggdt_workspace_status": (_c_int, [_vp, _vp]),
    "ggdt_set_spin_limit": (None, [ctypes.c_ulonglong]),
    "ggdt_profile_begin": (_c_int, [_c_int]),
    "ggdt_profile_end": (_c_int, [_vp, _c_int]),
    "ggdt_batched_plan": (_c_int, [_vp, _c_int, _vp, _vp, _vp]),
    "ggdt_batched_run": (_c_int, [_vp, _vp, _c_size, _vp]),
    "ggdt_batched_backward": (_c_int, [_vp, _vp, _c_size, _vp]),
    "ggdt_plan_destroy": (None, [_vp]),
    "ggdt_plan_info": (_c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
}


def load_library(path: str = LIB_PATH):
    """Load libggdt.so (after torch, so both use torch's HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run paper_2208_00001_amd.build.build() (or __graft_entry__.build())")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dims(shape):
    return (ctypes.c_int * len(shape))(*shape)


def _prep(image: torch.Tensor, softmask: torch.Tensor):
    if not (image.is_cuda and softmask.is_cuda):
        raise ValueError("image and softmask must be device tensors")
    if image.dtype != torch.float32 or softmask.dtype != torch.float32:
        raise TypeError("image and softmask must be float32")
    spatial = tuple(softmask.shape)
    if image.dim() == len(spatial):
        image = image.unsqueeze(0)
    if tuple(image.shape[1:]) != spatial or len(spatial) not in (2, 3):
        raise ValueError(f"shape mismatch: image {tuple(image.shape)} vs softmask {spatial}")
    return image.contiguous(), softmask.contiguous(), spatial


def workspace_bytes(spatial: Sequence[int], C: int) -> int:
    lib = load_library()
    return int(lib.ggdt_workspace_bytes(len(spatial), _dims(spatial), C))


def workspace_min_bytes(spatial: Sequence[int], C: int) -> int:
    """Smallest forward workspace: single-channel volumes then run the passes
    along the last axis in place instead of on scan-major copies."""
    lib = load_library()
    return int(lib.ggdt_workspace_min_bytes(len(spatial), _dims(spatial), C))


def records_bytes(spatial: Sequence[int], iterations: int) -> int:
    lib = load_library()
    return int(lib.ggdt_records_bytes(len(spatial), _dims(spatial), iterations))


def new_workspace(spatial, C, device, minimal=False) -> torch.Tensor:
    n = workspace_min_bytes(spatial, C) if minimal else workspace_bytes(spatial, C)
    if n == 0:
        raise ValueError(f"invalid shape {tuple(spatial)} with C={C}")
    return torch.empty(n, dtype=torch.uint8, device=device)


def _check_out(out, spatial, device, what="out"):
    """A caller-supplied output must be exactly what the kernels write: float32,
    contiguous, on the inputs' device, of the spatial shape (the C ABI takes no
    buffer lengths, so a wrong size would be written past)."""
    if out.dtype != torch.float32:
        raise ValueError(f"{what} must be float32, got {out.dtype}")
    if not out.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if out.device != device:
        raise ValueError(f"{what} is on {out.device}, the inputs on {device}")
    if tuple(out.shape) != tuple(spatial):
        raise ValueError(f"{what} has shape {tuple(out.shape)}, expected {tuple(spatial)}")
    return out


def _check_records(records, spatial, iterations, device):
    """Records: uint8, contiguous, on the device, iterations * 2 * ndim * prod(spatial) bytes."""
    if records.dtype != torch.uint8:
        raise ValueError(f"records must be uint8, got {records.dtype}")
    if not records.is_contiguous():
        raise ValueError("records must be contiguous")
    if records.device != device:
        raise ValueError(f"records are on {records.device}, the inputs on {device}")
    n = int(iterations) * 2 * len(spatial)
    for s in spatial:
        n *= int(s)
    if records.numel() != n:
        raise ValueError(f"records hold {records.numel()} bytes, the schedule of {iterations} iterations needs {n}")
    return records


def _check_workspace(workspace, device):
    """A caller's workspace: a contiguous uint8 tensor on the inputs' device (its
    numel is passed as the byte count the library checks)."""
    if workspace.dtype != torch.uint8 or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 tensor")
    if workspace.device != device:
        raise ValueError(f"workspace is on {workspace.device}, the inputs on {device}")
    return workspace


def _raise_if_watchdog(workspace, what):
    """Synchronise the stream and raise if an inter-workgroup wait of the call
    that used `workspace` expired (its results are then invalid)."""
    rc = load_library().ggdt_workspace_status(_ptr(workspace), _stream())
    if rc != GGDT_OK:
        raise GGDTError(rc, what)


def _spacing(spacing, nd):
    sp = tuple(float(s) for s in spacing)
    if len(sp) != nd:
        raise ValueError(f"spacing needs {nd} values")
    return (ctypes.c_float * nd)(*sp)


def _forward(image, softmask, spacing, v, lamb, iterations, out, workspace, records, check=False):
    lib = load_library()
    image, softmask, spatial = _prep(image, softmask)
    nd, C = len(spatial), image.shape[0]
    if out is None:
        out = torch.empty(spatial, dtype=torch.float32, device=softmask.device)
    else:
        _check_out(out, spatial, softmask.device)
    if records is not None:
        _check_records(records, spatial, iterations, softmask.device)
    if workspace is None:
        workspace = new_workspace(spatial, C, softmask.device)
    else:
        _check_workspace(workspace, softmask.device)
    sp = _spacing(spacing, nd)
    args = [_ptr(image), _ptr(softmask), sp, float(v), float(lamb), int(iterations), _ptr(out)]
    if records is not None:
        args.append(_ptr(records))
    args += [C, *spatial, _ptr(workspace), workspace.numel(), _stream()]
    if records is None:
        fn = lib.ggdt2d if nd == 2 else lib.ggdt3d
    else:
        fn = lib.ggdt2d_forward_rec if nd == 2 else lib.ggdt3d_forward_rec
    rc = fn(*args)
    if rc != GGDT_OK:
        raise GGDTError(rc, fn.__name__)
    if check:
        _raise_if_watchdog(workspace, fn.__name__)
    return out


def ggdt2d(image, softmask, spacing=(1.0, 1.0), v=1e10, lamb=1.0, iterations=2, out=None, workspace=None,
           check=False):
    """2D GGDT of image (C, H, W) or (H, W) with soft seed mask (H, W); returns D (H, W).

    Asynchronous on torch's current stream.  check=True synchronises and raises
    GGDTError if an inter-workgroup wait expired (the watchdog); otherwise that
    is reported only by workspace_status(workspace)."""
    if softmask.dim() != 2:
        raise ValueError("softmask must be (H, W)")
    return _forward(image, softmask, spacing, v, lamb, iterations, out, workspace, None, check)


def ggdt3d(image, softmask, spacing=(1.0, 1.0, 1.0), v=1e10, lamb=1.0, iterations=2, out=None, workspace=None,
           check=False):
    """3D GGDT of image (C, D, H, W) or (D, H, W) with soft seed mask (D, H, W); returns D.
    check as in ggdt2d."""
    if softmask.dim() != 3:
        raise ValueError("softmask must be (D, H, W)")
    return _forward(image, softmask, spacing, v, lamb, iterations, out, workspace, None, check)


GGDT_IMAGE_BF16, GGDT_IMAGE_F16 = 1, 2


def ggdt_half(image, softmask, spacing, v=1e10, lamb=1.0, iterations=2, out=None, workspace=None, check=False):
    """The forward with a 16-bit image: image is a torch.bfloat16 or torch.float16
    tensor ((C,) + spatial or spatial), widened to fp32 exactly inside the kernels;
    the result equals ggdt2d/ggdt3d on image.float() bit for bit.  2D with up to 3
    channels, 3D with one channel.  check as in ggdt2d."""
    lib = load_library()
    fmt = {torch.bfloat16: GGDT_IMAGE_BF16, torch.float16: GGDT_IMAGE_F16}.get(image.dtype)
    if fmt is None:
        raise TypeError(f"image must be bfloat16 or float16, got {image.dtype}")
    if not (image.is_cuda and softmask.is_cuda) or softmask.dtype != torch.float32:
        raise ValueError("image and softmask must be device tensors, softmask float32")
    spatial = tuple(softmask.shape)
    if image.dim() == len(spatial):
        image = image.unsqueeze(0)
    if tuple(image.shape[1:]) != spatial or len(spatial) not in (2, 3):
        raise ValueError(f"shape mismatch: image {tuple(image.shape)} vs softmask {spatial}")
    image, softmask = image.contiguous(), softmask.contiguous()
    nd, C = len(spatial), image.shape[0]
    if out is None:
        out = torch.empty(spatial, dtype=torch.float32, device=softmask.device)
    else:
        _check_out(out, spatial, softmask.device)
    if workspace is None:
        workspace = new_workspace(spatial, C, softmask.device)
    else:
        _check_workspace(workspace, softmask.device)
    fn = lib.ggdt2d_half if nd == 2 else lib.ggdt3d_half
    rc = fn(_ptr(image), fmt, _ptr(softmask), _spacing(spacing, nd), float(v), float(lamb), int(iterations),
            _ptr(out), C, *spatial, _ptr(workspace), workspace.numel(), _stream())
    if rc != GGDT_OK:
        raise GGDTError(rc, fn.__name__)
    if check:
        _raise_if_watchdog(workspace, fn.__name__)
    return out


def ggdt_toivanen(image, softmask, spacing, v=1e10, lamb=1.0, iterations=2, out=None, workspace=None, check=False):
    """Toivanen's raster scan (forward then backward raster sweep per iteration,
    in place over the preceding half of the 8/26-neighbourhood), run on the GPU by
    hyperplanes; image ((C,) + spatial or spatial) and softmask (spatial) float32
    device tensors, 2D or 3D.  check as in ggdt2d."""
    lib = load_library()
    image, softmask, spatial = _prep(image, softmask)
    nd, C = len(spatial), image.shape[0]
    if out is None:
        out = torch.empty(spatial, dtype=torch.float32, device=softmask.device)
    else:
        _check_out(out, spatial, softmask.device)
    if workspace is None:
        workspace = new_workspace(spatial, C, softmask.device, minimal=True)
    else:
        _check_workspace(workspace, softmask.device)
    fn = lib.ggdt2d_toivanen if nd == 2 else lib.ggdt3d_toivanen
    rc = fn(_ptr(image), _ptr(softmask), _spacing(spacing, nd), float(v), float(lamb), int(iterations), _ptr(out), C,
            *spatial, _ptr(workspace), workspace.numel(), _stream())
    if rc != GGDT_OK:
        raise GGDTError(rc, fn.__name__)
    if check:
        _raise_if_watchdog(workspace, fn.__name__)
    return out


def ggdt_converge(image, softmask, spacing, v=1e10, lamb=1.0, max_iterations=100, out=None, workspace=None):
    """Forward run to its fixed point (2D or 3D by the mask's rank).  Returns
    (D, iterations): the number of iterations that lowered some value, or -1 if
    max_iterations passed without reaching the fixed point.  Synchronises."""
    lib = load_library()
    image, softmask, spatial = _prep(image, softmask)
    nd, C = len(spatial), image.shape[0]
    if out is None:
        out = torch.empty(spatial, dtype=torch.float32, device=softmask.device)
    else:
        _check_out(out, spatial, softmask.device)
    if workspace is None:
        workspace = new_workspace(spatial, C, softmask.device)
    else:
        _check_workspace(workspace, softmask.device)
    fn = lib.ggdt2d_converge if nd == 2 else lib.ggdt3d_converge
    rc = fn(_ptr(image), _ptr(softmask), _spacing(spacing, nd), float(v), float(lamb), int(max_iterations),
            _ptr(out), C, *spatial, _ptr(workspace), workspace.numel(), _stream())
    if rc != GGDT_OK:
        raise GGDTError(rc, fn.__name__)
    n = ctypes.c_int(0)
    rc = lib.ggdt_workspace_iterations(_ptr(workspace), _stream(), ctypes.byref(n))
    if rc != GGDT_OK:
        raise GGDTError(rc, "ggdt_workspace_iterations")
    return out, n.value


def _composed(kind, image, softmask, spacing, v, lamb, iterations, thetas, out, workspace, check=False):
    lib = load_library()
    image, softmask, spatial = _prep(image, softmask)
    nd, C = len(spatial), image.shape[0]
    if out is None:
        out = torch.empty(spatial, dtype=torch.float32, device=softmask.device)
    else:
        _check_out(out, spatial, softmask.device)
    if workspace is None:
        q = lib.ggdt_signed_workspace_bytes if kind == "signed" else lib.ggdt_gsf_workspace_bytes
        n = int(q(nd, _dims(spatial), C))
        if n == 0:
            raise ValueError(f"invalid shape {tuple(spatial)} with C={C}")
        workspace = torch.empty(n, dtype=torch.uint8, device=softmask.device)
    else:
        _check_workspace(workspace, softmask.device)
    fn = getattr(lib, f"ggdt{nd}d_{kind}")
    rc = fn(_ptr(image), _ptr(softmask), _spacing(spacing, nd), *[float(t) for t in thetas], float(v), float(lamb),
            int(iterations), _ptr(out), C, *spatial, _ptr(workspace), workspace.numel(), _stream())
    if rc != GGDT_OK:
        raise GGDTError(rc, fn.__name__)
    if check:
        _raise_if_watchdog(workspace, fn.__name__)
    return out


def ggdt_signed(image, softmask, spacing, v=1e10, lamb=1.0, iterations=2, out=None, workspace=None, check=False):
    """Signed distance D(I; M) - D(I; 1 - M) (2D or 3D by the mask's rank); check as in ggdt2d."""
    return _composed("signed", image, softmask, spacing, v, lamb, iterations, (), out, workspace, check)


def ggdt_gsf(image, softmask, theta_d, theta_e, spacing, v=1e10, lamb=1.0, iterations=2, out=None, workspace=None,
             check=False):
    """Geodesic symmetric filter (S_d + S_e) + (theta_e - theta_d); the filtered object is where it is < 0.
    check as in ggdt2d."""
    return _composed("gsf", image, softmask, spacing, v, lamb, iterations, (theta_d, theta_e), out, workspace, check)


def ggdt_forward_rec(image, softmask, spacing, v=1e10, lamb=1.0, iterations=2, out=None, records=None,
                     workspace=None, check=False):
    """Forward that also returns the argmin records, uint8 (passes, *spatial); check as in ggdt2d."""
    _, sm, spatial = _prep(image, softmask)
    npass = iterations * 2 * len(spatial)
    if records is None:
        records = torch.empty((npass,) + spatial, dtype=torch.uint8, device=sm.device)
    out = _forward(image, softmask, spacing, v, lamb, iterations, out, workspace, records, check)
    return out, records


def ggdt_backward(image, records, grad_out, spacing, v, lamb, iterations, workspace=None, check=False):
    """Reverse of the recorded schedule: returns (dL/dI with image's shape, dL/dM); check as in ggdt2d."""
    lib = load_library()
    squeeze = image.dim() == grad_out.dim()
    image, grad_out, spatial = _prep(image, grad_out)
    nd, C = len(spatial), image.shape[0]
    _check_records(records, spatial, iterations, image.device)
    gi = torch.empty_like(image)
    gm = torch.empty(spatial, dtype=torch.float32, device=image.device)
    if workspace is None:
        n = int(lib.ggdt_backward_workspace_bytes(nd, _dims(spatial), C))
        if n == 0:
            raise ValueError(f"invalid shape {spatial} with C={C} for the backward")
        workspace = torch.empty(n, dtype=torch.uint8, device=image.device)
    else:
        _check_workspace(workspace, image.device)
    fn = lib.ggdt2d_backward if nd == 2 else lib.ggdt3d_backward
    rc = fn(_ptr(image), _ptr(records), _ptr(grad_out), _spacing(spacing, nd), float(v), float(lamb),
            int(iterations), _ptr(gi), _ptr(gm), C, *spatial, _ptr(workspace), workspace.numel(), _stream())
    if rc != GGDT_OK:
        raise GGDTError(rc, fn.__name__)
    if check:
        _raise_if_watchdog(workspace, fn.__name__)
    return (gi[0] if squeeze else gi), gm


def workspace_status(workspace) -> int:
    lib = load_library()
    return int(lib.ggdt_workspace_status(_ptr(workspace), _stream()))


def profile_begin(n: int) -> None:
    rc = load_library().ggdt_profile_begin(int(n))
    if rc != GGDT_OK:
        raise GGDTError(rc, "ggdt_profile_begin")


def profile_end(capacity: int):
    """Durations (ms) of the pass kernels launched since profile_begin."""
    buf = (ctypes.c_float * max(1, capacity))()
    n = load_library().ggdt_profile_end(buf, capacity)
    if n < 0:
        raise GGDTError(n, "ggdt_profile_end")
    return [buf[i] for i in range(min(n, capacity))]


def set_spin_limit(polls: int) -> None:
    load_library().ggdt_set_spin_limit(int(polls))


class GGDTFunction(torch.autograd.Function):
    """D = GGDT(image, softmask) with gradients for image and softmask."""

    @staticmethod
    def forward(ctx, image, softmask, spacing, v, lamb, iterations):
        _, sm, spatial = _prep(image.detach(), softmask.detach())
        ws = new_workspace(spatial, 1 if image.dim() == len(spatial) else image.shape[0], sm.device)
        out, rec = ggdt_forward_rec(image.detach(), softmask.detach(), spacing, v, lamb, iterations, workspace=ws)
        ctx.save_for_backward(image.detach(), rec)
        ctx.fwd_workspace = ws
        ctx.params = (tuple(spacing), float(v), float(lamb), int(iterations))
        return out

    @staticmethod
    def backward(ctx, grad_out):
        image, rec = ctx.saved_tensors
        spacing, v, lamb, iterations = ctx.params
        # The forward ran asynchronously: its watchdog word is read now, before
        # its records are trusted.
        _raise_if_watchdog(ctx.fwd_workspace, "GGDTFunction forward")
        gi, gm = ggdt_backward(image, rec, grad_out.contiguous().float(), spacing, v, lamb, iterations, check=True)
        return gi, gm, None, None, None, None


def ggdt_batched(*args, **kwargs):  # defined in batched.py once available
    from . import batched
    return batched.ggdt_batched(*args, **kwargs)


def BatchedPlan(*args, **kwargs):
    from . import batched
    return batched.BatchedPlan(*args, **kwargs)
