"""Batched ragged GGDT: many 2D/3D instances of uneven size in one persistent
launch (ggdt_batched_plan / ggdt_batched_run), optionally captured in a HIP
graph.  Marshalling only; the work runs in libggdt.so."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from .binding import (GGDT_OK, GGDTError, GGDTInstance, GGDTTuning, _check_out, _check_records, _prep,
                      _ptr, _raise_if_watchdog, _stream, load_library)


class BatchedPlan:
    """A plan over a list of instances.  Each instance is a dict with
    image ((C,) + spatial or spatial), softmask (spatial), spacing, v, lam, iterations
    and optionally out (preallocated D) and records (True to allocate a records
    tensor, or a uint8 tensor).  Tensors must stay alive as long as the plan."""

    def __init__(self, instances: Sequence[dict], tuning: Optional[dict] = None):
        self.lib = load_library()
        n = len(instances)
        if n == 0:
            raise ValueError("empty batch")
        arr = (GGDTInstance * n)()
        self.inst = []
        for i, d in enumerate(instances):
            img, m, spatial = _prep(d["image"], d["softmask"])
            if m.device != instances[0]["softmask"].device:
                raise ValueError(f"instance {i} is on {m.device}, instance 0 on {instances[0]['softmask'].device}")
            out = d.get("out")
            if out is None:
                out = torch.empty(spatial, dtype=torch.float32, device=m.device)
            else:
                _check_out(out, spatial, m.device, what=f"instance {i} out")
            rec = d.get("records")
            if rec is True:
                rec = torch.empty((d["iterations"] * 2 * len(spatial),) + spatial, dtype=torch.uint8, device=m.device)
            elif rec is False:
                rec = None
            elif rec is not None:
                _check_records(rec, spatial, d["iterations"], m.device)
            nd = len(spatial)
            e = arr[i]
            e.ndim, e.C = nd, img.shape[0]
            for b in range(3):
                e.dims[b] = spatial[b] if b < nd else 1
            e.image, e.softmask, e.out = img.data_ptr(), m.data_ptr(), out.data_ptr()
            sp = tuple(float(s) for s in d["spacing"])
            for b in range(3):
                e.spacing[b] = sp[b] if b < nd else 1.0
            e.v, e.lam, e.iterations = float(d["v"]), float(d["lam"]), int(d["iterations"])
            e.records = rec.data_ptr() if rec is not None else None
            go = d.get("grad_out")
            gi = gm = None
            if go is not None:
                _check_out(go.contiguous(), spatial, m.device, what=f"instance {i} grad_out")
                go = go.contiguous()
                gi = torch.empty_like(img)
                gm = torch.empty(spatial, dtype=torch.float32, device=m.device)
            e.grad_out = go.data_ptr() if go is not None else None
            e.grad_image = gi.data_ptr() if gi is not None else None
            e.grad_softmask = gm.data_ptr() if gm is not None else None
            self.inst.append(dict(image=img, softmask=m, out=out, records=rec, spacing=sp, v=float(d["v"]),
                                  lam=float(d["lam"]), iterations=int(d["iterations"]), grad_out=go, grad_image=gi,
                                  grad_softmask=gm))
        self._arr = arr
        tun = None
        if tuning:
            tun = GGDTTuning(int(tuning.get("tile_p", 0)), int(tuning.get("tile_q", 0)), int(tuning.get("chunk", 0)),
                             int(tuning.get("wg_per_cu", 0)))
        self.tuning = dict(tuning or {})
        plan = ctypes.c_void_p()
        wsb = ctypes.c_size_t()
        rc = self.lib.ggdt_batched_plan(ctypes.byref(arr), n, ctypes.byref(tun) if tun else None, ctypes.byref(plan),
                                        ctypes.byref(wsb))
        if rc != GGDT_OK:
            raise GGDTError(rc, "ggdt_batched_plan")
        self._plan = plan
        self.workspace = torch.empty(int(wsb.value), dtype=torch.uint8, device=instances[0]["softmask"].device)
        self.graph = None

    @property
    def outputs(self):
        return [d["out"] for d in self.inst]

    @property
    def records(self):
        return [d["records"] for d in self.inst]

    def run(self):
        rc = self.lib.ggdt_batched_run(self._plan, _ptr(self.workspace), self.workspace.numel(), _stream())
        if rc != GGDT_OK:
            raise GGDTError(rc, "ggdt_batched_run")
        return self.outputs

    def backward(self):
        """Reverse of every instance's recorded schedule in one launch: fills each
        instance's grad_image and grad_softmask from its grad_out (read at call time)."""
        rc = self.lib.ggdt_batched_backward(self._plan, _ptr(self.workspace), self.workspace.numel(), _stream())
        if rc != GGDT_OK:
            raise GGDTError(rc, "ggdt_batched_backward")
        return [(d["grad_image"], d["grad_softmask"]) for d in self.inst]

    def capture(self) -> torch.cuda.CUDAGraph:
        """Capture run() into a HIP graph (replay with .replay())."""
        self.run()  # warm (kernel attributes, code objects)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()
        return self.outputs

    def info(self) -> dict:
        n, g, bg = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        l, bl = ctypes.c_size_t(), ctypes.c_size_t()
        self.lib.ggdt_plan_info(self._plan, ctypes.byref(n), ctypes.byref(g), ctypes.byref(bg), ctypes.byref(l),
                                ctypes.byref(bl))
        return {"instances": n.value, "grid": g.value, "bwd_grid": bg.value, "lds": l.value, "bwd_lds": bl.value}

    def status(self) -> int:
        return int(self.lib.ggdt_workspace_status(_ptr(self.workspace), _stream()))

    def close(self):
        if getattr(self, "_plan", None):
            self.lib.ggdt_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self):
        """Synchronise and raise GGDTError if an inter-workgroup wait of the last
        run or backward expired (the watchdog): the results are then invalid."""
        _raise_if_watchdog(self.workspace, "batched launch")


def ggdt_batched(instances: Sequence[dict], tuning: Optional[dict] = None):
    """Run a ragged batch once; returns the list of distance maps.  Synchronises,
    and raises GGDTError if the watchdog fired."""
    plan = BatchedPlan(instances, tuning)
    out = plan.run()
    plan.check()
    plan.close()
    return out
