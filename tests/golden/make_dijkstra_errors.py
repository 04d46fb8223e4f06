"""Write tests/golden/dijkstra_errors.json: for every benchmark workload (each
lambda), the error of the FP32 directional-pass schedule (which the GPU equals
bit for bit, checked by the parity tests) and of the FP64 schedule against the
FP64 multi-source Dijkstra on the same 8/26-connected grid with the same edge
costs, i.e. the converged transform.  Calls only the oracle and the seeded
input generators.

    python tests/golden/make_dijkstra_errors.py [config1 config2 config3 config4 config5]

Relative error per voxel |D - D*| / D* over the voxels with D* > 0 (hard seeds
have D = D* = 0 exactly); the maximum and the mean are reported, and for
batches the maximum over instances and the voxel-weighted mean.
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2208_00001_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dijkstra_errors.json")


def rel_errors(D, ref):
    D = np.asarray(D, dtype=np.float64)
    sel = ref > 0
    if not sel.any():
        return 0.0, 0.0, 0
    r = np.abs(D[sel] - ref[sel]) / ref[sel]
    return float(r.max()), float(r.mean()), int(sel.sum())


def one_case(c):
    t = time.time()
    dij = oracle.dijkstra(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], "f64")
    d32 = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32")
    d64 = oracle.ggdt(c["image"].astype(np.float64), c["mask"].astype(np.float64), c["spacing"], c["v"], c["lam"],
                      c["iterations"], "f64")
    mx32, mean32, n = rel_errors(d32, dij)
    mx64, mean64, _ = rel_errors(d64, dij)
    return {"name": c["name"], "lambda": c["lam"], "iterations": c["iterations"], "voxels": int(c["mask"].size),
            "voxels_compared": n, "f32_max_rel": mx32, "f32_mean_rel": mean32, "f64_max_rel": mx64,
            "f64_mean_rel": mean64, "seconds": round(time.time() - t, 1)}


def _config4_case(i):
    return one_case(synth.config4()[i])


def _config5_case(i):
    return one_case(synth.config5()[i])


def batch_summary(entries):
    w = np.array([e["voxels_compared"] for e in entries], dtype=np.float64)
    return {"instances": len(entries),
            "f32_max_rel": max(e["f32_max_rel"] for e in entries),
            "f32_mean_rel": float(np.sum(w * [e["f32_mean_rel"] for e in entries]) / max(w.sum(), 1.0)),
            "f64_max_rel": max(e["f64_max_rel"] for e in entries),
            "f64_mean_rel": float(np.sum(w * [e["f64_mean_rel"] for e in entries]) / max(w.sum(), 1.0)),
            "per_instance": entries}


def main(which):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    workers = max(1, min(8, os.cpu_count() or 1))
    if "config1" in which:
        data["config1"] = [one_case(synth.config1(lam)) for lam in (0.0, 1.0)]
        print("config1", data["config1"], flush=True)
    if "config2" in which:
        with ProcessPoolExecutor(max_workers=3) as ex:
            data["config2"] = list(ex.map(one_case, [synth.config2(lam) for lam in (0.0, 0.5, 1.0)]))
        print("config2", data["config2"], flush=True)
    if "config3" in which:
        data["config3"] = [one_case(synth.config3())]
        print("config3", data["config3"], flush=True)
    if "config4" in which:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            entries = list(ex.map(_config4_case, range(len(synth.config4()))))
        data["config4"] = batch_summary(entries)
        print("config4", {k: v for k, v in data["config4"].items() if k != "per_instance"}, flush=True)
    if "config5" in which:
        with ProcessPoolExecutor(max_workers=4) as ex:
            entries = list(ex.map(_config5_case, range(len(synth.config5()))))
        data["config5"] = batch_summary(entries)
        print("config5", {k: v for k, v in data["config5"].items() if k != "per_instance"}, flush=True)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["config1", "config2", "config3", "config4", "config5"])
