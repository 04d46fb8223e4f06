"""Write tests/golden/digests.json: SHA-256 digests of the CPU oracle's FP32 outputs
on the full-size synthetic workloads (for the 4 x 128^3 gradient workload also
the records and the FP32 reverse pass), plus digests of the inputs they were
computed from.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_digests.py [config3] [config4] [config5]

A GPU test whose input digests match compares the GPU output's digest with the
stored one (bitwise parity); if inputs differ it recomputes with the oracle.
"""
from __future__ import annotations

import hashlib
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "digests.json")


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def entry(c):
    t = time.time()
    D = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32")
    return {
        "name": c["name"], "seed": c["seed"], "shape": list(c["mask"].shape),
        "image_sha256": sha(c["image"]), "mask_sha256": sha(c["mask"]), "out_sha256": sha(D),
        "out_sum": float(D.astype(np.float64).sum()), "oracle_seconds": round(time.time() - t, 2),
    }


def _config4_entry(i):
    return entry(synth.config4()[i])


def config5_entry(c):
    """Forward with records and the FP32 reverse pass of L = sum(W * D)."""
    t = time.time()
    D, rec = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32",
                         records=True)
    gi, gm = oracle.backward(c["image"], rec, c["weight"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32")
    return {
        "name": c["name"], "seed": c["seed"], "shape": list(c["mask"].shape),
        "image_sha256": sha(c["image"]), "mask_sha256": sha(c["mask"]), "weight_sha256": sha(c["weight"]),
        "out_sha256": sha(D), "records_sha256": sha(rec), "grad_image_sha256": sha(gi), "grad_mask_sha256": sha(gm),
        "out_sum": float(D.astype(np.float64).sum()), "oracle_seconds": round(time.time() - t, 2),
    }


def _config5_entry(i):
    return config5_entry(synth.config5()[i])


def main(which):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    if "config3" in which:
        data["config3"] = entry(synth.config3())
        print("config3", data["config3"], flush=True)
    if "config4" in which:
        n = len(synth.config4())
        with ProcessPoolExecutor(max_workers=max(1, min(6, os.cpu_count() or 1))) as ex:
            data["config4"] = list(ex.map(_config4_entry, range(n)))
        print("config4", len(data["config4"]), "instances", flush=True)
    if "config5" in which:
        with ProcessPoolExecutor(max_workers=4) as ex:
            data["config5"] = list(ex.map(_config5_entry, range(len(synth.config5()))))
        print("config5", [e["out_sha256"][:12] for e in data["config5"]], flush=True)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["config3"])
