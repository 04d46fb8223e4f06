"""Oracle references for the full-size GPU parity tests.

For a workload whose oracle output is stored as a digest (tests/golden/
digests.json, written by tests/golden/make_digests.py from the oracle alone),
the reference is that digest when the regenerated inputs hash to the stored
input digests; otherwise the oracle is run live on this machine's cores (a
thread pool: the oracle's C calls release the GIL).  Either way every output is
compared with the oracle, never with another GPU launch."""
import hashlib
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "digests.json")


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _stored(key):
    with open(GOLDEN) as f:
        return json.load(f).get(key)


def _threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _inputs_match(entry, c, extra=()):
    if not entry or entry["image_sha256"] != sha(c["image"]) or entry["mask_sha256"] != sha(c["mask"]):
        return False
    return all(entry.get(f"{k}_sha256") == sha(c[k]) for k in extra)


def forward_digests(key, cases):
    """Digest of the oracle's FP32 forward for every case (stored or live).
    Returns (digests, number computed live)."""
    stored = _stored(key) or []
    out = [None] * len(cases)
    live = []
    for i, c in enumerate(cases):
        e = stored[i] if i < len(stored) else None
        if _inputs_match(e, c):
            out[i] = e["out_sha256"]
        else:
            live.append(i)

    def run(i):
        c = cases[i]
        return i, sha(oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32"))

    with ThreadPoolExecutor(max_workers=_threads()) as ex:
        for i, d in ex.map(run, live):
            out[i] = d
    return out, len(live)


def gradient_digests(key, cases):
    """Digests of the oracle's FP32 forward, records and reverse pass of
    L = sum(weight * D) for every case (stored or live).  Returns (list of dicts
    with out, records, grad_image, grad_mask, number computed live)."""
    stored = _stored(key) or []
    out = [None] * len(cases)
    live = []
    for i, c in enumerate(cases):
        e = stored[i] if i < len(stored) else None
        if _inputs_match(e, c, extra=("weight",)):
            out[i] = {k: e[f"{k}_sha256"] for k in ("out", "records", "grad_image", "grad_mask")}
        else:
            live.append(i)

    def run(i):
        c = cases[i]
        D, rec = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32",
                             records=True)
        gi, gm = oracle.backward(c["image"], rec, c["weight"], c["spacing"], c["v"], c["lam"], c["iterations"],
                                 "f32")
        return i, {"out": sha(D), "records": sha(rec), "grad_image": sha(gi), "grad_mask": sha(gm)}

    with ThreadPoolExecutor(max_workers=_threads()) as ex:
        for i, d in ex.map(run, live):
            out[i] = d
    return out, len(live)
