"""Benchmark of the GGDT hot path on one MI355X.

A step is one whole forward transform of the 3D workload: a 256^3 fp32 volume
(C = 1), spacing (1, 1, 2.5), a 12^3 hard-seed cube, v = 1e10, lambda = 1,
4 iterations of 6 directional passes, inputs resident in HBM.  The metric is
voxel-updates/s = voxels x directional passes x iterations / time.

Also reported (same JSON line):
  batched       64 ragged 2D/3D instances (48 volumes U[64,192]x U[64,192] x U[64,96],
                16 images U[256,1024]^2, lambda U[0,1], spacing U[0.5,3], 2-4 iterations)
                in one autotuned persistent launch replayed from a HIP graph, vs
                the same instances as 64 plain per-instance calls on one stream
  backward      4 x 128^3 volumes, lambda 0.7, soft mask, 3 iterations: batched
                forward-with-records + batched backward (one launch each) vs
                per-volume forward-with-records + backward launches
  roofline      the directional-pass kernel's algorithmic bytes (12 B per voxel
                update: read I(x), read D_old(x), write D(x)) per launch over its
                average launch duration, timed with HIP events on its stream,
                against the MI355X HBM peak (8 TB/s) and against the measured rate
                of a streaming kernel on 2 GiB; traffic from rocprofv3 counters
                when a summary for the current kernel source exists
  dijkstra_error  relative error of the FP32 schedule against exact (FP64 Dijkstra) distances
                for every workload, from the stored table written by the oracle, after checking
                that this run's output has the oracle's digest
  half          the same volume with its image stored as fp16 and as bf16 (10 B per voxel
                update): time and the change against the fp32 image's result
  toivanen_gpu  Toivanen's raster scan on the GPU (hyperplane sweeps), one iteration of the
                same volume; the CPU leg checks its output against the oracle's sweeps
  converge      the same volume run to its fixed point (iterations and time)
  configs_2d    the 128^2 and 2048^2 x 3 images, voxel-updates/s per lambda
  composed      signed distance and geodesic symmetric filter of the same volume
  cpu_baseline  the CPU oracle (single thread, and OpenMP over each plane) on a bounded sample: one
                iteration (6 passes) of the same volume; Toivanen's scan on one thread

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-updates/s + HBM GB/s vs peak, 3D 256³ GGDT; batched & backward vs plain"
HBM_PEAK_GBS = 8000.0
BYTES_PER_VU = 12  # lambda = 1, C = 1: image(x) 4 + D_old(x) 4 + D(x) 4
# backward, C = 1: record 1 + image(x) 4 + adjoint read 4 / write 4 + image gradient read 4 / write 4
BWD_BYTES_PER_VU = 21
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pass_kernel_3d_256_pmc.json")


# Sources that define and launch the forward pass kernels and the scale kernel
# the counters are calibrated with: a change to any of them makes the stored
# counter summary stale.
PASS_KERNEL_SOURCES = ("forward.hip", "ggdt_internal.h", "pass_cell.h", "pass_device.h")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for name in PASS_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2208_00001_amd", "csrc", name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()


def traffic_from_counters(n_voxels):
    """HBM bytes per pass launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    with open(PMC_SUMMARY) as f:
        s = json.load(f)
    if s.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return s.get("hbm_bytes_per_pass_launch")


def cpu_baseline(c, toiv_gpu=None):
    import oracle
    t = time.perf_counter()
    oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], 1, "f32")
    dt = time.perf_counter() - t
    vu = c["mask"].size * 6
    out = {"value": vu / dt, "unit": "voxel-updates/s", "cores": 1, "kind": "oracle",
           "sample": f"1 iteration (6 passes) of the {c['name']} volume, {vu} voxel-updates in {dt:.1f} s",
           "cpu": cpu_model()}
    # The paper's CPU scheme: the same oracle with each plane's voxels shared
    # among OpenMP threads (OMP_NUM_THREADS, else every host core).
    t = time.perf_counter()
    _, threads = oracle.ggdt_omp(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], 1)
    dt = time.perf_counter() - t
    out["openmp"] = {"value": vu / dt, "unit": "voxel-updates/s", "cores": threads,
                     "sample": f"the same iteration in {dt:.2f} s"}
    out["toivanen"] = toivanen_comparison(c, toiv_gpu)
    return out


def toivanen_comparison(c, toiv_gpu=None):
    """Toivanen's sequential raster scan (the paper's comparison method, one
    thread): its rate on one iteration of the volume (two raster sweeps over
    half of the 26-neighbourhood), and the iterations each method needs to
    reach its fixed point on smaller synthetic inputs."""
    import oracle
    from paper_2208_00001_amd import synth
    t = time.perf_counter()
    ref = oracle.toivanen(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], 1, "f32")
    dt = time.perf_counter() - t
    res = {"voxel_visits_per_s": 2 * c["mask"].size / dt, "cores": 1,
           "sample": f"1 iteration (2 sweeps) of the {c['name']} volume in {dt:.1f} s", "iterations_to_fixed_point": {}}
    if toiv_gpu is not None:
        res["gpu_output_equals_oracle"] = bool((toiv_gpu.view("u4") == ref.view("u4")).all())
    for cc in (synth.config1(1.0), synth.config1(0.0), synth.config3(size=64)):
        _, n_scan = oracle.until_converged(cc["image"], cc["mask"], cc["spacing"], cc["v"], cc["lam"])
        _, n_toiv = oracle.toivanen(cc["image"], cc["mask"], cc["spacing"], cc["v"], cc["lam"], 10000, "f32",
                                    converge=True)
        nd = cc["mask"].ndim
        res["iterations_to_fixed_point"][cc["name"]] = {
            "directional_scan": n_scan, "directional_passes": n_scan * 2 * nd,
            "toivanen": n_toiv, "toivanen_sweeps": n_toiv * 2}
    return res


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def calibrate_copy(mib):
    """One launch of the scale kernel over a (mib MiB) volume: reads the mask and
    writes the output once each, a plain streaming copy of known size."""
    import torch

    from paper_2208_00001_amd import binding as B

    dev = "cuda:0"
    plane = 512 * 512
    n = max(1, mib * 2**20 // 4 // plane) * plane
    shape = (n // plane, 512, 512)
    src = torch.rand(shape, device=dev)
    dst = torch.empty(shape, device=dev)
    ws = B.new_workspace(shape, 1, dev)
    torch.cuda.synchronize()
    B.ggdt3d(src, src, (1.0, 1.0, 1.0), 2.0, 1.0, 0, out=dst, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(dst, src * 2.0)
    return {"kernel": "scale_kernel", "bytes_read": 4 * n, "bytes_written": 4 * n}


def copy_bandwidth(gib=2, reps=5):
    """GB/s of the library's streaming scale kernel (read 4 B + write 4 B per
    element) over a buffer larger than the 256 MB memory-side cache: the
    achievable HBM rate that the pass kernel's algorithmic rate is compared to."""
    import torch

    from paper_2208_00001_amd import binding as B

    dev = "cuda:0"
    plane = 512 * 512
    n = gib * 2**30 // 4 // plane * plane
    shape = (n // plane, 512, 512)
    src = torch.ones(shape, device=dev)
    dst = torch.empty(shape, device=dev)
    ws = B.new_workspace(shape, 1, dev)

    def run():
        B.ggdt3d(src, src, (1.0, 1.0, 1.0), 1.0, 1.0, 0, out=dst, workspace=ws)

    run()
    ms = _time(run, reps)
    del src, dst
    torch.cuda.empty_cache()
    return {"kernel": "scale_kernel (D = v*M)", "bytes": 8 * n, "ms": ms, "gbs": 8 * n / (ms * 1e-3) / 1e9}


def bench_small_configs(reps=5):
    """Voxel-updates/s of the 2D configurations (reported, not targeted): the
    128^2 correctness case and the 2048^2 x 3-channel case, per lambda."""
    import numpy as np
    import torch

    from paper_2208_00001_amd import binding as B
    from paper_2208_00001_amd import synth

    dev = "cuda:0"
    res = {}
    for name, cases in (("2d-128^2-c1", [synth.config1(lam) for lam in (0.0, 1.0)]),
                        ("2d-2048^2-c3", [synth.config2(lam) for lam in (0.0, 0.5, 1.0)])):
        for c in cases:
            img = torch.from_numpy(c["image"]).to(dev)
            m = torch.from_numpy(c["mask"]).to(dev)
            out = torch.empty_like(m)
            ws = B.new_workspace(tuple(m.shape), img.shape[0] if img.dim() > m.dim() else 1, dev)

            def run():
                B.ggdt2d(img, m, c["spacing"], c["v"], c["lam"], c["iterations"], out=out, workspace=ws)

            run()
            ms = _time(run, reps)
            vu = int(np.prod(m.shape)) * 4 * c["iterations"]
            res[f"{name}-lam{c['lam']:g}"] = {"ms": ms, "value": vu / (ms * 1e-3), "unit": "voxel-updates/s"}
    return res


def bench_converge(c, reps=3):
    """The 3D volume run to its fixed point (the exact grid shortest-path
    distance): iterations needed and time."""
    import numpy as np
    import torch

    from paper_2208_00001_amd import binding as B

    dev = "cuda:0"
    img = torch.from_numpy(c["image"]).to(dev)
    m = torch.from_numpy(c["mask"]).to(dev)
    out = torch.empty_like(m)
    ws = B.new_workspace(tuple(m.shape), 1, dev)
    _, n = B.ggdt_converge(img, m, c["spacing"], c["v"], c["lam"], 200, out=out, workspace=ws)
    ms = _time(lambda: B.ggdt_converge(img, m, c["spacing"], c["v"], c["lam"], 200, out=out, workspace=ws), reps)
    vu = int(np.prod(m.shape)) * 6 * (n + 1)
    return {"workload": c["name"] + " to its fixed point", "iterations_changing": n,
            "iterations_run": n + 1, "ms": ms, "voxel_updates": vu, "value": vu / (ms * 1e-3),
            "unit": "voxel-updates/s"}


def _time(fn, reps):
    import torch
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def bench_batched(reps):
    import numpy as np
    import torch

    from paper_2208_00001_amd import binding as B
    from paper_2208_00001_amd import synth, tune
    from paper_2208_00001_amd.batched import BatchedPlan

    dev = "cuda:0"
    cases = synth.config4()
    inst = [dict(image=torch.from_numpy(c["image"]).to(dev), softmask=torch.from_numpy(c["mask"]).to(dev),
                 spacing=c["spacing"], v=c["v"], lam=c["lam"], iterations=c["iterations"]) for c in cases]
    vu = sum(int(np.prod(c["mask"].shape)) * 2 * c["mask"].ndim * c["iterations"] for c in cases)
    best = tune.tune(inst, use_cache=False)
    plan = BatchedPlan(inst, best["tuning"])
    plan.capture()
    plan.replay()
    ms_b = _time(plan.replay, reps)
    assert plan.status() == 0, "watchdog fired (batched)"
    outs = [torch.empty_like(d["softmask"]) for d in inst]
    wss = [B.new_workspace(tuple(d["softmask"].shape), 1, dev) for d in inst]

    def plain():
        for d, c, o, w in zip(inst, cases, outs, wss):
            fn = B.ggdt3d if c["mask"].ndim == 3 else B.ggdt2d
            fn(d["image"], d["softmask"], c["spacing"], c["v"], c["lam"], c["iterations"], out=o, workspace=w)

    plain()
    ms_p = _time(plain, reps)
    same = all(torch.equal(o, b) for o, b in zip(outs, plan.outputs))
    plan.close()
    gbs = BYTES_PER_VU * vu / (ms_b * 1e-3) / 1e9
    return {"workload": "64 ragged instances (48 3D + 16 2D), lambda U[0,1], 2-4 iterations",
            "voxel_updates": vu, "batched_ms": ms_b, "plain_ms": ms_p, "speedup": ms_p / ms_b,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "bytes_per_voxel_update": BYTES_PER_VU,
                         "note": "whole batched launch (graph replay), algorithmic bytes"},
            "batched_value": vu / (ms_b * 1e-3), "plain_value": vu / (ms_p * 1e-3), "unit": "voxel-updates/s",
            "tuning": best["tuning"], "tuning_trials": best["trials"], "outputs_identical": same}


def bench_backward(reps):
    import numpy as np
    import torch

    from paper_2208_00001_amd import binding as B
    from paper_2208_00001_amd import synth
    from paper_2208_00001_amd.batched import BatchedPlan

    dev = "cuda:0"
    cases = synth.config5()
    inst = [dict(image=torch.from_numpy(c["image"]).to(dev), softmask=torch.from_numpy(c["mask"]).to(dev),
                 spacing=c["spacing"], v=c["v"], lam=c["lam"], iterations=c["iterations"], records=True,
                 grad_out=torch.from_numpy(c["weight"]).to(dev)) for c in cases]
    vu = sum(int(np.prod(c["mask"].shape)) * 6 * c["iterations"] for c in cases)
    plan = BatchedPlan(inst)

    def batched():
        plan.run()
        plan.backward()

    def plain():
        for d, c in zip(inst, cases):
            out, rec = B.ggdt_forward_rec(d["image"], d["softmask"], c["spacing"], c["v"], c["lam"], c["iterations"])
            B.ggdt_backward(d["image"], rec, d["grad_out"], c["spacing"], c["v"], c["lam"], c["iterations"])

    batched()
    plain()
    ms_b = _time(batched, reps)
    ms_p = _time(plain, reps)
    ms_bf = _time(plan.run, reps)
    ms_bb = _time(plan.backward, reps)
    assert plan.status() == 0, "watchdog fired (backward)"
    plan.close()
    gbs = BWD_BYTES_PER_VU * vu / (ms_bb * 1e-3) / 1e9
    return {"workload": "4 x 128^3, lambda 0.7, soft mask, v 10, 3 iterations, L = sum(W * D)",
            "voxel_updates_forward": vu, "batched_fwd_bwd_ms": ms_b, "plain_fwd_bwd_ms": ms_p,
            "speedup": ms_p / ms_b, "batched_forward_ms": ms_bf, "batched_backward_ms": ms_bb,
            "unit": "ms per forward+backward",
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "bytes_per_voxel_update": BWD_BYTES_PER_VU,
                         "note": "batched backward launch, algorithmic bytes"}}


def bench_composed(c, reps):
    """Signed distance (2 transforms) and geodesic symmetric filter (6) of the
    benchmark volume; voxel-updates count every pass of every transform."""
    import numpy as np
    import torch
    from paper_2208_00001_amd import binding as B
    dev = "cuda:0"
    shape = c["mask"].shape
    img = torch.from_numpy(c["image"]).to(dev)
    m = torch.from_numpy(c["mask"]).to(dev)
    out = torch.empty(shape, dtype=torch.float32, device=dev)
    lib = B.load_library()
    dims = B._dims(shape)
    vu1 = int(np.prod(shape)) * 6 * c["iterations"]
    res = {"workload": f"{c['name']}, signed distance and GSF (theta_d 8, theta_e 4)"}
    for kind, q, ntr, run in (
            ("signed", lib.ggdt_signed_workspace_bytes, 2,
             lambda ws: B.ggdt_signed(img, m, c["spacing"], c["v"], c["lam"], c["iterations"], out=out,
                                      workspace=ws)),
            ("gsf", lib.ggdt_gsf_workspace_bytes, 6,
             lambda ws: B.ggdt_gsf(img, m, 8.0, 4.0, c["spacing"], c["v"], c["lam"], c["iterations"], out=out,
                                   workspace=ws))):
        ws = torch.empty(int(q(3, dims, 1)), dtype=torch.uint8, device=dev)
        run(ws)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            run(ws)
        b.record()
        torch.cuda.synchronize()
        assert B.workspace_status(ws) == 0, f"watchdog fired ({kind})"
        ms = a.elapsed_time(b) / reps
        res[kind] = {"ms": ms, "transforms": ntr, "ms_per_transform": ms / ntr,
                     "value": ntr * vu1 / (ms * 1e-3), "unit": "voxel-updates/s"}
    return res


def dijkstra_error(out):
    """Error of each workload's transform against the FP64 multi-source Dijkstra
    (the converged transform), from tests/golden/dijkstra_errors.json (written
    by the oracle alone).  Those are the oracle's FP32 outputs, which the GPU
    equals bit for bit: checked here for the benchmark volume through the stored
    oracle digest of this very output."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "dijkstra_errors.json")
    dig = os.path.join(ROOT, "tests", "golden", "digests.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    res = {}
    for key, val in sorted(table.items()):
        entries = val if isinstance(val, list) else [dict(val, name=f"{val['instances']} instances")]
        res[key] = [{"workload": e["name"], "lambda": e.get("lambda"), "max_rel": e["f32_max_rel"],
                     "mean_rel": e["f32_mean_rel"], "fp64_schedule_max_rel": e["f64_max_rel"]} for e in entries]
    with open(dig) as f:
        want = json.load(f)["config3"]["out_sha256"]
    got = hashlib.sha256(np.ascontiguousarray(out.cpu().numpy()).tobytes()).hexdigest()
    res["benchmark_output_equals_oracle"] = got == want
    return res


def bench_half(c, img, m, out32, reps):
    """The benchmark volume with its image stored in 16 bits (10 bytes per voxel
    update instead of 12), as IEEE binary16 and as bfloat16: time per transform,
    and the difference from the fp32 image's result (the effect of rounding the
    image; bfloat16's 8 significant bits are coarse for the small intensity
    steps of a smooth volume at lambda = 1)."""
    import numpy as np
    import torch

    from paper_2208_00001_amd import binding as B
    dev = img.device
    N = int(np.prod(tuple(m.shape)))
    vu = N * 6 * c["iterations"]
    ref = out32.double()
    sel = ref > 0
    res = {"workload": c["name"] + " with a 16-bit image", "bytes_per_voxel_update": 10, "unit": "voxel-updates/s"}
    for name, dtype in (("f16", torch.float16), ("bf16", torch.bfloat16)):
        img16 = img.to(dtype)
        out = torch.empty_like(out32)
        ws = B.new_workspace(tuple(m.shape), 1, dev)

        def run():
            B.ggdt_half(img16, m, c["spacing"], c["v"], c["lam"], c["iterations"], out=out, workspace=ws)

        ms = _time(run, reps)
        assert B.workspace_status(ws) == 0, f"watchdog fired ({name} image)"
        rel = (out.double() - ref).abs()[sel] / ref[sel]
        res[name] = {"ms": ms, "value": vu / (ms * 1e-3), "algorithmic_gbs": 10 * vu / (ms * 1e-3) / 1e9,
                     "rel_diff_vs_fp32_image": {"max": float(rel.max()), "mean": float(rel.mean())}}
    return res


def bench_toivanen(c, img, m, reps):
    """Toivanen's raster scan on the GPU (hyperplane sweeps, one persistent
    launch) on the benchmark volume: one iteration (a forward and a backward
    sweep over half of the 26-neighbourhood each).  Returns the line's entry and
    the output, which the CPU leg compares with the oracle's sequential sweeps."""
    import numpy as np
    import torch

    from paper_2208_00001_amd import binding as B
    out = torch.empty_like(m)
    ws = B.new_workspace(tuple(m.shape), 1, img.device, minimal=True)

    def run():
        B.ggdt_toivanen(img, m, c["spacing"], c["v"], c["lam"], 1, out=out, workspace=ws)

    ms = _time(run, reps)
    assert B.workspace_status(ws) == 0, "watchdog fired (Toivanen)"
    N = int(np.prod(tuple(m.shape)))
    res = {"workload": c["name"] + ", Toivanen's raster scan, 1 iteration (2 sweeps)", "ms": ms,
           "voxel_visits_per_s": 2 * N / (ms * 1e-3),
           "hyperplanes_per_sweep": 4 * (m.shape[0] - 1) + 2 * (m.shape[1] - 1) + (m.shape[2] - 1) + 1}
    return res, out.cpu().numpy()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched and backward comparisons")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the measurements, run the elementwise scale kernel (D = v*M, zero iterations) once "
                         "over a MIB-sized volume: one read and one write of known size, the reference for scaling "
                         "HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this path has no multi-GPU mode (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2208_00001_amd import binding as B
    from paper_2208_00001_amd import synth

    B.load_library()
    dev = "cuda:0"
    c = synth.config3()
    shape = c["mask"].shape
    N = int(np.prod(shape))
    passes = 6 * c["iterations"]
    img = torch.from_numpy(c["image"]).to(dev)
    m = torch.from_numpy(c["mask"]).to(dev)
    out = torch.empty(shape, dtype=torch.float32, device=dev)
    ws = B.new_workspace(shape, 1, dev)

    def step():
        B.ggdt3d(img, m, c["spacing"], c["v"], c["lam"], c["iterations"], out=out, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert B.workspace_status(ws) == 0, "watchdog fired during warmup"

    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        step()
    end.record()
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(end)
    assert B.workspace_status(ws) == 0, "watchdog fired during the timed steps"
    ms_per_step = ms_total / args.steps
    vu_per_step = N * passes
    value = vu_per_step / (ms_per_step * 1e-3)

    # Pass-kernel durations: HIP events around each pass launch, on the launch stream.
    B.profile_begin(args.steps * passes)
    for _ in range(args.steps):
        step()
    durs = B.profile_end(args.steps * passes)
    torch.cuda.synchronize()
    avg_ms_events = float(np.mean(durs))
    # The event pairs around each launch add a little time of their own: the
    # per-launch figure is capped by the clean timed window's share per pass.
    avg_ms = min(avg_ms_events, ms_per_step / passes)
    achieved = BYTES_PER_VU * N / (avg_ms * 1e-3) / 1e9
    traffic = traffic_from_counters(N)

    copy = copy_bandwidth()

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": c["name"], "shape": list(shape), "channels": 1, "lambda": c["lam"], "v": c["v"],
                   "spacing": list(c["spacing"]), "iterations": c["iterations"], "directional_passes": passes,
                   "voxel_updates_per_step": vu_per_step, "seed": c["seed"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "copy_gbs": copy["gbs"], "frac_of_copy": achieved / copy["gbs"],
                     "kernel": "directional pass (3D, lambda=1 C=1 path)", "bytes_per_voxel_update": BYTES_PER_VU,
                     "launches_timed": len(durs), "avg_launch_ms": avg_ms, "avg_launch_ms_events": avg_ms_events},
        "dijkstra_error": dijkstra_error(out),
    }
    line["half"] = bench_half(c, img, m, out, max(3, min(args.steps, 10)))
    line["toivanen_gpu"], toiv_out = bench_toivanen(c, img, m, 3)
    if not args.no_batched:
        line["converge"] = bench_converge(c)
        line["configs_2d"] = bench_small_configs()
        line["batched"] = bench_batched(max(3, min(args.steps, 10)))
        line["backward"] = bench_backward(max(3, min(args.steps, 10)))
        line["composed"] = bench_composed(c, 3)
    if args.calibrate_copy > 0:
        line["calibration"] = calibrate_copy(args.calibrate_copy)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(c, toiv_out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
