"""GPU backward (reverse of the recorded schedule) vs the CPU oracle.

The kernels accumulate every adjoint in the same order as the oracle's FP32
reverse pass, so dL/dI and dL/dM are expected bitwise equal (the bar is 1e-5
relative).  The oracle's FP64 gradient is pinned to central finite differences
in test_oracle.py; here the GPU gradient is also checked against FP64 central
differences directly, away from argmin ties."""
import numpy as np
import pytest
import torch

import oracle
import oracle_ref
from gpu_util import assert_parity, to_dev, to_host
from paper_2208_00001_amd import synth

pytestmark = pytest.mark.gpu

CASES = [((23, 31, 19), 1, 0.7, 2), ((17, 40, 36), 1, 1.0, 2), ((30, 21, 18), 1, 0.0, 1), ((19, 26, 33), 2, 0.4, 1),
         ((300, 270), 1, 0.7, 2), ((270, 300), 2, 0.5, 2), ((1, 40, 37), 1, 0.6, 1), ((33, 1, 20), 1, 1.0, 2),
         ((5, 6, 7), 1, 0.8, 3), ((64, 17, 35), 3, 0.3, 1)]


def gpu_fwd_bwd(c, W):
    from paper_2208_00001_amd import binding as B
    img, m = to_dev(c["image"]), to_dev(c["mask"])
    out, rec = B.ggdt_forward_rec(img, m, c["spacing"], c["v"], c["lam"], c["iterations"])
    gi, gm = B.ggdt_backward(img, rec, to_dev(W), c["spacing"], c["v"], c["lam"], c["iterations"])
    return to_host(out), to_host(rec), to_host(gi), to_host(gm)


@pytest.mark.parametrize("shape,C,lam,it", CASES, ids=lambda v: str(v))
def test_backward_matches_oracle_f32(shape, C, lam, it):
    c = synth.small_case(shape, C=C, seed=700 + len(shape) * 7 + C, lam=lam, iterations=it, soft=True, v=10.0)
    W = np.random.default_rng(701).standard_normal(shape).astype(np.float32)
    print(f"case {c['name']} lam={c['lam']} it={it}", flush=True)
    out, rec, gi, gm = gpu_fwd_bwd(c, W)
    ref, ref_rec = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], it, "f32", records=True)
    assert np.array_equal(out, ref) and np.array_equal(rec, ref_rec)
    rgi, rgm = oracle.backward(c["image"], ref_rec, W, c["spacing"], c["v"], c["lam"], it, "f32")
    assert assert_parity(gm, rgm, what="dL/dM"), "dL/dM not bitwise"
    assert assert_parity(gi.reshape(rgi.shape), rgi, what="dL/dI"), "dL/dI not bitwise"


@pytest.mark.parametrize("shape,lam,it", [((23, 31, 19), 0.7, 2), ((9, 40, 66), 1.0, 1), ((30, 21, 130), 0.4, 2)],
                         ids=lambda v: str(v))
def test_records_and_backward_scan_major_and_in_place(shape, lam, it):
    """Single-channel volumes: the forward with records and the backward with
    their full workspaces (the last-axis passes and their reverses on
    scan-major copies, records moved to the array layout) and with the minimal
    ones (in place) both give the oracle's records and gradients bit for bit."""
    from paper_2208_00001_amd import binding as B
    c = synth.small_case(shape, C=1, seed=720 + sum(shape), lam=lam, iterations=it, soft=True, v=10.0)
    W = np.random.default_rng(721).standard_normal(shape).astype(np.float32)
    ref, ref_rec = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], lam, it, "f32", records=True)
    rgi, rgm = oracle.backward(c["image"], ref_rec, W, c["spacing"], c["v"], lam, it, "f32")
    img, m = to_dev(c["image"]), to_dev(c["mask"])
    nd = (3 * __import__("ctypes").c_int)(*shape)
    lib = B.load_library()
    assert lib.ggdt_backward_workspace_bytes(3, nd, 1) > lib.ggdt_backward_workspace_min_bytes(3, nd, 1)
    for minimal in (False, True):
        print(f"case {shape} lam={lam} it={it} minimal={minimal}", flush=True)
        ws = B.new_workspace(shape, 1, img.device, minimal=minimal)
        out, rec = B.ggdt_forward_rec(img, m, c["spacing"], c["v"], lam, it, workspace=ws, check=True)
        nb = (lib.ggdt_backward_workspace_min_bytes if minimal else lib.ggdt_backward_workspace_bytes)(3, nd, 1)
        bws = torch.empty(int(nb), dtype=torch.uint8, device=img.device)
        gi, gm = B.ggdt_backward(img, rec, to_dev(W), c["spacing"], c["v"], lam, it, workspace=bws, check=True)
        assert np.array_equal(to_host(out), ref) and np.array_equal(to_host(rec), ref_rec), f"minimal={minimal}"
        assert assert_parity(to_host(gm), rgm, what="dL/dM"), f"dL/dM not bitwise, minimal={minimal}"
        assert assert_parity(to_host(gi).reshape(rgi.shape), rgi, what="dL/dI"), f"dL/dI not bitwise, minimal={minimal}"


def test_autograd_function():
    from paper_2208_00001_amd.binding import GGDTFunction
    c = synth.small_case((20, 24, 22), C=1, seed=702, lam=0.7, iterations=2, soft=True, v=10.0)
    W = np.random.default_rng(703).standard_normal(c["mask"].shape).astype(np.float32)
    img = to_dev(c["image"][0]).requires_grad_(True)
    m = to_dev(c["mask"]).requires_grad_(True)
    D = GGDTFunction.apply(img, m, c["spacing"], c["v"], c["lam"], c["iterations"])
    (D * to_dev(W)).sum().backward()
    _, rec = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], 2, "f32", records=True)
    rgi, rgm = oracle.backward(c["image"], rec, W, c["spacing"], c["v"], c["lam"], 2, "f32")
    assert np.array_equal(to_host(m.grad), rgm)
    assert np.array_equal(to_host(img.grad), rgi[0])


def test_gpu_gradient_vs_central_differences():
    """FP64 central differences (eps = 1e-3 on M and on I) on voxels whose FP64
    records do not change under +-eps; GPU FP32 gradient within 1e-3 relative."""
    c = synth.small_case((14, 15, 13), C=1, seed=704, lam=0.7, iterations=3, soft=True, v=10.0)
    W = np.random.default_rng(705).standard_normal(c["mask"].shape)
    _, _, gi, gm = gpu_fwd_bwd(c, W.astype(np.float32))
    img = c["image"].astype(np.float64)
    msk = c["mask"].astype(np.float64)

    def loss(i2, m2):
        D, rec = oracle.ggdt(i2, m2, c["spacing"], c["v"], c["lam"], 3, "f64", records=True)
        return float(np.sum(W * D)), rec

    _, rec0 = loss(img, msk)
    rgi64, rgm64 = oracle.backward(img, rec0, W, c["spacing"], c["v"], c["lam"], 3, "f64")
    rng = np.random.default_rng(706)
    eps = 1e-3
    checked = 0
    for _ in range(120):
        idx = tuple(int(rng.integers(0, s)) for s in msk.shape)
        for which in ("M", "I"):
            vals, same = [], True
            for sgn in (1, -1):
                i2, m2 = img.copy(), msk.copy()
                if which == "M":
                    m2[idx] += sgn * eps
                else:
                    i2[(0,) + idx] += sgn * eps
                L, rec = loss(i2, m2)
                same &= np.array_equal(rec, rec0)
                vals.append(L)
            if not same:
                continue
            fd = (vals[0] - vals[1]) / (2 * eps)
            an64 = rgm64[idx] if which == "M" else rgi64[(0,) + idx]
            an = gm[idx] if which == "M" else gi.reshape(img.shape)[(0,) + idx]
            if abs(an - an64) > 1e-4 * max(abs(an64), 1.0):
                continue  # FP32 and FP64 schedules took different argmins on this voxel's paths
            assert abs(an - fd) <= 1e-3 * abs(fd) + 1e-3, (which, idx, an, fd)
            checked += 1
    assert checked >= 100


def test_config5_batched_forward_backward():
    """4 x 128^3, lambda 0.7, soft mask, v = 10: one batched forward (with records)
    and one batched backward; for every volume the forward, the records, dL/dI and
    dL/dM equal the oracle's FP32 forward and reverse pass bit for bit (stored
    digests, or a live oracle run when the regenerated inputs differ), and the
    single-instance launches give the same bits."""
    from paper_2208_00001_amd import binding as B
    from paper_2208_00001_amd.batched import BatchedPlan
    cases = synth.config5()
    ref, nlive = oracle_ref.gradient_digests("config5", cases)
    print(f"config5: {len(cases)} volumes, {nlive} oracle references computed live", flush=True)
    inst = [dict(image=to_dev(c["image"]), softmask=to_dev(c["mask"]), spacing=c["spacing"], v=c["v"], lam=c["lam"],
                 iterations=c["iterations"], records=True, grad_out=to_dev(c["weight"])) for c in cases]
    plan = BatchedPlan(inst)
    print("plan", plan.info(), flush=True)
    plan.run()
    assert plan.status() == 0, "watchdog fired in the batched forward"
    grads = plan.backward()
    torch.cuda.synchronize()
    assert plan.status() == 0, "watchdog fired in the batched backward"
    for k, (c, d) in enumerate(zip(cases, plan.inst)):
        got = {"out": to_host(d["out"]), "records": to_host(d["records"]),
               "grad_image": to_host(grads[k][0]).reshape(c["image"].shape), "grad_mask": to_host(grads[k][1])}
        for name, arr in got.items():
            assert oracle_ref.sha(arr) == ref[k][name], f"volume {k}: {name} differs from the oracle"
        out, rec = B.ggdt_forward_rec(d["image"], d["softmask"], c["spacing"], c["v"], c["lam"], c["iterations"])
        gi, gm = B.ggdt_backward(d["image"], rec, d["grad_out"], c["spacing"], c["v"], c["lam"], c["iterations"])
        assert torch.equal(out, d["out"]) and torch.equal(rec, d["records"]), f"volume {k} forward"
        assert torch.equal(gi, grads[k][0]) and torch.equal(gm, grads[k][1]), f"volume {k} backward"
    plan.close()


@pytest.mark.parametrize("shape,C,scale", [((21, 26, 19), 2, 1.0), ((140, 90), 3, 1.0), ((18, 22, 20), 2, 2.0 ** -30)],
                         ids=lambda v: str(v))
def test_backward_lam1_multichannel_root_forms(shape, C, scale):
    """The reverse pass at lambda 1 with several channels and a quantised image
    (equal neighbours: a zero root argument), in the normal-range root's domain
    and, with values near 2^-30, outside it."""
    c = synth.small_case(shape, C=C, seed=720 + C, lam=1.0, iterations=2, soft=True, v=10.0)
    c["image"] = (np.round(c["image"] * 2.0) * np.float32(scale)).astype(np.float32)
    W = np.random.default_rng(721).standard_normal(shape).astype(np.float32)
    print(f"case {c['name']} C={C} scale={scale}", flush=True)
    out, rec, gi, gm = gpu_fwd_bwd(c, W)
    ref, ref_rec = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], 1.0, 2, "f32", records=True)
    assert np.array_equal(out, ref) and np.array_equal(rec, ref_rec)
    rgi, rgm = oracle.backward(c["image"], ref_rec, W, c["spacing"], c["v"], 1.0, 2, "f32")
    assert assert_parity(gm, rgm, what="dL/dM"), "dL/dM not bitwise"
    assert assert_parity(gi.reshape(rgi.shape), rgi, what="dL/dI"), "dL/dI not bitwise"
