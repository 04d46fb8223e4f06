"""A seeded sweep of random small problems through every GPU entry point,
each result against the oracle bit for bit: the plain forward (full and
minimal workspace), the forward with records and the backward, the 16-bit
image entry, Toivanen's scan, and all instances together in one batched plan
(forward, then forward with records and the batched backward).  Shapes mix 2D
and 3D, unit and ragged dimensions; lambda is drawn with its exact regimes (0,
1) included; iterations 0-3; hard seeds or soft masks."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_parity, to_dev, to_host
from paper_2208_00001_amd import synth

pytestmark = pytest.mark.gpu

N_CASES = 32


def draw_cases(seed):
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(N_CASES):
        nd = 3 if rng.random() < 0.6 else 2
        if nd == 3:
            shape = tuple(int(x) for x in rng.integers(1, 40, size=3))
        else:
            shape = tuple(int(x) for x in rng.integers(1, 300, size=2))
        C = 1 if rng.random() < 0.7 else int(rng.integers(2, 4))
        lam = float(rng.choice([0.0, 1.0, rng.random()]))
        it = int(rng.integers(0, 4))
        soft = bool(rng.random() < 0.5)
        cases.append(synth.small_case(shape, C=C, seed=int(seed * 100 + k), lam=lam, iterations=it, soft=soft,
                                      v=8.0 if soft else 1e10))
    return cases


@pytest.mark.parametrize("seed", [11, 12, 13, 14])
def test_random_problems_every_entry_point(seed):
    from paper_2208_00001_amd import binding as B
    from paper_2208_00001_amd.batched import BatchedPlan
    cases = draw_cases(seed)
    for c in cases:
        shape, C, lam, it = c["mask"].shape, c["image"].shape[0], c["lam"], c["iterations"]
        print(f"case {c['name']} lam={lam} it={it} seed={c['seed']}", flush=True)
        img, m = to_dev(c["image"]), to_dev(c["mask"])
        ref = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], lam, it, "f32")
        fwd = B.ggdt2d if len(shape) == 2 else B.ggdt3d
        for minimal in (False, True):
            ws = B.new_workspace(shape, C, img.device, minimal=minimal)
            got = to_host(fwd(img, m, c["spacing"], c["v"], lam, it, workspace=ws, check=True))
            assert assert_parity(got, ref, what=f"{c['name']} minimal={minimal}"), "forward not bitwise"
        if it > 0:
            W = np.random.default_rng(c["seed"]).standard_normal(shape).astype(np.float32)
            out, rec = B.ggdt_forward_rec(img, m, c["spacing"], c["v"], lam, it, check=True)
            ref_o, ref_rec = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], lam, it, "f32", records=True)
            assert np.array_equal(to_host(out), ref_o) and np.array_equal(to_host(rec), ref_rec), "records differ"
            gi, gm = B.ggdt_backward(img, rec, to_dev(W), c["spacing"], c["v"], lam, it, check=True)
            rgi, rgm = oracle.backward(c["image"], ref_rec, W, c["spacing"], c["v"], lam, it, "f32")
            assert assert_parity(to_host(gm), rgm, what="dL/dM") and \
                assert_parity(to_host(gi).reshape(rgi.shape), rgi, what="dL/dI"), "gradients not bitwise"
        if (len(shape) == 3 and C == 1) or (len(shape) == 2 and C <= 3):
            t16 = torch.from_numpy(np.ascontiguousarray(c["image"])).to(torch.bfloat16)
            got = to_host(B.ggdt_half(t16.to("cuda"), m, c["spacing"], c["v"], lam, it, check=True))
            ref16 = oracle.ggdt(t16.float().numpy(), c["mask"], c["spacing"], c["v"], lam, it, "f32")
            assert assert_parity(got, ref16, what="bf16"), "16-bit image not bitwise"
        tv = to_host(B.ggdt_toivanen(img, m, c["spacing"], c["v"], lam, it, check=True))
        tref = oracle.toivanen(c["image"], c["mask"], c["spacing"], c["v"], lam, it, "f32")
        assert np.array_equal(tv.view(np.uint32), tref.view(np.uint32)), "Toivanen not bitwise"
    # every case in one batched plan (channel counts within the batched kernels' limits)
    bcases = [c for c in cases if c["image"].shape[0] <= 3]
    inst = [dict(image=to_dev(c["image"]), softmask=to_dev(c["mask"]), spacing=c["spacing"], v=c["v"], lam=c["lam"],
                 iterations=c["iterations"]) for c in bcases]
    plan = BatchedPlan(inst)
    plan.run()
    plan.check()
    for c, d in zip(bcases, plan.inst):
        ref = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32")
        assert assert_parity(to_host(d["out"]), ref, what=f"batched {c['name']}"), "batched not bitwise"
    plan.close()
