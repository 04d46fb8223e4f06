"""Batched ragged GGDT on the GPU: one persistent launch for many instances of
uneven size, each with its own lambda, v, spacing and iteration count.

Checked against the CPU oracle per instance (bitwise, within the 1e-5 bar), for
records too, for HIP-graph replays, and at the full 64-instance workload
against the oracle (stored digests or a live run) and the plain per-instance
launches."""
import numpy as np
import pytest
import torch

import oracle
import oracle_ref
from gpu_util import assert_parity, to_dev, to_host
from paper_2208_00001_amd import synth

pytestmark = pytest.mark.gpu


def small_batch(records=False):
    specs = [((37, 29, 41), 1, 0.7, 2), ((16, 16, 16), 1, 1.0, 3), ((300, 517), 1, 0.0, 2), ((20, 70, 33), 1, 0.0, 1),
             ((260, 33), 1, 0.45, 2), ((9, 40, 66), 1, 1.0, 1), ((1, 30, 40), 1, 0.3, 2), ((5, 6, 7), 1, 0.9, 0),
             ((2, 300), 1, 0.8, 3), ((48, 33, 20), 1, 0.6, 2)]
    cases = []
    for k, (shape, C, lam, it) in enumerate(specs):
        c = synth.small_case(shape, C=C, seed=300 + k, lam=lam, iterations=it, soft=(k % 3 == 1), v=6.0 if k % 3 == 1
                             else 1e10)
        cases.append(c)
    return cases


def to_instances(cases, records=False):
    return [dict(image=to_dev(c["image"]), softmask=to_dev(c["mask"]), spacing=c["spacing"], v=c["v"], lam=c["lam"],
                 iterations=c["iterations"], records=records) for c in cases]


# default class (16 x 16 volume tiles, K = 8), the multi-channel class forced
# (K = 4 tile passes), and 24 x 24 volume tiles with K = 4
TUNINGS = [None, {"chunk": 4}, {"chunk": 4, "tile_p": 24}]


@pytest.mark.parametrize("tuning", TUNINGS, ids=["default", "k4", "wide"])
@pytest.mark.parametrize("records", [False, True])
def test_small_ragged_batch_matches_oracle(records, tuning):
    from paper_2208_00001_amd.batched import BatchedPlan
    cases = small_batch()
    plan = BatchedPlan(to_instances(cases, records), tuning)
    print("plan", tuning, plan.info(), flush=True)
    plan.run()
    assert plan.status() == 0
    for c, d in zip(cases, plan.inst):
        print(f"instance {c['name']} lam={c['lam']} it={c['iterations']}", flush=True)
        got = to_host(d["out"])
        ref = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32",
                          records=records)
        if records:
            ref, ref_rec = ref
            if c["iterations"] > 0:
                assert np.array_equal(to_host(d["records"]), ref_rec), c["name"]
        assert assert_parity(got, ref, what=c["name"]), f"{c['name']}: not bitwise"
    plan.close()


def test_graph_replay_is_deterministic():
    from paper_2208_00001_amd.batched import BatchedPlan
    cases = small_batch()
    plan = BatchedPlan(to_instances(cases))
    eager = [to_host(o).copy() for o in plan.run()]
    plan.capture()
    for rep in range(3):
        for o in plan.outputs:
            o.fill_(-1.0)  # eager work between replays
        torch.cuda.synchronize()
        plan.replay()
        torch.cuda.synchronize()
        assert plan.status() == 0
        for e, o in zip(eager, plan.outputs):
            assert np.array_equal(e, to_host(o)), f"replay {rep} differs"
    plan.close()


@pytest.mark.parametrize("tuning", [None, {"chunk": 4, "tile_p": 24}], ids=["default", "wide"])
def test_config4_batch_equals_oracle_and_plain_launches(tuning):
    """The 64-instance ragged workload in one graph-replayed launch: every
    instance equals the oracle's FP32 forward bit for bit (stored digest, or a
    live oracle run when the regenerated inputs differ from the stored ones), and
    the plain per-instance launches give the same bits."""
    from paper_2208_00001_amd import binding as B
    from paper_2208_00001_amd.batched import BatchedPlan
    cases = synth.config4()
    ref, nlive = oracle_ref.forward_digests("config4", cases)
    print(f"config4: {len(cases)} instances, {nlive} oracle references computed live", flush=True)
    plan = BatchedPlan(to_instances(cases), tuning)
    plan.capture()
    plan.replay()
    torch.cuda.synchronize()
    assert plan.status() == 0
    for i, (c, d) in enumerate(zip(cases, plan.inst)):
        got = to_host(d["out"])
        assert oracle_ref.sha(got) == ref[i], f"instance {i} {c['name']}: differs from the oracle"
        fn = B.ggdt3d if c["mask"].ndim == 3 else B.ggdt2d
        plain = to_host(fn(d["image"], d["softmask"], c["spacing"], c["v"], c["lam"], c["iterations"]))
        assert np.array_equal(got, plain), f"instance {i} {c['name']}: batched != plain launch"
    plan.close()


@pytest.mark.parametrize("kind", ["mixed", "volumes", "volumes-wide"])
def test_small_ragged_batch_backward(kind):
    """Batched forward with records + batched backward for every instance, vs the
    single-instance launches and the oracle's FP32 reverse pass (bitwise).
    'mixed': 2D and 3D, 1-3 channels (tile reverse passes); 'volumes':
    single-channel volumes of different shapes only (thread-per-cell reverse
    pass, with more workgroups than some passes have tiles); 'volumes-wide':
    the same after a forward on 24 x 24 tiles (the reverse pass's 16 x 16
    tiles then need more exchange words than the forward's)."""
    from paper_2208_00001_amd import binding as B
    from paper_2208_00001_amd.batched import BatchedPlan
    if kind == "volumes-wide":
        # 65-cell planes: 9 tiles of 24 x 24 (5184 cells) against 25 of 16 x 16 (6400)
        specs = [((65, 65, 40), 1, 0.7, 2), ((19, 65, 65), 1, 1.0, 1), ((50, 26, 49), 1, 0.3, 2)]
    elif kind == "mixed":
        specs = [((29, 23, 31), 1, 0.7, 2), ((200, 137), 2, 0.5, 2), ((17, 40, 22), 3, 0.4, 1), ((90, 301), 1, 1.0, 2),
                 ((12, 13, 70), 1, 0.0, 2)]  # channel counts within the batched reverse pass's LDS (2D <= 2, 3D <= 3)
    else:
        specs = [((40, 33, 71), 1, 0.7, 2), ((19, 64, 17), 1, 1.0, 2), ((70, 18, 23), 1, 0.3, 1),
                 ((33, 33, 33), 1, 0.0, 2)]
    cases = []
    for k, (shape, C, lam, it) in enumerate(specs):
        c = synth.small_case(shape, C=C, seed=400 + k, lam=lam, iterations=it, soft=True, v=8.0)
        c["weight"] = np.random.default_rng(400 + k).standard_normal(c["mask"].shape).astype(np.float32)
        cases.append(c)
    inst = to_instances(cases, True)
    for d, c in zip(inst, cases):
        d["grad_out"] = to_dev(c["weight"])
    plan = BatchedPlan(inst, {"chunk": 4, "tile_p": 24} if kind == "volumes-wide" else None)
    print("plan", plan.info(), flush=True)
    plan.run()
    grads = plan.backward()
    torch.cuda.synchronize()
    assert plan.status() == 0
    for k, (c, d) in enumerate(zip(cases, plan.inst)):
        print(f"instance {c['name']} lam={c['lam']} it={c['iterations']}", flush=True)
        gi, gm = B.ggdt_backward(d["image"], d["records"], d["grad_out"], c["spacing"], c["v"], c["lam"],
                                 c["iterations"])
        assert torch.equal(gi, grads[k][0]) and torch.equal(gm, grads[k][1]), c["name"]
        _, ref_rec = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32",
                                 records=True)
        rgi, rgm = oracle.backward(c["image"], ref_rec, c["weight"], c["spacing"], c["v"], c["lam"], c["iterations"],
                                   "f32")
        assert assert_parity(to_host(grads[k][1]), rgm, what="dL/dM"), c["name"]
        assert assert_parity(to_host(grads[k][0]).reshape(rgi.shape), rgi, what="dL/dI"), c["name"]
    plan.close()


def test_batch_lam1_multichannel_root_forms():
    """lambda 1 with several channels in one batch: each instance's own image
    classification picks the normal-range root (quantised images, zero root
    arguments) or the full root (values near 2^-30)."""
    from paper_2208_00001_amd.batched import BatchedPlan
    cases = []
    for k, (shape, C, scale) in enumerate([((80, 70), 3, 1.0), ((17, 21, 19), 2, 1.0), ((16, 20, 18), 2, 2.0 ** -30),
                                           ((90, 60), 2, 2.0 ** -30)]):
        c = synth.small_case(shape, C=C, seed=330 + k, lam=1.0, iterations=2)
        c["image"] = (np.round(c["image"] * 2.0) * np.float32(scale)).astype(np.float32)
        cases.append(c)
    plan = BatchedPlan(to_instances(cases))
    plan.run()
    assert plan.status() == 0
    for c, d in zip(cases, plan.inst):
        print(f"instance {c['name']} C={c['image'].shape[0]}", flush=True)
        ref = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], 1.0, 2, "f32")
        assert np.array_equal(to_host(d["out"]).view(np.uint32), ref.view(np.uint32)), c["name"]
    plan.close()
