"""Failure handling on the GPU, forced from the host: a spin limit of one poll
makes the bounded inter-workgroup waits give up (every kernel still exits
normally), and the watchdog must then be reported as GGDT_ERR_WATCHDOG by the
status query and as GGDTError by the binding; with the limit restored, the same
workspace gives the oracle's result again."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import to_dev, to_host
from paper_2208_00001_amd import synth

pytestmark = pytest.mark.gpu

GGDT_ERR_WATCHDOG = -6


@pytest.fixture
def tiny_spin_limit():
    from paper_2208_00001_amd import binding as B
    B.load_library()
    B.set_spin_limit(1)
    yield
    B.set_spin_limit(0)  # restores the default


def test_watchdog_reported_for_plain_forward(tiny_spin_limit):
    from paper_2208_00001_amd import binding as B
    # two channels: the tile kernel, whose waits give up after one unsuccessful poll
    c = synth.small_case((40, 150, 170), C=2, seed=901, lam=0.5, iterations=1)
    img, m = to_dev(c["image"]), to_dev(c["mask"])
    ws = B.new_workspace(c["mask"].shape, 2, img.device)
    fired = 0
    for attempt in range(3):
        print(f"attempt {attempt}: forward with a spin limit of 1 poll", flush=True)
        try:
            B.ggdt3d(img, m, c["spacing"], c["v"], c["lam"], c["iterations"], workspace=ws, check=True)
        except B.GGDTError as e:
            assert e.code == GGDT_ERR_WATCHDOG, e
            assert B.workspace_status(ws) == GGDT_ERR_WATCHDOG
            fired += 1
            break
    assert fired, "no bounded wait gave up with a spin limit of one poll"
    B.set_spin_limit(0)
    out = B.ggdt3d(img, m, c["spacing"], c["v"], c["lam"], c["iterations"], workspace=ws, check=True)
    assert B.workspace_status(ws) == 0
    ref = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32")
    assert np.array_equal(to_host(out), ref)


def test_watchdog_reported_for_batched_launch(tiny_spin_limit):
    from paper_2208_00001_amd import binding as B
    from paper_2208_00001_amd.batched import BatchedPlan
    cases = [synth.small_case(s, C=1, seed=910 + k, lam=1.0, iterations=2) for k, s in
             enumerate([(40, 70, 90), (60, 50, 40), (300, 280)])]
    inst = [dict(image=to_dev(c["image"]), softmask=to_dev(c["mask"]), spacing=c["spacing"], v=c["v"], lam=c["lam"],
                 iterations=c["iterations"]) for c in cases]
    plan = BatchedPlan(inst)
    fired = 0
    for attempt in range(3):
        print(f"attempt {attempt}: batched launch with a spin limit of 1 poll", flush=True)
        plan.run()
        try:
            plan.check()
        except B.GGDTError as e:
            assert e.code == GGDT_ERR_WATCHDOG, e
            fired += 1
            break
    assert fired, "no bounded wait gave up with a spin limit of one poll"
    B.set_spin_limit(0)
    plan.run()
    plan.check()
    for c, d in zip(cases, plan.inst):
        ref = oracle.ggdt(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], c["iterations"], "f32")
        assert np.array_equal(to_host(d["out"]), ref), c["name"]
    plan.close()


def test_watchdog_reported_for_toivanen_grid(tiny_spin_limit):
    """Toivanen's scan on a pipeline of several row blocks: the waits for the
    neighbouring block's progress are bounded like every other wait."""
    from paper_2208_00001_amd import binding as B
    c = synth.small_case((80, 81, 20), C=1, seed=930, lam=1.0, iterations=1)  # 7 slabs of 12 planes
    img, m = to_dev(c["image"]), to_dev(c["mask"])
    ws = B.new_workspace(c["mask"].shape, 1, img.device, minimal=True)
    fired = 0
    for attempt in range(3):
        print(f"attempt {attempt}: Toivanen with a spin limit of 1 poll", flush=True)
        try:
            B.ggdt_toivanen(img, m, c["spacing"], c["v"], c["lam"], 1, workspace=ws, check=True)
        except B.GGDTError as e:
            assert e.code == GGDT_ERR_WATCHDOG, e
            fired += 1
            break
    assert fired, "no wait gave up with a spin limit of one poll"
    B.set_spin_limit(0)
    out = B.ggdt_toivanen(img, m, c["spacing"], c["v"], c["lam"], 1, workspace=ws, check=True)
    ref = oracle.toivanen(c["image"], c["mask"], c["spacing"], c["v"], c["lam"], 1, "f32")
    assert np.array_equal(to_host(out), ref)


def test_binding_rejects_wrong_buffers():
    from paper_2208_00001_amd import binding as B
    c = synth.small_case((8, 9, 10), C=1, seed=920, lam=0.7, iterations=1)
    img, m = to_dev(c["image"]), to_dev(c["mask"])
    args = (img, m, c["spacing"], c["v"], c["lam"], c["iterations"])
    for bad in (torch.empty((8, 9, 11), device=img.device), torch.empty((8, 9, 10), dtype=torch.float64,
                                                                          device=img.device),
                torch.empty((8, 9, 10)), torch.empty((8, 10, 9), device=img.device).transpose(1, 2)):
        with pytest.raises(ValueError):
            B.ggdt3d(*args, out=bad)
    rec_ok = torch.empty((6, 8, 9, 10), dtype=torch.uint8, device=img.device)
    for bad in (torch.empty((5, 8, 9, 10), dtype=torch.uint8, device=img.device),
                torch.empty((6, 8, 9, 10), dtype=torch.int32, device=img.device),
                torch.empty((6, 8, 9, 10), dtype=torch.uint8)):
        with pytest.raises(ValueError):
            B.ggdt_forward_rec(*args, records=bad)
    _, rec = B.ggdt_forward_rec(*args, records=rec_ok)
    with pytest.raises(ValueError):  # records of one iteration, backward over two
        B.ggdt_backward(img, rec, torch.ones_like(m), c["spacing"], c["v"], c["lam"], 2)
    with pytest.raises(ValueError):
        B.ggdt3d(*args, workspace=torch.empty(4096, dtype=torch.uint8))
