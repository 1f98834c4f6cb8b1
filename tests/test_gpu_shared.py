"""The shared-tensor (FP32 MFMA) path against the FP64 oracle.

A group of plates shares one coupling tensor up to per-row scales; the
library stores it once and evaluates the force as a dense product over the
group.  Bar: relative L2 error of each output signal <= 1e-5 against the
FP64 oracle, which runs every member with its own explicitly scaled tensor.
Members not run on the oracle are compared with the per-instance streaming
path of the same library (both within 1e-5 of the oracle, so within 2e-5 of
each other)."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import instances as OI
from oracle import simulate as OS

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel_l2(y, ref):
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_05940_amd import modal, physics
    return modal, physics


def _instances(group, physics):
    """Product instances (one shared float32 tensor object plus row scales)
    and a builder of oracle instances (each with its own FP64 scaled
    tensor), made only for the members the oracle runs."""
    p0 = physics.plate_instance(group["base"])
    H0 = np.ascontiguousarray(p0["Ht"], dtype=np.float32)
    pins = []
    for m in group["members"]:
        p = dict(p0, Ht=H0, h_row_scale=m["row_scale"], omega=p0["omega"] * m["omega_factor"],
                 gamma=p0["gamma"] * m["gamma_factor"], x0=p0["x0"] * m["amp_factor"],
                 xm1=p0["xm1"] * m["amp_factor"])
        if "b_ext" in m:
            p.update(b_ext=m["b_ext"], e_ext=m["e_ext"])
        pins.append(p)
    o0 = OI.plate_instance(group["base"])

    def oracle(b):
        m = group["members"][b]
        o = dict(o0, Ht=o0["Ht"] * m["row_scale"][:, None, None], omega=o0["omega"] * m["omega_factor"],
                 gamma=o0["gamma"] * m["gamma_factor"], x0=o0["x0"] * m["amp_factor"],
                 xm1=o0["xm1"] * m["amp_factor"])
        if "b_ext" in m:
            o.update(b_ext=m["b_ext"], e_ext=m["e_ext"].astype(float))
        return o
    return pins, oracle


def test_shared_group_full_second(gpu):
    modal, physics = gpu
    g = W.plate_group(batch=48, n_t=40, forced=2)
    pins, oins = _instances(g, physics)
    steps = g["n_steps"]
    _say(f"case: shared group 48 x (40/40), {steps} steps")
    sim = modal.Sim(pins, g["fs"])
    info = sim.info()
    assert info["shared"] == 1 and info["units"] == 64 and info["workgroups"] == 1, info
    y = sim.run(steps).double().cpu().numpy()
    sim.check()
    for b in (0, 1, 17, 47):  # both forced members and two free ones
        ref = OS.run(oins(b), steps, g["fs"])
        assert rel_l2(y[b], ref) < TOL, (b, rel_l2(y[b], ref))
    ys = modal.Sim(pins, g["fs"], flags=modal.FLAG_NO_SHARED)
    assert ys.info()["shared"] == 0
    y2 = ys.run(steps).double().cpu().numpy()
    errs = [rel_l2(y[b], y2[b]) for b in range(len(pins))]
    assert max(errs) < 2 * TOL, max(errs)


@pytest.mark.parametrize("scheme", ["sv", "tf"])
def test_shared_ragged_groups(gpu, scheme):
    """Two groups of different widths in one launch (16-row tiles 2 and 4,
    K steps 6 and 13), partially filled workgroups, forcing, both schemes."""
    modal, physics = gpu
    ga = W.plate_group(seed=11, batch=20, n_t=24, n_in=18, n_steps=3000, forced=1)
    gb = W.plate_group(seed=12, batch=70, n_t=50, n_in=30, n_steps=3000, forced=3)
    pa, oa = _instances(ga, physics)
    pb, ob = _instances(gb, physics)
    pins = pa + pb

    def oins(b):
        return oa(b) if b < len(pa) else ob(b - len(pa))
    _say(f"case: shared ragged groups 20 x 24/18 + 70 x 50/30, 3000 steps, {scheme}")
    sim = modal.Sim(pins, 44100.0, scheme=scheme)
    info = sim.info()
    assert info["shared"] == 1 and info["workgroups"] == 3, info
    y = sim.run(3000).double().cpu().numpy()
    for b in (0, 7, 19, 20, 22, 23, 60, 89):
        ref = OS.run(oins(b), 3000, 44100.0, scheme=scheme)
        assert rel_l2(y[b], ref) < TOL, (b, rel_l2(y[b], ref))
    y2 = modal.Sim(pins, 44100.0, scheme=scheme, flags=modal.FLAG_NO_SHARED).run(3000)
    y2 = y2.double().cpu().numpy()
    errs = [rel_l2(y[b], y2[b]) for b in range(len(pins))]
    assert max(errs) < 2 * TOL, max(errs)


def test_shared_two_column_tiles(gpu):
    """A group large enough for two 16-column tiles per wave (128 columns per
    workgroup, one workgroup per CU): sampled members against the oracle."""
    modal, physics = gpu
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    B = 128 * cus - 5
    g = W.plate_group(seed=13, batch=B, n_t=16, n_in=8, n_steps=400)
    pins, oins = _instances(g, physics)
    _say(f"case: shared group of {B} x (16/8), 400 steps")
    sim = modal.Sim(pins, 44100.0)
    info = sim.info()
    assert info["shared"] == 1 and info["units"] == 128 * cus and info["workgroups"] == cus, info
    y = sim.run(400).double().cpu().numpy()
    for b in (0, 129, B // 2, B - 1):
        ref = OS.run(oins(b), 400, 44100.0)
        assert rel_l2(y[b], ref) < TOL, (b, rel_l2(y[b], ref))


def test_shared_resume_reset_graph_and_state(gpu):
    modal, physics = gpu
    g = W.plate_group(seed=14, batch=40, n_t=33, n_in=21, n_steps=500, forced=1)
    pins, oins = _instances(g, physics)
    _say("case: shared group 40 x 33/21, resume / reset / graph / state")
    sim = modal.Sim(pins, 44100.0)
    assert sim.info()["shared"] == 1
    a = sim.run(300).cpu().numpy()
    b = sim.run(200).cpu().numpy()
    x, xm = sim.state()
    sim.reset()
    whole = sim.run(500).cpu().numpy()
    assert np.array_equal(np.concatenate([a, b], axis=1), whole)
    gs = modal.Sim(pins, 44100.0, flags=modal.FLAG_GRAPH)
    for _ in range(2):
        gs.reset()
        assert np.array_equal(gs.run(500).cpu().numpy(), whole)
    # state q^500, q^499 of member 0 (forced) and member 39
    off = np.cumsum([0] + sim.n_t)
    for m in (0, 39):
        _, st = OS.run(oins(m), 500, 44100.0, return_states=True)
        assert rel_l2(x[off[m]:off[m + 1]], st[500]) < TOL
        assert rel_l2(xm[off[m]:off[m + 1]], st[499]) < TOL


def test_shared_path_selection_and_nonfinite(gpu):
    modal, physics = gpu
    g = W.plate_group(seed=15, batch=20, n_t=12, n_in=6, n_steps=100)
    pins, _ = _instances(g, physics)
    _say("case: shared path selection, non-finite report")
    assert modal.Sim(pins[:15], 44100.0).info()["shared"] == 0       # under 16 per tensor
    assert modal.Sim(pins, 44100.0, flags=modal.FLAG_GRAD).info()["shared"] == 0
    assert modal.Sim(pins, 44100.0, flags=modal.FLAG_NO_SHARED).info()["shared"] == 0
    sim = modal.Sim(pins, 44100.0)
    assert sim.info()["shared"] == 1
    sim.run(50)
    big = [dict(p) for p in pins]
    big[3]["x0"] = big[3]["x0"] * 1e6
    big[3]["xm1"] = big[3]["xm1"] * 1e6
    bad = modal.Sim(big, 44100.0)
    assert bad.info()["shared"] == 1
    with pytest.raises(modal.ModalError) as e:
        bad.run(2000)
    assert e.value.status == "ENONFINITE"
