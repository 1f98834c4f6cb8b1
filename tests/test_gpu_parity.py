"""Parity of the HIP time loop (through the C ABI) with the FP64 oracle.

Bar: relative L2 error of each output signal <= 1e-5 against the unmodified
FP64 oracle (each side builds its own modes, tensors and coefficients from
the same seeded parameters)."""
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


def test_string_kc_full_length(gpu):
    modal, physics = gpu
    wl = W.string_kc()
    _say("case: KC string 30 modes, 22050 steps")
    sim = modal.Sim([physics.string_instance(wl)], wl["fs"])
    y = sim.run(wl["n_steps"])[0].double().cpu().numpy()
    ref = OS.run(OI.string_instance(wl), wl["n_steps"], wl["fs"])
    assert rel_l2(y, ref) < TOL, rel_l2(y, ref)


@pytest.mark.parametrize("family", ["clamped", "sine"])
def test_plate_vk_single_full_second(gpu, family):
    modal, physics = gpu
    wl = W.plate_vk(family=family)
    _say(f"case: vK plate 40/40 {family}, 44100 steps")
    sim = modal.Sim([physics.plate_instance(wl)], wl["fs"])
    y = sim.run(wl["n_steps"])[0].double().cpu().numpy()
    ref = OS.run(OI.plate_instance(wl), wl["n_steps"], wl["fs"])
    assert rel_l2(y, ref) < TOL, rel_l2(y, ref)


@pytest.mark.parametrize("n", [10, 50, 100])
def test_paper_sweep_shapes(gpu, n):
    modal, physics = gpu
    steps = 44100 if n <= 50 else 8820
    wl = W.plate_sweep(n, n_steps=steps)
    _say(f"case: vK sweep N={n}, {steps} steps")
    sim = modal.Sim([physics.plate_instance(wl)], wl["fs"])
    y = sim.run(steps)[0].double().cpu().numpy()
    ref = OS.run(OI.plate_instance(wl), steps, wl["fs"])
    assert rel_l2(y, ref) < TOL, rel_l2(y, ref)


def _ragged_batch():
    """Mixed kinds and ragged sizes: tensor widths that are and are not
    multiples of 4, single-row and multi-row in-plane counts."""
    out = []
    for i, (nt, nin) in enumerate([(3, 2), (5, 7), (17, 9), (33, 33), (40, 20), (64, 64), (65, 30), (90, 90)]):
        wl = W.plate_vk(seed=100 + i, n_t=nt, n_in=nin, family="sine", grid=None, n_steps=3000)
        wl["strike"]["amplitude"] = 2e-3
        out.append(wl)
    return out


@pytest.mark.parametrize("max_wg,waves", [(0, 4), (0, 1), (7, 4), (7, 1), (3, 4), (0, 8), (7, 8)])
def test_ragged_batch_split_and_packed(gpu, max_wg, waves):
    """max_workgroups 7 and 3 force instances to be cut into row slabs that
    exchange partial forces every step, next to instances packed whole; one,
    four or eight waves per workgroup share a unit's rows."""
    modal, physics = gpu
    wls = _ragged_batch()
    steps = 3000
    insts = [physics.plate_instance(w) for w in wls]
    s = W.string_kc(seed=7, n_modes=23)
    insts.append(physics.string_instance(s))
    lin = physics.string_instance(W.string_kc(seed=8, n_modes=9))
    lin["kind"] = "linear"
    insts.append(lin)
    _say(f"case: ragged batch of {len(insts)}, max_workgroups={max_wg}, waves={waves}")
    sim = modal.Sim(insts, 44100.0, max_workgroups=max_wg, flags=modal.FLAG_SPLIT_ANY, waves=waves)
    info = sim.info()
    if max_wg:
        assert info["workgroups"] <= max_wg and info["split_instances"] >= 1, info
    y = sim.run(steps).double().cpu().numpy()
    oinst = [OI.plate_instance(w) for w in wls] + [OI.string_instance(s)]
    ol = OI.string_instance(W.string_kc(seed=8, n_modes=9))
    ol["kind"] = "linear"
    oinst.append(ol)
    for b, oi in enumerate(oinst):
        ref = OS.run(oi, steps, 44100.0)
        assert rel_l2(y[b], ref) < TOL, (b, rel_l2(y[b], ref))


def test_resume_and_determinism(gpu):
    modal, physics = gpu
    wls = _ragged_batch()[2:6]
    insts = [physics.plate_instance(w) for w in wls]
    a = modal.Sim(insts, 44100.0, max_workgroups=5, flags=modal.FLAG_SPLIT_ANY)
    y_full = a.run(2000).cpu().numpy()
    b = modal.Sim(insts, 44100.0, max_workgroups=5, flags=modal.FLAG_SPLIT_ANY)
    y1 = b.run(700).cpu().numpy()
    y2 = b.run(1300).cpu().numpy()
    assert np.array_equal(y_full, np.concatenate([y1, y2], axis=1))
    a.reset()
    assert np.array_equal(a.run(2000).cpu().numpy(), y_full)


def test_graph_replay_matches_eager(gpu):
    modal, physics = gpu
    wls = _ragged_batch()[3:5]
    insts = [physics.plate_instance(w) for w in wls]
    import torch
    eager = modal.Sim(insts, 44100.0, max_workgroups=4, flags=modal.FLAG_SPLIT_ANY)
    graph = modal.Sim(insts, 44100.0, max_workgroups=4, flags=modal.FLAG_GRAPH | modal.FLAG_SPLIT_ANY,
                      chunk_steps=250)
    out = torch.empty((2, 500), device="cuda")
    for rep in range(3):
        ye = eager.run(500).cpu().numpy()
        graph.run(500, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ye), rep


def test_forced_linear_and_tf_scheme(gpu):
    modal, physics = gpu
    rng = np.random.default_rng(11)
    n = 13
    om = np.sort(rng.uniform(2 * np.pi * 50, 2 * np.pi * 5000, n))
    base = dict(kind="linear", omega=om, gamma=1 + 0.002 * om, x0=np.zeros(n), xm1=np.zeros(n),
                c=rng.normal(size=n), b_ext=rng.normal(size=n), e_ext=rng.normal(size=500).astype(np.float32))
    for scheme in ("sv", "tf"):
        sim = modal.Sim([base], 44100.0, scheme=scheme)
        y = sim.run(3000)[0].double().cpu().numpy()
        oi = dict(base, e_ext=base["e_ext"].astype(np.float64))
        ref = OS.run(oi, 3000, 44100.0, scheme=scheme)
        assert rel_l2(y, ref) < TOL, (scheme, rel_l2(y, ref))
    wl = W.plate_vk(n_t=20, family="sine", grid=None, n_steps=4000)
    sim = modal.Sim([physics.plate_instance(wl)], 44100.0, scheme="tf")
    y = sim.run(4000)[0].double().cpu().numpy()
    ref = OS.run(OI.plate_instance(wl), 4000, 44100.0, scheme="tf")
    assert rel_l2(y, ref) < TOL, rel_l2(y, ref)


def test_state_readback_matches_oracle_state(gpu):
    modal, physics = gpu
    wl = W.plate_vk(n_t=16, family="sine", grid=None, n_steps=1000)
    sim = modal.Sim([physics.plate_instance(wl)], 44100.0)
    sim.run(1000)
    x, xm = sim.state()
    _, states = OS.run(OI.plate_instance(wl), 1000, 44100.0, return_states=True)
    assert np.linalg.norm(x - states[-1]) / np.linalg.norm(states[-1]) < TOL
    assert np.linalg.norm(xm - states[-2]) / np.linalg.norm(states[-2]) < TOL


def test_nonfinite_is_reported(gpu):
    modal, physics = gpu
    wl = W.plate_vk(n_t=12, family="sine", grid=None, n_steps=2000)
    inst = physics.plate_instance(wl)
    inst["x0"] = inst["x0"] * 1e4  # tens of metres: the explicit scheme blows up
    inst["xm1"] = inst["x0"].copy()
    sim = modal.Sim([inst], 44100.0)
    with pytest.raises(modal.ModalError) as e:
        sim.run(2000)
    assert e.value.status == "ENONFINITE"
    sim.reset()
    sim.check()


def test_asymmetric_tensor_rejected(gpu):
    modal, physics = gpu
    wl = W.plate_vk(n_t=8, family="sine", grid=None)
    inst = physics.plate_instance(wl)
    H = inst["Ht"].copy()
    H[2, 1, 5] += 1e-3 * np.abs(H).max()  # one entry, not its mirror
    inst["Ht"] = H
    with pytest.raises(modal.ModalError) as e:
        modal.Sim([inst], 44100.0)
    assert e.value.status == "EINVAL"


def test_latency_plan_single_and_small_batches(gpu):
    """Latency-bound batches (at most one instance per CU, small dense
    tensors, default shape) beyond the on-chip limits (more than 64 modes):
    a lone plate runs dense in slabs of about eight in-plane rows on their
    own workgroups; a batch of more than 16 keeps each plate whole on one
    workgroup.  Both match the FP64 oracle."""
    modal, physics = gpu
    wl = W.plate_vk(seed=31, n_t=72, family="sine", grid=None, n_steps=1500)
    p = physics.plate_instance(wl)
    o = OI.plate_instance(wl)
    _say("case: latency plan, one 72/72 plate")
    sim = modal.Sim([p], 44100.0)
    info = sim.info()
    assert info["path"] == 0 and info["blocked_instances"] == 0, info
    assert info["workgroups"] == 9 and info["split_instances"] == 1, info
    y = sim.run(1500).double().cpu().numpy()[0]
    assert rel_l2(y, OS.run(o, 1500, 44100.0)) < TOL
    _say("case: latency plan, 20 plates of 66/12")
    wls = [W.plate_vk(seed=40 + i, n_t=66, n_in=12, family="sine", grid=None, n_steps=800) for i in range(20)]
    sim = modal.Sim([physics.plate_instance(w) for w in wls], 44100.0)
    info = sim.info()
    assert info["path"] == 0 and info["workgroups"] == 20 and info["split_instances"] == 0, info
    y = sim.run(800).double().cpu().numpy()
    for i in (0, 7, 19):
        assert rel_l2(y[i], OS.run(OI.plate_instance(wls[i]), 800, 44100.0)) < TOL
