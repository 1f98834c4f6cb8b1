"""The on-chip plan: forward-only, latency-bound batches whose instances have
at most 64 modes step each instance in one workgroup that holds its coupling
tensor in registers for the whole launch (modal_info path 3).

Bar: relative L2 error of each output signal <= 1e-5 against the FP64
oracle; the read-back state to the same bar; graph replays and
modal_run_noalloc bit-identical to eager modal_run of the same plan."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import instances as OI
from oracle import simulate as OS

pytestmark = pytest.mark.gpu

TOL = 1e-5
PATH_CHIP = 3


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


def test_c2_plate_full_second_on_chip(gpu):
    """The 40/40 clamped-family plate (the latency configuration) over 1 s,
    its modes grouped by parity class like a sine-family plate's."""
    modal, physics = gpu
    wl = W.plate_vk()
    _say("case: on-chip 40/40 clamped plate, 44100 steps")
    sim = modal.Sim([physics.plate_instance(wl)], wl["fs"])
    assert sim.info()["path"] == PATH_CHIP
    assert sim.info()["workgroups"] == 1
    y = sim.run(wl["n_steps"])[0].double().cpu().numpy()
    _, states = OS.run(OI.plate_instance(wl), wl["n_steps"], wl["fs"], return_states=True)
    ref = OS.run(OI.plate_instance(wl), wl["n_steps"], wl["fs"])
    e = rel_l2(y, ref)
    _say(f"  rel L2 {e:.2e}")
    assert e < TOL, e
    x, xm = sim.state()
    assert rel_l2(x, states[-1]) < TOL
    assert rel_l2(xm, states[-2]) < TOL


@pytest.mark.parametrize("n", [40, 50, 60])
def test_sine_plates_full_second_on_chip(gpu, n):
    """Sine-family plates up to the paper's 50-mode benchmark shape and
    beyond (Sec. 4.2): modes grouped by parity class so that a lane holds
    only the quarter of each row that can be nonzero against its mode."""
    modal, physics = gpu
    wl = W.plate_sweep(n)
    _say(f"case: on-chip {n}/{n} sine plate, 44100 steps")
    sim = modal.Sim([physics.plate_instance(wl)], wl["fs"])
    assert sim.info()["path"] == PATH_CHIP
    y = sim.run(wl["n_steps"])[0].double().cpu().numpy()
    ref = OS.run(OI.plate_instance(wl), wl["n_steps"], wl["fs"])
    e = rel_l2(y, ref)
    _say(f"  rel L2 {e:.2e}")
    assert e < TOL, e


def _mixed():
    """Ragged small instances of every kind: sine-family vK plates (modes
    grouped by class) whose mode counts are and are not multiples of 4 and
    whose in-plane rows fill one to five rows per wave, a clamped-family
    plate given without its classes (held whole), a tension-modulated string,
    and a forced linear system."""
    out = []
    for i, (nt, nin) in enumerate([(3, 2), (10, 10), (17, 9), (33, 33), (40, 40), (24, 31)]):
        wl = W.plate_vk(seed=300 + i, n_t=nt, n_in=nin, family="sine", grid=None, n_steps=6000)
        wl["strike"]["amplitude"] = 2e-3
        out.append(("plate", wl))
    wl = W.plate_vk(seed=299, n_t=16, n_steps=6000)  # clamped family, its classes withheld: held whole
    wl["strike"]["amplitude"] = 2e-3
    out.append(("plate_whole", wl))
    out.append(("string", W.string_kc(n_steps=6000)))
    rng = np.random.default_rng(12)
    n = 13
    om = np.sort(rng.uniform(2 * np.pi * 50, 2 * np.pi * 5000, n))
    out.append(("linear", dict(kind="linear", omega=om, gamma=1 + 0.002 * om, x0=np.zeros(n), xm1=np.zeros(n),
                               c=rng.normal(size=n), b_ext=rng.normal(size=n),
                               e_ext=rng.normal(size=500).astype(np.float32))))
    return out


def _product(physics, kind, wl):
    if kind == "plate":
        return physics.plate_instance(wl)
    if kind == "plate_whole":
        inst = physics.plate_instance(wl)
        inst.pop("mode_class", None)
        return inst
    if kind == "string":
        return physics.string_instance(wl)
    return wl


def _oracle(kind, wl, steps):
    if kind in ("plate", "plate_whole"):
        return OS.run(OI.plate_instance(wl), steps, wl["fs"])
    if kind == "string":
        return OS.run(OI.string_instance(wl), steps, wl["fs"])
    return OS.run(dict(wl, e_ext=wl["e_ext"].astype(np.float64)), steps, 44100.0)


@pytest.mark.parametrize("scheme", ["sv", "tf"])
def test_mixed_batch_on_chip(gpu, scheme):
    modal, physics = gpu
    cases = _mixed()
    steps = 6000
    _say(f"case: on-chip mixed batch of {len(cases)} ({scheme}), {steps} steps")
    sim = modal.Sim([_product(physics, k, w) for k, w in cases], 44100.0, scheme=scheme)
    assert sim.info()["path"] == PATH_CHIP
    y = sim.run(steps).double().cpu().numpy()
    for b, (kind, wl) in enumerate(cases):
        ref = (_oracle(kind, wl, steps) if scheme == "sv" else
               OS.run(OI.plate_instance(wl) if kind in ("plate", "plate_whole") else
                      OI.string_instance(wl) if kind == "string" else
                      dict(wl, e_ext=wl["e_ext"].astype(np.float64)), steps, 44100.0, scheme="tf"))
        e = rel_l2(y[b], ref)
        _say(f"  {b} {kind}: rel L2 {e:.2e}")
        assert e < TOL, (b, kind, e)


def test_chunks_graphs_and_noalloc_match_eager(gpu):
    import torch
    modal, physics = gpu
    cases = _mixed()
    insts = [_product(physics, k, w) for k, w in cases]
    B, steps = len(insts), 1500
    _say("case: on-chip eager vs chunked graph vs modal_run_noalloc, 3 x 1500 steps")
    eager = modal.Sim(insts, 44100.0)
    graph = modal.Sim(insts, 44100.0, flags=modal.FLAG_GRAPH, chunk_steps=441)
    noal = modal.Sim(insts, 44100.0)
    for s in (eager, graph, noal):
        assert s.info()["path"] == PATH_CHIP
    out = torch.empty((B, steps), device="cuda")
    out2 = torch.empty((B, steps), device="cuda")
    for rep in range(3):
        ye = eager.run(steps).cpu().numpy()
        graph.run(steps, out=out)
        noal.run_noalloc(steps, out2)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ye), rep
        assert np.array_equal(out2.cpu().numpy(), ye), rep


def test_streaming_plan_is_still_chosen_when_it_must_be(gpu):
    """Instances beyond the on-chip limits, an explicit launch shape, and
    gradient contexts keep the streaming kernel."""
    modal, physics = gpu
    small = physics.plate_instance(W.plate_vk(n_t=20, family="sine", grid=None))
    big = physics.plate_instance(W.plate_sweep(100))
    assert modal.Sim([small], 44100.0).info()["path"] == PATH_CHIP
    assert modal.Sim([big], 44100.0).info()["path"] == 0
    assert modal.Sim([small, big], 44100.0).info()["path"] == 0
    assert modal.Sim([small], 44100.0, waves=8).info()["path"] == 0
    assert modal.Sim([small], 44100.0, flags=modal.FLAG_GRAD).info()["path"] == 0


def test_nonfinite_is_reported_on_chip(gpu):
    modal, physics = gpu
    wl = W.plate_vk(n_t=12, family="sine", grid=None, n_steps=2000)
    inst = physics.plate_instance(wl)
    inst["x0"] = inst["x0"] * 1e4  # tens of metres: the explicit scheme blows up
    sim = modal.Sim([inst], 44100.0)
    assert sim.info()["path"] == PATH_CHIP
    with pytest.raises(modal.ModalError, match="non-finite"):
        sim.run(2000)


def _plain():
    """Instances without a tensor, beyond 64 modes too: the 100-mode Berger
    plate of the paper's Fig. 2, a Kirchhoff-Carrier string and a forced
    linear system of 130 modes whose 1500-sample forcing ends inside a
    64-sample chunk."""
    rng = np.random.default_rng(31)
    n = 130
    om = np.sort(rng.uniform(2 * np.pi * 50, 2 * np.pi * 8000, n))
    lin = dict(kind="linear", omega=om, gamma=1 + 0.002 * om, x0=np.zeros(n), xm1=np.zeros(n),
               c=rng.normal(size=n), b_ext=rng.normal(size=n), e_ext=rng.normal(size=1500).astype(np.float32))
    return [("berger", W.plate_berger(n_t=100, n_steps=4000)), ("string", W.string_kc(n_steps=4000)),
            ("linear", lin)]


def test_wave_path_for_instances_without_tensor(gpu):
    """A batch with no tensor (tension-modulated and linear instances of up
    to 256 modes) steps one wave per instance (modal_info path 3); parity
    with the oracle, and eager, chunked-graph and modal_run_noalloc runs
    bit-identical over launches that start inside a 64-sample chunk."""
    import torch
    modal, physics = gpu
    cases = _plain()
    prod = {"berger": physics.plate_berger_instance, "string": physics.string_instance, "linear": lambda w: w}
    orac = {"berger": OI.plate_berger_instance, "string": OI.string_instance,
            "linear": lambda w: dict(w, e_ext=w["e_ext"].astype(np.float64))}
    insts = [prod[k](w) for k, w in cases]
    steps = 4000
    _say(f"case: one-wave on-chip path, {len(insts)} instances, {steps} steps")
    sim = modal.Sim(insts, 44100.0, flags=modal.FLAG_RECURSE)
    assert sim.info()["path"] == PATH_CHIP and sim.info()["workgroups"] == len(insts)
    y = sim.run(steps).double().cpu().numpy()
    for b, (kind, wl) in enumerate(cases):
        ref = OS.run(orac[kind](wl), steps, 44100.0)
        e = rel_l2(y[b], ref)
        _say(f"  {kind}: rel L2 {e:.2e}")
        assert e < TOL, (kind, e)
    graph = modal.Sim(insts, 44100.0, flags=modal.FLAG_RECURSE | modal.FLAG_GRAPH, chunk_steps=441)
    noal = modal.Sim(insts, 44100.0, flags=modal.FLAG_RECURSE)
    out = torch.empty((len(insts), steps), device="cuda")
    out2 = torch.empty((len(insts), steps), device="cuda")
    graph.run(steps, out=out)
    noal.run_noalloc(steps, out2)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), y.astype(np.float32))
    assert np.array_equal(out2.cpu().numpy(), y.astype(np.float32))
