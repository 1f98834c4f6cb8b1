"""Latency-bound plans keep each workgroup's unit state and coefficients in LDS
for a whole launch and write the state back at its end.  Checked through the
C ABI: the plan reports it; runs cut into launches of any length give the same
bits as one long run; the output matches the FP64 oracle (relative L2 <= 1e-5)
and the state matches a plan that keeps it in global memory; a gradient
context on such a plan (checkpoints and the recorded trajectory written from
LDS) matches the oracle's reverse pass (relative L2 <= 1e-4)."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as OA
from oracle import instances as OI
from oracle import simulate as OS

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_05940_amd import modal, physics
    return modal, physics, torch


def test_resident_state_across_launches(gpu):
    modal, physics, _ = gpu
    # more than 64 modes: beyond the on-chip plan, so the streaming kernel's
    # latency plan with LDS-resident state
    wl = W.plate_vk(seed=17, n_t=72, family="sine", grid=None, n_steps=1500)
    p = physics.plate_instance(wl)
    _say("case: resident state, one 72/72 plate, 1500 steps in one and in four launches")
    whole = modal.Sim([p], 44100.0)
    info = whole.info()
    assert info["resident_floats"] >= 72 and info["split_instances"] == 1, info
    y1 = whole.run(1500).cpu().numpy()[0]
    chunked = modal.Sim([p], 44100.0)
    parts = [chunked.run(k).cpu().numpy()[0] for k in (1, 37, 500, 962)]
    assert np.array_equal(np.concatenate(parts), y1)
    xa, xma = whole.state()
    xb, xmb = chunked.state()
    assert np.array_equal(xa, xb) and np.array_equal(xma, xmb)
    assert rel(y1, OS.run(OI.plate_instance(wl), 1500, 44100.0)) < 1e-5
    _say("case: same plate, state in global memory (explicit waves)")
    glob = modal.Sim([p], 44100.0, waves=8, max_workgroups=7, flags=modal.FLAG_SPLIT_ANY)
    assert glob.info()["resident_floats"] == 0
    y2 = glob.run(1500).cpu().numpy()[0]
    assert rel(y2, y1) < 1e-5
    xg, xmg = glob.state()
    assert rel(xg, xa) < 1e-5 and rel(xmg, xma) < 1e-5
    # a Berger plate and a string in the same latency plan
    wb = W.plate_berger(n_t=80, n_steps=1000)
    ws = W.string_kc(n_modes=20, n_steps=1000)
    insts = [physics.string_instance(ws), physics.plate_berger_instance(wb)]
    oinsts = [OI.string_instance(ws), OI.plate_berger_instance(wb)]
    _say("case: resident state, a KC string and a Berger plate")
    # a gradient context keeps the streaming kernel (a forward-only batch
    # without tensors would step on chip, one wave per instance)
    sim = modal.Sim(insts, 44100.0, flags=modal.FLAG_GRAD)
    assert sim.info()["resident_floats"] > 0
    y = np.concatenate([sim.run(k).cpu().numpy() for k in (300, 700)], axis=1)
    for b, o in enumerate(oinsts):
        assert rel(y[b], OS.run(o, 1000, 44100.0)) < 1e-5, b


def test_resident_gradient_context(gpu):
    modal, physics, torch = gpu
    wl = W.plate_vk(n_t=14, n_in=11, family="sine", grid=None, n_steps=600)
    wl["strike"]["amplitude"] = 3e-3
    steps = 600
    o = OI.plate_instance(wl)
    g = np.random.default_rng(9).normal(size=(1, steps)) / np.abs(o["x0"]).max()
    _say("case: gradient on a resident plan, vK 14/11, 600 steps, checkpoints every 128")
    sim = modal.Sim([physics.plate_instance(wl)], 44100.0, flags=modal.FLAG_GRAD)
    assert sim.info()["resident_floats"] > 0
    res = sim.grad(steps, torch.tensor(g, dtype=torch.float32, device="cuda"), ckpt_every=128)
    r = OA.reverse(o, steps, 44100.0, g[0].astype(np.float32).astype(float))
    om, ga = OA.sv_omega_gamma_grads(r, o["omega"], o["gamma"], 1 / 44100.0)
    ref = dict(omega=om, gamma=ga, c=r["c"], x0=r["x0"], xm1=r["xm1"])
    for k, v in ref.items():
        assert rel(res[k][0], v) < 1e-4, (k, rel(res[k][0], v))
