"""Tension-modulated (Berger) plates through the tension kernel, against
the FP64 oracle: the benchmark shapes of the paper's Fig. 2 (bottom panel,
10/50/100 modes), both schemes, and a mixed launch of Berger, von Karman,
Kirchhoff-Carrier and linear instances.  Bar: relative L2 <= 1e-5."""
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


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available()
    from paper_2505_05940_amd import modal, physics
    return modal, physics


@pytest.mark.parametrize("n,scheme", [(10, "sv"), (50, "sv"), (100, "sv"), (50, "tf")])
def test_berger_plate_fig2_shapes(gpu, n, scheme):
    modal, physics = gpu
    steps = 44100
    wl = W.plate_berger(n_t=n, n_steps=steps)
    print(f"case: Berger plate N={n}, {steps} steps, {scheme}", flush=True)
    sim = modal.Sim([physics.plate_berger_instance(wl)], wl["fs"], scheme=scheme)
    assert sim.info()["path"] == 3  # one wave on chip: no tensor
    y = sim.run(steps)
    ref = OS.run(OI.plate_berger_instance(wl), steps, wl["fs"], scheme=scheme)
    assert rel_l2(y[0].double().cpu().numpy(), ref) < TOL


def test_mixed_kinds_in_one_launch(gpu):
    modal, physics = gpu
    steps = 3000
    wb = W.plate_berger(seed=21, n_t=30, n_steps=steps)
    wv = W.plate_vk(seed=22, n_t=24, n_in=24, family="sine", grid=None, n_steps=steps)
    ws = W.string_kc(seed=23, n_modes=20)
    lin = dict(kind="linear", omega=2 * np.pi * np.array([110.0, 220.0, 330.0]),
               gamma=np.array([2.0, 3.0, 4.0]), x0=np.array([1e-3, -5e-4, 2e-4]),
               xm1=np.array([1e-3, -5e-4, 2e-4]), c=np.array([1.0, 0.5, 0.25]))
    pins = [physics.plate_berger_instance(wb), physics.plate_instance(wv), physics.string_instance(ws), lin]
    oins = [OI.plate_berger_instance(wb), OI.plate_instance(wv), OI.string_instance(ws), dict(lin)]
    print("case: mixed Berger / vK / KC / linear launch, 3000 steps", flush=True)
    y = modal.Sim(pins, 44100.0).run(steps).double().cpu().numpy()
    for b in range(4):
        ref = OS.run(oins[b], steps, 44100.0)
        assert rel_l2(y[b], ref) < TOL, (b, rel_l2(y[b], ref))
