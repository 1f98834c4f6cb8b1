"""Parity at the sizes the benchmark and the paper's shapes are quoted on,
against stored FP64 oracle outputs (``tests/golden/``, written by
``tests/golden/make_golden.py``, which calls only ``oracle/``).

* The 256-plate batch (seed 3, N ~ U{50..400}) in exactly the launch
  configuration ``bench.py`` times (library default plan, 441-sample
  launches replayed from a hipGraph), run for one second: every plate over
  its first 2205 steps, and 8 plates at evenly spaced ranks of N (the
  smallest and the 400-mode plate included) over all 44 100 steps.
* The paper's benchmark shape at 100 modes (Sec. 4.2, Fig. 2): the von
  Karman and the Berger plate over one second.

Bar: relative L2 error of each output signal <= 1e-5 against the FP64
oracle (the stored outputs are FP32-rounded oracle values: about 6e-8
relative, far below the bar)."""
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel_l2(y, ref):
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.fail(f"{path} missing: run tests/golden/make_golden.py")
    return np.load(path)


@pytest.mark.timeout(900)
def test_benchmark_batch_all_plates_one_second():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_05940_amd import modal, physics
    head = _load("batch_head.npz")
    full = _load("batch_full.npz")
    wls = W.plate_batch(seed=3, batch=256)
    n = np.array([w["n_t"] for w in wls])
    assert np.array_equal(n, head["n_t"])
    _say("case: benchmark batch, 256 plates, default plan, 100 x 441-step graph launches")
    insts = [physics.plate_instance(w) for w in wls]
    sim = modal.Sim(insts, 44100.0, flags=modal.FLAG_GRAPH | modal.FLAG_ASYNC, chunk_steps=441)
    assert sim.info()["blocked_instances"] == 256
    del insts
    S, steps = 441, 44100
    y = torch.empty((256, steps), device="cuda")
    buf = torch.empty((256, S), device="cuda")  # the benchmark's output buffer
    for i in range(steps // S):
        sim.run(S, out=buf)
        y[:, i * S:(i + 1) * S].copy_(buf)
    sim.check()
    sim.close()
    y = y.double().cpu().numpy()
    hs = int(head["steps"])
    errs = np.array([rel_l2(y[b, :hs], head["y"][b].astype(float)) for b in range(256)])
    worst = int(np.argmax(errs))
    _say(f"  all 256 plates, {hs} steps: worst rel L2 {errs[worst]:.2e} (plate {worst}, N={n[worst]})")
    assert errs.max() < TOL, (worst, n[worst], errs[worst])
    for k, b in enumerate(full["index"]):
        e = rel_l2(y[b], full["y"][k].astype(float))
        _say(f"  plate {b} (N={n[b]}), 44100 steps: rel L2 {e:.2e}")
        assert e < TOL, (b, n[b], e)


@pytest.mark.timeout(600)
def test_paper_shape_100_modes_one_second():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_05940_amd import modal, physics
    g = _load("sweep_100.npz")
    steps = int(g["steps"])
    for name, inst in (("vK plate 100/100", physics.plate_instance(W.plate_sweep(100))),
                       ("Berger plate 100", physics.plate_berger_instance(W.plate_berger(n_t=100)))):
        _say(f"case: {name}, {steps} steps, default plan")
        sim = modal.Sim([inst], 44100.0)
        y = sim.run(steps)[0].double().cpu().numpy()
        sim.close()
        ref = (g["vk"] if name.startswith("vK") else g["berger"]).astype(float)
        e = rel_l2(y, ref)
        _say(f"  rel L2 {e:.2e}")
        assert e < TOL, (name, e)
