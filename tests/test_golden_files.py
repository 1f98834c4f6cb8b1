"""Consistency of the stored oracle outputs (tests/golden/, written by
tests/golden/make_golden.py from oracle/ only) before any GPU test uses them:
shapes and workloads match the generators, and the stored config-4 gradient
of the reverse recursion agrees with the stored central differences where
differences are a valid derivative estimate (Sec. 4.3: gradients through the
time loop)."""
import json
import os

import numpy as np

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _json(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_batch_outputs_cover_every_plate_and_the_largest_for_one_second():
    head = np.load(os.path.join(GOLDEN, "batch_head.npz"))
    full = np.load(os.path.join(GOLDEN, "batch_full.npz"))
    n = np.array([w["n_t"] for w in W.plate_batch(seed=3, batch=256)])
    assert np.array_equal(head["n_t"], n)
    assert head["y"].shape == (256, int(head["steps"])) and int(head["steps"]) >= 2205
    idx = np.asarray(full["index"])
    assert full["y"].shape == (len(idx), 44100) and len(idx) >= 8
    assert n[idx].max() == n.max()  # the 400-mode plate is among them
    assert np.all(np.isfinite(head["y"])) and np.all(np.isfinite(full["y"]))
    # the one-second records start with the 2205-step ones (same oracle run)
    for k, b in enumerate(idx):
        assert np.array_equal(full["y"][k][:int(head["steps"])], head["y"][b])


def test_sweep_outputs_are_one_second():
    g = np.load(os.path.join(GOLDEN, "sweep_100.npz"))
    assert int(g["steps"]) == 44100
    assert g["vk"].shape == (44100,) and g["berger"].shape == (44100,)


def test_config4_reverse_gradient_matches_fine_differences():
    """The spectral-convergence loss is smooth where no STFT bin vanishes;
    its central differences at a relative step of 1e-6 agree with the
    reverse recursion + chain rule to 1e-3 per component.  At the configured
    step 1e-4 they do not (the phase of a 5 kHz mode moves by about 1.6 rad
    over the second per 1e-4 of D^), which the stored values show too."""
    sc = _json("gradient_200_sc.json")
    full = _json("gradient_200.json")
    assert sc["theta0"] == full["theta0"] and sc["steps"] == full["steps"] == 44100
    rev, fd6, fd4 = (np.asarray(sc[k]) for k in ("grad_reverse", "grad_fd_1e6", "grad_fd"))
    err6 = np.abs(rev - fd6) / np.abs(rev)
    assert err6.max() < 1e-3, err6
    assert (np.abs(rev - fd4) / np.abs(rev)).max() > 0.1
    # the full loss: same signs and magnitudes from both, but not to 1e-3
    rf, ff = np.asarray(full["grad_reverse"]), np.asarray(full["grad_fd_1e6"])
    assert np.all(np.sign(rf) == np.sign(ff))
    assert (np.abs(rf - ff) / np.abs(rf)).max() < 2e-2
