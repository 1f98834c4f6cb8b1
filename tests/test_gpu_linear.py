"""Linear batches on the closed-form path (time-parallel FP64 evaluation of
each mode's recursion from the roots of its characteristic polynomial)
against the FP64 oracle's step-by-step recursion.  Bar: relative L2 <= 1e-5
per output signal (the closed form is exact up to FP64 rounding; the FP32
output limits it to about 1e-7)."""
import numpy as np
import pytest

import workloads as W
from oracle import simulate as OS

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel_l2(y, ref):
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available()
    from paper_2505_05940_amd import modal
    return modal


@pytest.mark.parametrize("scheme", ["sv", "tf"])
def test_linear_batch_full_second(gpu, scheme):
    modal = gpu
    wl = W.linear_batch(batch=24, n_steps=44100)
    insts = wl["instances"]
    print(f"case: linear batch of 24 strings, 44100 steps, {scheme}", flush=True)
    sim = modal.Sim(insts, wl["fs"], scheme=scheme)
    assert sim.info()["path"] == 2
    y = sim.run(44100).double().cpu().numpy()
    for b in (0, 3, 7, 8, 23):  # forced and free strings
        ref = OS.run(dict(insts[b]), 44100, wl["fs"], scheme=scheme)
        assert rel_l2(y[b], ref) < TOL, (b, rel_l2(y[b], ref))
    yr = modal.Sim(insts, wl["fs"], scheme=scheme, flags=modal.FLAG_RECURSE)
    assert yr.info()["path"] in (0, 3)  # the recursion (streaming or on-chip)
    y2 = yr.run(44100).double().cpu().numpy()
    assert max(rel_l2(y[b], y2[b]) for b in range(24)) < 2 * TOL


def test_linear_resume_and_state(gpu):
    modal = gpu
    wl = W.linear_batch(seed=10, batch=6, n_steps=2000, forced=3)
    insts = wl["instances"]
    print("case: linear resume and state", flush=True)
    sim = modal.Sim(insts, wl["fs"])
    a = sim.run(700).double().cpu().numpy()
    b = sim.run(1300).double().cpu().numpy()
    x, xm = sim.state()
    sim.reset()
    whole = sim.run(2000).double().cpu().numpy()
    assert np.abs(np.concatenate([a, b], axis=1) - whole).max() <= 1e-6 * np.abs(whole).max()
    off = np.cumsum([0] + sim.n_t)
    for i in (0, 4):
        _, st = OS.run(dict(insts[i]), 2000, wl["fs"], return_states=True)
        assert rel_l2(x[off[i]:off[i + 1]], st[2000]) < TOL
        assert rel_l2(xm[off[i]:off[i + 1]], st[1999]) < TOL


def test_double_root_keeps_the_recursion(gpu):
    """A critically damped SV mode (double root of z^2 - g z - p, up to
    rounding) sends the batch to the recursion, which still matches."""
    modal = gpu
    fs, T = 44100.0, 1 / 44100.0
    gam = 300.0
    # SV: r = T^2/(1+gT), p = -(1-gT)/(1+gT), g = r (2/T^2 - w^2); g^2 = -4p
    p = -(1 - gam * T) / (1 + gam * T)
    r = T * T / (1 + gam * T)
    g = np.sqrt(-4 * p)
    w = np.sqrt(2 / T ** 2 - g / r)
    inst = dict(kind="linear", omega=np.array([w, 2 * w]), gamma=np.array([gam, gam]),
                x0=np.array([1e-3, 1e-3]), xm1=np.array([1e-3, 1e-3]), c=np.array([1.0, 1.0]))
    sim = modal.Sim([inst], fs)
    assert sim.info()["path"] in (0, 3)  # the recursion (streaming or on-chip)
    y = sim.run(500).double().cpu().numpy()[0]
    assert rel_l2(y, OS.run(dict(inst), 500, fs)) < TOL


def _sv_disc(w, gam, fs=44100.0):
    T = 1 / fs
    r = T * T / (1 + gam * T)
    p = -(1 - gam * T) / (1 + gam * T)
    g = r * (2 / T ** 2 - w * w)
    return g * g + 4 * p, g, p


def test_real_roots_groups_and_windows(gpu):
    """Real root pairs (positive, negative and of both signs) beside more than
    64 complex-conjugate pairs in one forced instance, and an unforced
    instance, run in uneven windows that split at the end of the excitation
    and inside a 64-step lane stride."""
    modal = gpu
    fs = 44100.0
    rng = np.random.default_rng(21)
    w = 2 * np.pi * np.linspace(100.0, 11000.0, 70)
    gam = 1.0 + 2e-8 * w * w
    # overdamped: two positive roots; two negative roots; one of each sign
    w = np.concatenate([w, [600.0, 80000.0, 1000.0]])
    gam = np.concatenate([gam, [2e4, 4e4, 5e4]])
    disc, g, p = _sv_disc(w, gam)
    assert (disc[:70] < 0).all() and (disc[70:] > 0).all()
    assert g[70] > 0 and g[71] < 0 and p[72] > 0
    n = len(w)
    x0 = 1e-3 * rng.normal(size=n)
    forced = dict(kind="linear", omega=w, gamma=gam, x0=x0, xm1=0.9 * x0, c=rng.normal(size=n),
                  b_ext=rng.normal(size=n), e_ext=(1e2 * rng.normal(size=300)).astype(np.float32))
    free = dict(kind="linear", omega=w[::2].copy(), gamma=gam[::2].copy(), x0=x0[::2].copy(),
                xm1=x0[::2].copy(), c=np.ones(len(w[::2])))
    insts = [forced, free]
    sim = modal.Sim(insts, fs)
    assert sim.info()["path"] == 2
    print("case: real roots, 73 modes, windows 100/37/163/2700", flush=True)
    y = np.concatenate([sim.run(k).double().cpu().numpy() for k in (100, 37, 163, 2700)], axis=1)
    for i in range(2):
        ref = OS.run(dict(insts[i]), 3000, fs)
        assert rel_l2(y[i], ref) < TOL, (i, rel_l2(y[i], ref))
        assert np.abs(y[i, :400] - ref[:400]).max() < TOL * np.abs(ref[:400]).max()
