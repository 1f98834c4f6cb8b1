"""Writes the stored oracle results that the GPU parity tests compare with.

Every value here comes from the FP64 oracle (``oracle/``) on the seeded
workloads (``workloads``); nothing is read from the product.  Run on the CPU:

    python tests/golden/make_golden.py batch      # 256 plates x 2205 steps, 8 x 1 s
    python tests/golden/make_golden.py sweep      # 100-mode vK and Berger plates, 1 s
    python tests/golden/make_golden.py gradient   # 200/200 plate: MR-STFT theta-gradient
    python tests/golden/make_golden.py gradient_sc  # the same for the spectral-convergence terms
    python tests/golden/make_golden.py all

Files (outputs stored as float32: their rounding, about 6e-8 relative, is far
below the 1e-5 parity bar):

* ``batch_head.npz``: outputs of all 256 plates of the batched workload
  (seed 3, N ~ U{50..400}) for the first 2205 steps.
* ``batch_full.npz``: 8 of those plates, chosen at evenly spaced ranks of N
  (the smallest and the 400-mode plate included), for 44 100 steps (1 s).
* ``sweep_100.npz``: the single plate's geometry at 100/100 modes (sine
  in-plane family) and the 100-mode Berger plate, 44 100 steps each.
* ``gradient_200.json`` + ``gradient_200.npz``: the 200/200-mode fitting
  plate (seed 4).  The target is the oracle's output at the perturbed
  parameters; at the base parameters theta0 = (T0/rho_s, D/rho_s, a,
  d1/(2 rho_s), d3/(2 rho_s)) the file holds the MR-STFT loss, its gradient
  by the oracle's reverse recursion and the chain rule through the
  parameterised plate, and central differences of the loss at relative
  steps of 1e-4 (the configured step) and 1e-6; the npz holds the target and
  the output at theta0.
* ``gradient_200_sc.json``: the same for the loss's spectral-convergence
  terms alone.  The log-magnitude term is only piecewise differentiable (an
  absolute value per STFT bin), and at the configured relative step of 1e-4
  the central differences of the full loss cross enough of its kinks to
  miss the derivative by tens of per cent for D^ and a; without it the loss
  is smooth and the differences are a valid check.
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

FS = 44100.0
HEAD_STEPS = 2205
FULL_STEPS = 44100


def _limit_threads(n):
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(n)
    except ImportError:
        pass


def _plate_output(args):
    """Output of batch plate ``index`` over ``steps`` steps (worker)."""
    index, steps, threads = args
    _limit_threads(threads)
    import workloads as W
    from oracle import adjoint as OA
    from oracle import instances as OI
    wl = W.plate_batch(seed=3, batch=256)[index]
    t0 = time.time()
    y = OA.forward(OI.plate_instance(wl), steps, FS)[0]
    print(f"  plate {index} (N={wl['n_t']}): {steps} steps in {time.time() - t0:.0f} s", flush=True)
    return index, y.astype(np.float32)


def full_indices():
    """8 plates at evenly spaced ranks of N (stable order)."""
    import workloads as W
    n = np.array([w["n_t"] for w in W.plate_batch(seed=3, batch=256)])
    order = np.argsort(n, kind="stable")
    return [int(order[i]) for i in np.round(np.linspace(0, len(n) - 1, 8)).astype(int)]


def batch(workers):
    import workloads as W
    n = np.array([w["n_t"] for w in W.plate_batch(seed=3, batch=256)])
    threads = max(1, 8 // workers)
    # largest first, so that the pool drains evenly
    jobs = [(int(i), HEAD_STEPS, threads) for i in np.argsort(-n, kind="stable")]
    y = np.zeros((256, HEAD_STEPS), np.float32)
    with ProcessPoolExecutor(workers) as ex:
        for i, yi in ex.map(_plate_output, jobs):
            y[i] = yi
    np.savez(os.path.join(HERE, "batch_head.npz"), y=y, n_t=n, steps=HEAD_STEPS, seed=3)
    idx = full_indices()
    jobs = [(i, FULL_STEPS, threads) for i in sorted(idx, key=lambda i: -n[i])]
    yf = {}
    with ProcessPoolExecutor(workers) as ex:
        for i, yi in ex.map(_plate_output, jobs):
            yf[i] = yi
    np.savez(os.path.join(HERE, "batch_full.npz"), index=np.array(idx),
             y=np.stack([yf[i] for i in idx]), n_t=n[idx], steps=FULL_STEPS, seed=3)


def sweep():
    import workloads as W
    from oracle import adjoint as OA
    from oracle import instances as OI
    vk = OA.forward(OI.plate_instance(W.plate_sweep(100)), FULL_STEPS, FS)[0]
    berger = OA.forward(OI.plate_berger_instance(W.plate_berger(n_t=100)), FULL_STEPS, FS)[0]
    np.savez(os.path.join(HERE, "sweep_100.npz"), vk=vk.astype(np.float32),
             berger=berger.astype(np.float32), steps=FULL_STEPS)


def _loss_at(args):
    theta, target, threads, log_term = args
    _limit_threads(threads)
    import workloads as W
    from oracle import adjoint as OA
    from oracle import losses as OL
    from oracle import params as OP
    fit = W.plate_fit()
    y = OA.forward(OP.plate_from_theta(fit, np.asarray(theta)), FULL_STEPS, FS)[0]
    return float(OL.mrstft_loss(y, target, log_term=log_term))


def gradient(workers, log_term=True):
    """Theta-gradient of the MR-STFT loss of the 200/200 plate at theta0
    (log_term=False: of its spectral-convergence terms alone, a loss that is
    differentiable wherever no STFT bin vanishes, so that central
    differences at the configured step are a valid check)."""
    import workloads as W
    from oracle import adjoint as OA
    from oracle import losses as OL
    from oracle import params as OP
    fit = W.plate_fit()
    th0 = np.asarray(fit["theta0"], float)
    tht = np.asarray(fit["theta_target"], float)
    t0 = time.time()
    target = OA.forward(OP.plate_from_theta(fit, tht), FULL_STEPS, FS)[0]
    inst = OP.plate_from_theta(fit, th0)
    y0 = OA.forward(inst, FULL_STEPS, FS)[0]
    L0 = float(OL.mrstft_loss(y0, target, log_term=log_term))
    ybar = OL.mrstft_loss_grad(y0, target, log_term=log_term)
    print(f"  forward passes and loss {L0:.6f} in {time.time() - t0:.0f} s", flush=True)
    # derivatives of the parameterised plate's pieces by central differences
    # (smooth maps without a time loop), step 1e-6 relative
    keys = ("omega", "gamma", "x0", "c", "Ht")
    dpiece = []
    for j in range(5):
        e = 1e-6 * th0[j]
        tp, tm = th0.copy(), th0.copy()
        tp[j] += e
        tm[j] -= e
        a, b = OP.plate_from_theta(fit, tp), OP.plate_from_theta(fit, tm)
        dpiece.append({k: (a[k] - b[k]) / (2 * e) for k in keys})
    t0 = time.time()
    g = OA.reverse(inst, FULL_STEPS, FS, ybar, Hdot=[d["Ht"] for d in dpiece])
    print(f"  reverse pass in {time.time() - t0:.0f} s", flush=True)
    T = 1.0 / FS
    g_omega, g_gamma = OA.sv_omega_gamma_grads(g, inst["omega"], inst["gamma"], T)
    grad = np.array([
        np.sum(g_omega * d["omega"]) + np.sum(g_gamma * d["gamma"])
        + np.sum((g["x0"] + g["xm1"]) * d["x0"]) + np.sum(g["c"] * d["c"]) + g["theta"][j]
        for j, d in enumerate(dpiece)])
    # central differences of the loss at the configured relative step 1e-4,
    # and at 1e-6: the log-magnitude term is not differentiable where a bin's
    # log difference changes sign, and a larger step crosses more such kinks
    fd = {}
    Ls = {}
    for eps in (1e-4, 1e-6):
        jobs = []
        for j in range(5):
            for s in (1.0, -1.0):
                th = th0.copy()
                th[j] += s * eps * th0[j]
                jobs.append((th.tolist(), target, max(1, 8 // workers), log_term))
        t0 = time.time()
        with ProcessPoolExecutor(workers) as ex:
            L = list(ex.map(_loss_at, jobs))
        fd[eps] = [(L[2 * j] - L[2 * j + 1]) / (2 * eps * th0[j]) for j in range(5)]
        Ls[eps] = L
        print(f"  differences at {eps:g} in {time.time() - t0:.0f} s", flush=True)
    rec = dict(
        workload="von Karman plate, 200 transverse and 200 in-plane sine modes, area 0.12 m^2, "
                 "1 mm steel, 44100 steps at 44.1 kHz, strike 1 h; target from the perturbed "
                 "parameters (seed 4)",
        loss_terms="spectral convergence + log magnitude" if log_term else "spectral convergence only",
        params=["T0/rho_s", "D/rho_s", "aspect", "d1/(2 rho_s)", "d3/(2 rho_s)"],
        theta0=th0.tolist(), theta_target=tht.tolist(), steps=FULL_STEPS, loss=L0,
        grad_reverse=grad.tolist(), grad_fd=fd[1e-4], grad_fd_1e6=fd[1e-6], fd_rel_step=1e-4,
        loss_fd=Ls[1e-4], loss_fd_1e6=Ls[1e-6],
        note="oracle only: reverse recursion + chain rule, and central differences")
    name = "gradient_200" if log_term else "gradient_200_sc"
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(rec, f, indent=1)
    if log_term:
        np.savez(os.path.join(HERE, "gradient_200.npz"), target=target.astype(np.float32),
                 y0=y0.astype(np.float32))
    print(json.dumps({k: rec[k] for k in ("loss", "grad_reverse", "grad_fd", "grad_fd_1e6")}),
          flush=True)


def ybar():
    """The config-4 adjoint inputs in FP64: the oracle's output at theta0 and
    the target's, and dL/dy of the MR-STFT loss (with and without its
    log-magnitude term) at them, so that a test can drive the product's
    reverse pass with exactly the oracle's dL/dy (the log-magnitude term's
    dL/dy responds to FP32 rounding of the output in near-silent bins)."""
    import workloads as W
    from oracle import adjoint as OA
    from oracle import losses as OL
    from oracle import params as OP
    fit = W.plate_fit()
    th0 = np.asarray(fit["theta0"], float)
    tht = np.asarray(fit["theta_target"], float)
    t0 = time.time()
    target = OA.forward(OP.plate_from_theta(fit, tht), FULL_STEPS, FS)[0]
    y0 = OA.forward(OP.plate_from_theta(fit, th0), FULL_STEPS, FS)[0]
    print(f"  forward passes in {time.time() - t0:.0f} s", flush=True)
    np.savez(os.path.join(HERE, "gradient_200_ybar.npz"), y0=y0, target=target,
             ybar=OL.mrstft_loss_grad(y0, target, log_term=True),
             ybar_sc=OL.mrstft_loss_grad(y0, target, log_term=False))


def main():
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    workers = int(os.environ.get("GOLDEN_WORKERS", "4"))
    if what in ("sweep", "all"):
        sweep()
    if what in ("gradient", "all"):
        gradient(workers)
    if what in ("gradient_sc", "all"):
        gradient(workers, log_term=False)
    if what in ("ybar", "all"):
        ybar()
    if what in ("batch", "all"):
        batch(workers)


if __name__ == "__main__":
    main()
