"""FP64 time loop of the modal system with the nonlinear modal force.

Paper, Sec. 3.2: q^{n+1} = g . q^n + p . q^{n-1} + r . (f_ext^n - f_nl^n)
(Stormer-Verlet, modal oscillator update; the impulse-invariant recursion
has the same shape with other coefficients).  Output y^n = sum_k c_k q_k^n
(modal to physical transform at one point, Sec. 4.1).

Nonlinear forces (Sec. 3.1):
* tension-modulated string / membrane (modal string-membrane equation): with
  normalised modes, f_nl,mu = kappa lambda_mu q_mu sum_nu lambda_nu q_nu^2,
  kappa = tau / rho_s.
* von Karman plate (nonlinear plate equation) with the scaled tensor H~:
  eta_n = sum_pq H~[n,p,q] q_p q_q, then f_nl,k = sum_{n,q} H~[n,k,q] q_q eta_n.

An instance is a dict with
    kind: 'linear' | 'tension' | 'vk'
    omega, gamma: [N] rad/s and 1/s
    lam, kappa:  tension only
    Ht: [N_in, N, N] scaled coupling tensor (vk only)
    x0, xm1: [N] initial state q^0 and q^-1
    c: [N] output weights
    b_ext [N], e_ext [n_exc] (optional): f_ext^n = b_ext * e_ext[n]
"""
from __future__ import annotations

import numpy as np

from .scheme import sv_coefficients, tf_coefficients


def force_tension(X, lam, kappa):
    """f_mu = kappa lambda_mu X_mu sum_nu lambda_nu X_nu^2."""
    return kappa * lam * X * np.sum(lam * X * X)


def force_vk(X, Ht):
    """The two contractions against H~: eta_n = sum_pq H~[n,p,q] X_p X_q,
    f_k = sum_{n,q} H~[n,k,q] X_q eta_n."""
    n_in, n, _ = Ht.shape
    eta = Ht.reshape(n_in, n * n) @ np.outer(X, X).ravel()
    return np.tensordot(eta, Ht, axes=(0, 0)) @ X


def modal_force(inst, X):
    kind = inst["kind"]
    if kind == "linear":
        return np.zeros_like(X)
    if kind == "tension":
        return force_tension(X, inst["lam"], inst["kappa"])
    if kind == "vk":
        return force_vk(X, inst["Ht"])
    raise ValueError(kind)


def coefficients(inst, fs, scheme="sv"):
    T = 1.0 / fs
    if scheme == "sv":
        return sv_coefficients(inst["omega"], inst["gamma"], T)
    if scheme == "tf":
        return tf_coefficients(inst["omega"], inst["gamma"], T)
    raise ValueError(scheme)


def external_force(inst, n):
    e = inst.get("e_ext")
    if e is None or n >= len(e):
        return 0.0
    return inst["b_ext"] * e[n]


def run(inst, n_steps, fs, scheme="sv", return_states=False):
    """Direct two-step recursion in FP64.  Returns y [n_steps] (and the
    states q^0..q^n_steps if asked)."""
    g, p, r = coefficients(inst, fs, scheme)
    Xm = np.array(inst["xm1"], dtype=float)
    X = np.array(inst["x0"], dtype=float)
    c = inst["c"]
    y = np.empty(n_steps)
    states = [X.copy()] if return_states else None
    for n in range(n_steps):
        y[n] = c @ X
        F = modal_force(inst, X)
        Xn = g * X + p * Xm + r * (external_force(inst, n) - F)
        Xm, X = X, Xn
        if return_states:
            states.append(X.copy())
    if return_states:
        return y, np.array(states)
    return y


def run_increment(inst, n_steps, fs, scheme="sv"):
    """The same recursion in increment form, d = q^n - q^{n-1}:
    d^{n+1} = (g + p - 1) q^n - p d^n + r (f_ext - f_nl), q^{n+1} = q^n + d^{n+1}.
    Algebraically identical to ``run``."""
    g, p, r = coefficients(inst, fs, scheme)
    m = g + p - 1.0
    X = np.array(inst["x0"], dtype=float)
    d = X - np.array(inst["xm1"], dtype=float)
    c = inst["c"]
    y = np.empty(n_steps)
    for n in range(n_steps):
        y[n] = c @ X
        F = modal_force(inst, X)
        d = m * X - p * d + r * (external_force(inst, n) - F)
        X = X + d
    return y


def run_batch(insts, n_steps, fs, scheme="sv"):
    """Independent instances, one after the other."""
    return [run(i, n_steps, fs, scheme) for i in insts]
