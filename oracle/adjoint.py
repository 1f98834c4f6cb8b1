"""Reverse-mode gradient of the time loop (back-propagation through time),
FP64, plus the complex-step derivative it is checked against.

Paper, Sec. 4.3 (plate experiments): parameters are fitted by propagating
gradients through the time integrator.  The loop of Sec. 3.2 in increment
form, d = q^n - q^{n-1}, is
    y^n     = c . q^n
    d^{n+1} = m q^n - p d^n + r (f_ext^n - F(q^n))
    q^{n+1} = q^n + d^{n+1}
with m = g + p - 1.  Writing qb^n = dL/dq^n and db^n = dL/dd^n for the total
derivatives of a loss L(y^0..y^{N-1}), and qb^N = db^{N+1} = 0:
    db^{n+1} = qb^{n+1} - p db^{n+2}
    u^n      = r db^{n+1}
    qb^n     = ybar^n c + qb^{n+1} + m db^{n+1} - J(q^n) u^n,   J = dF/dq
and the coefficient gradients are
    dL/dm = sum_n db^{n+1} q^n,  dL/dp = -sum_n db^{n+1} d^n,
    dL/dr = sum_n db^{n+1} (f_ext^n - F^n).
J is symmetric (F is the gradient of a potential).  For the von Karman force
with V = H~ q per in-plane row, eta = V . q:
    (J u)_k = sum_i 2 (V_i . u) V_ik + eta_i (H~_i u)_k.
A force scale s (F proportional to s) gets dL/ds = -sum_n u^n . F^n / s; a
tensor direction Hdot gets dL/dtheta = -sum_n u^n . dF^n with
dF_k = sum_i (Vdot_i . q) V_ik + eta_i Vdot_ik, Vdot = Hdot q.
The gradient with respect to every entry of the tensor (each entry taken as
an independent parameter, Sec. 4.3 fits of the coupling tensor) follows from
d eta_i / dH~[i][a][b] = q_a q_b and d V_ik / dH~[i][a][b] = delta_ka q_b:
    dL/dH~[i][a][b] = -sum_n ((V_i . u) q_a + eta_i u_a) q_b   (at step n).
"""
from __future__ import annotations

import numpy as np

from .scheme import sv_coefficients, tf_coefficients


def _coeffs(inst, fs, scheme):
    T = 1.0 / fs
    if scheme == "sv":
        return sv_coefficients(inst["omega"], inst["gamma"], T)
    return tf_coefficients(inst["omega"], inst["gamma"], T)


def _force(inst, X):
    kind = inst["kind"]
    if kind == "linear":
        return np.zeros_like(X)
    if kind == "tension":
        lam = inst["lam"]
        return inst["kappa"] * lam * X * np.sum(lam * X * X)
    Ht = inst["Ht"]
    n_in, n, _ = Ht.shape
    V = Ht.reshape(n_in * n, n) @ X
    V = V.reshape(n_in, n)
    eta = V @ X
    return eta @ V


def _jvp(inst, X, u):
    """J(X) u with J = dF/dX."""
    kind = inst["kind"]
    if kind == "linear":
        return np.zeros_like(u)
    if kind == "tension":
        lam, kap = inst["lam"], inst["kappa"]
        S = np.sum(lam * X * X)
        return kap * lam * (u * S + X * 2.0 * np.sum(lam * X * u))
    Ht = inst["Ht"]
    n_in, n, _ = Ht.shape
    V = (Ht.reshape(n_in * n, n) @ X).reshape(n_in, n)
    W = (Ht.reshape(n_in * n, n) @ u).reshape(n_in, n)
    eta = V @ X
    w = V @ u
    return 2.0 * (w @ V) + eta @ W


def _ext(inst, n, like):
    e = inst.get("e_ext")
    if e is None or n >= len(e):
        return np.zeros_like(like)
    return inst["b_ext"] * e[n]


def forward(inst, n_steps, fs, scheme="sv"):
    """Increment-form loop (any float or complex dtype).  Returns y [N] and
    the states q^n, d^n and forces F^n for n < N."""
    g, p, r = _coeffs(inst, fs, scheme)
    m = g + p - 1.0
    X = np.array(inst["x0"])
    d = X - np.array(inst["xm1"])
    c = inst["c"]
    dt = np.result_type(X, d, m, p, r, c, *(np.asarray(inst[k]) for k in ("Ht", "kappa", "lam")
                                         if inst.get(k) is not None))
    y = np.empty(n_steps, dtype=dt)
    Xs = np.empty((n_steps, len(X)), dtype=dt)
    ds = np.empty_like(Xs)
    Fs = np.empty_like(Xs)
    for n in range(n_steps):
        y[n] = c @ X
        F = _force(inst, X)
        Xs[n], ds[n], Fs[n] = X, d, F
        d = m * X - p * d + r * (_ext(inst, n, X) - F)
        X = X + d
    return y, Xs, ds, Fs


def reverse(inst, n_steps, fs, ybar, scheme="sv", Hdot=None, full_tensor=False):
    """Gradients of L with dL/dy^n = ybar[n].

    Returns dict: m, p, r (per mode), x0, xm1 (per mode), c (per mode),
    scale (force scale s, the nonlinearity's prefactor), theta (if Hdot;
    Hdot may also be a list of tangent tensors, one theta per entry),
    and for a von Karman instance row (per in-plane mode n): dL/d log s_n for
    a factor s_n on row n of the scaled tensor.  That factor scales V_n and
    eta_n together, so the force term eta_n V_n goes as s_n^2 and
    dL/d log s_n = -2 sum over steps of eta_n (V_n . u).
    With full_tensor, also H: dL/dH~ entry by entry, [n_in][n][n].
    """
    g, p, r = _coeffs(inst, fs, scheme)
    m = g + p - 1.0
    _, Xs, ds, Fs = forward(inst, n_steps, fs, scheme)
    c = inst["c"]
    n = len(c)
    qb = np.zeros(n)
    db_next = np.zeros(n)  # db^{n+2}
    gm, gp, gr, gc = (np.zeros(n) for _ in range(4))
    gs = 0.0
    many = isinstance(Hdot, (list, tuple))
    Hdots = list(Hdot) if many else ([] if Hdot is None else [Hdot])
    gth = np.zeros(len(Hdots))
    vk = inst["kind"] == "vk"
    grow = np.zeros(inst["Ht"].shape[0]) if vk else None
    gH = np.zeros(inst["Ht"].shape) if (vk and full_tensor) else None
    for k in range(n_steps - 1, -1, -1):
        db = qb - p * db_next          # db^{k+1}
        u = r * db
        X = Xs[k]
        gm += db * X
        gp -= db * ds[k]
        gr += db * (_ext(inst, k, X) - Fs[k])
        gc += ybar[k] * X
        gs -= u @ Fs[k]
        if vk:
            n_in = inst["Ht"].shape[0]
            V = (inst["Ht"].reshape(n_in * n, n) @ X).reshape(n_in, n)
            grow = grow - 2.0 * (V @ X) * (V @ u)
            if gH is not None:
                eta, w = V @ X, V @ u
                for i in range(n_in):
                    gH[i] -= np.outer(w[i] * X + eta[i] * u, X)
        for j, Hd in enumerate(Hdots):
            n_in = Hd.shape[0]
            V = (inst["Ht"].reshape(n_in * n, n) @ X).reshape(n_in, n)
            Vd = (Hd.reshape(n_in * n, n) @ X).reshape(n_in, n)
            eta, etad = V @ X, Vd @ X
            dF = etad @ V + eta @ Vd
            gth[j] -= u @ dF
        qb = ybar[k] * c + qb + m * db - _jvp(inst, X, u)
        db_next = db
    d0b = -p * db_next  # d^0 only feeds d^1
    theta = list(gth) if many else (float(gth[0]) if Hdots else 0.0)
    return dict(m=gm, p=gp, r=gr, c=gc, x0=qb + d0b, xm1=-d0b, scale=gs, theta=theta, row=grow, H=gH)


def sv_omega_gamma_grads(g, omega, gamma, T):
    """Chain rule from (m, p, r) of Stormer-Verlet to (omega, gamma):
    r = T^2/(1 + gamma T), p = -(1 - gamma T)/(1 + gamma T), m = -r omega^2."""
    r = T * T / (1.0 + gamma * T)
    dr = -T ** 3 / (1.0 + gamma * T) ** 2
    dp = 2.0 * T / (1.0 + gamma * T) ** 2
    d_omega = g["m"] * (-2.0 * r * omega)
    d_gamma = g["m"] * (-omega ** 2 * dr) + g["p"] * dp + g["r"] * dr
    return d_omega, d_gamma


def complex_step(fn, theta, h=1e-30):
    """d fn / d theta by the complex step: Im(fn(theta + i h)) / h."""
    return np.imag(fn(theta + 1j * h)) / h
