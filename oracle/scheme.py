"""Modal ODE coefficients and the two time-stepping schemes.

Paper, Sec. 3.2 (integration in time).  Each mode obeys
    q'' + 2 gamma q' + omega^2 q = f_ext - f_nl          (modal oscillator)
with omega^2 = (D lambda^2 + T0 lambda) / rho_s and
gamma = (d1 + d3 lambda) / (2 rho_s), where rho_s is the mass per unit area
(plates) or length (strings).
"""
from __future__ import annotations

import numpy as np


def omega_from(lam, D, T0, rho_s):
    """Angular frequency omega = sqrt((D lambda^2 + T0 lambda) / rho_s)."""
    lam = np.asarray(lam) * 1.0
    return np.sqrt((D * lam ** 2 + T0 * lam) / rho_s)


def gamma_from_d(lam, d1, d3, rho_s):
    """Decay rate gamma = (d1 + d3 lambda) / (2 rho_s)."""
    return (d1 + d3 * np.asarray(lam)) / (2.0 * rho_s)


def gamma_affine_omega(omega, g0, g1):
    """Decay rate gamma_k = g0 + g1 omega_k (the workloads' damping law)."""
    return g0 + g1 * np.asarray(omega, dtype=float)


def sv_coefficients(omega, gamma, T):
    """Stormer-Verlet recursion q+ = g q + p q- + r (f_ext - f_nl)
    (Sec. 3.2, modal oscillator update):
        r = 2 T^2 / (2 + 2 gamma T)
        g = r (2 / T^2 - omega^2)
        p = r (-1 / T^2 + 2 gamma / (2 T)).
    """
    omega = np.asarray(omega) * 1.0  # real or complex (complex-step checks)
    gamma = np.asarray(gamma) * 1.0
    r = 2.0 * T * T / (2.0 + 2.0 * gamma * T)
    g = r * (2.0 / (T * T) - omega ** 2)
    p = r * (-1.0 / (T * T) + 2.0 * gamma / (2.0 * T))
    return g, p, r


def tf_coefficients(omega, gamma, T):
    """Impulse-invariant recursion (Sec. 3.2, transfer function and its
    update) written as q+ = g q + p q- + r (f_ext - f_nl).

    The discrete transfer function has denominator z^2 + a1 z + a2 with
    a1 = -2 e^{-gamma T} cos(w T), a2 = e^{-2 gamma T}, w = sqrt(omega^2 -
    gamma^2); the matching recursion is q+ = -a1 q - a2 q- + b1 f.  The input
    gain is b1 = T e^{-gamma T} sin(w T) / w for a force per unit mass (the
    impulse response of the continuous oscillator sampled and scaled by T).
    """
    omega = np.asarray(omega, dtype=float)
    gamma = np.asarray(gamma, dtype=float)
    w = np.sqrt(omega ** 2 - gamma ** 2)
    a1 = -2.0 * np.exp(-gamma * T) * np.cos(w * T)
    a2 = np.exp(-2.0 * gamma * T)
    b1 = T * np.exp(-gamma * T) * np.sin(w * T) / w
    return -a1, -a2, b1
