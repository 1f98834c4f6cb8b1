"""Transfer-function route of the linear string fits, plain FP64.

Paper, Sec. 3.2 (transfer function): with impulse invariance each mode is the
discrete system H_mu(z) = b_mu1 z / (z^2 + a_mu1 z + a_mu2), with
a_mu1 = -2 e^{-gamma T} cos(w T), a_mu2 = e^{-2 gamma T}, w^2 = omega^2 - gamma^2
(the coefficients of ``scheme.tf_coefficients``).  Sec. 4.3 (linear string,
first approach): the target's spectral envelope is taken by high-order linear
prediction (LPC) and sampled on the Bark scale; the model's magnitude response
is sampled the same way and compared with the loss of Sec. 4.3 with the STFT
magnitude replaced by these samples.  The extended model adds a second
numerator coefficient b_mu2 per mode (unknown initial conditions) and free
output weights per mode instead of mode shapes:
    H(z) = sum_mu w_mu (b_mu1 z + b_mu2) / (z^2 + a_mu1 z + a_mu2).
The Bark scale is Traunmueller's formula z = 26.81 f / (1960 + f) - 0.53.
This module is test infrastructure: only the tests and the benchmark's CPU
baseline use it.
"""
from __future__ import annotations

import numpy as np


def response(a1, a2, b1, b2, w, Omega):
    """H(e^{i Omega_k}) for the modes given as arrays (one entry per mode);
    Omega in radians per sample.  Returns a complex array [K]."""
    H = np.zeros(len(Omega), dtype=complex)
    for k, Om in enumerate(Omega):
        z = np.exp(1j * Om)
        for m in range(len(a1)):
            H[k] += w[m] * (b1[m] * z + b2[m]) / (z * z + a1[m] * z + a2[m])
    return H


def response_grad(a1, a2, b1, b2, w, Omega, g):
    """Gradient of L = sum_k Re(conj(g_k) H_k) with respect to each mode's
    (a1, a2, b1, b2, w), as an array [modes, 5]: with N = b1 z + b2 and
    D = z^2 + a1 z + a2, dH/dw = N/D, dH/db1 = w z/D, dH/db2 = w/D,
    dH/da1 = -w N z/D^2, dH/da2 = -w N/D^2."""
    out = np.zeros((len(a1), 5))
    for m in range(len(a1)):
        for k, Om in enumerate(Omega):
            z = np.exp(1j * Om)
            N = b1[m] * z + b2[m]
            D = z * z + a1[m] * z + a2[m]
            d = [-w[m] * N * z / D ** 2, -w[m] * N / D ** 2, w[m] * z / D, w[m] / D, N / D]
            for j in range(5):
                out[m, j] += (np.conj(g[k]) * d[j]).real
    return out


def lpc(x, order):
    """Linear prediction by the autocorrelation method and the
    Levinson-Durbin recursion: returns (a [order + 1] with a[0] = 1, so that
    A(z) = sum_k a_k z^{-k}, and the final prediction-error power)."""
    x = np.asarray(x, dtype=float)
    n = len(x)
    r = np.array([np.dot(x[:n - k], x[k:]) for k in range(order + 1)])
    a = np.zeros(order + 1)
    a[0] = 1.0
    err = r[0]
    for i in range(1, order + 1):
        acc = r[i]
        for j in range(1, i):
            acc += a[j] * r[i - j]
        k = -acc / err
        prev = a.copy()
        for j in range(1, i):
            a[j] = prev[j] + k * prev[i - j]
        a[i] = k
        err *= 1.0 - k * k
    return a, err


def lpc_envelope(a, err, Omega):
    """Magnitude of the all-pole model sqrt(err) / |A(e^{i Omega})|."""
    out = np.empty(len(Omega))
    for k, Om in enumerate(Omega):
        A = sum(a[j] * np.exp(-1j * Om * j) for j in range(len(a)))
        out[k] = np.sqrt(err) / abs(A)
    return out


def hz_to_bark(f):
    f = np.asarray(f, dtype=float)
    return 26.81 * f / (1960.0 + f) - 0.53


def bark_to_hz(z):
    z = np.asarray(z, dtype=float)
    return 1960.0 * (z + 0.53) / (26.28 - z)


def bark_grid(n, f_lo, f_hi, fs):
    """n frequencies equally spaced in Bark between f_lo and f_hi (Hz), as
    radians per sample."""
    zb = np.linspace(hz_to_bark(f_lo), hz_to_bark(f_hi), n)
    return 2.0 * np.pi * bark_to_hz(zb) / fs
