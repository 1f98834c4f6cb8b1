"""Transfer-function fits of linear strings (paper: Sec. 4.3, linear string,
first approach; Sec. 3.2, impulse-invariant transfer function).

The target's spectral envelope is taken by high-order linear prediction and
sampled at frequencies equally spaced on the Bark scale (Traunmueller's
formula).  The model is the string's transfer function
    H(z) = sum_mu w_mu (b1_mu z + b2_mu) / (z^2 + a1_mu z + a2_mu),
    a1 = -2 e^{-gamma T} cos(w T), a2 = e^{-2 gamma T},
    b1 = T e^{-gamma T} sin(w T) / w, w^2 = omega^2 - gamma^2,
    omega_mu^2 = D^ lambda_mu^2 + T0^ lambda_mu, gamma_mu = (d1^ + d3^ lambda_mu) / 2,
    lambda_mu = (mu pi)^2  (unit length; the length is absorbed in T0^, D^),
with free output weights w_mu and b2_mu = beta_mu b1_mu (the second numerator
coefficient, for unknown initial conditions).  Its magnitude on the same
grid is compared with the envelope by spectral convergence plus the mean
absolute log difference (the loss of Sec. 4.3 with the STFT magnitude
replaced by the Bark-sampled magnitude).  No time-domain simulation runs.

The response and its gradient run in the library's HIP kernels
(modal_tf_response, modal_tf_grad), in float-float arithmetic; the FP64 chain
from (T0^, D^, d1^, d3^, w, beta) to the coefficients and the loss is torch
on the host (a few hundred modes and frequencies).  The envelope of the
target (linear prediction) is host preprocessing done once.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from .modal import ModalError, _stream_handle
from .modal import lib as _lib


def _check(code):
    if code != 0:
        raise ModalError(code, _lib.modal_last_error().decode())


def bark_grid(n: int, f_lo: float, f_hi: float, fs: float) -> np.ndarray:
    """n frequencies equally spaced in Bark over [f_lo, f_hi] Hz, in radians
    per sample (Bark z = 26.81 f / (1960 + f) - 0.53)."""
    z0 = 26.81 * f_lo / (1960.0 + f_lo) - 0.53
    z1 = 26.81 * f_hi / (1960.0 + f_hi) - 0.53
    zb = np.linspace(z0, z1, n)
    f = 1960.0 * (zb + 0.53) / (26.28 - zb)
    return 2.0 * math.pi * f / fs


def lpc(x, order: int):
    """Linear prediction coefficients (a[0] = 1, A(z) = sum a_j z^-j) and the
    prediction-error power, by the autocorrelation method: autocorrelation
    through the FFT, then the Levinson-Durbin recursion."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    nfft = 1 << int(math.ceil(math.log2(2 * n)))
    X = np.fft.rfft(x, nfft)
    r = np.fft.irfft(X * np.conj(X), nfft)[:order + 1]
    a = np.zeros(order + 1)
    a[0] = 1.0
    e = r[0]
    for i in range(1, order + 1):
        k = -(r[i] + np.dot(a[1:i], r[i - 1:0:-1])) / e
        a[1:i] = a[1:i] + k * a[i - 1:0:-1]
        a[i] = k
        e *= 1.0 - k * k
    return a, e


def lpc_envelope(a, err, Omega) -> np.ndarray:
    """sqrt(err) / |A(e^{i Omega})| on the given grid."""
    j = np.arange(len(a))
    A = np.exp(-1j * np.outer(Omega, j)) @ a
    return math.sqrt(err) / np.abs(A)


class TfResponse(torch.autograd.Function):
    """H [batch, n_freq, 2] (real, imaginary) from coef [modes, 5] =
    (a1, a2, b1, b2, w); host FP64 tensors in and out, evaluated by the
    library's float-float kernels; backward through modal_tf_grad."""

    @staticmethod
    def forward(ctx, coef, mode_off, omega, max_modes):
        assert not coef.is_cuda and coef.dtype == torch.float64 and coef.is_contiguous() and coef.shape[1] == 5
        assert mode_off.dtype == torch.int32 and omega.dtype == torch.float64 and not omega.is_cuda
        B, K = mode_off.numel() - 1, omega.numel()
        H = torch.empty((B, K, 2), dtype=torch.float64)
        cf = coef.detach()
        _check(_lib.modal_tf_response(C.c_void_p(cf.data_ptr()), C.c_void_p(mode_off.data_ptr()), B,
                                      C.c_void_p(omega.data_ptr()), K, C.c_void_p(H.data_ptr()),
                                      _stream_handle(None)))
        ctx.save_for_backward(cf, mode_off, omega)
        ctx.max_modes = int(max_modes)
        return H

    @staticmethod
    def backward(ctx, gH):
        coef, mode_off, omega = ctx.saved_tensors
        gH = gH.contiguous().to(torch.float64)
        g = torch.zeros_like(coef)
        _check(_lib.modal_tf_grad(C.c_void_p(coef.data_ptr()), C.c_void_p(mode_off.data_ptr()),
                                  mode_off.numel() - 1, ctx.max_modes, C.c_void_p(omega.data_ptr()),
                                  omega.numel(), C.c_void_p(gH.data_ptr()), C.c_void_p(g.data_ptr()),
                                  _stream_handle(None)))
        return g, None, None, None


def string_coefficients(theta: torch.Tensor, n_modes: int, fs: float):
    """(a1, a2, b1) of the first n_modes modes of a string with
    theta = (T0^, D^, d1^, d3^)."""
    T = 1.0 / fs
    mu = torch.arange(1, n_modes + 1, dtype=torch.float64, device=theta.device)
    lam = (mu * math.pi) ** 2
    om2 = theta[1] * lam ** 2 + theta[0] * lam
    gam = 0.5 * (theta[2] + theta[3] * lam)
    wd = torch.sqrt(om2 - gam ** 2)
    dec = torch.exp(-gam * T)
    return -2.0 * dec * torch.cos(wd * T), dec * dec, T * dec * torch.sin(wd * T) / wd


def tf_loss(M: torch.Tensor, E: torch.Tensor, eps: float = 1e-5) -> torch.Tensor:
    """Spectral convergence plus mean absolute log difference of two sampled
    magnitude responses."""
    return (torch.linalg.vector_norm(E - M) / torch.linalg.vector_norm(E)
            + (torch.log(E + eps) - torch.log(M + eps)).abs().mean())


def fit_tf(target, fs: float, n_modes: int, theta0, iters: int = 600, lr: float = 0.003,
           lr_modes: float = 0.02, order: int = 200, n_freq: int = 512, f_lo: float = 60.0,
           f_hi: float = 15000.0, callback=None):
    """Fits (T0^, D^, d1^, d3^), the per-mode weights and the second numerator
    coefficients of a string's transfer function to the target's
    Bark-sampled LPC envelope with Adam (logs of the physical parameters).
    Returns (theta, weights, beta, loss history)."""
    dev = torch.device("cpu")  # the chain and the loss; the sums run on the GPU
    Om = bark_grid(n_freq, f_lo, f_hi, fs)
    a, err = lpc(np.asarray(target, dtype=np.float64), order)
    E = torch.tensor(lpc_envelope(a, err, Om), device=dev)
    E = E / E.pow(2).mean().sqrt()
    omega = torch.tensor(Om, device=dev)
    mode_off = torch.tensor([0, n_modes], dtype=torch.int32, device=dev)
    z = torch.tensor(np.log(np.asarray(theta0, dtype=np.float64)), device=dev, requires_grad=True)
    w = torch.ones(n_modes, dtype=torch.float64, device=dev)
    beta = torch.zeros(n_modes, dtype=torch.float64, device=dev, requires_grad=True)

    def magnitude(z, w, beta):
        a1, a2, b1 = string_coefficients(torch.exp(z), n_modes, fs)
        coef = torch.stack([a1, a2, b1, beta * b1, w], dim=1).contiguous()
        H = TfResponse.apply(coef, mode_off, omega, n_modes)[0]
        return torch.sqrt(H[:, 0] ** 2 + H[:, 1] ** 2)

    with torch.no_grad():  # weights start at the envelope's level
        w *= E.pow(2).mean().sqrt() / magnitude(z, w, beta).pow(2).mean().sqrt()
    w.requires_grad_(True)
    opt = torch.optim.Adam([{"params": [z], "lr": lr}, {"params": [w, beta], "lr": lr_modes}])
    hist = []
    for it in range(iters):
        L = tf_loss(magnitude(z, w, beta), E)
        opt.zero_grad(set_to_none=True)
        L.backward()
        opt.step()
        hist.append(float(L.detach()))
        if callback:
            callback(it, hist[-1])
    return torch.exp(z).detach().cpu().numpy(), w.detach().cpu().numpy(), beta.detach().cpu().numpy(), hist
