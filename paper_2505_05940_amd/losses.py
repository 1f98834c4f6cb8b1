"""Spectral losses and features on the caller's side of the C ABI (torch).

Paper, Sec. 4.3 (loss functions): with Y = |STFT(x)| and Yh = |STFT(xh)|,
    L_log = || log(Y + eps) - log(Yh + eps) ||_1
    L_sc  = || Y - Yh ||_F / || Y ||_F.
The multi-resolution loss used here averages L_sc + L_log over FFT sizes
256 / 1024 / 4096 with hop n_fft/4 and a Hann window; the L1 norm is taken as
a mean over bins and eps = 1e-7.

The learned proposal reads a 128-bin log-mel spectrogram of 1 s of audio
averaged over 8 equal time slices (8 x 128 = 1024 features).
"""
from __future__ import annotations

import math

import torch

FFT_SIZES = (256, 1024, 4096)
EPS = 1e-7


def stft_mag(x: torch.Tensor, n_fft: int) -> torch.Tensor:
    """|STFT| of x [..., T] with a Hann window and hop n_fft/4."""
    win = torch.hann_window(n_fft, device=x.device, dtype=x.dtype)
    X = torch.stft(x.reshape(-1, x.shape[-1]), n_fft, hop_length=n_fft // 4, window=win,
                   center=True, return_complex=True)
    return X.abs().reshape(*x.shape[:-1], *X.shape[-2:])


def mrstft_loss(y: torch.Tensor, target: torch.Tensor, reduce: bool = True,
                log_term: bool = True) -> torch.Tensor:
    """Multi-resolution STFT loss of y against target ([..., T] each).
    Returns the mean over the leading dims (or per item if reduce=False).
    log_term=False keeps only the spectral-convergence terms."""
    total = 0.0
    for n in FFT_SIZES:
        Y = stft_mag(target, n)
        Yh = stft_mag(y, n)
        dims = (-2, -1)
        sc = torch.linalg.vector_norm(Y - Yh, dim=dims) / torch.linalg.vector_norm(Y, dim=dims).clamp_min(1e-30)
        total = total + sc
        if log_term:
            total = total + (torch.log(Y + EPS) - torch.log(Yh + EPS)).abs().mean(dim=dims)
    out = total / len(FFT_SIZES)
    return out.mean() if reduce else out


def _hz_to_mel(f):
    return 2595.0 * math.log10(1.0 + f / 700.0)


def mel_filterbank(n_mels: int, n_fft: int, fs: float, device=None, dtype=torch.float32):
    """HTK-style triangular mel filters [n_mels, n_fft//2 + 1]."""
    n_bins = n_fft // 2 + 1
    mels = torch.linspace(_hz_to_mel(0.0), _hz_to_mel(fs / 2), n_mels + 2, dtype=torch.float64)
    hz = 700.0 * (10.0 ** (mels / 2595.0) - 1.0)
    freqs = torch.linspace(0, fs / 2, n_bins, dtype=torch.float64)
    fb = torch.zeros(n_mels, n_bins, dtype=torch.float64)
    for i in range(n_mels):
        lo, c, hi = hz[i], hz[i + 1], hz[i + 2]
        up = (freqs - lo) / (c - lo)
        down = (hi - freqs) / (hi - c)
        fb[i] = torch.clamp(torch.minimum(up, down), min=0.0)
    return fb.to(device=device, dtype=dtype)


def logmel_features(y: torch.Tensor, fs: float = 44100.0, n_mels: int = 128, slices: int = 8,
                    n_fft: int = 2048, hop: int = 512) -> torch.Tensor:
    """[B, T] -> [B, slices * n_mels]: log(mel power + 1e-5), frames averaged
    in `slices` equal groups in time."""
    win = torch.hann_window(n_fft, device=y.device, dtype=y.dtype)
    X = torch.stft(y, n_fft, hop_length=hop, window=win, center=True, return_complex=True)
    P = X.abs() ** 2  # [B, bins, frames]
    fb = mel_filterbank(n_mels, n_fft, fs, device=y.device, dtype=y.dtype)
    M = torch.log(torch.einsum("mb,nbt->nmt", fb, P) + 1e-5)
    frames = M.shape[-1]
    edges = [round(i * frames / slices) for i in range(slices + 1)]
    parts = [M[..., edges[i]:max(edges[i + 1], edges[i] + 1)].mean(dim=-1) for i in range(slices)]
    return torch.stack(parts, dim=1).reshape(y.shape[0], slices * n_mels)
