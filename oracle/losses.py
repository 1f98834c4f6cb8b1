"""FP64 spectral losses (paper, Sec. 4.3 loss functions), written plainly
with numpy FFTs for checking the torch implementation.

|STFT|: frames of n_fft samples every n_fft/4 samples after reflect-padding
by n_fft/2 at both ends, multiplied by the periodic Hann window
0.5 - 0.5 cos(2 pi i / n_fft), real FFT, magnitude.
L_sc = ||Y - Yh||_F / ||Y||_F, L_log = mean |log(Y + eps) - log(Yh + eps)|,
eps = 1e-7; the multi-resolution loss averages L_sc + L_log over
n_fft = 256, 1024, 4096.
"""
from __future__ import annotations

import numpy as np

FFT_SIZES = (256, 1024, 4096)
EPS = 1e-7


def stft_mag(x, n_fft):
    x = np.asarray(x, dtype=float)
    pad = n_fft // 2
    xp = np.concatenate([x[pad:0:-1], x, x[-2:-pad - 2:-1]])
    hop = n_fft // 4
    n_frames = 1 + (len(xp) - n_fft) // hop
    win = 0.5 - 0.5 * np.cos(2 * np.pi * np.arange(n_fft) / n_fft)
    frames = np.stack([xp[t * hop:t * hop + n_fft] * win for t in range(n_frames)], axis=1)
    return np.abs(np.fft.rfft(frames, axis=0))  # [bins, frames]


def mrstft_loss(y, target, log_term=True):
    """The multi-resolution loss; log_term=False keeps only the spectral
    convergence terms (differentiable wherever no STFT bin of y vanishes)."""
    total = 0.0
    for n in FFT_SIZES:
        Y = stft_mag(target, n)
        Yh = stft_mag(y, n)
        sc = np.linalg.norm(Y - Yh) / np.linalg.norm(Y)
        lg = np.mean(np.abs(np.log(Y + EPS) - np.log(Yh + EPS))) if log_term else 0.0
        total += sc + lg
    return total / len(FFT_SIZES)


def _reflect_pad(x, pad):
    """x extended by ``pad`` mirrored samples at each end (edge not repeated)."""
    return np.concatenate([x[pad:0:-1], x, x[-2:-pad - 2:-1]])


def mrstft_loss_grad(y, target, log_term=True):
    """dL/dy of ``mrstft_loss`` by the chain rule through each step written
    out by hand: the loss terms' derivatives with respect to the magnitudes,
    |Z| with respect to the complex spectrum, the real DFT, the window, the
    framing (overlap-add of frame gradients) and the reflect padding (mirrored
    samples fold back onto their sources).

    With Z_k = sum_i f_i e^{-2 pi i k i/n} (k = 0..n/2) and G_k = dL/d|Z_k|,
    dL/df_i = Re( sum_k G_k conj(Z_k)/|Z_k| e^{-2 pi i k i/n} ).
    """
    y = np.asarray(y, dtype=float)
    T = len(y)
    grad = np.zeros(T)
    for n in FFT_SIZES:
        pad, hop = n // 2, n // 4
        win = 0.5 - 0.5 * np.cos(2 * np.pi * np.arange(n) / n)
        tp = _reflect_pad(np.asarray(target, dtype=float), pad)
        yp = _reflect_pad(y, pad)
        n_frames = 1 + (len(yp) - n) // hop
        fy = np.stack([yp[t * hop:t * hop + n] * win for t in range(n_frames)], axis=1)
        ft = np.stack([tp[t * hop:t * hop + n] * win for t in range(n_frames)], axis=1)
        Zh = np.fft.rfft(fy, axis=0)
        Yh = np.abs(Zh)
        Y = np.abs(np.fft.rfft(ft, axis=0))
        diff = Y - Yh
        nd = np.linalg.norm(diff)
        # L_sc = |Y - Yh| / |Y|;  L_log = mean |log(Y+eps) - log(Yh+eps)|
        G = -diff / (nd * np.linalg.norm(Y)) if nd > 0 else np.zeros_like(Yh)
        if log_term:
            G = G - np.sign(np.log(Y + EPS) - np.log(Yh + EPS)) / ((Yh + EPS) * Yh.size)
        G = G / len(FFT_SIZES)
        A = np.where(Yh > 0, G * np.conj(Zh) / np.where(Yh > 0, Yh, 1.0), 0.0)
        k = np.arange(n // 2 + 1)
        i = np.arange(n)
        E = np.exp(-2j * np.pi * np.outer(i, k) / n)      # [n, bins]
        gf = np.real(E @ A) * win[:, None]                # [n, frames]
        gp = np.zeros(len(yp))
        for t in range(n_frames):
            gp[t * hop:t * hop + n] += gf[:, t]
        g = gp[pad:pad + T].copy()
        # left mirror: padded sample j < pad holds y[pad - j]
        for j in range(pad):
            g[pad - j] += gp[j]
        # right mirror: padded sample pad + T + j holds y[T - 2 - j]
        for j in range(pad):
            g[T - 2 - j] += gp[pad + T + j]
        grad += g
    return grad


def hz_to_mel(f):
    """HTK mel scale: 2595 log10(1 + f / 700)."""
    return 2595.0 * np.log10(1.0 + np.asarray(f, dtype=float) / 700.0)


def mel_to_hz(m):
    return 700.0 * (10.0 ** (np.asarray(m, dtype=float) / 2595.0) - 1.0)


def mel_filters(n_mels, n_fft, fs):
    """Triangular filters on the DFT bin frequencies k fs / n_fft, one per
    mel band, with n_mels + 2 edge frequencies equally spaced in mel from 0
    to fs/2: filter i rises linearly from edge i to edge i+1 and falls to
    edge i+2.  Written as a double loop over bands and bins."""
    edges = mel_to_hz(np.linspace(hz_to_mel(0.0), hz_to_mel(fs / 2.0), n_mels + 2))
    n_bins = n_fft // 2 + 1
    fb = np.zeros((n_mels, n_bins))
    for i in range(n_mels):
        lo, c, hi = edges[i], edges[i + 1], edges[i + 2]
        for k in range(n_bins):
            f = k * fs / n_fft
            if lo < f <= c:
                fb[i, k] = (f - lo) / (c - lo)
            elif c < f < hi:
                fb[i, k] = (hi - f) / (hi - c)
    return fb


def logmel(y, fs=44100.0, n_mels=128, slices=8, n_fft=2048, hop=512):
    """Log-mel features of one signal: power spectrum of Hann-windowed frames
    (reflect-padded by n_fft/2, hop ``hop``) by a direct DFT sum, mel filter
    energies, log(. + 1e-5), then the frames averaged in ``slices`` groups of
    consecutive frames, group g spanning frames [round(g F/S), round((g+1)F/S)).
    Returns [slices * n_mels], slice-major."""
    y = np.asarray(y, dtype=float)
    yp = _reflect_pad(y, n_fft // 2)
    n_frames = 1 + (len(yp) - n_fft) // hop
    win = 0.5 - 0.5 * np.cos(2 * np.pi * np.arange(n_fft) / n_fft)
    k = np.arange(n_fft // 2 + 1)
    E = np.exp(-2j * np.pi * np.outer(k, np.arange(n_fft)) / n_fft)   # direct DFT matrix
    frames = np.stack([yp[t * hop:t * hop + n_fft] * win for t in range(n_frames)], axis=1)
    P = np.abs(E @ frames) ** 2                                       # [bins, frames]
    M = np.log(mel_filters(n_mels, n_fft, fs) @ P + 1e-5)             # [mels, frames]
    out = []
    for g in range(slices):
        a = int(round(g * n_frames / slices))
        b = max(int(round((g + 1) * n_frames / slices)), a + 1)
        out.append(M[:, a:b].mean(axis=1))
    return np.concatenate(out)
