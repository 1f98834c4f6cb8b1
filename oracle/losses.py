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


def mrstft_loss(y, target):
    total = 0.0
    for n in FFT_SIZES:
        Y = stft_mag(target, n)
        Yh = stft_mag(y, n)
        sc = np.linalg.norm(Y - Yh) / np.linalg.norm(Y)
        lg = np.mean(np.abs(np.log(Y + EPS) - np.log(Yh + EPS)))
        total += sc + lg
    return total / len(FFT_SIZES)
