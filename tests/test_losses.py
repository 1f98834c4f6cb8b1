"""The torch MR-STFT loss against the FP64 numpy oracle: value, and the
autograd gradient against central differences of the oracle; the oracle's
|STFT| against a direct DFT sum."""
import numpy as np
import pytest
import torch

from oracle import losses as OL


def test_oracle_stft_is_a_windowed_dft():
    rng = np.random.default_rng(0)
    x = rng.normal(size=1000)
    n = 256
    S = OL.stft_mag(x, n)
    xp = np.pad(x, n // 2, mode="reflect")
    win = np.hanning(n + 1)[:-1]  # periodic Hann
    t = 3
    frame = xp[t * n // 4:t * n // 4 + n] * win
    k = np.arange(n // 2 + 1)
    dft = np.abs(np.exp(-2j * np.pi * np.outer(k, np.arange(n)) / n) @ frame)
    assert np.allclose(S[:, t], dft, atol=1e-9)


def test_torch_loss_matches_oracle_value_and_gradient():
    from paper_2505_05940_amd import losses
    rng = np.random.default_rng(1)
    T = 6000
    t = np.arange(T) / 44100.0
    target = np.exp(-5 * t) * np.sin(2 * np.pi * 440 * t) + 0.01 * rng.normal(size=T)
    y = np.exp(-6 * t) * np.sin(2 * np.pi * 452 * t) + 0.01 * rng.normal(size=T)
    yt = torch.tensor(y, dtype=torch.float64, requires_grad=True)
    L = losses.mrstft_loss(yt[None], torch.tensor(target)[None])
    L.backward()
    Lo = OL.mrstft_loss(y, target)
    assert abs(L.item() - Lo) < 1e-10 * abs(Lo)
    for i in (10, 2000, 5999):
        e = 1e-6
        yp, ym = y.copy(), y.copy()
        yp[i] += e
        ym[i] -= e
        fd = (OL.mrstft_loss(yp, target) - OL.mrstft_loss(ym, target)) / (2 * e)
        assert abs(fd - yt.grad[i].item()) < 1e-4 * np.abs(yt.grad.numpy()).max()


def test_loss_is_zero_on_identical_signals_and_positive_otherwise():
    from paper_2505_05940_amd import losses
    x = torch.randn(2, 5000, dtype=torch.float64)
    assert losses.mrstft_loss(x, x).item() == 0.0
    assert losses.mrstft_loss(x, 1.1 * x).item() > 0.0


def test_logmel_shape_and_slices():
    from paper_2505_05940_amd import losses
    y = torch.randn(3, 44100)
    f = losses.logmel_features(y)
    assert f.shape == (3, 1024) and torch.isfinite(f).all()
    fb = losses.mel_filterbank(128, 2048, 44100.0)
    assert fb.shape == (128, 1025) and (fb >= 0).all() and (fb.sum(1) > 0).all()


def test_logmel_matches_oracle():
    """The product's log-mel features (torch STFT, mel matrix product) against
    the oracle's direct-DFT, double-loop-filter version of the same
    definition, at the proposal network's settings (1 s, 128 bands, 8
    slices, n_fft 2048, hop 512)."""
    from oracle import losses as OL
    from paper_2505_05940_amd import losses
    rng = np.random.default_rng(11)
    t = np.arange(44100) / 44100.0
    f = rng.uniform(60.0, 9000.0, size=12)
    y = sum(np.exp(-rng.uniform(1, 20) * t) * np.sin(2 * np.pi * fk * t + rng.uniform(0, 6)) for fk in f)
    y = 1e-4 * (y + 0.01 * rng.normal(size=t.size))
    got = losses.logmel_features(torch.tensor(y[None], dtype=torch.float64)).numpy()[0]
    ref = OL.logmel(y)
    assert got.shape == ref.shape == (1024,)
    assert np.abs(got - ref).max() < 1e-6 * np.abs(ref).max(), np.abs(got - ref).max()
