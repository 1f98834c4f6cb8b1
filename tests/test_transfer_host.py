"""Host preprocessing of the transfer-function fits (linear prediction by
FFT autocorrelation and a vectorised Levinson-Durbin recursion, the Bark
grid, the envelope) against the oracle's plain loops."""
import numpy as np

from oracle import transfer as OT


def test_lpc_bark_and_envelope_match_the_oracle():
    from paper_2505_05940_amd import transfer
    rng = np.random.default_rng(4)
    x = np.convolve(rng.normal(size=6000), [1.0, -0.9, 0.4], mode="same")
    for order in (1, 7, 40):
        a, e = transfer.lpc(x, order)
        ao, eo = OT.lpc(x, order)
        assert np.allclose(a, ao, rtol=1e-9, atol=1e-11) and abs(e - eo) < 1e-9 * eo
    Om = transfer.bark_grid(100, 60, 15000, 44100.0)
    assert np.allclose(Om, OT.bark_grid(100, 60, 15000, 44100.0), rtol=1e-13, atol=0)
    a, e = transfer.lpc(x, 12)
    assert np.allclose(transfer.lpc_envelope(a, e, Om), OT.lpc_envelope(a, e, Om), rtol=1e-11)
