"""Pins of the oracle's transfer-function route: the response against the
discrete-time Fourier transform of the time-domain recursion's impulse
response (both numerator terms), its gradient against central differences,
the Levinson-Durbin recursion against a direct Toeplitz solve and against a
known all-pole process, and the Bark formula against the critical-band
table."""
import numpy as np
from scipy.linalg import solve_toeplitz

from oracle import scheme
from oracle import simulate as OS
from oracle import transfer as TF

FS = 44100.0


def _modes(n=5, seed=0):
    rng = np.random.default_rng(seed)
    omega = 2 * np.pi * np.sort(rng.uniform(100, 5000, n))
    gamma = rng.uniform(60, 200, n)
    return omega, gamma, rng


def _dtft(y, Omega):
    n = np.arange(len(y))
    return np.array([np.sum(y * np.exp(-1j * Om * n)) for Om in Omega])


def test_response_is_the_dtft_of_the_recursion():
    omega, gamma, rng = _modes()
    T = 1 / FS
    g, p, b1 = scheme.tf_coefficients(omega, gamma, T)  # q+ = g q + p q- + b1 f
    a1, a2 = -g, -p
    w = rng.normal(size=len(omega))
    Omega = TF.bark_grid(40, 50, 15000, FS)
    steps = 12000  # every mode decayed below 1e-9
    assert np.exp(-gamma.min() * steps * T) < 1e-9
    inst = dict(kind="linear", omega=omega, gamma=gamma, x0=np.zeros(5), xm1=np.zeros(5), c=w,
                b_ext=np.ones(5), e_ext=np.array([1.0]))
    y = OS.run(inst, steps, FS, scheme="tf")
    H = TF.response(a1, a2, b1, np.zeros(5), w, Omega)
    assert np.abs(_dtft(y, Omega) - H).max() < 1e-9 * np.abs(H).max()
    # b2 z^{-1} ... : the b2 term is the b1 term's impulse response delayed one
    # sample, with b1 replaced by b2
    b2 = rng.normal(size=5) * b1
    inst2 = dict(inst, c=w * b2 / b1)
    y2 = np.concatenate([[0.0], OS.run(inst2, steps, FS, scheme="tf")[:-1]])
    H2 = TF.response(a1, a2, np.zeros(5), b2, w, Omega)
    assert np.abs(_dtft(y2, Omega) - H2).max() < 1e-9 * np.abs(H2).max()


def test_response_gradient_matches_differences():
    omega, gamma, rng = _modes(4, seed=1)
    g, p, b1 = scheme.tf_coefficients(omega, gamma, 1 / FS)
    a1, a2 = -g, -p
    b2 = 0.3 * b1
    w = rng.normal(size=4)
    Omega = TF.bark_grid(30, 50, 15000, FS)
    g = rng.normal(size=30) + 1j * rng.normal(size=30)
    G = TF.response_grad(a1, a2, b1, b2, w, Omega, g)
    P = np.stack([a1, a2, b1, b2, w], axis=1)

    def L(P):
        return float(np.sum((np.conj(g) * TF.response(*P.T, Omega)).real))

    for m in range(4):
        for j in range(5):
            h = 1e-8 * max(abs(P[m, j]), 1e-3)
            Pp, Pm = P.copy(), P.copy()
            Pp[m, j] += h
            Pm[m, j] -= h
            fd = (L(Pp) - L(Pm)) / (2 * h)
            assert abs(fd - G[m, j]) < 1e-5 * max(abs(fd), 1e-6 * np.abs(G[:, j]).max()), (m, j, fd, G[m, j])


def test_levinson_matches_toeplitz_solve_and_recovers_an_all_pole_process():
    rng = np.random.default_rng(3)
    x = rng.normal(size=4000)
    a, err = TF.lpc(x, 12)
    r = np.array([np.dot(x[:len(x) - k], x[k:]) for k in range(13)])
    direct = solve_toeplitz(r[:12], -r[1:13])
    assert np.allclose(a[1:], direct, rtol=1e-10, atol=1e-12)
    assert abs(err - (r[0] + np.dot(a[1:], r[1:13]))) < 1e-9 * r[0]
    # x[n] = 1.6 x[n-1] - 0.8 x[n-2] + e[n]
    e = rng.normal(size=200000)
    xs = np.zeros_like(e)
    for n in range(2, len(e)):
        xs[n] = 1.6 * xs[n - 1] - 0.8 * xs[n - 2] + e[n]
    a2, err2 = TF.lpc(xs, 2)
    assert np.allclose(a2, [1.0, -1.6, 0.8], atol=5e-3)
    assert abs(err2 / len(xs) - 1.0) < 0.02
    # the envelope of the all-pole model at a frequency, by its definition
    Om = np.array([0.3])
    A = 1 - 1.6 * np.exp(-0.3j) + 0.8 * np.exp(-0.6j)
    assert abs(TF.lpc_envelope(np.array([1, -1.6, 0.8]), 4.0, Om)[0] - 2.0 / abs(A)) < 1e-12


def test_bark_formula_against_the_critical_band_table():
    # upper edges (Hz) of critical bands 1..20 of the classical table
    edges = [100, 200, 300, 400, 510, 630, 770, 920, 1080, 1270, 1480, 1720, 2000, 2320, 2700,
             3150, 3700, 4400, 5300, 6400]
    z = TF.hz_to_bark(edges)
    assert np.abs(z[1:] - np.arange(2, 21)).max() < 0.25
    zz = np.linspace(0.5, 23, 50)
    assert np.allclose(TF.hz_to_bark(TF.bark_to_hz(zz)), zz, rtol=0, atol=1e-12)
    Om = TF.bark_grid(64, 40, 16000, FS)
    assert np.all(np.diff(Om) > 0) and abs(Om[0] - 2 * np.pi * 40 / FS) < 1e-12
