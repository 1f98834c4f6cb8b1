"""Pins of the oracle's time-stepping schemes (Sec. 3.2) against closed forms,
an independent high-order integrator, and exact discrete energy identities."""
import numpy as np
import pytest

from oracle import scheme, simulate


def _linear_inst(omega, gamma, x0, xm1):
    n = len(omega)
    return dict(kind="linear", omega=np.asarray(omega, float), gamma=np.asarray(gamma, float),
                x0=np.asarray(x0, float), xm1=np.asarray(xm1, float), c=np.ones(n))


def test_sv_linear_matches_characteristic_roots():
    """With no nonlinear force the SV recursion q+ = g q + p q- has the exact
    solution A z1^n + B z2^n, z roots of z^2 - g z - p, fixed by q^0, q^-1."""
    fs = 44100.0
    T = 1 / fs
    omega = np.array([2 * np.pi * 100.0, 2 * np.pi * 3000.0, 2 * np.pi * 9000.0])
    gamma = np.array([0.5, 7.0, 40.0])
    x0 = np.array([1.0, -0.3, 0.2])
    xm1 = np.array([0.9, -0.25, 0.1])
    inst = _linear_inst(omega, gamma, x0, xm1)
    n = 3000
    _, states = simulate.run(inst, n, fs, return_states=True)
    g, p, r = scheme.sv_coefficients(omega, gamma, T)
    for k in range(3):
        z = np.roots([1.0, -g[k], -p[k]]).astype(complex)
        # q^n = A z1^n + B z2^n with q^0 = x0, q^-1 = xm1
        M = np.array([[1.0, 1.0], [1 / z[0], 1 / z[1]]])
        A, B = np.linalg.solve(M, np.array([x0[k], xm1[k]], dtype=complex))
        nn = np.arange(n + 1)
        exact = (A * z[0] ** nn + B * z[1] ** nn).real
        err = np.abs(states[:, k] - exact).max() / np.abs(exact).max()
        assert err < 1e-10, (k, err)
    # the discrete decay per step is sqrt(-p) = sqrt((1 - gamma T)/(1 + gamma T))
    assert np.allclose(np.abs(np.roots([1.0, -g[2], -p[2]])),
                       np.sqrt((1 - gamma[2] * T) / (1 + gamma[2] * T)), rtol=1e-12)


def test_sv_coefficients_are_centred_differences():
    """(q+ - 2q + q-)/T^2 + 2 gamma (q+ - q-)/(2T) + omega^2 q = f solved for
    q+ gives exactly the printed g, p, r."""
    rng = np.random.default_rng(0)
    T = 1 / 44100.0
    om = rng.uniform(10, 2e4, 5)
    ga = rng.uniform(0, 100, 5)
    q, qm, f = rng.normal(size=(3, 5))
    g, p, r = scheme.sv_coefficients(om, ga, T)
    qp = g * q + p * qm + r * f
    resid = (qp - 2 * q + qm) / T ** 2 + 2 * ga * (qp - qm) / (2 * T) + om ** 2 * q - f
    # every term is of size |q|/T^2; the residual is rounding of that size
    assert np.abs(resid).max() < 1e-12 * np.abs(q).max() / T ** 2
    assert np.allclose(g + p - 1.0, -r * om ** 2, rtol=1e-9, atol=1e-15)


def test_tf_is_exact_for_free_damped_oscillator():
    """Impulse-invariant recursion with the sign reading q+ = -a1 q - a2 q-:
    fed two exact samples of e^{-gamma t} cos(w t + phi), it reproduces the
    continuous solution at every later sample."""
    fs = 44100.0
    T = 1 / fs
    omega = np.array([2 * np.pi * 440.0, 2 * np.pi * 7000.0])
    gamma = np.array([3.0, 80.0])
    w = np.sqrt(omega ** 2 - gamma ** 2)
    phi = np.array([0.3, -1.1])
    xt = lambda t: np.exp(-gamma * t) * np.cos(w * t + phi)
    inst = _linear_inst(omega, gamma, xt(0.0), xt(-T))
    n = 5000
    _, states = simulate.run(inst, n, fs, scheme="tf", return_states=True)
    t = np.arange(n + 1)[:, None] * T
    exact = np.exp(-gamma * t) * np.cos(w * t + phi)
    assert np.abs(states - exact).max() < 1e-11


def test_tf_and_sv_forced_responses_agree_as_T_shrinks():
    """Input gain reading: with b1 = T e^{-gT} sin(wT)/w (force per unit mass)
    the TF and SV forced responses of the same oscillator converge to each
    other as T -> 0 (a missing factor T would leave them apart by 1/T)."""
    omega = np.array([2 * np.pi * 200.0])
    gamma = np.array([5.0])
    errs = []
    for fs in (44100.0, 88200.0, 176400.0):
        n = int(0.02 * fs)
        inst = _linear_inst(omega, gamma, [0.0], [0.0])
        inst["b_ext"] = np.array([1.0])
        inst["e_ext"] = np.ones(n)  # unit step force
        ysv = simulate.run(inst, n, fs, "sv")
        ytf = simulate.run(inst, n, fs, "tf")
        errs.append(np.abs(ysv - ytf).max() / np.abs(ysv).max())
    assert errs[0] < 0.02
    assert errs[1] < errs[0] / 1.8 and errs[2] < errs[1] / 1.8


def test_linear_discrete_energy_balance_is_exact():
    """E^{n+1/2} = 1/2 |(q^{n+1}-q^n)/T|^2 + 1/2 sum w^2 q^{n+1} q^n changes by
    T sum[-2 gamma (dq)^2 + f dq] per step, dq the centred difference
    (q^{n+1}-q^{n-1})/(2T).  The identity holds to rounding."""
    fs = 44100.0
    T = 1 / fs
    rng = np.random.default_rng(1)
    omega = rng.uniform(100, 2e4, 8)
    gamma = rng.uniform(0.0, 30.0, 8)
    x0 = rng.normal(size=8)
    inst = _linear_inst(omega, gamma, x0, x0 * 0.99)
    n = 4000
    inst["b_ext"] = rng.normal(size=8)
    inst["e_ext"] = rng.normal(size=n)
    _, q = simulate.run(inst, n, fs, return_states=True)
    qprev = np.vstack([inst["xm1"][None], q[:-1]])
    # E^{n+1/2} for n = 0..n-1 uses q^{n+1}, q^n
    E = 0.5 * np.sum(((q[1:] - q[:-1]) / T) ** 2, axis=1) + 0.5 * np.sum(omega ** 2 * q[1:] * q[:-1], axis=1)
    dE = E[1:] - E[:-1]
    dq = (q[2:] - q[:-2]) / (2 * T)
    f = inst["b_ext"][None] * inst["e_ext"][1:n, None]
    rhs = T * np.sum(-2 * gamma * dq ** 2 + f * dq, axis=1)
    scale = np.abs(E).max()
    assert np.abs(dE - rhs).max() < 1e-9 * scale
    # undamped, unforced: constant
    inst2 = _linear_inst(omega, 0 * gamma, x0, x0 * 0.99)
    _, q2 = simulate.run(inst2, n, fs, return_states=True)
    E2 = 0.5 * np.sum(((q2[1:] - q2[:-1]) / T) ** 2, axis=1) + 0.5 * np.sum(omega ** 2 * q2[1:] * q2[:-1], axis=1)
    assert np.abs(E2 - E2[0]).max() < 1e-10 * E2[0]


def test_direct_and_increment_forms_agree():
    """The two algebraically identical forms of the recursion agree in FP64."""
    import workloads as W
    from oracle import instances
    inst = instances.plate_instance(W.plate_vk(n_t=12, family="sine", grid=(60, 45)))
    y1 = simulate.run(inst, 3000, 44100.0)
    y2 = simulate.run_increment(inst, 3000, 44100.0)
    assert np.linalg.norm(y1 - y2) / np.linalg.norm(y1) < 1e-10
