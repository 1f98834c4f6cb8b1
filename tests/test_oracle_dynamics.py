"""Pins of the oracle's nonlinear time loop (Sec. 3.1-2.2): an independent
8th-order integrator (the paper's own DOP853 comparison, Fig. 1), energy
behaviour, invariances, and the workload constructions."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import workloads as W
from oracle import coupling, excitation, instances, modes, simulate


def _kc_small(n=10):
    wl = W.string_kc(n_modes=n)
    return wl, instances.string_instance(wl)


def test_kc_string_converges_to_dop853_at_second_order():
    """SV on the Kirchhoff-Carrier string against scipy's DOP853 on the same
    modal ODEs (rtol 1e-12).  The SV start uses the exact q(-T) so that the
    only error is the scheme's; halving T must cut it about four times."""
    wl, inst = _kc_small(10)
    om, ga, lam, kap = inst["omega"], inst["gamma"], inst["lam"], inst["kappa"]
    n = len(om)

    def rhs(t, z):
        q, v = z[:n], z[n:]
        f = kap * lam * q * np.sum(lam * q * q)
        return np.concatenate([v, -2 * ga * v - om ** 2 * q - f])

    t_end = 0.01
    z0 = np.concatenate([inst["x0"], np.zeros(n)])
    errs = []
    for fs in (44100.0, 88200.0, 176400.0):
        T = 1 / fs
        back = solve_ivp(rhs, (0, -T), z0, method="DOP853", rtol=1e-12, atol=1e-20)
        steps = int(round(t_end * fs))
        t = np.arange(steps) * T
        fwd = solve_ivp(rhs, (0, t[-1]), z0, method="DOP853", rtol=1e-12, atol=1e-20, t_eval=t)
        ref = inst["c"] @ fwd.y[:n]
        i2 = dict(inst, xm1=back.y[:n, -1])
        y = simulate.run(i2, steps, fs)
        # compare on the coarsest grid's sample times
        stride = int(round(fs / 44100.0))
        errs.append(np.linalg.norm((y - ref)[::stride]) / np.linalg.norm(ref[::stride]))
    assert errs[2] < 2e-2, errs
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7, errs


def _discrete_energy(inst, q, T):
    om = inst["omega"]
    kin = 0.5 * np.sum(((q[1:] - q[:-1]) / T) ** 2, axis=1)
    pot = 0.5 * np.sum(om ** 2 * q[1:] * q[:-1], axis=1)
    Ht = inst["Ht"]
    V = np.array([0.25 * np.sum(np.einsum("npq,p,q->n", Ht, x, x) ** 2) for x in q])
    return kin + pot + 0.5 * (V[1:] + V[:-1]), V


def test_vk_energy_drift_is_second_order_and_potential_nonnegative():
    """Undamped, unforced von Karman plate: the explicit scheme conserves
    the energy only approximately; the drift shrinks about 4x when T halves
    and the coupling potential 1/4 sum eta^2 is never negative."""
    wl = W.plate_vk(n_t=10, family="sine", grid=(80, 60))
    wl["strike"]["amplitude"] = 4e-3
    inst = instances.plate_instance(wl)
    inst["gamma"] = np.zeros_like(inst["gamma"])
    drift = []
    for fs in (44100.0, 88200.0):
        n = int(0.02 * fs)
        _, q = simulate.run(inst, n, fs, return_states=True)
        E, V = _discrete_energy(inst, q, 1 / fs)
        assert V.min() >= 0
        assert V.max() > 0.01 * E[0]  # the nonlinearity matters in this run
        drift.append(np.abs(E - E[0]).max() / E[0])
    assert drift[0] < 1e-2 and 3.0 < drift[0] / drift[1] < 5.0, drift


def test_mode_permutation_leaves_output_unchanged():
    wl = W.plate_vk(n_t=9, family="clamped", grid=(60, 45))
    inst = instances.plate_instance(wl)
    perm = np.random.default_rng(0).permutation(9)
    pin = np.random.default_rng(1).permutation(9)
    i2 = dict(inst)
    for k in ("omega", "gamma", "x0", "xm1", "c", "lam"):
        i2[k] = inst[k][perm]
    i2["Ht"] = inst["Ht"][pin][:, perm][:, :, perm]
    y1 = simulate.run(inst, 2000, 44100.0)
    y2 = simulate.run(i2, 2000, 44100.0)
    assert np.linalg.norm(y1 - y2) / np.linalg.norm(y1) < 1e-12


def test_string_projection_reconstructs_the_pluck():
    L = 0.65
    k, _ = modes.string_modes(L, 600)
    X = excitation.string_pluck_modal(k, L, 0.2, 1e-3, 0.065, 4096)
    x = np.linspace(0, L, 301)
    w = modes.string_phi(k, L, x).T @ X
    ref = excitation.raised_cosine_1d(x, 0.2, 1e-3, 0.065)
    assert np.abs(w - ref).max() < 1e-3 * 1e-3


def test_plate_projection_parseval():
    """For a strike resolved by the kept modes, sum X_k^2 equals the midpoint
    integral of w0^2 (the modes are orthonormal under that rule)."""
    Lx, Ly, nx, ny = 0.4, 0.3, 200, 150
    m, q, _ = modes.plate_modes(Lx, Ly, 1500)
    X = excitation.plate_strike_modal(m, q, Lx, Ly, nx, ny, 0.2, 0.15, 1e-3, 0.06)
    x, y, dA = modes.midpoint_grid(Lx, Ly, nx, ny)
    w0 = excitation.raised_cosine_2d(x, y, 0.2, 0.15, 1e-3, 0.06)
    assert abs(np.sum(X ** 2) / (dA * np.sum(w0 ** 2)) - 1) < 1e-3


def test_berger_tension_term_is_the_gradient_energy():
    """The Berger force's sum lambda q^2 equals the plate's gradient energy
    int |grad w|^2 = -int w lap(w) (w = 0 on the edges), by midpoint
    quadrature of the modal field; and the force is the gradient of
    kappa/4 (sum lambda q^2)^2."""
    wl = W.plate_berger(n_t=12, n_steps=10)
    inst = instances.plate_berger_instance(wl)
    rng = np.random.default_rng(4)
    qv = rng.normal(size=12)
    x, y, dA = modes.midpoint_grid(inst["Lx"], inst["Ly"], 400, 300)
    d = modes.plate_phi_derivs(inst["m"], inst["q"], inst["Lx"], inst["Ly"], x, y)
    w = qv @ d["phi"]
    lap = qv @ (d["xx"] + d["yy"])
    energy = -np.sum(w * lap) * dA
    assert abs(energy - np.sum(inst["lam"] * qv ** 2)) < 1e-4 * energy
    F = simulate.modal_force(inst, qv)
    V = lambda v: inst["kappa"] / 4 * np.sum(inst["lam"] * v ** 2) ** 2
    e = 1e-6
    g = np.array([(V(qv + e * np.eye(12)[k]) - V(qv - e * np.eye(12)[k])) / (2 * e) for k in range(12)])
    assert np.allclose(F, g, rtol=1e-6, atol=1e-9 * np.abs(g).max())


def test_batch_geometry_puts_top_mode_at_target():
    from oracle import scheme
    for wl in W.plate_batch(batch=4):
        Lx, Ly = instances.plate_geometry(wl)
        assert abs(Ly / Lx - wl["aspect"]) < 1e-12
        _, _, lam = modes.plate_modes(Lx, Ly, wl["n_t"])
        D = wl["E"] * wl["h"] ** 3 / (12 * (1 - wl["nu"] ** 2))
        om = scheme.omega_from(lam, D, wl["T0"], wl["rho"] * wl["h"])
        assert abs(om[-1] / (2 * np.pi) - wl["top_mode_hz"]) < 1e-6 * wl["top_mode_hz"]
