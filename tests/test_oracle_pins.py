"""Pins of the oracle's physical constants against textbook results and
against forces computed in physical space.

Each test fixes a part of the oracle by something other than its own
formula: closed-form natural frequencies of strings, membranes and
simply supported plates; the free decay rate of a viscously damped mode;
the Kirchhoff-Carrier, Berger and von Karman forces evaluated on a grid by
finite differences of the displacement field and projected onto the modes;
and the parameterised plate against the plate built from physical
parameters.  A wrong density reading (volumetric instead of per area), a
wrong tension prefactor or a wrong von Karman scale fails one of them.
"""
import numpy as np
import pytest
from scipy.signal import hilbert

import workloads as W
from oracle import instances as OI
from oracle import losses as OL
from oracle import modes as OM
from oracle import params as OP
from oracle import simulate as OS


def _plate_no_tensor(wl):
    """The oracle's plate with a zero coupling tensor passed in (frequencies,
    damping and excitation only)."""
    n_t, n_in = wl["n_t"], max(1, wl["n_in"])
    return OI.plate_instance(wl, H=(np.zeros((n_in, n_t, n_t)), np.ones(n_in)))


# --- natural frequencies (Sec. 3.2: omega^2 = (D lambda^2 + T0 lambda) / rho_s) ---

def test_string_fundamental_is_the_textbook_value():
    """Ideal string: f_k = (k / 2L) sqrt(T0 / (rho A)); at 0.65 m, 60 N and
    6e-4 kg/m the fundamental is 243.25 Hz."""
    wl = W.string_kc()
    f = OI.string_instance(wl)["omega"] / (2 * np.pi)
    assert abs(f[0] - 243.25) < 0.01
    k = np.arange(1, wl["n_modes"] + 1)
    assert np.allclose(f, k / (2 * wl["L"]) * np.sqrt(wl["T0"] / wl["rhoA"]), rtol=1e-13)


def test_stiff_string_inharmonicity_is_the_textbook_law():
    """Stiff string (Fletcher): f_k = k f0 sqrt(1 + B k^2) with
    B = pi^2 E I / (T0 L^2)."""
    wl = dict(W.string_kc(), EI=2e-4)
    f = OI.string_instance(wl)["omega"] / (2 * np.pi)
    k = np.arange(1, wl["n_modes"] + 1)
    f0 = np.sqrt(wl["T0"] / wl["rhoA"]) / (2 * wl["L"])
    B = np.pi ** 2 * wl["EI"] / (wl["T0"] * wl["L"] ** 2)
    assert np.allclose(f, k * f0 * np.sqrt(1 + B * k * k), rtol=1e-13)


def test_simply_supported_plate_frequencies_are_the_textbook_values():
    """Simply supported Kirchhoff plate (Leissa):
    f_mn = (pi / 2) ((m/Lx)^2 + (n/Ly)^2) sqrt(D / (rho h)),
    D = E h^3 / (12 (1 - nu^2)); the 0.4 x 0.3 m, 1 mm steel plate has its
    fundamental at 41.6 Hz."""
    wl = W.plate_vk(n_t=12, family="sine", grid=None)
    inst = _plate_no_tensor(wl)
    f = inst["omega"] / (2 * np.pi)
    D = wl["E"] * wl["h"] ** 3 / (12 * (1 - wl["nu"] ** 2))
    ref = 0.5 * np.pi * ((inst["m"] / wl["Lx"]) ** 2 + (inst["q"] / wl["Ly"]) ** 2) \
        * np.sqrt(D / (wl["rho"] * wl["h"]))
    assert np.allclose(f, ref, rtol=1e-13)
    assert abs(f[0] - 41.6) < 0.05


def test_membrane_frequencies_are_the_textbook_values():
    """Rectangular membrane under tension T (N/m), no bending stiffness:
    f_mn = (1/2) sqrt(T / (rho h)) sqrt((m/Lx)^2 + (n/Ly)^2)."""
    wl = dict(W.plate_vk(n_t=10, family="sine", grid=None), T0=80.0, E=1e-30)
    inst = _plate_no_tensor(wl)
    f = inst["omega"] / (2 * np.pi)
    ref = 0.5 * np.sqrt(wl["T0"] / (wl["rho"] * wl["h"])) * np.sqrt(
        (inst["m"] / wl["Lx"]) ** 2 + (inst["q"] / wl["Ly"]) ** 2)
    assert np.allclose(f, ref, rtol=1e-12)


def test_viscous_decay_rate_is_the_textbook_value():
    """A string with a damping force -(d1 - d3 w_xx) w_t per unit length: mode
    k decays as exp(-(d1 + d3 lambda_k) t / (2 rho A)).  Measured from the
    envelope of the oracle's free response of one mode."""
    d1, d3 = 4e-3, 2e-7
    wl = dict(W.string_kc(n_steps=22050), damping=("d1d3", d1, d3))
    inst = OI.string_instance(wl)
    inst["kind"] = "linear"
    k = 3
    x0 = np.zeros_like(inst["x0"])
    x0[k - 1] = 1e-3
    inst.update(x0=x0, xm1=x0.copy(), c=np.eye(len(x0))[k - 1])
    y = OS.run(inst, 22050, wl["fs"])
    env = np.abs(hilbert(y))
    t = np.arange(len(y)) / wl["fs"]
    sl = slice(2000, 20000)
    rate = -np.polyfit(t[sl], np.log(env[sl]), 1)[0]
    lam = (k * np.pi / wl["L"]) ** 2
    ref = (d1 + d3 * lam) / (2 * wl["rhoA"])
    assert abs(rate - ref) < 2e-3 * ref


# --- nonlinear forces projected from physical space ---

def _fd2(f, x, h):
    return (f(x + h) - 2 * f(x) + f(x - h)) / (h * h)


def _fd1(f, x, h):
    return (f(x + h) - f(x - h)) / (2 * h)


def test_kirchhoff_carrier_force_is_the_projected_physical_force():
    """Kirchhoff-Carrier string: rho A w_tt = (T0 + (E A / 2L) int w_x^2 dx) w_xx.
    The nonlinear part, moved to the left, is f = -(E A / 2L)(int w_x^2) w_xx;
    its modal force per unit mass is int f Phi_k dx / (rho A).  Derivatives
    by finite differences of the displacement field, integrals by the
    midpoint rule on a fine grid."""
    wl = W.string_kc(n_modes=8)
    inst = OI.string_instance(wl)
    L, n = wl["L"], 8
    rng = np.random.default_rng(3)
    X = 1e-3 * rng.normal(size=n) / np.arange(1, n + 1)
    k = np.arange(1, n + 1)

    def w(x):
        return X @ OM.string_phi(k, L, x)

    M = 20000
    x = (np.arange(M) + 0.5) * L / M
    h = 1e-4 * L
    wx = _fd1(w, x, h)
    wxx = _fd2(w, x, h)
    tension = wl["EA"] / (2 * L) * np.sum(wx ** 2) * (L / M)
    f_phys = -tension * wxx
    proj = OM.string_phi(k, L, x) @ f_phys * (L / M) / wl["rhoA"]
    F = OS.force_tension(X, inst["lam"], inst["kappa"])
    assert np.allclose(F, proj, rtol=1e-5, atol=1e-5 * np.abs(F).max())


def _plate_field(m, q, Lx, Ly, X):
    def w(x, y):
        return X @ OM.plate_phi_derivs(m, q, Lx, Ly, x, y)["phi"]
    return w


def _grid(Lx, Ly, nx, ny):
    x, y, dA = OM.midpoint_grid(Lx, Ly, nx, ny)
    return x, y, dA


def test_berger_force_is_the_projected_physical_force():
    """Berger plate: the in-plane stretching adds the membrane force
    N Delta w with N = E h / (2 S (1 - nu^2)) int |grad w|^2 dS; the nonlinear
    force on the left is f = -N Delta w and its modal force per unit mass is
    int f Phi_k dS / (rho h)."""
    wl = W.plate_berger(n_t=6)
    inst = OI.plate_berger_instance(wl)
    Lx, Ly, h = inst["Lx"], inst["Ly"], wl["h"]
    rng = np.random.default_rng(4)
    X = h * rng.normal(size=6)
    w = _plate_field(inst["m"], inst["q"], Lx, Ly, X)
    x, y, dA = _grid(Lx, Ly, 400, 300)
    e = 1e-4 * Lx
    wx = (w(x + e, y) - w(x - e, y)) / (2 * e)
    wy = (w(x, y + e) - w(x, y - e)) / (2 * e)
    lap = (w(x + e, y) + w(x - e, y) + w(x, y + e) + w(x, y - e) - 4 * w(x, y)) / (e * e)
    S = Lx * Ly
    N = wl["E"] * h / (2 * S * (1 - wl["nu"] ** 2)) * np.sum(wx ** 2 + wy ** 2) * dA
    phi = OM.plate_phi_derivs(inst["m"], inst["q"], Lx, Ly, x, y)["phi"]
    proj = phi @ (-N * lap) * dA / (wl["rho"] * h)
    F = OS.force_tension(X, inst["lam"], inst["kappa"])
    assert np.allclose(F, proj, rtol=2e-5, atol=2e-5 * np.abs(F).max())


def test_von_karman_force_is_the_projected_physical_force():
    """von Karman plate (Sec. 3, plate equations): rho h w_tt + D DD w =
    L(w, F), DD F = -(E h / 2) L(w, w), L(f, g) = f_xx g_yy + f_yy g_xx -
    2 f_xy g_xy.  With the sine in-plane family (F = Delta F = 0 on the
    edges) the biharmonic is diagonal in the sine modes, eigenvalue
    ((a pi/Lx)^2 + (b pi/Ly)^2)^2.  Physical-space evaluation: L(w, w) by
    finite differences, projected onto the first n_in sine modes and divided
    by their biharmonic eigenvalues gives F on the grid; L(w, F) by finite
    differences (F from its modal sum), projected onto Phi_k and divided by
    rho h, is the force.  It must equal the oracle's two contractions
    against the scaled tensor (volumetric rho in E / 2 rho)."""
    wl = W.plate_vk(n_t=5, n_in=5, family="sine", grid=None)
    inst = OI.plate_instance(wl)
    Lx, Ly, h, E, rho = wl["Lx"], wl["Ly"], wl["h"], wl["E"], wl["rho"]
    m, q = inst["m"], inst["q"]
    rng = np.random.default_rng(5)
    X = h * rng.normal(size=5)
    x, y, dA = _grid(Lx, Ly, 400, 300)
    e = 2e-4 * Lx

    def derivs(fun):
        f0 = fun(x, y)
        xx = (fun(x + e, y) - 2 * f0 + fun(x - e, y)) / (e * e)
        yy = (fun(x, y + e) - 2 * f0 + fun(x, y - e)) / (e * e)
        xy = (fun(x + e, y + e) - fun(x + e, y - e) - fun(x - e, y + e) + fun(x - e, y - e)) / (4 * e * e)
        return xx, yy, xy

    w = _plate_field(m, q, Lx, Ly, X)
    wxx, wyy, wxy = derivs(w)
    Lww = 2 * (wxx * wyy - wxy ** 2)
    a, b, _ = OM.plate_modes(Lx, Ly, 5)       # sine in-plane modes, same ordering rule
    psi = OM.plate_phi_derivs(a, b, Lx, Ly, x, y)["phi"]
    bih = ((a * np.pi / Lx) ** 2 + (b * np.pi / Ly) ** 2) ** 2
    coefF = -(E * h / 2) * (psi @ Lww) * dA / bih

    def Ffun(xx_, yy_):
        return coefF @ OM.plate_phi_derivs(a, b, Lx, Ly, xx_, yy_)["phi"]

    Fxx, Fyy, Fxy = derivs(Ffun)
    LwF = wxx * Fyy + wyy * Fxx - 2 * wxy * Fxy
    phi = OM.plate_phi_derivs(m, q, Lx, Ly, x, y)["phi"]
    proj = -(phi @ LwF) * dA / (rho * h)        # f_nl on the left-hand side
    F = OS.force_vk(X, inst["Ht"])
    assert np.allclose(F, proj, rtol=1e-4, atol=1e-4 * np.abs(F).max())


# --- the parameterised plate is the physical plate ---

@pytest.mark.parametrize("which", ["base", "target"])
def test_parameterised_plate_is_the_physical_plate(which):
    """theta = (T0/rho_s, D/rho_s, a, d1/(2 rho_s), d3/(2 rho_s)) (Sec. 4.3,
    density-normalised parameters) against the oracle's plate built from the
    physical T0, E, h, Lx, Ly, d1 and d3 that these stand for.  The target
    case takes the target's stiffness, tension and damping at aspect 0.7,
    where the mode sets fixed at the base aspect are still the physical
    plate's smallest eigenvalues (in another order: matched by index pair)."""
    fit = W.plate_fit(n_t=12, n_in=12)
    theta = np.array(fit["theta0"] if which == "base" else fit["theta_target"], dtype=float)
    theta[2] = fit["base_aspect"] if which == "base" else 0.7
    T0h, Dh, a, d1h, d3h = theta
    h, nu, rho = fit["h"], fit["nu"], fit["rho"]
    rho_s = rho * h
    S = fit["area"]
    Lx, Ly = np.sqrt(S / a), np.sqrt(S * a)
    E = 12 * (1 - nu ** 2) * Dh * rho_s / h ** 3
    xc, yc, amp, rr = fit["strike"]
    wl = dict(family="plate", model="vk", inplane="sine", grid=None, Lx=Lx, Ly=Ly, h=h,
              T0=T0h * rho_s, E=E, nu=nu, rho=rho, n_t=fit["n_t"], n_in=fit["n_in"],
              fs=fit["fs"], damping=("d1d3", 2 * rho_s * d1h, 2 * rho_s * d3h),
              strike=dict(xc=xc * Lx, yc=yc * Ly, amplitude=amp, radius=rr * min(Lx, Ly)),
              out=(fit["out"][0] * Lx, fit["out"][1] * Ly), proj_grid=fit["proj_grid"])
    phys = OI.plate_instance(wl)
    par = OP.plate_from_theta(fit, theta)
    m0, q0, a0, b0 = OP._mode_sets(fit)
    pos = {(int(mm), int(qq)): i for i, (mm, qq) in enumerate(zip(phys["m"], phys["q"]))}
    pt = np.array([pos[(int(mm), int(qq))] for mm, qq in zip(m0, q0)])
    ai, bi, _ = OM.plate_modes(Lx, Ly, fit["n_in"])
    pos_in = {(int(mm), int(qq)): i for i, (mm, qq) in enumerate(zip(ai, bi))}
    pi = np.array([pos_in[(int(mm), int(qq))] for mm, qq in zip(a0, b0)])
    assert (which == "base") == (np.array_equal(pt, np.arange(12)) and np.array_equal(pi, np.arange(12)))
    for key in ("omega", "gamma", "lam", "x0", "c"):
        assert np.allclose(par[key], phys[key][pt], rtol=1e-12, atol=1e-300), key
    Hp = phys["Ht"][pi][:, pt][:, :, pt]
    assert np.allclose(par["Ht"], Hp, rtol=1e-12, atol=1e-12 * np.abs(Hp).max())


# --- losses and features (Sec. 4.3 loss functions; the proposal's input) ---

def test_mrstft_gradient_matches_differences():
    """The oracle's hand-written chain rule of the MR-STFT loss against
    central differences of the loss (a smooth region of the loss: small
    steps, so that no |.| kink of the log term is crossed)."""
    rng = np.random.default_rng(1)
    T = 3000
    t = np.arange(T) / 44100.0
    tg = np.exp(-5 * t) * np.sin(2 * np.pi * 440 * t) + 0.01 * rng.normal(size=T)
    y = np.exp(-6 * t) * np.sin(2 * np.pi * 452 * t) + 0.01 * rng.normal(size=T)
    for log_term in (True, False):
        g = OL.mrstft_loss_grad(y, tg, log_term=log_term)
        for i in (0, 1, 5, 100, 1500, 2990, 2998, 2999):
            e = 1e-9 if log_term else 1e-6  # the smooth loss takes a larger step
            yp, ym = y.copy(), y.copy()
            yp[i] += e
            ym[i] -= e
            fd = (OL.mrstft_loss(yp, tg, log_term=log_term) - OL.mrstft_loss(ym, tg, log_term=log_term)) / (2 * e)
            assert abs(fd - g[i]) < 1e-5 * np.abs(g).max(), (log_term, i)


def test_htk_mel_scale_and_filters():
    """HTK mel: 1000 Hz is 1000 mel (to 0.02); the inverse is exact; inside
    the outermost centres the triangles of neighbouring bands sum to one."""
    assert abs(OL.hz_to_mel(1000.0) - 1000.0) < 0.02
    f = np.array([0.0, 123.0, 4000.0, 22050.0])
    assert np.allclose(OL.mel_to_hz(OL.hz_to_mel(f)), f, rtol=1e-13, atol=1e-9)
    fb = OL.mel_filters(128, 2048, 44100.0)
    edges = OL.mel_to_hz(np.linspace(0.0, OL.hz_to_mel(22050.0), 130))
    fk = np.arange(1025) * 44100.0 / 2048
    inside = (fk > edges[1]) & (fk <= edges[128])
    assert np.allclose(fb.sum(0)[inside], 1.0, atol=1e-12)
    assert (fb >= 0).all()


def test_logmel_direct_dft_matches_fft_and_slices():
    """The log-mel's direct DFT equals numpy's FFT of the same frames, and the
    slice means partition the frames."""
    rng = np.random.default_rng(2)
    y = rng.normal(size=6000)
    f = OL.logmel(y, n_mels=16, slices=4, n_fft=256, hop=64)
    yp = np.pad(y, 128, mode="reflect")
    n_frames = 1 + (len(yp) - 256) // 64
    win = np.hanning(257)[:-1]
    P = np.stack([np.abs(np.fft.rfft(yp[t * 64:t * 64 + 256] * win)) ** 2 for t in range(n_frames)], 1)
    M = np.log(OL.mel_filters(16, 256, 44100.0) @ P + 1e-5)
    edges = [int(round(g * n_frames / 4)) for g in range(5)]
    ref = np.concatenate([M[:, edges[g]:edges[g + 1]].mean(1) for g in range(4)])
    assert np.allclose(f, ref, rtol=1e-10, atol=1e-10)


def test_theta_gradient_matches_differences_of_the_loop():
    """The oracle's theta-gradient (reverse recursion + chain rule through
    the parameterised plate) against central differences of the oracle time
    loop itself, on a 10-mode plate over 1500 steps."""
    import workloads as W
    from oracle import adjoint as OA
    from oracle import params as OP
    fw = W.plate_fit(n_t=10)
    th = fw["theta0"] * np.array([1.0, 1.0, 1.0, 3.0, 1.0])
    steps = 1500
    rng = np.random.default_rng(5)
    gy = rng.normal(size=steps) / np.abs(OP.plate_from_theta(fw, th)["x0"]).max()
    g = OP.theta_gradient(fw, th, steps, 44100.0, gy)
    for i in range(5):
        h = 1e-5 * th[i]
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (gy @ OA.forward(OP.plate_from_theta(fw, tp), steps, 44100.0)[0]
              - gy @ OA.forward(OP.plate_from_theta(fw, tm), steps, 44100.0)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-5 * abs(fd), (i, fd, g[i])


def test_string_theta_gradient_matches_differences_of_the_loop():
    """The oracle's string theta-gradient (reverse recursion + chain rule
    through the parameterised Kirchhoff-Carrier string) against central
    differences of the oracle time loop, on a 10-mode string over 2000
    steps; and the parameterised string equals the physical one built from
    the same tension, stiffness, length and damping."""
    from oracle import adjoint as OA
    sf = W.string_fit(n_modes=10)
    th = sf["theta0"] * np.array([1.0, 50.0, 1.0, 3.0, 1.0])  # a stiffer string
    steps = 2000
    rng = np.random.default_rng(6)
    gy = rng.normal(size=steps) / np.abs(OP.string_from_theta(sf, th)["x0"]).max()
    g = OP.string_theta_gradient(sf, th, steps, 44100.0, gy)
    for i in range(5):
        h = 1e-5 * th[i]
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (gy @ OA.forward(OP.string_from_theta(sf, tp), steps, 44100.0)[0]
              - gy @ OA.forward(OP.string_from_theta(sf, tm), steps, 44100.0)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-5 * abs(fd), (i, fd, g[i])
    # the textbook stiff string: f_k = k f1 sqrt(1 + B k^2), f1 = sqrt(T0^)/(2L),
    # B = pi^2 EI^ / (T0^ L^2)
    inst = OP.string_from_theta(sf, th)
    T0h, EIh, L = th[0], th[1], th[2]
    k = np.arange(1, 11)
    f = k * np.sqrt(T0h) / (2 * L) * np.sqrt(1 + np.pi ** 2 * EIh / (T0h * L ** 2) * k ** 2)
    assert np.allclose(inst["omega"] / (2 * np.pi), f, rtol=1e-12)
    assert np.isclose(inst["kappa"], sf["EAhat"] / (2 * L), rtol=1e-14)
    assert np.allclose(inst["gamma"], th[3] + th[4] * (k * np.pi / L) ** 2, rtol=1e-13)
