"""Oracle-side construction of instances from the seeded workload parameters.

Follows the paper's chain: modes and eigenvalues (Sec. 3), coupling tensors
(Sec. 3.1), omega and gamma (Sec. 3.2), then the initial state and output
weights of the workload's excitation and pickup point.
"""
from __future__ import annotations

import numpy as np

from . import coupling, excitation, modes, scheme


def _gamma(wl, omega, lam, rho_s):
    kind = wl["damping"][0]
    if kind == "affine_omega":
        return scheme.gamma_affine_omega(omega, wl["damping"][1], wl["damping"][2])
    if kind == "d1d3":
        return scheme.gamma_from_d(lam, wl["damping"][1], wl["damping"][2], rho_s)
    raise ValueError(kind)


def string_instance(wl):
    """Kirchhoff-Carrier string: tau = EA / (2L) (Sec. 3.1), kappa = tau/rhoA."""
    k, lam = modes.string_modes(wl["L"], wl["n_modes"])
    omega = scheme.omega_from(lam, wl["EI"], wl["T0"], wl["rhoA"])
    gamma = _gamma(wl, omega, lam, wl["rhoA"])
    pl = wl["pluck"]
    x0 = excitation.string_pluck_modal(k, wl["L"], pl["x0"], pl["amplitude"],
                                       pl["width"], wl["proj_cells"])
    c = excitation.string_output(k, wl["L"], wl["x_out"])
    tau = wl["EA"] / (2.0 * wl["L"])
    return dict(kind="tension", omega=omega, gamma=gamma, lam=lam,
                kappa=tau / wl["rhoA"], x0=x0, xm1=x0.copy(), c=c)


def plate_geometry(wl):
    """(Lx, Ly): given directly, or from the aspect ratio a = Ly/Lx and the
    area S that puts transverse mode N at the target frequency:
    rho_s w^2 S^2 - T0 Lam S - D Lam^2 = 0, Lam = lambda_N at unit area."""
    if "Lx" in wl:
        return wl["Lx"], wl["Ly"]
    a = wl["aspect"]
    D = wl["E"] * wl["h"] ** 3 / (12.0 * (1.0 - wl["nu"] ** 2))
    rho_s = wl["rho"] * wl["h"]
    _, _, lam1 = modes.plate_modes(1.0 / np.sqrt(a), np.sqrt(a), wl["n_t"])
    Lam = lam1[-1]
    w = 2.0 * np.pi * wl["top_mode_hz"]
    T0 = wl["T0"]
    S = (T0 * Lam + np.sqrt((T0 * Lam) ** 2 + 4.0 * rho_s * w * w * D * Lam ** 2)) / (2.0 * rho_s * w * w)
    return np.sqrt(S / a), np.sqrt(S * a)


def plate_berger_instance(wl):
    """Tension-modulated (Berger) plate (Sec. 3, tension equation; Sec. 3.1,
    modal string/membrane expansion): f_mu = tau lambda_mu q_mu sum lambda q^2
    with normalised modes and tau_membrane = E h / (2 Lx Ly (1 - nu^2));
    divided by the areal density, kappa = tau / rho_s."""
    Lx, Ly = plate_geometry(wl)
    h, E, nu, rho = wl["h"], wl["E"], wl["nu"], wl["rho"]
    D = E * h ** 3 / (12.0 * (1.0 - nu ** 2))
    rho_s = rho * h
    m, q, lam = modes.plate_modes(Lx, Ly, wl["n_t"])
    omega = scheme.omega_from(lam, D, wl["T0"], rho_s)
    gamma = _gamma(wl, omega, lam, rho_s)
    st = wl["strike"]
    nx, ny = wl["proj_grid"]
    x0 = excitation.plate_strike_modal(m, q, Lx, Ly, nx, ny, st["xc"], st["yc"], st["amplitude"],
                                       st["radius"])
    c = excitation.plate_output(m, q, Lx, Ly, *wl["out"])
    tau = E * h / (2.0 * Lx * Ly * (1.0 - nu ** 2))
    return dict(kind="tension", omega=omega, gamma=gamma, lam=lam, kappa=tau / rho_s,
                x0=x0, xm1=x0.copy(), c=c, Lx=Lx, Ly=Ly, m=m, q=q)


def plate_instance(wl, H=None):
    """von Karman plate.  H (unscaled, [n_in, n_t, n_t]) may be passed in to
    avoid rebuilding it; otherwise it is computed by the midpoint rule on
    wl['grid'], or exactly (sine family) when wl['grid'] is None."""
    Lx, Ly = plate_geometry(wl)
    h, E, nu, rho = wl["h"], wl["E"], wl["nu"], wl["rho"]
    D = E * h ** 3 / (12.0 * (1.0 - nu ** 2))
    rho_s = rho * h
    n_t, n_in = wl["n_t"], wl["n_in"]
    m, q, lam = modes.plate_modes(Lx, Ly, n_t)
    if H is None:
        if wl["grid"] is None:
            assert wl["inplane"] == "sine"
            cp = coupling.coupling_sine_exact(Lx, Ly, n_t, n_in)
        else:
            cp = coupling.coupling_midpoint(Lx, Ly, n_t, n_in, *wl["grid"],
                                            family=wl["inplane"])
        H, zeta4 = cp["H"], cp["zeta4"]
    else:
        H, zeta4 = H
    Ht = coupling.scale_coupling(H, zeta4, E, rho)
    omega = scheme.omega_from(lam, D, wl["T0"], rho_s)
    gamma = _gamma(wl, omega, lam, rho_s)
    if "strike" in wl:
        st = wl["strike"]
        xc, yc, amp, rad = st["xc"], st["yc"], st["amplitude"], st["radius"]
        xo, yo = wl["out"]
    else:
        st = wl["strike_rel"]
        xc, yc, amp = st["xc"] * Lx, st["yc"] * Ly, st["amplitude"]
        rad = st["radius_rel"] * min(Lx, Ly)
        xo, yo = wl["out_rel"][0] * Lx, wl["out_rel"][1] * Ly
    nx, ny = wl["proj_grid"]
    x0 = excitation.plate_strike_modal(m, q, Lx, Ly, nx, ny, xc, yc, amp, rad)
    c = excitation.plate_output(m, q, Lx, Ly, xo, yo)
    return dict(kind="vk", omega=omega, gamma=gamma, lam=lam, Ht=Ht, H=H,
                zeta4=zeta4, x0=x0, xm1=x0.copy(), c=c, Lx=Lx, Ly=Ly, m=m, q=q)
