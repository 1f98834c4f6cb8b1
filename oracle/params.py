"""Oracle-side plate built from the five fitted parameters
theta = (T0/rho_s, D/rho_s, aspect a = Ly/Lx, d1/(2 rho_s), d3/(2 rho_s))
(paper, Sec. 4.3: density-normalised parameters; Sec. 3.2: omega^2 =
(D lambda^2 + T0 lambda)/rho_s and gamma = (d1 + d3 lambda)/(2 rho_s)).

Fixed: area S (Lx = sqrt(S/a), Ly = sqrt(S a)), thickness, Poisson ratio,
strike and pickup at relative positions, and the mode index sets, taken at
the base aspect.  The von Karman prefactor E/(2 rho) = 6 (1 - nu^2) D^/h^2
follows the bending stiffness.  Sine in-plane family, exact integrals.
"""
from __future__ import annotations

import numpy as np

from . import coupling, excitation, modes


def _mode_sets(fit):
    a0, S = fit["base_aspect"], fit["area"]
    Lx, Ly = np.sqrt(S / a0), np.sqrt(S * a0)
    m, q, _ = modes.plate_modes(Lx, Ly, fit["n_t"])
    a, b, _ = modes.plate_modes(Lx, Ly, fit["n_in"])
    return m, q, a, b


def plate_from_theta(fit, theta):
    T0h, Dh, asp, d1, d3 = theta
    S = fit["area"]
    Lx, Ly = np.sqrt(S / asp), np.sqrt(S * asp)
    m, q, ai, bi = _mode_sets(fit)
    lam = (m * np.pi / Lx) ** 2 + (q * np.pi / Ly) ** 2
    lam_in = (ai * np.pi / Lx) ** 2 + (bi * np.pi / Ly) ** 2
    omega = np.sqrt(Dh * lam ** 2 + T0h * lam)
    gamma = d1 + d3 * lam
    # exact sine-family integrals for the fixed index sets
    c = 2.0 / np.sqrt(Lx * Ly)
    al, be = m * np.pi / Lx, q * np.pi / Ly
    A = al[:, None] ** 2 * be[None, :] ** 2 + be[:, None] ** 2 * al[None, :] ** 2
    B = 2.0 * (al * be)[:, None] * (al * be)[None, :]
    H = np.empty((len(ai), len(m), len(m)))
    for k in range(len(ai)):
        H[k] = c ** 3 * (A * coupling._int_sss(ai[k], m[:, None], m[None, :], Lx)
                         * coupling._int_sss(bi[k], q[:, None], q[None, :], Ly)
                         - B * coupling._int_scc(ai[k], m[:, None], m[None, :], Lx)
                         * coupling._int_scc(bi[k], q[:, None], q[None, :], Ly))
    E_over_2rho = 6.0 * (1.0 - fit["nu"] ** 2) * Dh / fit["h"] ** 2
    Ht = np.sqrt(E_over_2rho) * H / lam_in[:, None, None]
    xc, yc, amp, rr = fit["strike"]
    x0 = excitation.plate_strike_modal(m, q, Lx, Ly, *fit["proj_grid"], xc * Lx, yc * Ly, amp,
                                       rr * min(Lx, Ly))
    cw = excitation.plate_output(m, q, Lx, Ly, fit["out"][0] * Lx, fit["out"][1] * Ly)
    return dict(kind="vk", omega=omega, gamma=gamma, lam=lam, Ht=Ht, x0=x0, xm1=x0.copy(), c=cw)


def theta_gradient(fit, theta, n_steps, fs, ybar, h_rel=1e-6):
    """dL/dtheta for a loss with dL/dy^n = ybar[n], by the chain rule: the
    reverse recursion of the time loop (``adjoint.reverse``) gives the
    gradients with respect to omega, gamma, q^0, q^-1, c and the tensor
    directions; the derivatives of those pieces with respect to each theta_j
    are central differences of ``plate_from_theta`` at a relative step h_rel
    (smooth maps with no time loop in them).  The tensor's derivative enters
    as one tangent tensor per parameter."""
    from . import adjoint
    theta = np.asarray(theta, dtype=float)
    inst = plate_from_theta(fit, theta)
    keys = ("omega", "gamma", "x0", "c", "Ht")
    dpiece = []
    for j in range(len(theta)):
        e = h_rel * theta[j]
        tp, tm = theta.copy(), theta.copy()
        tp[j] += e
        tm[j] -= e
        a, b = plate_from_theta(fit, tp), plate_from_theta(fit, tm)
        dpiece.append({k: (a[k] - b[k]) / (2.0 * e) for k in keys})
    g = adjoint.reverse(inst, n_steps, fs, np.asarray(ybar, dtype=float),
                        Hdot=[d["Ht"] for d in dpiece])
    g_omega, g_gamma = adjoint.sv_omega_gamma_grads(g, inst["omega"], inst["gamma"], 1.0 / fs)
    return np.array([
        np.sum(g_omega * d["omega"]) + np.sum(g_gamma * d["gamma"])
        + np.sum((g["x0"] + g["xm1"]) * d["x0"]) + np.sum(g["c"] * d["c"]) + g["theta"][j]
        for j, d in enumerate(dpiece)])


# ----------------------------------------------------------------------------
# Strings.  theta = (T0/rhoA, EI/rhoA, L, d1^, d3^) of a Kirchhoff-Carrier
# string (paper: Sec. 3, the tension-modulated string and tau = EA/(2L);
# Sec. 4.3, density-normalised parameters), gamma_k = d1^ + d3^ lambda_k, with
# EA/rhoA, the pluck and the pickup (relative positions) fixed.  Built through
# the oracle's own physical string with rho A = 1, so that the parameters
# are the physical quantities per unit mass.

def string_from_theta(sfit, theta):
    from . import instances
    T0h, EIh, L, d1, d3 = (float(v) for v in theta)
    xp, amp, w = sfit["pluck"]
    wl = dict(L=L, T0=T0h, EI=EIh, EA=sfit["EAhat"], rhoA=1.0, n_modes=sfit["n_modes"],
              damping=("d1d3", 2.0 * d1, 2.0 * d3),
              pluck=dict(x0=xp * L, amplitude=amp, width=w * L),
              x_out=sfit["out"] * L, proj_cells=sfit["proj_cells"])
    return instances.string_instance(wl)


def _force_scale(inst):
    """The string's nonlinear force kappa lambda_k q_k sum_j lambda_j q_j^2 is
    a fixed shape times kappa lambda_1^2 when every lambda scales alike."""
    return inst["kappa"] * inst["lam"][0] ** 2


def string_theta_gradient(sfit, theta, n_steps, fs, ybar, h_rel=1e-6):
    """dL/dtheta of a string for dL/dy^n = ybar[n]: the reverse recursion
    gives the gradients with respect to omega, gamma, q^0, q^-1, c and the
    force scale; the derivatives of those pieces with respect to theta are
    central differences of ``string_from_theta`` (for the force, of the log of
    its scale, after checking that the lambdas move by one common factor)."""
    from . import adjoint
    theta = np.asarray(theta, dtype=float)
    inst = string_from_theta(sfit, theta)
    g = adjoint.reverse(inst, n_steps, fs, np.asarray(ybar, dtype=float))
    g_omega, g_gamma = adjoint.sv_omega_gamma_grads(g, inst["omega"], inst["gamma"], 1.0 / fs)
    out = np.empty(len(theta))
    for j in range(len(theta)):
        e = h_rel * theta[j]
        tp, tm = theta.copy(), theta.copy()
        tp[j] += e
        tm[j] -= e
        a, b = string_from_theta(sfit, tp), string_from_theta(sfit, tm)
        ra = a["lam"] / inst["lam"]
        assert np.allclose(ra, ra[0], rtol=1e-12), "the lambdas do not move together"
        d = {k: (a[k] - b[k]) / (2.0 * e) for k in ("omega", "gamma", "x0", "c")}
        dlog_s = (np.log(_force_scale(a)) - np.log(_force_scale(b))) / (2.0 * e)
        out[j] = (np.sum(g_omega * d["omega"]) + np.sum(g_gamma * d["gamma"])
                  + np.sum((g["x0"] + g["xm1"]) * d["x0"]) + np.sum(g["c"] * d["c"]) + g["scale"] * dlog_s)
    return out
