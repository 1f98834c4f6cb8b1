"""Coupling tensors of the von Karman plate.

Paper, Sec. 3.1, coupling-coefficient equations:

    H^k_{ij} = int_S Psi_k L(Phi_i, Phi_j) dS / (|Psi_k| |Phi_i| |Phi_j|)
    C^s_{ij} = int_S Phi_s L(Phi_i, Psi_j) dS / (|Phi_s| |Phi_i| |Psi_j|)

with the von Karman operator L(f, g) = Delta f Delta g - grad grad f : grad
grad g (von Karman operator equation), which in Cartesian components is
f_xx g_yy + f_yy g_xx - 2 f_xy g_xy.  The oracle stores H as H[k, i, j]
(in-plane index first).

``coupling_midpoint`` evaluates the integrals with the midpoint rule on an
nx x ny grid, written as one matrix product of the in-plane mode samples with
the samples of L(Phi_i, Phi_j).  ``coupling_sine_exact`` gives the exact
integrals for the sine in-plane family through product-to-sum identities.
"""
from __future__ import annotations

import numpy as np

from .inplane import inplane_on_grid, sine_family
from .modes import midpoint_grid, plate_modes, plate_phi_derivs


def vk_operator(f, g):
    """L(f, g) for derivative dicts f, g with entries xx, yy, xy (broadcast)."""
    return f["xx"] * g["yy"] + f["yy"] * g["xx"] - 2.0 * f["xy"] * g["xy"]


def coupling_midpoint(Lx, Ly, n_t, n_in, nx, ny, family="clamped", K=None,
                      with_C=False):
    """H[k, i, j] by the midpoint rule on nx x ny cells (and C[s, i, j] if
    asked).  Norms use the same rule.  Returns dict with H, zeta4, modes.
    """
    m, q, lam = plate_modes(Lx, Ly, n_t)
    x, y, dA = midpoint_grid(Lx, Ly, nx, ny)
    zeta4, psi = inplane_on_grid(family, Lx, Ly, n_in, x, y, dA, K)
    phi = plate_phi_derivs(m, q, Lx, Ly, x, y)
    nphi = np.sqrt(dA * np.sum(phi["phi"] ** 2, axis=1))
    npsi = np.sqrt(dA * np.sum(psi["psi"] ** 2, axis=1))
    G = x.size
    H = np.empty((n_in, n_t, n_t))
    for i in range(n_t):
        fi = {k: v[i][None, :] for k, v in phi.items()}
        Lij = vk_operator(fi, phi)  # [n_t (j), G]
        H[:, i, :] = dA * (psi["psi"] @ Lij.T)
    H /= npsi[:, None, None] * nphi[None, :, None] * nphi[None, None, :]
    out = dict(H=H, zeta4=zeta4, m=m, q=q, lam=lam)
    if with_C:
        C = np.empty((n_t, n_t, n_in))
        for i in range(n_t):
            fi = {k: v[i][None, :] for k, v in phi.items()}
            Lik = vk_operator(fi, psi)  # [n_in (k), G]
            C[:, i, :] = dA * (phi["phi"] @ Lik.T)
        C /= nphi[:, None, None] * nphi[None, :, None] * npsi[None, None, :]
        out["C"] = C
    assert G == nx * ny
    return out


def _sin_int(k, L):
    """Exact integral over [0, L] of sin(k pi x / L) for integer k of any
    sign: L (1 - cos k pi) / (k pi), i.e. 2 L / (k pi) for odd k, else 0."""
    k = np.asarray(k)
    return 2.0 * L * (k % 2) / (np.pi * np.where(k == 0, 1, k))


def _int_sss(a, i, j, L):
    """Exact integral over [0, L] of sin(a u) sin(i u) sin(j u), u = pi x/L."""
    return 0.25 * (_sin_int(a + i - j, L) + _sin_int(a - i + j, L)
                   + _sin_int(-a + i + j, L) - _sin_int(a + i + j, L))


def _int_scc(a, i, j, L):
    """Exact integral over [0, L] of sin(a u) cos(i u) cos(j u), u = pi x/L."""
    return 0.25 * (_sin_int(a + i - j, L) + _sin_int(a - i + j, L)
                   + _sin_int(a + i + j, L) + _sin_int(a - i - j, L))


def coupling_sine_exact(Lx, Ly, n_t, n_in):
    """Exact H[k, i, j] for the sine in-plane family.

    With c = 2/sqrt(Lx Ly), alpha = m pi/Lx and beta = q pi/Ly, the modes are
    c sin(alpha x) sin(beta y) and
        L(Phi_i, Phi_j) = (a_i^2 b_j^2 + b_i^2 a_j^2) Phi_i Phi_j
                          - 2 a_i b_i a_j b_j c^2 cos cos cos cos,
    so each entry is a sum of two products of 1-D integrals of three
    trigonometric factors, each a sum of four sine integrals.
    """
    m, q, lam = plate_modes(Lx, Ly, n_t)
    a_k, b_k, zeta4 = sine_family(Lx, Ly, n_in)
    c = 2.0 / np.sqrt(Lx * Ly)
    al = m * np.pi / Lx
    be = q * np.pi / Ly
    A = al[:, None] ** 2 * be[None, :] ** 2 + be[:, None] ** 2 * al[None, :] ** 2
    B = 2.0 * (al * be)[:, None] * (al * be)[None, :]
    mi, mj = m[:, None], m[None, :]
    qi, qj = q[:, None], q[None, :]
    H = np.empty((n_in, n_t, n_t))
    for k in range(n_in):
        Sx = _int_sss(a_k[k], mi, mj, Lx)
        Sy = _int_sss(b_k[k], qi, qj, Ly)
        Cx = _int_scc(a_k[k], mi, mj, Lx)
        Cy = _int_scc(b_k[k], qi, qj, Ly)
        H[k] = c ** 3 * (A * Sx * Sy - B * Cx * Cy)
    return dict(H=H, zeta4=zeta4, m=m, q=q, lam=lam)


def scale_coupling(H, zeta4, E, rho):
    """Scaled tensor H~[n,p,q] = sqrt(E / (2 rho)) H[n,p,q] / zeta_n^2.

    From the von Karman modal force (Sec. 3.1, nonlinear plate equation)
    f_s = E/(2 rho) sum_n zeta_n^-4 (sum_qr H^n_qr X_q X_r)(sum_p C^s_pn X_p)
    with C^s_pn = H^n_ps (simply supported identity, Sec. 4.3): with H~,
    eta_n = sum_pq H~[n,p,q] X_p X_q and f_k = sum_{n,q} H~[n,k,q] X_q eta_n.
    rho is the volumetric density.
    """
    return np.sqrt(E / (2.0 * rho)) * H / np.sqrt(zeta4)[:, None, None]
