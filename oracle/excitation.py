"""Initial displacement projections and output weights (modal <-> physical).

The excitations of the workloads are raised-cosine initial displacements
released from rest; the output is the displacement at one point,
w(x_o) = sum_k q_k Phi_k(x_o).  Projections use the midpoint rule.
"""
from __future__ import annotations

import numpy as np

from .modes import midpoint_grid, plate_phi_derivs, string_phi


def raised_cosine_1d(x, x0, amplitude, width):
    """(A/2)(1 + cos(pi (x - x0) / (width/2))) for |x - x0| < width/2."""
    half = 0.5 * width
    d = np.abs(np.asarray(x) - x0)
    return np.where(d < half, 0.5 * amplitude * (1.0 + np.cos(np.pi * d / half)), 0.0)


def raised_cosine_2d(x, y, xc, yc, amplitude, radius):
    """(A/2)(1 + cos(pi r / r0)) for r < r0."""
    r = np.hypot(np.asarray(x) - xc, np.asarray(y) - yc)
    return np.where(r < radius, 0.5 * amplitude * (1.0 + np.cos(np.pi * r / radius)), 0.0)


def string_pluck_modal(k, L, x0, amplitude, width, cells):
    """X_k = int_0^L w0(x) Phi_k(x) dx by the midpoint rule on ``cells``."""
    x = (np.arange(cells) + 0.5) * L / cells
    w0 = raised_cosine_1d(x, x0, amplitude, width)
    return string_phi(k, L, x) @ w0 * (L / cells)


def plate_strike_modal(m, q, Lx, Ly, nx, ny, xc, yc, amplitude, radius):
    """X_k = int_S w0 Phi_k dS by the midpoint rule on an nx x ny grid."""
    x, y, dA = midpoint_grid(Lx, Ly, nx, ny)
    w0 = raised_cosine_2d(x, y, xc, yc, amplitude, radius)
    phi = plate_phi_derivs(m, q, Lx, Ly, x, y)["phi"]
    return phi @ w0 * dA


def string_output(k, L, x_out):
    """c_k = Phi_k(x_out)."""
    return string_phi(k, L, np.array([x_out]))[:, 0]


def plate_output(m, q, Lx, Ly, xo, yo):
    """c_k = Phi_k(xo, yo)."""
    return plate_phi_derivs(m, q, Lx, Ly, np.array([xo]), np.array([yo]))["phi"][:, 0]
