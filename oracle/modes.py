"""Transverse modes of a fixed string and a simply supported rectangular plate.

Paper, Sec. 3 (eigenvalue problem): Laplacian eigenpairs, Delta Phi = -lambda
Phi, analytic for a string fixed at both ends and a simply supported
rectangle.  Modes are L2-normalised so that the integral of Phi^2 over the
domain is one.
"""
from __future__ import annotations

import numpy as np


def string_modes(L: float, n: int):
    """Mode numbers k = 1..n, eigenvalues lambda_k = (k pi / L)^2."""
    k = np.arange(1, n + 1)
    return k, (k * np.pi / L) ** 2


def string_phi(k, L: float, x):
    """Normalised string mode sqrt(2/L) sin(k pi x / L) at points x.
    Returns [len(k), len(x)]."""
    k = np.asarray(k, dtype=float)[:, None]
    x = np.asarray(x, dtype=float)[None, :]
    return np.sqrt(2.0 / L) * np.sin(k * np.pi * x / L)


def plate_modes(Lx: float, Ly: float, n: int):
    """The n simply supported plate modes (m, q) with the smallest
    lambda = (m pi/Lx)^2 + (q pi/Ly)^2, ties broken by (lambda, m, q).

    Every candidate with m <= n and q <= n is listed: a mode with m > n lies
    above the n modes (1..n, 1), so none of the n smallest is missed.
    Returns (m [n], q [n], lambda [n]).
    """
    cands = []
    for m in range(1, n + 1):
        for q in range(1, n + 1):
            lam = (m * np.pi / Lx) ** 2 + (q * np.pi / Ly) ** 2
            cands.append((lam, m, q))
    cands.sort()
    sel = cands[:n]
    lam = np.array([c[0] for c in sel])
    m = np.array([c[1] for c in sel], dtype=np.int64)
    q = np.array([c[2] for c in sel], dtype=np.int64)
    return m, q, lam


def plate_phi_derivs(m, q, Lx: float, Ly: float, x, y):
    """Normalised plate modes (2/sqrt(Lx Ly)) sin(m pi x/Lx) sin(q pi y/Ly)
    and their second derivatives at the points (x[i], y[i]).

    Returns a dict of [n_modes, n_points] arrays: phi, xx, yy, xy.
    """
    a = (np.asarray(m, dtype=float) * np.pi / Lx)[:, None]
    b = (np.asarray(q, dtype=float) * np.pi / Ly)[:, None]
    x = np.asarray(x, dtype=float)[None, :]
    y = np.asarray(y, dtype=float)[None, :]
    c = 2.0 / np.sqrt(Lx * Ly)
    sx, cx = np.sin(a * x), np.cos(a * x)
    sy, cy = np.sin(b * y), np.cos(b * y)
    phi = c * sx * sy
    return dict(phi=phi, xx=-a * a * phi, yy=-b * b * phi, xy=c * a * b * cx * cy)


def midpoint_grid(Lx: float, Ly: float, nx: int, ny: int):
    """Cell centres of an nx x ny grid on [0,Lx] x [0,Ly], flattened with y
    fastest, and the cell area."""
    xs = (np.arange(nx) + 0.5) * Lx / nx
    ys = (np.arange(ny) + 0.5) * Ly / ny
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    return X.ravel(), Y.ravel(), Lx * Ly / (nx * ny)
