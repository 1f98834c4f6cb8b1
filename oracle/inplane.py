"""In-plane (Airy stress function) eigenpairs Psi_n, zeta_n^4.

Paper, Sec. 3.1 (coupling coefficients): Psi and zeta^4 are the
eigenfunctions and eigenvalues of the Airy stress function operator, i.e.
Delta Delta Psi = zeta^4 Psi on the plate.  The paper does not state the
in-plane boundary conditions.  Two families are provided:

* ``clamped``: Psi = d Psi / dn = 0 on the edges (in-plane edges free of
  traction).  Computed by a Rayleigh-Ritz method: the biharmonic energy
  integral of (Delta Psi)^2 against the integral of Psi^2, over the tensor
  basis X_a(x) Y_b(y) with X_a(t) = (1 - t^2)^2 P_a(t) (Legendre P_a, t
  mapped to [-1, 1]), which satisfies both conditions.  Both integrals are
  assembled on a 2-D Gauss-Legendre grid that integrates the polynomial
  integrands exactly.
* ``sine``: Psi = Delta Psi = 0 on the edges; Psi_ab has the same form as the
  transverse plate modes and zeta^4 = lambda_ab^2.

Each Psi_n is normalised to unit L2 norm under a caller-chosen midpoint rule
(the one the coupling tensor is built with) and its sign is fixed so that its
largest-magnitude sample on that grid is positive.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg

from .modes import plate_modes, plate_phi_derivs


def sine_family(Lx: float, Ly: float, n_in: int):
    """Sine in-plane family: (a [n], b [n], zeta4 [n]) for the n_in smallest
    lambda_ab, zeta^4 = lambda^2."""
    a, b, lam = plate_modes(Lx, Ly, n_in)
    return a, b, lam ** 2


def _clamped_basis_1d(K: int):
    """Legendre-series coefficients of X_a(t) = (1 - t^2)^2 P_a(t), a < K,
    and of their first and second t-derivatives."""
    w = npleg.poly2leg([1.0, 0.0, -2.0, 0.0, 1.0])  # (1 - t^2)^2
    funcs = []
    for a in range(K):
        pa = np.zeros(a + 1)
        pa[a] = 1.0
        c = npleg.legmul(w, pa)
        funcs.append((c, npleg.legder(c, 1), npleg.legder(c, 2)))
    return funcs


def _eval_1d(funcs, t, L: float):
    """Values, d/dx and d2/dx2 of the 1-D basis at t in [-1, 1] (x = L(t+1)/2)."""
    v = np.array([npleg.legval(t, f[0]) for f in funcs])
    d1 = np.array([npleg.legval(t, f[1]) for f in funcs]) * (2.0 / L)
    d2 = np.array([npleg.legval(t, f[2]) for f in funcs]) * (2.0 / L) ** 2
    return v, d1, d2


class ClampedFamily:
    """Rayleigh-Ritz clamped in-plane modes on [0,Lx] x [0,Ly].

    ``K`` basis functions per direction; the lowest ``n_in`` eigenpairs are
    kept in ascending zeta^4.
    """

    def __init__(self, Lx: float, Ly: float, n_in: int, K: int | None = None):
        if K is None:
            # largest half-wave count among the wanted modes, estimated from
            # the sine family of the same size, plus a margin
            a, b, _ = sine_family(Lx, Ly, n_in)
            K = 2 * int(max(a.max(), b.max())) + 8
        self.Lx, self.Ly, self.n_in, self.K = Lx, Ly, n_in, K
        self.fx = _clamped_basis_1d(K)
        self.fy = _clamped_basis_1d(K)
        ng = K + 6
        t, w = npleg.leggauss(ng)
        # 2-D Gauss grid, flattened with y fastest
        TX, TY = np.meshgrid(t, t, indexing="ij")
        WX, WY = np.meshgrid(w, w, indexing="ij")
        wts = (WX * WY).ravel() * (Lx / 2.0) * (Ly / 2.0)
        B, Bxx, Byy, _ = self._basis_2d(TX.ravel(), TY.ravel())
        lapB = Bxx + Byy
        # Rayleigh quotient: integral of (Delta Psi)^2 over integral of Psi^2
        Kmat = (lapB * wts) @ lapB.T
        Mmat = (B * wts) @ B.T
        from scipy.linalg import eigh
        vals, vecs = eigh(Kmat, Mmat)
        self.zeta4 = vals[:n_in]
        self.coef = vecs[:, :n_in].T  # [n_in, K*K]

    def _basis_2d(self, tx, ty):
        vx, dx1, dx2 = _eval_1d(self.fx, tx, self.Lx)
        vy, dy1, dy2 = _eval_1d(self.fy, ty, self.Ly)
        K = self.K
        # basis index a*K + b -> X_a(x) Y_b(y)
        B = (vx[:, None, :] * vy[None, :, :]).reshape(K * K, -1)
        Bxx = (dx2[:, None, :] * vy[None, :, :]).reshape(K * K, -1)
        Byy = (vx[:, None, :] * dy2[None, :, :]).reshape(K * K, -1)
        Bxy = (dx1[:, None, :] * dy1[None, :, :]).reshape(K * K, -1)
        return B, Bxx, Byy, Bxy

    def eval(self, x, y):
        """Psi_n and second derivatives at points (x, y) (unnormalised).
        Returns dict of [n_in, n_points]: psi, xx, yy, xy."""
        tx = 2.0 * np.asarray(x) / self.Lx - 1.0
        ty = 2.0 * np.asarray(y) / self.Ly - 1.0
        B, Bxx, Byy, Bxy = self._basis_2d(tx, ty)
        c = self.coef
        return dict(psi=c @ B, xx=c @ Bxx, yy=c @ Byy, xy=c @ Bxy)


def inplane_on_grid(family: str, Lx: float, Ly: float, n_in: int, x, y,
                    dA: float, K: int | None = None):
    """In-plane modes on the quadrature points (x, y) with cell area dA,
    normalised to unit midpoint-rule L2 norm, sign fixed by the largest
    sample.  Returns (zeta4 [n_in], dict of [n_in, G] arrays psi/xx/yy/xy).
    """
    if family == "sine":
        a, b, zeta4 = sine_family(Lx, Ly, n_in)
        d = plate_phi_derivs(a, b, Lx, Ly, x, y)
        d = dict(psi=d["phi"], xx=d["xx"], yy=d["yy"], xy=d["xy"])
    elif family == "clamped":
        fam = ClampedFamily(Lx, Ly, n_in, K)
        zeta4 = fam.zeta4
        d = fam.eval(x, y)
    else:
        raise ValueError(family)
    psi = d["psi"]
    norm = np.sqrt(dA * np.sum(psi * psi, axis=1))
    idx = np.argmax(np.abs(psi), axis=1)
    sign = np.sign(psi[np.arange(psi.shape[0]), idx])
    scale = (sign / norm)[:, None]
    return zeta4, {k: v * scale for k, v in d.items()}
