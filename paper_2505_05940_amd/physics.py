"""Host FP64 precompute that feeds the time loop: modes, in-plane
eigenpairs, coupling tensors, modal coefficients, excitation and pickup.

Paper: Sec. 3 (eigenvalue problem: analytic Laplacian modes of a fixed
string and a simply supported rectangle), Sec. 3.1 (tension-modulated force
constant tau; von Karman coupling coefficients H from the Airy-function
eigenpairs Psi, zeta^4), Sec. 3.2 (omega^2 = (D lambda^2 + T0 lambda)/rho_s,
gamma = (d1 + d3 lambda)/(2 rho_s)).  FP64 throughout; the scaled tensor is
handed to the GPU in FP32.

The sine in-plane family's tensor comes from the library's multi-threaded
host builder; the clamped family is a Rayleigh-Ritz solve in a Kronecker
basis followed by a separable midpoint evaluation of H.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L

from . import modal


# ------------------------------------------------------------------ modes
def string_eigs(L_len: float, n: int):
    k = np.arange(1, n + 1, dtype=np.float64)
    return k, (np.pi * k / L_len) ** 2


def plate_eigs(Lx: float, Ly: float, n: int):
    """Indices (m, q) and eigenvalues of the n lowest simply supported plate
    modes, ordered by (lambda, m, q).  Candidates live on a square index box
    that is grown until mode n is below every eigenvalue outside it."""
    K = int(np.ceil(np.sqrt(n))) + 2
    while True:
        mm, qq = np.meshgrid(np.arange(1, K + 1), np.arange(1, K + 1), indexing="ij")
        lam = (np.pi * mm / Lx) ** 2 + (np.pi * qq / Ly) ** 2
        order = np.lexsort((qq.ravel(), mm.ravel(), lam.ravel()))[:n]
        lam_n = lam.ravel()[order[-1]]
        outside = min((np.pi * (K + 1) / Lx) ** 2 + (np.pi / Ly) ** 2,
                      (np.pi / Lx) ** 2 + (np.pi * (K + 1) / Ly) ** 2)
        if len(order) == n and lam_n < outside:
            return mm.ravel()[order], qq.ravel()[order], lam.ravel()[order]
        K *= 2


def bending_stiffness(E, h, nu):
    return E * h ** 3 / (12.0 * (1.0 - nu * nu))


def plate_size(wl):
    """(Lx, Ly) of a plate workload: given, or from aspect a = Ly/Lx and the
    area S at which transverse mode N sits at the target frequency:
    omega_N^2 rho_s = D (Lam/S)^2 + T0 Lam/S with Lam the unit-area eigenvalue."""
    if "Lx" in wl:
        return float(wl["Lx"]), float(wl["Ly"])
    a = wl["aspect"]
    _, _, lam_unit = plate_eigs(1.0 / np.sqrt(a), np.sqrt(a), wl["n_t"])
    Lam = lam_unit[-1]
    D = bending_stiffness(wl["E"], wl["h"], wl["nu"])
    rs = wl["rho"] * wl["h"]
    w2 = (2.0 * np.pi * wl["top_mode_hz"]) ** 2
    # quadratic in u = 1/S:  D Lam^2 u^2 + T0 Lam u - rs w2 = 0
    A, B, Cc = D * Lam * Lam, wl["T0"] * Lam, -rs * w2
    u = (2.0 * -Cc) / (B + np.sqrt(B * B - 4.0 * A * Cc))
    S = 1.0 / u
    return np.sqrt(S / a), np.sqrt(S * a)


def damping(wl, omega, lam, rho_s):
    law = wl["damping"]
    if law[0] == "affine_omega":
        return law[1] + law[2] * omega
    if law[0] == "d1d3":
        return (law[1] + law[2] * lam) / (2.0 * rho_s)
    raise ValueError(law)


# ------------------------------------------------------------- excitation
def _raised_cosine(r, half, amp):
    return np.where(r < half, 0.5 * amp * (1.0 + np.cos(np.pi * r / half)), 0.0)


def string_initial(k, L_len, pluck, cells):
    """q_k^0 = midpoint projection of the raised-cosine pluck on sqrt(2/L) sin."""
    dx = L_len / cells
    x = dx * (np.arange(cells) + 0.5)
    w0 = _raised_cosine(np.abs(x - pluck["x0"]), 0.5 * pluck["width"], pluck["amplitude"])
    S = np.sin(np.outer(k, x) * (np.pi / L_len))
    return np.sqrt(2.0 / L_len) * dx * (S @ w0)


def plate_initial(m, q, Lx, Ly, grid, xc, yc, amp, radius):
    """q_k^0 = midpoint projection of a raised-cosine bump, separably:
    X_k = c dA sum_i sum_j sin(m_k x_i) w0[i,j] sin(q_k y_j)."""
    nx, ny = grid
    x = (np.arange(nx) + 0.5) * (Lx / nx)
    y = (np.arange(ny) + 0.5) * (Ly / ny)
    w0 = _raised_cosine(np.hypot(x[:, None] - xc, y[None, :] - yc), radius, amp)
    Sx = np.sin(np.outer(np.arange(1, m.max() + 1), x) * (np.pi / Lx))  # [M, nx]
    Sy = np.sin(np.outer(np.arange(1, q.max() + 1), y) * (np.pi / Ly))  # [Q, ny]
    T = Sx @ w0 @ Sy.T  # [M, Q]
    return T[m - 1, q - 1] * (2.0 / np.sqrt(Lx * Ly)) * (Lx * Ly / (nx * ny))


def plate_pickup(m, q, Lx, Ly, xo, yo):
    return 2.0 / np.sqrt(Lx * Ly) * np.sin(m * np.pi * xo / Lx) * np.sin(q * np.pi * yo / Ly)


# ---------------------------------------------- clamped in-plane family
class ClampedRitz:
    """Psi with Psi = dPsi/dn = 0 on the edges: Rayleigh-Ritz for the
    biharmonic operator in the basis (1 - t^2)^2 P_a(t) per direction,
    assembled as Kronecker products of 1-D Gauss integrals:
      K = A_x (x) M_y + B_x (x) B_y^T + B_x^T (x) B_y + M_x (x) A_y,
      M = M_x (x) M_y,
    A = int X'' X'', B[a,c] = int X_a'' X_c, M = int X X."""

    def __init__(self, Lx, Ly, n_in, K=None):
        if K is None:
            a, b, _ = plate_eigs(Lx, Ly, n_in)
            K = 2 * int(max(a.max(), b.max())) + 8
        self.Lx, self.Ly, self.K = Lx, Ly, K
        self.cx = self._series(K)
        mats_x = self._mats(self.cx, Lx)
        mats_y = self._mats(self.cx, Ly)
        Ax, Bx, Mx = mats_x
        Ay, By, My = mats_y
        Kmat = np.kron(Ax, My) + np.kron(Bx, By.T) + np.kron(Bx.T, By) + np.kron(Mx, Ay)
        Mmat = np.kron(Mx, My)
        from scipy.linalg import eigh
        w, v = eigh(Kmat, Mmat, subset_by_index=(0, n_in - 1))
        self.zeta4 = w
        self.coef = v.T.reshape(n_in, K, K)

    @staticmethod
    def _series(K):
        bump = L.poly2leg([1.0, 0.0, -2.0, 0.0, 1.0])
        return [L.legmul(bump, np.eye(a + 1)[a]) for a in range(K)]

    @staticmethod
    def _vals(series, t, Lseg, der=0):
        out = np.empty((len(series), len(t)))
        for i, c in enumerate(series):
            out[i] = L.legval(t, L.legder(c, der) if der else c)
        return out * (2.0 / Lseg) ** der

    def _mats(self, series, Lseg):
        t, w = L.leggauss(self.K + 8)
        w = w * (Lseg / 2.0)
        V0 = self._vals(series, t, Lseg, 0)
        V2 = self._vals(series, t, Lseg, 2)
        return (V2 * w) @ V2.T, (V2 * w) @ V0.T, (V0 * w) @ V0.T

    def on_grid(self, nx, ny):
        """Psi_n on the nx x ny cell centres: [n_in, nx, ny]."""
        tx = 2.0 * (np.arange(nx) + 0.5) / nx - 1.0
        ty = 2.0 * (np.arange(ny) + 0.5) / ny - 1.0
        Xv = self._vals(self.cx, tx, self.Lx)
        Yv = self._vals(self.cx, ty, self.Ly)
        return np.einsum("ax,nab,by->nxy", Xv, self.coef, Yv, optimize=True)


def coupling_clamped_midpoint(Lx, Ly, m, q, n_in, grid, K=None):
    """H[n,i,j] = dA sum_cells Psi_n L(Phi_i, Phi_j) with unit-norm Psi_n under
    the same rule (sign: largest sample positive), evaluated separably:
    P_n[(mi,mj),(qi,qj)] = sum_x sum_y s_mi s_mj Psi_n s_qi s_qj (and the
    cosine analogue), then gathered for every transverse pair."""
    nx, ny = grid
    fam = ClampedRitz(Lx, Ly, n_in, K)
    psi = fam.on_grid(nx, ny)
    dA = Lx * Ly / (nx * ny)
    nrm = np.sqrt(dA * np.einsum("nxy,nxy->n", psi, psi))
    flat = psi.reshape(n_in, -1)
    sgn = np.sign(flat[np.arange(n_in), np.argmax(np.abs(flat), axis=1)])
    psi = psi * (sgn / nrm)[:, None, None]
    x = (np.arange(nx) + 0.5) * (Lx / nx)
    y = (np.arange(ny) + 0.5) * (Ly / ny)
    M, Q = int(m.max()), int(q.max())
    sx = np.sin(np.outer(np.arange(1, M + 1), x) * np.pi / Lx)
    cx = np.cos(np.outer(np.arange(1, M + 1), x) * np.pi / Lx)
    sy = np.sin(np.outer(np.arange(1, Q + 1), y) * np.pi / Ly)
    cy = np.cos(np.outer(np.arange(1, Q + 1), y) * np.pi / Ly)
    SSx = (sx[:, None, :] * sx[None, :, :]).reshape(M * M, nx)
    CCx = (cx[:, None, :] * cx[None, :, :]).reshape(M * M, nx)
    SSy = (sy[:, None, :] * sy[None, :, :]).reshape(Q * Q, ny)
    CCy = (cy[:, None, :] * cy[None, :, :]).reshape(Q * Q, ny)
    Ps = np.einsum("ax,nxy,by->nab", SSx, psi, SSy, optimize=True)
    Pc = np.einsum("ax,nxy,by->nab", CCx, psi, CCy, optimize=True)
    al = m * np.pi / Lx
    be = q * np.pi / Ly
    c2 = 4.0 / (Lx * Ly)
    A = np.outer(al ** 2, be ** 2) + np.outer(be ** 2, al ** 2)
    B = 2.0 * np.outer(al * be, al * be)
    ii = (m[:, None] - 1) * M + (m[None, :] - 1)
    jj = (q[:, None] - 1) * Q + (q[None, :] - 1)
    H = c2 * dA * (A[None] * Ps[:, ii, jj] - B[None] * Pc[:, ii, jj])
    H = 0.5 * (H + H.transpose(0, 2, 1))  # exact symmetry (rounding only)
    return H, fam.zeta4


# ---------------------------------------------------------------- instances
def string_instance(wl):
    """Kirchhoff-Carrier string: tau = EA/(2L), kappa = tau / (rho A)."""
    k, lam = string_eigs(wl["L"], wl["n_modes"])
    omega = np.sqrt((wl["EI"] * lam * lam + wl["T0"] * lam) / wl["rhoA"])
    gamma = damping(wl, omega, lam, wl["rhoA"])
    x0 = string_initial(k, wl["L"], wl["pluck"], wl["proj_cells"])
    c = np.sqrt(2.0 / wl["L"]) * np.sin(k * np.pi * wl["x_out"] / wl["L"])
    return dict(kind="tension", omega=omega, gamma=gamma, lam=lam,
                kappa=wl["EA"] / (2.0 * wl["L"]) / wl["rhoA"], x0=x0, xm1=x0.copy(), c=c)


def plate_berger_instance(wl):
    """Tension-modulated (Berger) plate: plate modes, omega from bending
    stiffness and pre-tension, and kappa = tau / rho_s with the membrane
    tension tau = E h / (2 Lx Ly (1 - nu^2))."""
    Lx, Ly = plate_size(wl)
    E, h, nu, rho = wl["E"], wl["h"], wl["nu"], wl["rho"]
    rs = rho * h
    m, q, lam = plate_eigs(Lx, Ly, wl["n_t"])
    omega = np.sqrt((bending_stiffness(E, h, nu) * lam * lam + wl["T0"] * lam) / rs)
    gamma = damping(wl, omega, lam, rs)
    st = wl["strike"]
    x0 = plate_initial(m, q, Lx, Ly, wl["proj_grid"], st["xc"], st["yc"], st["amplitude"],
                       st["radius"])
    c = plate_pickup(m, q, Lx, Ly, *wl["out"])
    tau = E * h / (2.0 * Lx * Ly * (1.0 - nu * nu))
    return dict(kind="tension", omega=omega, gamma=gamma, lam=lam, kappa=tau / rs, x0=x0,
                xm1=x0.copy(), c=c)


def mode_classes(m, q):
    """Parity class 2 (m mod 2) + (q mod 2) of each transverse plate mode.
    With sine in-plane modes, each coupling integral over x (over y) is a sum
    of integrals of sin(k pi x / L) with k = a +- m_p +- m_q, all of one
    parity, which vanish for even k; so for in-plane row n the entries between
    modes of classes i and j vanish unless i xor j is fixed by (a_n, b_n):
    one block of columns per class of rows."""
    return (2 * (np.asarray(m) % 2) + (np.asarray(q) % 2)).astype(np.uint8)


def exact_parity_zeros(Ht, cls, tol=1e-5):
    """Clamped in-plane modes are even or odd about the plate's centre lines,
    like the sine ones, and the midpoint grid is symmetric about them, so the
    coupling integrals that the parities make odd vanish; the quadrature
    leaves rounding in their place (about 1e-11 to 1e-8 of the row's largest
    entry for 40 to 200 modes).  For every in-plane row, the rows of each
    class i couple to a single class j of columns (an involution i <-> j);
    when every other entry is below tol times that block's largest, they are
    set to zero, which lets the library store the tensor parity-blocked.
    Returns (Ht, True), or (Ht unchanged, False) if some row is not of that
    form (e.g. a mode that mixes parities)."""
    cls = np.asarray(cls)
    masks = [cls == i for i in range(4)]
    keep = np.zeros(Ht.shape, dtype=bool)
    for n in range(Ht.shape[0]):
        row = np.abs(Ht[n])
        pair = []
        for i in range(4):
            if not masks[i].any():
                pair.append(-1)
                continue
            mags = [row[np.ix_(masks[i], masks[j])].max() if masks[j].any() else 0.0 for j in range(4)]
            j = int(np.argmax(mags))
            if mags[j] > 0 and any(mags[k] > tol * mags[j] for k in range(4) if k != j):
                return Ht, False
            pair.append(j)
        for i, j in enumerate(pair):
            if j >= 0 and pair[j] != i:
                return Ht, False
            if j >= 0:
                keep[n][np.ix_(masks[i], masks[j])] = True
    return np.where(keep, Ht, np.float32(0.0)).astype(Ht.dtype), True


def plate_instance(wl, threads=0):
    """von Karman plate instance with the scaled tensor
    Ht = sqrt(E/(2 rho)) H / zeta^2 (rho volumetric) in float32."""
    Lx, Ly = plate_size(wl)
    E, h, nu, rho = wl["E"], wl["h"], wl["nu"], wl["rho"]
    rs = rho * h
    m, q, lam = plate_eigs(Lx, Ly, wl["n_t"])
    omega = np.sqrt((bending_stiffness(E, h, nu) * lam * lam + wl["T0"] * lam) / rs)
    gamma = damping(wl, omega, lam, rs)
    pref = np.sqrt(E / (2.0 * rho))
    blocked = False
    if wl["inplane"] == "sine":
        a, b, lam_in = plate_eigs(Lx, Ly, wl["n_in"])
        zeta2 = lam_in  # zeta^4 = lambda^2
        Ht = modal.vk_coupling_sine(Lx, Ly, m, q, a, b, pref / zeta2,
                                    grid=wl.get("grid"), threads=threads)
    elif wl["inplane"] == "clamped":
        H, zeta4 = coupling_clamped_midpoint(Lx, Ly, m, q, wl["n_in"], wl["grid"])
        Ht = (pref * H / np.sqrt(zeta4)[:, None, None]).astype(np.float32)
        Ht, blocked = exact_parity_zeros(Ht, mode_classes(m, q))
    else:
        raise ValueError(wl["inplane"])
    if "strike" in wl:
        st = wl["strike"]
        xc, yc, amp, rad = st["xc"], st["yc"], st["amplitude"], st["radius"]
        xo, yo = wl["out"]
    else:
        st = wl["strike_rel"]
        xc, yc, amp = st["xc"] * Lx, st["yc"] * Ly, st["amplitude"]
        rad = st["radius_rel"] * min(Lx, Ly)
        xo, yo = wl["out_rel"][0] * Lx, wl["out_rel"][1] * Ly
    x0 = plate_initial(m, q, Lx, Ly, wl["proj_grid"], xc, yc, amp, rad)
    c = plate_pickup(m, q, Lx, Ly, xo, yo)
    out = dict(kind="vk", omega=omega, gamma=gamma, lam=lam, Ht=Ht, x0=x0,
               xm1=x0.copy(), c=c, Lx=Lx, Ly=Ly, m=m, q=q)
    if wl["inplane"] == "sine" or blocked:
        out["mode_class"] = mode_classes(m, q)
    return out
