"""Pins of the oracle's modes, in-plane eigenpairs and coupling tensors
(Sec. 3 eigenvalue problem; Sec. 3.1 coupling coefficients) against closed
forms, brute force, textbook values and the paper's H-C identity."""
import json
import os

import numpy as np
import pytest

from oracle import coupling, inplane, modes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_plate_modes_are_the_smallest_eigenvalues():
    """Against an independent enumeration: all (m, q) on a large box, sorted."""
    Lx, Ly = 0.4, 0.3
    m, q, lam = modes.plate_modes(Lx, Ly, 60)
    M = np.arange(1, 80)
    grid = np.add.outer((M * np.pi / Lx) ** 2, (M * np.pi / Ly) ** 2)
    assert np.allclose(np.sort(grid.ravel())[:60], lam, rtol=1e-14)
    assert np.all(np.diff(lam) >= 0)
    # Delta Phi = -lambda Phi at random points (second derivatives analytic)
    rng = np.random.default_rng(0)
    x, y = rng.uniform(0, Lx, 7), rng.uniform(0, Ly, 7)
    d = modes.plate_phi_derivs(m, q, Lx, Ly, x, y)
    assert np.allclose(d["xx"] + d["yy"], -lam[:, None] * d["phi"], atol=1e-9 * lam.max())


def test_plate_mode_ties_ordered_by_index():
    m, q, lam = modes.plate_modes(1.0, 1.0, 6)
    assert list(zip(m, q)) == [(1, 1), (1, 2), (2, 1), (2, 2), (1, 3), (3, 1)]


def test_clamped_eigenvalues_match_textbook():
    ref = json.load(open(os.path.join(GOLDEN, "clamped_plate_eigenvalues.json")))
    for case in ref["cases"]:
        vals = np.array(case["values"])
        fam = inplane.ClampedFamily(case["a"], case["b"], len(vals), K=16)
        got = np.sqrt(fam.zeta4) * case["a"] ** 2
        assert np.allclose(got, vals, rtol=case["rel_tol"]), got


def test_clamped_ritz_decreases_with_basis_and_converges():
    prev = None
    for K in (8, 12, 16, 22):
        z = inplane.ClampedFamily(0.4, 0.3, 12, K=K).zeta4
        if prev is not None:
            assert np.all(z <= prev * (1 + 1e-12))
        prev = z
    zK = inplane.ClampedFamily(0.4, 0.3, 12, K=30).zeta4
    assert np.allclose(prev, zK, rtol=1e-8)


def test_clamped_modes_satisfy_boundary_conditions_and_orthonormality():
    Lx, Ly = 0.4, 0.3
    fam = inplane.ClampedFamily(Lx, Ly, 10)
    t = np.linspace(0, Ly, 11)
    for xb in (0.0, Lx):
        assert np.abs(fam.eval(np.full(11, xb), t)["psi"]).max() < 1e-12
    x, y, dA = modes.midpoint_grid(Lx, Ly, 200, 150)
    z4, d = inplane.inplane_on_grid("clamped", Lx, Ly, 10, x, y, dA)
    G = dA * d["psi"] @ d["psi"].T
    assert np.allclose(np.diag(G), 1.0, atol=1e-13)
    assert np.abs(G - np.eye(10)).max() < 1e-4  # midpoint rule, O(dx^2)


def test_H_is_symmetric_in_transverse_indices():
    cp = coupling.coupling_midpoint(0.4, 0.3, 15, 12, 80, 60, family="clamped")
    H = cp["H"]
    assert np.abs(H - H.transpose(0, 2, 1)).max() <= 1e-14 * np.abs(H).max()


def _sine_midpoint_closed_form(Lx, Ly, n_t, n_in, nx, ny):
    """The midpoint sum of the sine-family H in closed form, from
    sum_{i<M} sin(j pi (i+1/2)/M) = (1 - (-1)^j) / (2 sin(j pi / 2M)) and
    the vanishing cosine sums (0 < |j| < 2M); independent of the matrix
    product the oracle uses."""
    def msum(j, L, M):
        j = np.asarray(j)
        out = np.zeros(j.shape)
        nz = (j % (2 * M)) != 0
        jj = j[nz].astype(float)
        out[nz] = (1 - np.cos(jj * np.pi)) / (2 * np.sin(jj * np.pi / (2 * M)))
        return out * (L / M)
    def sss(a, i, j, L, M):
        return 0.25 * (msum(a + i - j, L, M) + msum(a - i + j, L, M) + msum(-a + i + j, L, M) - msum(a + i + j, L, M))
    def scc(a, i, j, L, M):
        return 0.25 * (msum(a + i - j, L, M) + msum(a - i + j, L, M) + msum(a + i + j, L, M) + msum(a - i - j, L, M))
    m, q, _ = modes.plate_modes(Lx, Ly, n_t)
    a, b, _ = inplane.sine_family(Lx, Ly, n_in)
    c = 2 / np.sqrt(Lx * Ly)
    al, be = m * np.pi / Lx, q * np.pi / Ly
    H = np.zeros((n_in, n_t, n_t))
    for k in range(n_in):
        for i in range(n_t):
            for j in range(n_t):
                t1 = (al[i] ** 2 * be[j] ** 2 + be[i] ** 2 * al[j] ** 2) * sss(a[k], m[i], m[j], Lx, nx) * sss(b[k], q[i], q[j], Ly, ny)
                t2 = 2 * al[i] * be[i] * al[j] * be[j] * scc(a[k], m[i], m[j], Lx, nx) * scc(b[k], q[i], q[j], Ly, ny)
                H[k, i, j] = c ** 3 * (t1 - t2)
    return H


def _align(Hq, Href):
    s = np.sign(np.sum(Hq * Href, axis=(1, 2)))
    s[s == 0] = 1
    return s[:, None, None] * Hq


def test_sine_midpoint_H_matches_discrete_closed_form():
    Lx, Ly = 0.4, 0.3
    cp = coupling.coupling_midpoint(Lx, Ly, 10, 8, 40, 30, family="sine")
    Href = _sine_midpoint_closed_form(Lx, Ly, 10, 8, 40, 30)
    H = _align(cp["H"], Href)
    assert np.abs(H - Href).max() < 1e-11 * np.abs(Href).max()


def test_sine_exact_H_is_the_limit_of_the_midpoint_rule():
    """Midpoint H converges to the exact closed form at second order."""
    Lx, Ly = 0.4, 0.3
    He = coupling.coupling_sine_exact(Lx, Ly, 10, 10)["H"]
    errs = []
    for nx, ny in ((60, 45), (120, 90), (240, 180)):
        Hm = _align(coupling.coupling_midpoint(Lx, Ly, 10, 10, nx, ny, family="sine")["H"], He)
        errs.append(np.abs(Hm - He).max() / np.abs(He).max())
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4, errs


def test_H_brute_force_tiny_grid():
    """Five nested loops straight from the definition of H on an 8 x 6 grid,
    with second derivatives by central finite differences of the mode
    functions (step 1e-4), against the oracle's matrix-product builder."""
    Lx, Ly, nx, ny, n = 0.4, 0.3, 8, 6, 4
    cp = coupling.coupling_midpoint(Lx, Ly, n, n, nx, ny, family="sine")
    m, q, _ = modes.plate_modes(Lx, Ly, n)
    a, b, _ = inplane.sine_family(Lx, Ly, n)
    c = 2 / np.sqrt(Lx * Ly)
    f = lambda mm, qq, x, y: c * np.sin(mm * np.pi * x / Lx) * np.sin(qq * np.pi * y / Ly)
    e = 1e-4
    def d2(mm, qq, x, y):
        fxx = (f(mm, qq, x + e, y) - 2 * f(mm, qq, x, y) + f(mm, qq, x - e, y)) / e ** 2
        fyy = (f(mm, qq, x, y + e) - 2 * f(mm, qq, x, y) + f(mm, qq, x, y - e)) / e ** 2
        fxy = (f(mm, qq, x + e, y + e) - f(mm, qq, x + e, y - e) - f(mm, qq, x - e, y + e) + f(mm, qq, x - e, y - e)) / (4 * e * e)
        return fxx, fyy, fxy
    dA = Lx * Ly / (nx * ny)
    H = np.zeros((n, n, n))
    for k in range(n):
        for i in range(n):
            for j in range(n):
                s = 0.0
                for ix in range(nx):
                    for iy in range(ny):
                        x, y = (ix + 0.5) * Lx / nx, (iy + 0.5) * Ly / ny
                        ixx, iyy, ixy = d2(m[i], q[i], x, y)
                        jxx, jyy, jxy = d2(m[j], q[j], x, y)
                        s += f(a[k], b[k], x, y) * (ixx * jyy + iyy * jxx - 2 * ixy * jxy) * dA
                H[k, i, j] = s
    # the tiny grid is too coarse for unit midpoint norms of every mode, so
    # divide by the same-rule norms as the definition asks
    xs, ys, _ = modes.midpoint_grid(Lx, Ly, nx, ny)
    nphi = np.sqrt(dA * np.sum(f(m[:, None], q[:, None], xs, ys) ** 2, axis=1))
    npsi = np.sqrt(dA * np.sum(f(a[:, None], b[:, None], xs, ys) ** 2, axis=1))
    H /= npsi[:, None, None] * nphi[None, :, None] * nphi[None, None, :]
    Hq = _align(cp["H"], H)
    assert np.abs(Hq - H).max() < 2e-6 * np.abs(H).max()


def test_H_C_identity():
    """C^j_{ik} = H^k_{ij} for modes vanishing on the edges (Sec. 4.3): the
    independently integrated C tends to H as the grid is refined."""
    for fam in ("sine", "clamped"):
        errs = []
        for nx, ny in ((80, 60), (160, 120)):
            cp = coupling.coupling_midpoint(0.4, 0.3, 8, 8, nx, ny, family=fam, with_C=True)
            H, C = cp["H"], cp["C"]  # H[k,i,j], C[s,i,k]
            diff = C - H.transpose(2, 1, 0)  # C[j,i,k] vs H[k,i,j]
            errs.append(np.abs(diff).max() / np.abs(H).max())
        assert errs[1] < errs[0] / 3.0 and errs[1] < 2e-3, (fam, errs)


def test_H_parity_zeros():
    """Each mode is even or odd about both centre lines, so H[k,i,j] vanishes
    unless the x parities and the y parities each combine evenly: 3/4 of the
    entries are structural zeros for the sine family."""
    cp = coupling.coupling_sine_exact(0.4, 0.3, 24, 24)
    H = cp["H"]
    m, q = cp["m"], cp["q"]
    a, b, _ = inplane.sine_family(0.4, 0.3, 24)
    # mode sin(m pi x/L) is even about the centre iff m is odd
    px = (a[:, None, None] + m[None, :, None] + m[None, None, :]) % 2
    py = (b[:, None, None] + q[None, :, None] + q[None, None, :]) % 2
    allowed = (px == 1) & (py == 1)
    assert np.all(np.abs(H[~allowed]) < 1e-12 * np.abs(H).max())
    assert np.all(np.abs(H[allowed]) > 0)


def test_sign_of_inplane_mode_does_not_change_the_force():
    from oracle import simulate
    rng = np.random.default_rng(3)
    Ht = coupling.coupling_sine_exact(0.4, 0.3, 10, 10)["H"]
    X = rng.normal(size=10)
    F = simulate.force_vk(X, Ht)
    Ht2 = Ht.copy()
    Ht2[[1, 4, 7]] *= -1
    assert np.array_equal(F, simulate.force_vk(X, Ht2))


def test_forces_are_gradients_of_their_potentials():
    """f_vk = grad of 1/4 sum eta_n^2 and f_kc = grad of kappa/4 (sum lam X^2)^2,
    by central differences."""
    from oracle import simulate
    rng = np.random.default_rng(4)
    Ht = coupling.coupling_sine_exact(0.4, 0.3, 8, 6)["H"] * 1e-3
    X = rng.normal(size=8)
    V = lambda X: 0.25 * np.sum(np.einsum("npq,p,q->n", Ht, X, X) ** 2)
    lam = rng.uniform(1, 3, 8)
    U = lambda X: 0.25 * 2.0 * np.sum(lam * X * X) ** 2
    e = 1e-6
    gV = np.array([(V(X + e * np.eye(8)[k]) - V(X - e * np.eye(8)[k])) / (2 * e) for k in range(8)])
    gU = np.array([(U(X + e * np.eye(8)[k]) - U(X - e * np.eye(8)[k])) / (2 * e) for k in range(8)])
    assert np.allclose(simulate.force_vk(X, Ht), gV, rtol=1e-7, atol=1e-9 * np.abs(gV).max())
    assert np.allclose(simulate.force_tension(X, lam, 2.0), gU, rtol=1e-7)


def test_scaled_tensor_reproduces_the_paper_force_form():
    """f_s = E/(2 rho) sum_n zeta_n^-4 (sum_qr H^n_qr X_q X_r)(sum_p C^s_pn X_p)
    with C from its own quadrature equals the H~ contraction used by the
    time loop, up to the quadrature error of the H-C identity."""
    from oracle import simulate
    cp = coupling.coupling_midpoint(0.4, 0.3, 8, 8, 320, 240, family="clamped", with_C=True)
    H, C, z4 = cp["H"], cp["C"], cp["zeta4"]
    E, rho = 2e11, 7860.0
    Ht = coupling.scale_coupling(H, z4, E, rho)
    X = np.random.default_rng(5).normal(size=8) * 1e-6
    eta = np.einsum("nqr,q,r->n", H, X, X)
    f_paper = E / (2 * rho) * np.einsum("n,spn,p->s", eta / z4, C, X)
    f_ht = simulate.force_vk(X, Ht)
    assert np.abs(f_paper - f_ht).max() < 1e-3 * np.abs(f_ht).max()
