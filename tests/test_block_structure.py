"""The block structure the library exploits for von Karman plates, checked on
the product's own tensor builder (CPU): with transverse modes grouped by the
parities of their two indices, every in-plane row holds, for each class of
rows, nonzero entries in exactly one class of columns, and that class is the
row class xor a fixed class of the in-plane mode; three quarters of the
entries are exact zeros when the classes are balanced.  Sine in-plane modes
give the zeros exactly; clamped ones after the builder zeroes the quadrature's
rounding."""
import numpy as np

import workloads as W


def test_sine_tensor_blocks_by_parity_class():
    from paper_2505_05940_amd import physics
    for n_t, n_in in ((17, 9), (40, 40), (64, 30)):
        wl = W.plate_vk(seed=7, n_t=n_t, n_in=n_in, family="sine", grid=None, n_steps=10)
        p = physics.plate_instance(wl)
        H = p["Ht"]
        cls = p["mode_class"]
        assert cls.dtype == np.uint8 and cls.max() <= 3
        for n in range(n_in):
            cols_of = []
            for i in range(4):
                rows = np.flatnonzero(cls == i)
                if len(rows) == 0:
                    continue
                nzcls = {int(cls[k]) for k in np.flatnonzero(np.any(H[n][rows] != 0, axis=0))}
                assert len(nzcls) <= 1, (n, i, nzcls)
                cols_of.append((i, nzcls))
            targets = {i ^ next(iter(c)) for i, c in cols_of if c}
            assert len(targets) <= 1, (n, targets)  # one xor class per in-plane row
        zero = float(np.mean(H == 0))
        assert zero > 0.6, zero


def _check_blocks(H, cls):
    for n in range(H.shape[0]):
        cols_of = []
        for i in range(4):
            rows = np.flatnonzero(cls == i)
            if len(rows) == 0:
                continue
            nzcls = {int(cls[k]) for k in np.flatnonzero(np.any(H[n][rows] != 0, axis=0))}
            assert len(nzcls) <= 1, (n, i, nzcls)
            cols_of.append((i, nzcls))
        targets = {i ^ next(iter(c)) for i, c in cols_of if c}
        assert len(targets) <= 1, (n, targets)


def test_clamped_plates_get_exact_parity_zeros():
    """Clamped in-plane modes have the parities of the sine ones about the
    plate's centre lines; midpoint quadrature leaves rounding where the
    integrals vanish.  The builder zeroes those entries (each below 1e-5 of
    its row's largest) and marks the classes, so the tensor blocks like a
    sine-family one; a row that mixes classes is left alone."""
    from paper_2505_05940_amd import physics
    wl = W.plate_vk(seed=8, n_t=40, n_in=40, family="clamped", n_steps=10)
    p = physics.plate_instance(wl)
    assert "mode_class" in p
    H, cls = p["Ht"], p["mode_class"]
    _check_blocks(H, cls)
    assert float(np.mean(H == 0)) > 0.6
    # what was zeroed was rounding: the raw quadrature tensor differs from it
    # by less than 1e-5 of each in-plane row's largest entry
    Lx, Ly = physics.plate_size(wl)
    Hr, zeta4 = physics.coupling_clamped_midpoint(Lx, Ly, p["m"], p["q"], wl["n_in"], wl["grid"])
    Hr = (np.sqrt(wl["E"] / (2.0 * wl["rho"])) * Hr / np.sqrt(zeta4)[:, None, None]).astype(np.float32)
    dev = np.abs(Hr - H).reshape(len(Hr), -1).max(axis=1) / np.abs(Hr).reshape(len(Hr), -1).max(axis=1)
    assert dev.max() < 1e-5, dev.max()
    # a coupling across the classes is not rounding: nothing is zeroed
    bad = Hr.copy()
    k0 = int(np.flatnonzero(cls == 0)[0])
    k1 = int(np.flatnonzero(cls == 1)[0])
    k2 = int(np.flatnonzero(cls == 2)[0])
    big = np.abs(bad[0]).max()
    for a, b in ((k0, k1), (k1, k0), (k0, k2), (k2, k0)):
        bad[0, a, b] += 1e-2 * big
    out, ok = physics.exact_parity_zeros(bad, cls)
    assert not ok and np.array_equal(out, bad)
