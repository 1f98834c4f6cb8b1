"""Pins of the oracle's reverse-mode gradient: complex-step derivatives
(exact to rounding for an analytic loop), central differences, and the
symmetry of the force Jacobian."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, coupling, instances


def _vk_small(n=6, steps=400, amp=3e-3):
    wl = W.plate_vk(n_t=n, family="sine", grid=None, n_steps=steps)
    wl["strike"]["amplitude"] = amp
    return instances.plate_instance(wl)


def _loss_grad(y, w):
    # L = 1/2 sum w_n y_n^2 ; dL/dy = w y
    return w * y


def test_force_jacobian_is_symmetric_and_matches_differences():
    inst = _vk_small()
    rng = np.random.default_rng(0)
    X = inst["x0"] * 3
    u, v = rng.normal(size=(2, len(X)))
    Ju, Jv = adjoint._jvp(inst, X, u), adjoint._jvp(inst, X, v)
    assert abs(v @ Ju - u @ Jv) < 1e-12 * np.abs(Ju).max() * np.abs(v).sum()
    e = 1e-7 * np.abs(X).max()
    fd = (adjoint._force(inst, X + e * u) - adjoint._force(inst, X - e * u)) / (2 * e)
    assert np.allclose(Ju, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())
    kc = instances.string_instance(W.string_kc(n_modes=8))
    X = kc["x0"] * 2
    u, v = rng.normal(size=(2, 8))
    Ju, Jv = adjoint._jvp(kc, X, u), adjoint._jvp(kc, X, v)
    assert abs(v @ Ju - u @ Jv) < 1e-12 * np.abs(Ju).max() * np.abs(v).sum()


@pytest.mark.parametrize("kind", ["vk", "tension"])
def test_reverse_gradient_matches_complex_step(kind):
    fs, steps = 44100.0, 400
    if kind == "vk":
        inst = _vk_small(steps=steps)
    else:
        inst = instances.string_instance(W.string_kc(n_modes=8))
    w = np.linspace(1, 2, steps) / np.abs(inst["x0"]).max() ** 2
    y, *_ = adjoint.forward(inst, steps, fs)
    g = adjoint.reverse(inst, steps, fs, _loss_grad(y.real, w))
    d_om, d_ga = adjoint.sv_omega_gamma_grads(g, inst["omega"], inst["gamma"], 1 / fs)

    def L_of(key, k):
        def f(t):
            i2 = dict(inst)
            v = np.array(inst[key], dtype=complex)
            v[k] = t
            i2[key] = v
            yy = adjoint.forward(i2, steps, fs)[0]
            return 0.5 * np.sum(w * yy * yy)
        return f

    for k in (0, len(inst["omega"]) // 2, len(inst["omega"]) - 1):
        cs = adjoint.complex_step(L_of("omega", k), inst["omega"][k])
        assert abs(cs - d_om[k]) <= 1e-8 * abs(cs) + 1e-12 * np.abs(d_om).max(), (k, cs, d_om[k])
        cs = adjoint.complex_step(L_of("gamma", k), inst["gamma"][k])
        assert abs(cs - d_ga[k]) <= 1e-8 * abs(cs) + 1e-12 * np.abs(d_ga).max(), (k, cs, d_ga[k])
        cs = adjoint.complex_step(L_of("x0", k), inst["x0"][k])
        assert abs(cs - g["x0"][k]) <= 1e-8 * abs(cs) + 1e-12 * np.abs(g["x0"]).max()
        cs = adjoint.complex_step(L_of("xm1", k), inst["xm1"][k])
        assert abs(cs - g["xm1"][k]) <= 1e-8 * abs(cs) + 1e-12 * np.abs(g["xm1"]).max()
        cs = adjoint.complex_step(L_of("c", k), inst["c"][k])
        assert abs(cs - g["c"][k]) <= 1e-8 * abs(cs) + 1e-12 * np.abs(g["c"]).max()
    # the nonlinear force scale (Ht ~ sqrt(s), kappa ~ s)
    def L_scale(t):
        i2 = dict(inst)
        if kind == "vk":
            i2["Ht"] = inst["Ht"] * np.sqrt(t + 0j)
        else:
            i2["kappa"] = inst["kappa"] * t
        yy = adjoint.forward(i2, steps, fs)[0]
        return 0.5 * np.sum(w * yy * yy)
    cs = adjoint.complex_step(L_scale, 1.0)
    assert abs(cs - g["scale"]) <= 1e-7 * abs(cs), (cs, g["scale"])


def test_row_scale_gradient_matches_complex_step():
    """dL/d log s_n for a factor s_n on row n of the scaled tensor, and its
    sum over rows against the whole-tensor direction Hdot = Ht."""
    fs, steps = 44100.0, 400
    inst = _vk_small(steps=steps)
    w = np.linspace(1, 2, steps) / np.abs(inst["x0"]).max() ** 2
    y, *_ = adjoint.forward(inst, steps, fs)
    g = adjoint.reverse(inst, steps, fs, _loss_grad(y.real, w), Hdot=inst["Ht"])
    for n in (0, 2, 5):
        def L(t, n=n):
            i2 = dict(inst)
            Ht = np.array(inst["Ht"], dtype=complex)
            Ht[n] *= np.exp(t)
            i2["Ht"] = Ht
            yy = adjoint.forward(i2, steps, fs)[0]
            return 0.5 * np.sum(w * yy * yy)
        cs = adjoint.complex_step(L, 0.0)
        assert abs(cs - g["row"][n]) <= 1e-7 * abs(cs), (n, cs, g["row"][n])
    assert abs(g["row"].sum() - g["theta"]) <= 1e-10 * abs(g["theta"])


def test_tensor_direction_matches_complex_step():
    fs, steps = 44100.0, 300
    inst = _vk_small(steps=steps)
    rng = np.random.default_rng(2)
    Hd = rng.normal(size=inst["Ht"].shape)
    Hd = 0.5 * (Hd + Hd.transpose(0, 2, 1)) * np.abs(inst["Ht"]).max()
    w = np.ones(steps) / np.abs(inst["x0"]).max() ** 2
    y, *_ = adjoint.forward(inst, steps, fs)
    g = adjoint.reverse(inst, steps, fs, w * y, Hdot=Hd)

    def L(t):
        i2 = dict(inst, Ht=inst["Ht"] + t * Hd)
        yy = adjoint.forward(i2, steps, fs)[0]
        return 0.5 * np.sum(w * yy * yy)
    cs = adjoint.complex_step(L, 0.0)
    assert abs(cs - g["theta"]) <= 1e-7 * abs(cs), (cs, g["theta"])


def test_central_differences_agree_at_the_configured_step():
    """Central differences with a 1e-4 relative step agree with the reverse
    gradient to 1e-3 (the gradient-check tolerance) in FP64."""
    fs, steps = 44100.0, 600
    inst = _vk_small(steps=steps)
    w = np.ones(steps) / np.abs(inst["x0"]).max() ** 2
    y, *_ = adjoint.forward(inst, steps, fs)
    g = adjoint.reverse(inst, steps, fs, w * y)
    d_om, _ = adjoint.sv_omega_gamma_grads(g, inst["omega"], inst["gamma"], 1 / fs)
    k = 2
    h = 1e-4 * inst["omega"][k]
    def L(o):
        i2 = dict(inst)
        om = inst["omega"].copy()
        om[k] = o
        i2["omega"] = om
        yy = adjoint.forward(i2, steps, fs)[0]
        return 0.5 * np.sum(w * yy * yy)
    fd = (L(inst["omega"][k] + h) - L(inst["omega"][k] - h)) / (2 * h)
    assert abs(fd - d_om[k]) < 1e-3 * abs(d_om[k])


def test_full_tensor_gradient_matches_complex_step_and_differences():
    """dL/dH~ entry by entry: single entries (off-diagonal in the last two
    indices too, each entry an independent parameter) against the complex
    step, and the contraction with a random direction against central
    differences of the plain forward loop."""
    inst = _vk_small(n=5, steps=300, amp=4e-3)
    steps, fs = 300, 44100.0
    rng = np.random.default_rng(7)
    wts = rng.uniform(0.5, 1.5, size=steps)
    y0 = adjoint.forward(inst, steps, fs)[0]
    ybar = _loss_grad(y0, wts)
    G = adjoint.reverse(inst, steps, fs, ybar, full_tensor=True)["H"]
    assert G.shape == inst["Ht"].shape
    scale = np.abs(G).max()

    def loss(Ht):
        y = adjoint.forward(dict(inst, Ht=Ht), steps, fs)[0]
        return 0.5 * np.sum(wts * y * y)

    for (i, a, b) in [(0, 0, 0), (1, 2, 4), (3, 4, 2), (4, 1, 1)]:
        E = np.zeros(inst["Ht"].shape)
        E[i, a, b] = 1.0
        cs = adjoint.complex_step(lambda t: loss(inst["Ht"] + t * E), 0.0)
        assert abs(cs - G[i, a, b]) < 1e-9 * scale, (i, a, b, cs, G[i, a, b])
    D = rng.normal(size=inst["Ht"].shape)
    h = 1e-4 / np.abs(D).max() * np.abs(inst["Ht"]).max()
    fd = (loss(inst["Ht"] + h * D) - loss(inst["Ht"] - h * D)) / (2 * h)
    assert abs(fd - np.sum(G * D)) < 1e-6 * abs(fd)
