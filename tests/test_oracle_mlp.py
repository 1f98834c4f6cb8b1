"""Pins of the FP64 MLP reference: gradient by central differences, Adam by
its closed form after one step."""
import numpy as np

from oracle import mlp as OM


def test_mlp_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    dims = [7, 6, 5, 3]
    n = sum(i * j + j for i, j in zip(dims[:-1], dims[1:]))
    theta = rng.normal(size=n) * 0.5
    x = rng.normal(size=(4, 7))
    dy = rng.normal(size=(4, 3))
    g = OM.backward(theta, dims, x, dy)
    f = lambda t: float(np.sum(OM.forward(t, dims, x)[0] * dy))
    for i in rng.choice(n, 15, replace=False):
        e = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[i] += e
        tm[i] -= e
        assert abs((f(tp) - f(tm)) / (2 * e) - g[i]) < 1e-6 * max(1.0, abs(g[i]))


def test_adam_first_step_is_sign_times_lr():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    p1, m, v = OM.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.1, eps=0.0)
    assert np.allclose(p1, p - 0.1 * np.sign(g))
