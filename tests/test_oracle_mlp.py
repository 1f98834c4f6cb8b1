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


def test_bf16_rounding_and_operand_rounded_network():
    """BF16 keeps 7 fraction bits (spacing 2^-7 at 1): 1 + 2^-8 and
    1 + 3 2^-8 are ties and round to the neighbour with an even last bit (1
    and 1 + 2^-6); values already on the grid pass unchanged.  With every weight and input on the
    BF16 grid (small integers and halves), the operand-rounded network equals
    the plain FP64 network exactly in its first layer and its gradient."""
    from oracle import mlp as OM
    v = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -7, -2.5, 3.0e38], np.float32)
    r = OM.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1 + 2.0 ** -6) and r[3] == np.float32(1 + 2.0 ** -7)
    assert r[4] == -2.5
    rng = np.random.default_rng(0)
    dims = [6, 4, 3]
    theta = rng.integers(-4, 5, size=6 * 4 + 4 + 4 * 3 + 3) / 2.0
    x = rng.integers(-3, 4, size=(5, 6)).astype(float)
    acts = OM.forward_bf16_operands(theta, dims, x)
    y, _ = OM.forward(theta, dims, x)
    # first-layer activations are small half-integers (on the grid), so the
    # second product's operands are exact too
    assert np.array_equal(acts[-1], y)
    dy = rng.integers(-2, 3, size=(5, 3)).astype(float)
    assert np.array_equal(OM.backward_bf16_operands(theta, dims, acts, dy), OM.backward(theta, dims, x, dy))
