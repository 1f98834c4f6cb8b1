"""The proposal network's HIP kernels (through the C ABI) against the FP64
reference.  Operands are rounded to BF16 inside the GEMMs (FP32 accumulate),
so the bar is a relative error of 2e-2 on outputs and gradients computed from
BF16-representable inputs and weights (the reference sees the same values)."""
import numpy as np
import pytest

from oracle import mlp as OM

pytestmark = pytest.mark.gpu


def _bf16(a):
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("dims,B", [([1024, 512, 512, 512, 512, 5], 256), ([37, 70, 3], 45)])
def test_forward_backward_adam_match_reference(dims, B):
    import torch
    from paper_2505_05940_amd.mlp import MLP
    rng = np.random.default_rng(1)
    net = MLP(dims, max_batch=B)
    net.init_params(seed=2)
    theta = _bf16(net.params())
    net.set_params(theta)
    x = _bf16(rng.normal(size=(B, dims[0])))
    y = net.forward(torch.tensor(x, device="cuda")).cpu().numpy()
    y_ref, _ = OM.forward(theta.astype(float), dims, x.astype(float))
    assert np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref) < 2e-2
    dy = _bf16(rng.normal(size=(B, dims[-1])))
    net.backward(torch.tensor(dy, device="cuda"))
    g = net.grads()
    g_ref = OM.backward(theta.astype(float), dims, x.astype(float), dy.astype(float))
    assert np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref) < 2e-2
    net.adam_step(1e-3)
    p1 = net.params()
    p_ref, _, _ = OM.adam(theta.astype(float), g.astype(float), 0 * g_ref, 0 * g_ref, 1, lr=1e-3)
    assert np.abs(p1 - p_ref).max() < 1e-6
    net.close()


def test_gemm_layout_on_identity():
    """One linear layer with W = I and b = 0 returns x exactly (BF16 inputs):
    catches any transposition or lane-layout slip in the MFMA tiles."""
    import torch
    from paper_2505_05940_amd.mlp import MLP
    n = 96
    net = MLP([n, n], max_batch=70)
    net.set_params(np.concatenate([np.eye(n).ravel(), np.zeros(n)]))
    x = _bf16(np.random.default_rng(3).normal(size=(70, n)))
    y = net.forward(torch.tensor(x, device="cuda")).cpu().numpy()
    assert np.array_equal(y, x)
    net.close()
