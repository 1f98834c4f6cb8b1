"""FP64 reference of the proposal network: a multilayer perceptron with ReLU
between layers and a linear output, its gradients by the chain rule, and
Adam (Kingma & Ba 2015, bias-corrected).  Parameters are W_l [out, in] and
b_l [out] per layer, flattened layer by layer as W_l then b_l."""
from __future__ import annotations

import numpy as np


def unflatten(theta, dims):
    out, o = [], 0
    for i, j in zip(dims[:-1], dims[1:]):
        W = theta[o:o + i * j].reshape(j, i)
        o += i * j
        b = theta[o:o + j]
        o += j
        out.append((W, b))
    return out


def forward(theta, dims, x):
    """Returns the output and the list of layer inputs (activations)."""
    acts = [np.asarray(x, float)]
    layers = unflatten(np.asarray(theta, float), dims)
    for l, (W, b) in enumerate(layers):
        z = acts[-1] @ W.T + b
        acts.append(np.maximum(z, 0.0) if l + 1 < len(layers) else z)
    return acts[-1], acts


def backward(theta, dims, x, dy):
    """Gradient of sum_b dy[b] . y[b] with respect to theta (flattened)."""
    _, acts = forward(theta, dims, x)
    layers = unflatten(np.asarray(theta, float), dims)
    g = np.asarray(dy, float)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (g.T @ acts[l], g.sum(axis=0))
        if l > 0:
            g = (g @ W) * (acts[l] > 0)
    return np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return p, m, v


# ----------------------------------------------------------------------------
# The same network with each matrix product's operands rounded to BF16 first
# (products then summed exactly in FP64), the arithmetic of a BF16 matrix
# unit with FP32 accumulation up to the order of its sums.  Bias, ReLU and
# the bias gradients stay in full precision.  Test infrastructure: it gives
# the GEMM path a reference that differs from it only by accumulation order,
# so that its bar need not absorb the BF16 rounding itself, which compounds
# over the layers of the back-propagated signal (2^-8 per product).

def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float32."""
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def forward_bf16_operands(theta, dims, x):
    """Activations [x, a_1, ..., y] with BF16-rounded matrix operands."""
    acts = [x]
    layers = unflatten(theta, dims)
    for l, (W, b) in enumerate(layers):
        z = bf16(acts[-1]).astype(float) @ bf16(W).astype(float).T + b
        acts.append(np.maximum(z, 0.0) if l + 1 < len(layers) else z)
    return acts


def backward_bf16_operands(theta, dims, acts, dy):
    """Flattened gradient of sum(dy * y) with BF16-rounded matrix operands
    (acts from forward_bf16_operands)."""
    layers = unflatten(theta, dims)
    g = dy
    out = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        gb = bf16(g).astype(float)
        out[l] = np.concatenate([(gb.T @ bf16(acts[l]).astype(float)).ravel(), g.sum(axis=0)])
        if l > 0:
            g = (gb @ bf16(W).astype(float)) * (acts[l] > 0)
    return np.concatenate(out)
