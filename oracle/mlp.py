"""FP64 NumPy model of the spatial-factor network -- TEST INFRASTRUCTURE ONLY.

The network maps (x1, x2, theta_ell, s) to the 16 complex spatial factors
alpha_t(x) of wedge ell at phase scale s.  It has a fixed periodic feature
map (16 inputs), three hidden layers of width 128 with the tanh form of
GELU, and 32 real outputs (real and imaginary parts of 16 factors):

    z1 = f W1 + b1, a1 = gelu(z1); z2 = a1 W2 + b2, a2 = gelu(z2);
    z3 = a2 W3 + b3, a3 = gelu(z3); y = a3 W4 + b4.

The loss is the mean over samples of the squared error summed over the 32
outputs; the optimiser is Adam.  `bf16=True` rounds every matrix-product
operand to bfloat16 (round to nearest even) the way the GPU kernels feed
their BF16 matrix cores, so that the two can be compared closely.
"""
from __future__ import annotations

import math

import numpy as np

DIMS = (16, 128, 128, 128, 32)
GELU_C = math.sqrt(2.0 / math.pi)
GELU_A = 0.044715


def features(x1, x2, theta, s):
    """Periodic feature map: harmonics 1, 2 of x1 and x2, of theta, and the scale."""
    x1 = np.asarray(x1, float)
    x2 = np.asarray(x2, float)
    th = np.broadcast_to(np.asarray(theta, float), x1.shape)
    sc = np.broadcast_to(np.asarray(s, float), x1.shape)
    t = 2.0 * math.pi
    cols = [np.sin(t * x1), np.cos(t * x1), np.sin(t * x2), np.cos(t * x2),
            np.sin(2 * t * x1), np.cos(2 * t * x1), np.sin(2 * t * x2), np.cos(2 * t * x2),
            np.cos(th), np.sin(th), np.cos(2 * th), np.sin(2 * th),
            sc - 1.0, (sc - 1.0) ** 2, np.ones_like(x1), np.zeros_like(x1)]
    return np.stack(cols, axis=-1)


def bf16(a):
    """Round float64/float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + GELU_A * z ** 3)))


def gelu_grad(z):
    t = np.tanh(GELU_C * (z + GELU_A * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * z * z)


def init_params(rng, dims=DIMS):
    """He-style normal initialisation, zero biases: [(W1, b1), ..., (W4, b4)]."""
    ps = []
    for i in range(len(dims) - 1):
        W = rng.standard_normal((dims[i], dims[i + 1])) * math.sqrt(2.0 / dims[i])
        ps.append((W, np.zeros(dims[i + 1])))
    return ps


def forward(params, f, bf16_ops=False):
    """Returns (y, cache) with cache = [(input, z), ...] per layer."""
    rnd = bf16 if bf16_ops else (lambda v: v)
    a = np.asarray(f, float)
    cache = []
    n = len(params)
    for i, (W, b) in enumerate(params):
        z = rnd(a) @ rnd(W) + b
        cache.append((a, z))
        a = gelu(z) if i < n - 1 else z
    return a, cache


def loss_and_grads(params, f, target, bf16_ops=False):
    """Mean squared error (sum over outputs, mean over samples) and its gradients."""
    rnd = bf16 if bf16_ops else (lambda v: v)
    y, cache = forward(params, f, bf16_ops)
    n = y.shape[0]
    diff = y - target
    loss = float(np.sum(diff * diff) / n)
    dz = 2.0 * diff / n
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        a_in, z = cache[i]
        W, _ = params[i]
        gW = rnd(a_in).T @ rnd(dz)
        gb = dz.sum(axis=0)
        grads[i] = (gW, gb)
        if i > 0:
            da = rnd(dz) @ rnd(W).T
            dz = da * gelu_grad(cache[i - 1][1])
    return loss, grads


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (state: dict with 't', 'm', 'v'); returns new params."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    if "m" not in state:
        state["m"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        state["v"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    out = []
    for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        (mW, mb), (vW, vb) = state["m"][i], state["v"][i]
        mW = b1 * mW + (1 - b1) * gW
        mb = b1 * mb + (1 - b1) * gb
        vW = b2 * vW + (1 - b2) * gW * gW
        vb = b2 * vb + (1 - b2) * gb * gb
        state["m"][i] = (mW, mb)
        state["v"][i] = (vW, vb)
        c1 = 1 - b1 ** t
        c2 = 1 - b2 ** t
        W = W - lr * (mW / c1) / (np.sqrt(vW / c2) + eps)
        b = b - lr * (mb / c1) / (np.sqrt(vb / c2) + eps)
        out.append((W, b))
    return out


def flatten(params):
    """Concatenate W1, b1, ..., W4, b4 (row-major) into one float64 vector."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflatten(vec, dims=DIMS):
    ps = []
    o = 0
    for i in range(len(dims) - 1):
        nW = dims[i] * dims[i + 1]
        W = np.asarray(vec[o:o + nW], float).reshape(dims[i], dims[i + 1])
        o += nW
        b = np.asarray(vec[o:o + dims[i + 1]], float)
        o += dims[i + 1]
        ps.append((W, b))
    return ps


def factor_targets(A_cols, V, s1):
    """Training targets of the network for one wedge: alpha*(x) = A(x, C) V / s1.

    A_cols: (n_x, r) residual-kernel columns at the wedge's sampled column set C,
    V: (r, 16) leading right singular vectors of the columns stacked over the
    training scales, s1: the leading singular value.  Returns (n_x, 32) reals
    (real and imaginary part interleaved per factor).
    """
    al = A_cols @ V / s1
    out = np.empty((al.shape[0], 2 * al.shape[1]))
    out[:, 0::2] = al.real
    out[:, 1::2] = al.imag
    return out
