"""Pins of the network oracle (oracle/mlp.py): finite differences, GELU closed
form, bfloat16 rounding rule, Adam on a quadratic."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_tanh_form_matches_definition_and_erf_gelu():
    z = np.linspace(-6, 6, 1001)
    ref = 0.5 * z * (1 + np.tanh(math.sqrt(2 / math.pi) * (z + 0.044715 * z ** 3)))
    np.testing.assert_allclose(mlp.gelu(z), ref, rtol=0, atol=1e-15)
    erf_gelu = 0.5 * z * (1 + np.array([math.erf(v / math.sqrt(2)) for v in z]))
    assert np.max(np.abs(mlp.gelu(z) - erf_gelu)) < 5e-4   # the tanh form approximates the erf form
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, atol=1e-8)


def test_bf16_rounding_rule():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -3.14159, 1e-20, 65504.0])
    out = mlp.bf16(vals)
    assert out[0] == 1.0
    assert out[1] == 1.0                  # tie -> even (1.0)
    assert out[2] == 1.0 + 2 ** -7        # representable
    assert out[3] == 1.0 + 2 ** -6        # tie -> even mantissa
    assert abs(out[4] - (-3.140625)) < 1e-12
    rel = np.abs(mlp.bf16(np.linspace(0.1, 100, 1000)) / np.linspace(0.1, 100, 1000) - 1)
    assert rel.max() <= 2 ** -8          # half an ulp of an 8-bit significand


def test_gradients_against_central_differences():
    rng = np.random.default_rng(0)
    dims = (16, 8, 8, 8, 6)
    params = mlp.init_params(rng, dims)
    f = rng.standard_normal((20, 16))
    target = rng.standard_normal((20, 6))
    loss, grads = mlp.loss_and_grads(params, f, target)
    vec = mlp.flatten(params)
    gvec = mlp.flatten(grads)
    idx = rng.choice(vec.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        vp = vec.copy()
        vp[i] += h
        vm = vec.copy()
        vm[i] -= h
        lp, _ = mlp.loss_and_grads(mlp.unflatten(vp, dims), f, target)
        lm, _ = mlp.loss_and_grads(mlp.unflatten(vm, dims), f, target)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gvec[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gvec[i])


def test_adam_minimises_a_quadratic():
    rng = np.random.default_rng(1)
    dims = (16, 4, 4, 4, 2)
    params = mlp.init_params(rng, dims)
    f = rng.standard_normal((64, 16))
    target = f[:, :2] * 0.3
    state = {}
    l0, _ = mlp.loss_and_grads(params, f, target)
    for _ in range(400):
        _, g = mlp.loss_and_grads(params, f, target)
        params = mlp.adam_step(params, g, state, 1e-2)
    l1, _ = mlp.loss_and_grads(params, f, target)
    assert l1 < 0.05 * l0


def test_feature_map_is_periodic():
    rng = np.random.default_rng(2)
    x1, x2 = rng.random(50), rng.random(50)
    a = mlp.features(x1, x2, 0.3, 1.2)
    b = mlp.features(x1 + 1, x2 - 2, 0.3 + 2 * math.pi, 1.2)
    np.testing.assert_allclose(a, b, atol=1e-12)
    assert a.shape == (50, 16)


def test_adam_first_step_and_constant_gradient_closed_forms():
    """Bias-corrected Adam: with a constant gradient g every step moves each
    parameter by exactly lr * g / (|g| + eps), whatever the scale of g, since
    the corrected moments are then g and g^2 at every t."""
    rng = np.random.default_rng(3)
    dims = (4, 3, 3, 3, 2)
    params = mlp.init_params(rng, dims)
    g = mlp.init_params(rng, dims)
    g = [(gW * 10.0 ** rng.integers(-3, 3), gb + 0.5) for gW, gb in g]
    state = {}
    lr, eps = 1e-2, 1e-8
    cur = params
    for t in range(1, 6):
        nxt = mlp.adam_step(cur, g, state, lr, eps=eps)
        for (W0, b0), (W1, b1), (gW, gb) in zip(cur, nxt, g):
            np.testing.assert_allclose(W0 - W1, lr * gW / (np.abs(gW) + eps), rtol=1e-9, atol=1e-15)
            np.testing.assert_allclose(b0 - b1, lr * gb / (np.abs(gb) + eps), rtol=1e-9, atol=1e-15)
        cur = nxt
    assert state["t"] == 5


def test_adam_second_step_by_hand():
    """Two scalar steps worked out by hand: g1 = 1, g2 = -3, b1 = 0.9, b2 = 0.999.
    t = 1: m = 0.1, v = 0.001, corrected 1 and 1 -> step lr.
    t = 2: m = 0.09 - 0.3 = -0.21, v = 0.000999 + 0.009 = 0.009999;
           corrected m = -0.21/0.19, v = 0.009999/0.001999 -> step lr (-0.21/0.19)/sqrt(0.009999/0.001999)."""
    p = [(np.array([[2.0]]), np.array([0.0]))]
    state = {}
    lr = 0.1
    p1 = mlp.adam_step(p, [(np.array([[1.0]]), np.array([1.0]))], state, lr, eps=0.0)
    assert abs(p1[0][0][0, 0] - (2.0 - lr)) < 1e-15
    p2 = mlp.adam_step(p1, [(np.array([[-3.0]]), np.array([-3.0]))], state, lr, eps=0.0)
    step = lr * (-0.21 / 0.19) / math.sqrt(0.009999 / 0.001999)
    assert abs(p2[0][0][0, 0] - (2.0 - lr - step)) < 1e-14
    assert abs(p2[0][1][0] - (0.0 - lr - step)) < 1e-14


def test_factor_targets_equal_left_singular_vectors_times_singular_values():
    """alpha* = A(:, C) V / s1 is U S / s1 of the SVD A(:, C) = U S V^H: the
    columns are orthogonal, the first has unit norm, and their norms are the
    singular values over s1 (an independent construction through numpy's SVD)."""
    rng = np.random.default_rng(4)
    n, r = 300, 24
    A = rng.standard_normal((n, 5)) @ rng.standard_normal((5, r)) + 1j * rng.standard_normal((n, r)) * 0.1
    U, S, Vh = np.linalg.svd(A, full_matrices=False)
    V = Vh.conj().T[:, :16]
    out = mlp.factor_targets(A, V, S[0])
    al = out[:, 0::2] + 1j * out[:, 1::2]
    np.testing.assert_allclose(al, U[:, :16] * (S[:16] / S[0]), atol=1e-12)
    G = al.conj().T @ al
    np.testing.assert_allclose(np.abs(G - np.diag(np.diag(G))), 0, atol=1e-12)
    assert abs(np.linalg.norm(al[:, 0]) - 1.0) < 1e-12
    # interleaving: real part at even columns, imaginary part at odd ones
    assert np.array_equal(out[:, 0], al[:, 0].real) and np.array_equal(out[:, 1], al[:, 0].imag)
