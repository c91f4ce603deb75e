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
