"""Pins of the proposal-network oracle: finite differences in binary64,
the Gaussian NLL's closed-form minimiser, and Adam's first step."""
import math

import numpy as np
import pytest

import synth.mlp_init as mi
from oracle import mlp


def _small(seed=0, din=20, h=8):
    p = {k: v.astype(np.float64) for k, v in mi.init_params(seed, din, h, 12).items()}
    rng = np.random.default_rng(seed + 1)
    p["W3"] = rng.standard_normal(p["W3"].shape) * 0.3
    p["b1"] = rng.standard_normal(h) * 0.1
    X = rng.standard_normal((5, din))
    Y = rng.standard_normal((5, 6)) * 0.2
    return p, X, Y


def test_gradients_match_central_differences():
    p, X, Y = _small()
    _, g = mlp.loss_and_grads(p, X, Y)
    rng = np.random.default_rng(7)
    for k in mlp.NAMES:
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in p[k].shape)
            h = 1e-6
            old = p[k][idx]
            p[k][idx] = old + h
            lp, _ = mlp.loss_and_grads(p, X, Y)
            p[k][idx] = old - h
            lm, _ = mlp.loss_and_grads(p, X, Y)
            p[k][idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, g[k][idx])


def test_gelu_closed_forms():
    z = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    phi = 0.5 * (1 + np.array([math.erf(v / math.sqrt(2)) for v in z]))
    assert np.allclose(mlp.gelu(z), z * phi, rtol=0, atol=1e-15)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5)


def test_nll_minimiser_is_the_sample_statistics():
    """For a constant prediction, the NLL is minimised at mu = mean(y) and
    exp(2 l) = mean((y - mu)^2): the gradient vanishes there."""
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((400, 6)) * np.array([0.1, 0.2, 0.3, 0.05, 0.5, 1.0]) + 0.2
    mu = Y.mean(0)
    var = ((Y - mu) ** 2).mean(0)
    out = np.tile(np.concatenate([mu, 0.5 * np.log(var)]), (400, 1))
    _, d = mlp.loss_and_dout(out, Y)
    assert np.abs(d.sum(0)).max() < 1e-12


def test_adam_first_step_is_signed_lr():
    p = {k: np.ones(2) for k in mlp.NAMES}
    g = {k: np.array([0.3, -2.0]) for k in mlp.NAMES}
    m = {k: np.zeros(2) for k in mlp.NAMES}
    v = {k: np.zeros(2) for k in mlp.NAMES}
    mlp.adam_step(p, g, m, v, 1, lr=0.01, eps=0.0)
    for k in mlp.NAMES:
        assert np.allclose(p[k], [0.99, 1.01], atol=1e-15)


def test_bf16_rounding_pins():
    """Round to nearest, ties to even, on the upper 16 bits of binary32:
    1 + 2^-8 (a tie) goes down to 1, 1 + 3 * 2^-8 (a tie) up to 1 + 2^-6,
    1 + 2^-8 + 2^-20 up to 1 + 2^-7; bfloat16 values are kept; the relative
    error is at most half a unit in the 8th bit, 2^-8."""
    v = np.array([1 + 2.0**-8, 1 + 3 * 2.0**-8, 1 + 2.0**-8 + 2.0**-20, -(1 + 2.0**-8), 0.0, 3.5])
    r = mlp.bf16_round(v)
    assert list(r) == [1.0, 1 + 2.0**-6, 1 + 2.0**-7, -1.0, 0.0, 3.5]
    rng = np.random.default_rng(3)
    x = rng.standard_normal(10000) * 10.0 ** rng.uniform(-6, 6, 10000)
    rx = mlp.bf16_round(x)
    x32 = x.astype(np.float32).astype(np.float64)
    assert np.all(np.abs(rx - x32) <= np.abs(x32) * 2.0**-8)
    assert np.array_equal(mlp.bf16_round(rx), rx)


def test_bf16_products_of_bf16_values_are_exact():
    """Operands already in bfloat16 (small integers times powers of two)
    give the same products in both modes; other operands do not."""
    rng = np.random.default_rng(4)
    A = rng.integers(-64, 64, (7, 33)) * 2.0**-5
    B = rng.integers(-64, 64, (33, 5)) * 2.0**-3
    assert np.array_equal(mlp.mm(A, B, bf16=True), A @ B)
    C = rng.standard_normal((7, 33))
    assert not np.array_equal(mlp.mm(C, B, bf16=True), C @ B)
