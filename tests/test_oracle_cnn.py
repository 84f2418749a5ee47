"""Pins of the warm-start network oracle (oracle/cnn.py): the convolution
against scipy's periodic 2-D correlation, the backward pass against central
finite differences, Adam against its closed first step, the parameter
count, and the bfloat16 rounding against hand-worked values."""
import numpy as np
import pytest
from scipy.signal import correlate2d

import ibgen
from oracle import cnn


def test_parameter_count():
    # 5->32, four 32->32, 32->3, 3x3 kernels with biases
    assert cnn.n_params() == (32 * 5 * 9 + 32) + 4 * (32 * 32 * 9 + 32) + (3 * 32 * 9 + 3) == 39331
    th = ibgen.cnn_init(3)
    assert th.shape == (39331,) and th.dtype == np.float32
    W6, b6 = cnn.unpack(th)[-1]
    assert not W6.any() and not b6.any()
    assert np.allclose(cnn.pack(cnn.unpack(th)), th)


def test_conv_matches_periodic_correlation():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((4, 9, 7))
    W = rng.standard_normal((3, 4, 3, 3))
    b = rng.standard_normal(3)
    z = cnn.conv3(a, W, b)
    for o in range(3):
        ref = b[o] + sum(correlate2d(a[c], W[o, c], mode="same", boundary="wrap") for c in range(4))
        assert np.allclose(z[o], ref, rtol=1e-13, atol=1e-13)


def test_conv_transpose_is_adjoint():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((4, 8, 8))
    g = rng.standard_normal((3, 8, 8))
    W = rng.standard_normal((3, 4, 3, 3))
    lhs = np.sum(cnn.conv3(a, W, np.zeros(3)) * g)
    rhs = np.sum(a * cnn.conv3_transpose(g, W))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    N = 6
    th = rng.standard_normal(cnn.n_params()) * 0.2
    x = rng.standard_normal((5, N, N))
    t = rng.standard_normal((3, N, N))
    L, g = cnn.loss_grad(th, x, t)
    # indices in every layer's weights and biases
    sizes = [co * ci * 9 + co for ci, co in cnn.LAYERS]
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    idx = []
    for s0, sz in zip(starts, sizes):
        idx += [s0 + 5, s0 + sz // 2, s0 + sz - 1]
    h = 1e-5
    for k in idx:
        e = np.zeros_like(th)
        e[k] = h
        fd = (cnn.loss_grad(th + e, x, t)[0] - cnn.loss_grad(th - e, x, t)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_relu_kills_gradient_of_dead_units():
    # a hidden layer with all-negative pre-activations passes no gradient
    rng = np.random.default_rng(4)
    th = rng.standard_normal(cnn.n_params()) * 0.1
    layers = cnn.unpack(th)
    W1, b1 = layers[0]
    layers[0] = (np.zeros_like(W1), -np.ones_like(b1))
    th2 = cnn.pack(layers)
    _, g = cnn.loss_grad(th2, rng.standard_normal((5, 5, 5)), rng.standard_normal((3, 5, 5)))
    assert not g[: 32 * 5 * 9 + 32].any()


def test_adam_first_step_closed_form():
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    t1, m, v = cnn.adam(th, np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    # bias-corrected moments equal g and g^2 after one step
    assert np.allclose(t1, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


@pytest.mark.parametrize("x,want", [
    (1.0, 1.0), (1.0 + 2 ** -8, 1.0), (1.0 + 3 * 2 ** -8, 1.0 + 2 ** -6),
    (1.0 + 2 ** -7, 1.0 + 2 ** -7), (-3.140625, -3.140625), (1e-3, 0.00099945068359375)])
def test_bf16_rounding(x, want):
    assert cnn.bf16(x) == want
