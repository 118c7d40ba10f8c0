"""Pins of the FP64 network oracle: back-propagation against central finite
differences, and the BF16 rounding helper against exactly representable
cases (round to nearest, ties to even)."""
import numpy as np

from oracle import mlp_oracle as M


def test_bf16_rounding_ties_to_even():
    one = 1.0
    assert M.bf16_round(one) == 1.0
    assert M.bf16_round(1.0 + 2.0 ** -8) == 1.0                  # tie -> even mantissa
    assert M.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie -> even mantissa
    assert M.bf16_round(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7      # representable
    assert M.bf16_round(-3.0) == -3.0
    x = np.random.default_rng(1).normal(size=1000)
    assert np.all(np.abs(M.bf16_round(x) - x) <= np.abs(x) * 2.0 ** -8)


def test_backprop_matches_central_differences():
    shape = (5, 7, 2, 2)
    g = np.random.default_rng(2)
    L, din, dout = M.dims(*shape)
    n_par = sum(a * b for a, b in zip(din, dout)) + sum(dout)
    p = 0.5 * g.normal(size=n_par)
    X = g.uniform(-1, 1, size=(6, 5))
    Y = g.normal(size=(6, 2))
    loss, grad = M.loss_and_grads(p, X, Y, shape)
    h = 1e-6
    num = np.zeros(n_par)
    for k in range(n_par):
        e = np.zeros(n_par)
        e[k] = h
        num[k] = (M.loss_and_grads(p + e, X, Y, shape)[0] - M.loss_and_grads(p - e, X, Y, shape)[0]) / (2 * h)
    assert np.abs(num - grad).max() < 1e-6 * max(1.0, np.abs(grad).max())


def test_silu_derivative():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    assert np.abs((M.silu(z + h) - M.silu(z - h)) / (2 * h) - M.dsilu(z)).max() < 1e-8
