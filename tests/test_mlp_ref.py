"""CPU pins of the network reference: sizes, the GELU derivative and the full
parameter gradient against central finite differences."""
import math

import numpy as np

from oracle import mlp_oracle as R


def test_parameter_count():
    assert R.NPARAMS == 18817


def test_gelu_values_and_derivative():
    z = np.linspace(-4, 4, 41)
    # Phi(z) z with Phi the normal CDF; GELU(0) = 0, GELU(z) -> z for large z
    assert abs(R.gelu(np.array([0.0]))[0]) == 0.0
    assert abs(R.gelu(np.array([6.0]))[0] - 6.0) < 1e-7
    h = 1e-6
    fd = (R.gelu(z + h) - R.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(R.gelu_grad(z), fd, atol=1e-8)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = R.init(1) + 0.05 * rng.standard_normal(R.NPARAMS)
    X = rng.standard_normal((7, R.NIN))
    t = rng.standard_normal(7)
    g = R.grad(p, X, t)
    idx = np.concatenate([rng.choice(R.NPARAMS, 60, replace=False), [R.NPARAMS - 1, 0, 2048]])
    h = 1e-6
    for i in idx:
        e = np.zeros(R.NPARAMS)
        e[i] = h
        fd = (R.loss(p + e, X, t) - R.loss(p - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_moves_by_lr():
    p = np.zeros(3)
    g = np.array([1.0, -2.0, 0.5])
    p1, m, v = R.adam(p, np.zeros(3), np.zeros(3), g, 1, 1e-3)
    # bias-corrected first step is lr * sign(g) (up to eps)
    np.testing.assert_allclose(p1, -1e-3 * np.sign(g), rtol=1e-6)
