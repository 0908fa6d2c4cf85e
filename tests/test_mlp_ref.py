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


def _bf16_by_enumeration(x32):
    """Nearest BF16 value of a binary32 number by exact rational comparison of
    the two BF16 neighbours (ties to the even mantissa), from the format's
    definition: BF16 is binary32 with the low 16 mantissa bits zero."""
    from fractions import Fraction
    import struct
    bits = struct.unpack("<I", struct.pack("<f", float(x32)))[0]
    lo_bits = bits & 0xFFFF0000
    hi_bits = lo_bits + 0x10000
    f = lambda b: struct.unpack("<f", struct.pack("<I", b & 0xFFFFFFFF))[0]
    x = Fraction(float(x32))
    a, b = Fraction(f(lo_bits)), Fraction(f(hi_bits))
    da, db = abs(x - a), abs(b - x)
    if da < db:
        return float(a)
    if db < da:
        return float(b)
    return float(a) if ((lo_bits >> 16) & 1) == 0 else float(b)


def test_bf16_rounding_follows_the_format():
    # hand cases: spacing 2^-7 at 1, ties to even, carry into the exponent
    cases = {1.0: 1.0, 1.0 + 2 ** -8: 1.0, 1.0 + 3 * 2 ** -8: 1.0 + 2 ** -6,
             1.0 + 2 ** -8 + 2 ** -20: 1.0 + 2 ** -7, -3.140625: -3.140625, 65504.0: 65536.0,
             2.0 - 2 ** -9: 2.0, 0.0: 0.0}
    for x, want in cases.items():
        assert R.to_bf16(np.array([x]))[0] == want, x
    rng = np.random.default_rng(7)
    xs = np.concatenate([rng.standard_normal(400) * 10.0 ** rng.integers(-6, 6, 400),
                         np.float32(1.0) + np.arange(-64, 64) * np.float32(2.0 ** -12)])
    xs = xs.astype(np.float32)
    got = R.to_bf16(xs)
    for x, g in zip(xs, got):
        assert g == _bf16_by_enumeration(x), x


def test_bf16_forward_within_its_rounding_bound():
    """forward_bf16 against the exact forward: each BF16 rounding is within
    2^-9 relative, so the output stays within a bound built from the layer
    magnitudes; with operands already representable and a linear path the two
    agree except for the hidden roundings."""
    rng = np.random.default_rng(3)
    p = R.init(4) + 0.02 * rng.standard_normal(R.NPARAMS)
    X = rng.standard_normal((50, R.NIN))
    y, (Z1, A1, Z2, A2) = R.forward(p, X)
    yb, (A1b, A2b) = R.forward_bf16(p, X)
    q = R.unpack(p)
    u = 2.0 ** -8  # two roundings' worth of relative error per operand
    bound1 = u * (np.abs(X) @ np.abs(q["W1"]).T) * 1.2  # |dZ1|, GELU' <= 1.13
    dA1 = u * np.abs(A1) + bound1
    dA2 = u * np.abs(A2) + 1.2 * (dA1 @ np.abs(q["W2"]).T + u * np.abs(A1) @ np.abs(q["W2"]).T)
    bound = dA2 @ np.abs(q["w3"]) + u * np.abs(A2) @ np.abs(q["w3"])
    assert np.all(np.abs(yb - y) <= bound)
    assert np.max(np.abs(yb - y)) > 0.0
    np.testing.assert_array_equal(R.to_bf16(A1b), A1b)  # hidden values are BF16
