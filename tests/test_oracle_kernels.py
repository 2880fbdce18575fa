"""Pins of the oracle's kernel functions (matrix entries of eq. (2)).

The Matern kernel of Section 6.2 with beta - d/2 = 1 needs s K_1(s); the
oracle's series / trapezoidal evaluation is checked against scipy's K_1
(a library routine) and mpmath at 40 digits, on both sides of the switch at
s = 2, down to the underflow of e^-s and up to s -> 0, and the kernel's
value at r = 0 against the closed form 1 / (2^(d/2) Gamma(1 + d/2))."""
import math

import numpy as np
import pytest
from scipy.special import k1

import oracle


S_GRID = np.concatenate([10.0 ** np.arange(-300, 0, 7.0), np.linspace(0.01, 2.0, 57),
                         [np.nextafter(2.0, 0), 2.0, np.nextafter(2.0, 3)],
                         np.linspace(2.0, 40.0, 77), [60.0, 100.0, 300.0, 650.0, 700.0]])


def test_xk1_against_scipy():
    worst = 0.0
    for s in S_GRID:
        ref = s * k1(s)
        got = oracle.xk1(s)
        rel = abs(got - ref) / ref
        worst = max(worst, rel)
        assert rel <= 4e-15, (s, got, ref, rel)
    print("worst relative deviation from scipy.special.k1: %.2e" % worst)
    assert oracle.xk1(0.0) == 1.0


def test_xk1_against_mpmath():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    for s in [1e-12, 1e-3, 0.3, 1.0, 1.999, 2.001, 3.7, 11.0, 55.0, 400.0]:
        ref = float(mpmath.mpf(s) * mpmath.besselk(1, s))
        assert abs(oracle.xk1(s) - ref) <= 3e-15 * ref, s


@pytest.mark.parametrize("d", [1, 2, 3])
def test_matern_nu1_kernel(d):
    beta = 1.0 + d / 2.0
    norm = 2.0 ** (beta - 1.0) * math.gamma(beta)
    closed = {1: math.sqrt(2.0 / math.pi), 2: 0.5, 3: 1.0 / (1.5 * math.sqrt(2.0 * math.pi))}
    x = np.array([0.3, -0.2, 0.7][:d])
    assert abs(oracle.kernel("matern_nu1", 0.4, x, x) - closed[d]) <= 1e-15
    g = np.random.default_rng(5 + d)
    for _ in range(50):
        y = g.random(d) * 3.0
        ell = 10.0 ** g.uniform(-2, 1)
        r = float(np.sqrt(((x - y) ** 2).sum()))
        ref = (r / ell) * k1(r / ell) / norm
        got = oracle.kernel("matern_nu1", ell, x, y)
        assert abs(got - ref) <= 5e-15 * ref + 1e-300, (r, ell, got, ref)
        assert got == oracle.kernel("matern_nu1", ell, y, x)  # symmetric
