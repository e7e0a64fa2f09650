"""Pins for the oracle's Lagrange basis on GLL nodes and the Bernstein
transform used for element boxes: Kronecker property, partition of unity,
exact reproduction and differentiation of polynomials of degree <= N, and
the Bernstein form's endpoint/linear-precision identities."""
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9, 15])
def test_kronecker_at_nodes(N):
    z, _ = oracle.gll(N)
    for m in range(N + 1):
        h, _ = oracle.lagrange(N, z[m])
        ref = np.zeros(N + 1)
        ref[m] = 1.0
        assert np.array_equal(h, ref)


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9, 15])
def test_partition_of_unity(N):
    rng = np.random.default_rng(N)
    for r in rng.uniform(-1, 1, 20):
        h, dh = oracle.lagrange(N, r)
        assert abs(h.sum() - 1.0) <= 1e-13
        assert abs(dh.sum()) <= 1e-11 * max(1.0, np.abs(dh).max())


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7, 9])
def test_polynomial_reproduction(N):
    """sum_i p(z_i) h_i(r) = p(r) and sum_i p(z_i) h_i'(r) = p'(r) for deg p <= N."""
    rng = np.random.default_rng(100 + N)
    z, _ = oracle.gll(N)
    for _ in range(5):
        c = rng.uniform(-1, 1, N + 1)          # p(x) = sum c_a x^a
        p = np.polynomial.Polynomial(c)
        dp = p.deriv()
        for r in rng.uniform(-1, 1, 10):
            h, dh = oracle.lagrange(N, r)
            assert abs(np.dot(p(z), h) - p(r)) <= 1e-13 * max(1, np.abs(c).sum())
            assert abs(np.dot(p(z), dh) - dp(r)) <= 1e-11 * max(1, np.abs(c).sum())


def test_degree_N_plus_1_is_not_reproduced():
    N = 4
    z, _ = oracle.gll(N)
    h, _ = oracle.lagrange(N, 0.3)
    assert abs(np.dot(z ** (N + 1), h) - 0.3 ** (N + 1)) > 1e-6


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9])
def test_bernstein_inverse(N):
    """Binv maps nodal values to Bernstein coefficients on [-1, 1]."""
    z, _ = oracle.gll(N)
    Binv = oracle.bernstein_inverse(N)
    B = np.array([[math.comb(N, k) * ((1 + x) / 2) ** k * ((1 - x) / 2) ** (N - k)
                   for k in range(N + 1)] for x in z])
    assert np.max(np.abs(B @ Binv - np.eye(N + 1))) <= 1e-12
    # constant -> all coefficients 1; x -> coefficients -1 + 2k/N
    assert np.max(np.abs(Binv @ np.ones(N + 1) - 1.0)) <= 1e-12
    assert np.max(np.abs(Binv @ z - (-1.0 + 2.0 * np.arange(N + 1) / N))) <= 1e-12
    # endpoint interpolation: first/last coefficient equal the end values
    v = np.random.default_rng(N).uniform(-1, 1, N + 1)
    c = Binv @ v
    assert abs(c[0] - v[0]) <= 1e-12 and abs(c[-1] - v[-1]) <= 1e-12
