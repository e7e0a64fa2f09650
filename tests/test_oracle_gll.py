"""Pins for the oracle's GLL nodes and weights (Section 2: nodal bases on the
GLL points): textbook closed forms, numpy's Legendre roots and exactness of
the Lobatto quadrature."""
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "gll_closed_forms.txt")


def _closed_forms():
    rows = {}
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        n, x, w = (s.strip() for s in line.split(";"))
        ev = lambda s: eval(s, {"__builtins__": {}}, {"sqrt": math.sqrt})
        rows.setdefault(int(n), []).append((ev(x), ev(w)))
    return rows


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_closed_forms(N):
    z, w = oracle.gll(N)
    for x, wt in _closed_forms()[N]:
        for sgn in (1.0, -1.0):
            i = int(np.argmin(np.abs(z - sgn * x)))
            assert abs(z[i] - sgn * x) <= 2e-16, (N, x, z)
            assert abs(w[i] - wt) <= 4e-16, (N, wt, w)


@pytest.mark.parametrize("N", range(1, 16))
def test_against_numpy_legendre(N):
    z, w = oracle.gll(N)
    inner = np.sort(np.real(np.polynomial.legendre.Legendre.basis(N).deriv().roots()))
    ref = np.concatenate([[-1.0], inner, [1.0]])
    assert np.all(np.diff(z) > 0)
    assert np.max(np.abs(z - ref)) <= 1e-13
    assert np.array_equal(z, -z[::-1])
    assert abs(w.sum() - 2.0) <= 1e-14
    # endpoint weight 2 / (N (N + 1))
    assert abs(w[0] - 2.0 / (N * (N + 1))) <= 1e-15


@pytest.mark.parametrize("N", range(1, 16))
def test_quadrature_exact_to_degree_2N_minus_1(N):
    z, w = oracle.gll(N)
    for k in range(0, 2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, z ** k) - exact) <= 1e-14, (N, k)
    if N >= 1:
        # degree 2N is NOT integrated exactly: the rule really has order 2N-1
        k = 2 * N
        assert abs(np.dot(w, z ** k) - 2.0 / (k + 1)) > 1e-12


def test_out_of_range():
    with pytest.raises(ValueError):
        oracle.gll(0)
    with pytest.raises(ValueError):
        oracle.gll(16)
