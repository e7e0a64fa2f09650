"""Pins of the interface-data oracle (flux correction, time extrapolation)
against closed forms: GLL surface quadrature of a box is exact for the
polynomial fields used, so the fluxes are known exactly."""
import numpy as np
import pytest

from helpers import box_surface as _box_surface
from oracle.interface import extrapolate, flux_correct


def test_flux_of_divergence_free_field_is_zero():
    x, w, n = _box_surface((0, 0, 0), (1, 2, 3))
    u = np.stack([x[1] ** 2, x[2] * x[0], np.ones_like(x[0])])  # div = 0
    g, out = flux_correct(w, n, np.ones(w.size, bool), u)
    assert abs(g) <= 1e-14
    assert np.max(np.abs(out - u)) <= 1e-14


def test_gamma_closed_form_all_interface():
    # u = (x, 0, 0): boundary flux = volume = 6, area = 2 (1*2 + 1*3 + 2*3) = 22
    x, w, n = _box_surface((0, 0, 0), (1, 2, 3))
    u = np.stack([x[0], np.zeros_like(x[0]), np.zeros_like(x[0])])
    g, out = flux_correct(w, n, np.ones(w.size, bool), u)
    assert abs(g - (-6.0 / 22.0)) <= 1e-14
    flux = np.sum(w * np.sum(out * n, axis=0))
    assert abs(flux) <= 1e-13


def test_gamma_closed_form_partial_interface():
    # only the face x = 1 is interpolated (area 6): gamma = -6 / 6 = -1 and
    # only that face's values change
    x, w, n = _box_surface((0, 0, 0), (1, 2, 3))
    u = np.stack([x[0], np.zeros_like(x[0]), np.zeros_like(x[0])])
    iface = (n[0] > 0.5)
    g, out = flux_correct(w, n, iface, u)
    assert abs(g + 1.0) <= 1e-14
    assert np.array_equal(out[:, ~iface], u[:, ~iface])
    assert abs(np.sum(w * np.sum(out * n, axis=0))) <= 1e-13


def test_no_interface_leaves_data():
    x, w, n = _box_surface((0, 0, 0), (1, 1, 1))
    u = np.stack([x[0], x[1], x[2]])
    g, out = flux_correct(w, n, np.zeros(w.size, bool), u)
    assert g == 0.0 and np.array_equal(out, u)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_extrapolation_exact_for_degree_below_order(m):
    rng = np.random.default_rng(m)
    c = rng.standard_normal((m, 50))  # per-point polynomial in time, degree m-1
    def val(t):
        return sum(c[d] * t ** d for d in range(m))
    hist = [val(1.0 - q) for q in range(m)]  # t = 1, 0, -1, ...
    assert np.max(np.abs(extrapolate(hist, m) - val(2.0))) <= 1e-12
    if m > 1:  # and not for degree m
        bad = [val(1.0 - q) + (1.0 - q) ** m for q in range(m)]
        assert np.max(np.abs(extrapolate(bad, m) - (val(2.0) + 2.0 ** m))) > 0.5
