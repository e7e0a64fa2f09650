"""Pins for the oracle's isoparametric map and Jacobian (Section 2): affine
closed form, an analytic polynomial map reproduced exactly, and central
finite differences on the curved annulus."""
import numpy as np

import oracle
import workloads as w
from helpers import box_affine, box_elem_ids, dphi_np, phi_np


def test_affine_closed_form():
    n, lo, hi = (3, 2, 2), (-1.0, 0.5, 2.0), (2.0, 1.5, 2.6)
    m = w.box_mesh(*n, lo=lo, hi=hi, N=4)
    om = oracle.OracleMesh.from_mesh(m)
    ex, ey, ez = box_elem_ids(m.E, n)
    rng = np.random.default_rng(0)
    for e in range(m.E):
        r = rng.uniform(-1, 1, 3)
        x, J = om.map(e, r)
        ref = box_affine(ex[e], ey[e], ez[e], n, lo, hi, r)
        assert np.max(np.abs(x - ref)) <= 1e-14
        dj = (np.asarray(hi) - np.asarray(lo)) / np.asarray(n) / 2.0
        assert np.max(np.abs(J - np.diag(dj))) <= 1e-13


def test_polynomial_map_exact():
    n = (2, 2, 2)
    m, _ = w.poly_map_mesh(*n, N=3)
    om = oracle.OracleMesh.from_mesh(m)
    ex, ey, ez = box_elem_ids(m.E, n)
    rng = np.random.default_rng(1)
    for e in range(m.E):
        for _ in range(4):
            r = rng.uniform(-1, 1, 3)
            a = box_affine(ex[e], ey[e], ez[e], n, (0, 0, 0), (1, 1, 1), r)
            ref = np.array(phi_np(*a))
            x, J = om.map(e, r)
            assert np.max(np.abs(x - ref)) <= 1e-14
            Jref = dphi_np(*a) @ np.diag(np.full(3, 0.5 / 2.0))
            assert np.max(np.abs(J - Jref)) <= 1e-13


def test_curved_jacobian_finite_differences():
    m = w.annulus_mesh(2, 8, 2, N=5)
    om = oracle.OracleMesh.from_mesh(m)
    rng = np.random.default_rng(2)
    eps = 1e-6
    for e in rng.integers(0, m.E, 6):
        r = rng.uniform(-0.9, 0.9, 3)
        _, J = om.map(e, r)
        for d in range(3):
            rp, rm = r.copy(), r.copy()
            rp[d] += eps
            rm[d] -= eps
            fd = (om.map(e, rp)[0] - om.map(e, rm)[0]) / (2 * eps)
            assert np.max(np.abs(fd - J[:, d])) <= 1e-8


def test_annulus_map_close_to_circle():
    """The degree-5 interpolant of a 45-degree arc is within ~1e-7 of it."""
    m = w.annulus_mesh(2, 8, 2, N=5)
    om = oracle.OracleMesh.from_mesh(m)
    rng = np.random.default_rng(3)
    for e in range(m.E):
        r = rng.uniform(-1, 1, 3)
        x, _ = om.map(e, r)
        er, et, ez = e % 2, (e // 2) % 8, e // 16
        rho = 0.5 + 0.5 * (er + (r[0] + 1) / 2) / 2
        assert abs(np.hypot(x[0], x[1]) - rho) <= 1e-6
