"""Pins for the oracle's owner selection (Section 2.1: session-id exclusion
and the distance-to-boundary discriminator, Fig. 2) and for findpts_eval
(tensor-product Lagrange interpolation): a hand-computable three-session
case, exactness on per-element polynomials of degree <= N, nodal values."""
import numpy as np
import pytest
import torch

import oracle
import workloads as w


def _three_sessions():
    """Three one-element boxes of order 2 with linear distance fields:
    session 0: [0,3]x[0,1]^2, delta = 100; session 1: [0,2]x[0,1]^2,
    delta = 2 - x; session 2: [1,3]x[0,1]^2, delta = x - 1."""
    boxes = [((0, 0, 0), (3, 1, 1)), ((0, 0, 0), (2, 1, 1)), ((1, 0, 0), (3, 1, 1))]
    ms = [w.box_mesh(1, 1, 1, lo, hi, N=2) for lo, hi in boxes]
    x = torch.cat([m.x for m in ms]); y = torch.cat([m.y for m in ms])
    z = torch.cat([m.z for m in ms])
    delta = torch.cat([torch.full_like(ms[0].x, 100.0), 2.0 - ms[1].x, ms[2].x - 1.0])
    sess = torch.tensor([0, 1, 2], dtype=torch.int32)
    return w.Mesh("three", 2, x, y, z, sess, delta)


def test_distance_discriminator_three_sessions():
    m = _three_sessions()
    om = oracle.OracleMesh.from_mesh(m)
    xs = np.array([0.5, 1.2, 1.4, 1.5, 1.6, 1.9, 2.5])
    pts = np.stack([xs, np.full_like(xs, 0.3), np.full_like(xs, 0.7)], 1)
    # tag 0: session 0 excluded; in the overlap [1, 2] the larger of
    # 2 - x (session 1) and x - 1 (session 2) wins, x = 1.5 ties -> session 1
    code, el, _, _ = om.findpts(pts, np.zeros(len(xs), np.int32))
    assert np.all(code == 0)
    assert list(el) == [1, 1, 1, 1, 2, 2, 2]
    # tag 1: only session 0 and 2 eligible; session 0's delta = 100 wins
    code, el, _, _ = om.findpts(pts, np.ones(len(xs), np.int32))
    assert list(el) == [0] * len(xs)
    # no exclusion (tag -1): session 0 wins everywhere
    code, el, _, _ = om.findpts(pts, np.full(len(xs), -1, np.int32))
    assert list(el) == [0] * len(xs)


def test_session_exclusion_without_delta():
    m = _three_sessions()
    m.delta = None
    om = oracle.OracleMesh.from_mesh(m)
    pts = np.array([[1.5, 0.5, 0.5], [0.5, 0.5, 0.5], [2.5, 0.5, 0.5]])
    code, el, _, _ = om.findpts(pts, np.array([0, 0, 0], np.int32))
    # smallest INSIDE element id among non-excluded sessions
    assert list(code) == [0, 0, 0] and list(el) == [1, 1, 2]
    code, el, _, _ = om.findpts(pts, np.array([1, 1, 1], np.int32))
    assert list(el) == [0, 0, 0]
    code, el, _, _ = om.findpts(pts, np.array([0, 2, 1], np.int32))
    assert list(el) == [1, 0, 0]


def _mono(coef, r):
    a = np.arange(coef.shape[-1])
    pr, ps, pt = r[0] ** a, r[1] ** a, r[2] ** a
    return np.einsum("cba,c,b,a->", coef, pt, ps, pr)


@pytest.mark.parametrize("case", ["polymap", "annulus", "c1"])
def test_eval_exact_on_reference_polynomials(case):
    if case == "polymap":
        m, _ = w.poly_map_mesh(2, 2, 2, N=4)
    elif case == "annulus":
        m = w.annulus_mesh(2, 4, 2, N=7)
    else:
        m = w.cube_c1()
    fields, coef = w.ref_poly_fields(m, 2, seed=5)
    om = oracle.OracleMesh.from_mesh(m)
    rng = np.random.default_rng(5)
    P = 300
    el = rng.integers(0, m.E, P).astype(np.int32)
    rst = rng.uniform(-1, 1, (P, 3))
    code = np.zeros(P, np.int32)
    code[::50] = 2
    out = om.eval(code, el, rst, [f.numpy() for f in fields])
    for f in range(2):
        for p in range(P):
            if code[p] == 2:
                assert np.isnan(out[f, p])
                continue
            ref = _mono(coef[f, el[p]], rst[p])
            scale = np.abs(coef[f, el[p]]).sum()
            assert abs(out[f, p] - ref) <= 1e-14 * scale


def test_eval_at_nodes_returns_nodal_values():
    m = w.annulus_mesh(2, 4, 2, N=5)
    fields, _ = w.ref_poly_fields(m, 1, seed=6)
    F = fields[0].numpy()
    om = oracle.OracleMesh.from_mesh(m)
    z, _ = oracle.gll(5)
    rng = np.random.default_rng(6)
    el = rng.integers(0, m.E, 100).astype(np.int32)
    ijk = rng.integers(0, 6, (100, 3))
    rst = z[ijk]
    out = om.eval(np.zeros(100, np.int32), el, rst, [F])
    ref = F[el, ijk[:, 2], ijk[:, 1], ijk[:, 0]]
    assert np.array_equal(out[0], ref)
