"""Pins for the oracle's point location (Section 2.1: hash, boxes, Newton
from the closest mapped GLL node, inside / border / not-found):
exact recovery of points generated as x^e(r_true) through an analytic
polynomial map, the affine closed form (inside and border), the unit cube,
and brute force over all elements with many Newton starts."""
import numpy as np
import pytest

import oracle
import workloads as w
from helpers import box_affine, box_elem_ids, phi_np, spiral_exact_points


def _residual(om, e, r, p):
    x, _ = om.map(e, r)
    return float(np.linalg.norm(x - p))


def test_exact_recovery_polynomial_map():
    n, N = (3, 3, 3), 4
    m, _ = w.poly_map_mesh(*n, N=N, amp=0.04)
    om = oracle.OracleMesh.from_mesh(m)
    _, h = om.bbox()
    ex, ey, ez = box_elem_ids(m.E, n)
    rng = np.random.default_rng(11)
    P = 600
    et = rng.integers(0, m.E, P)
    rt = rng.uniform(-1, 1, (P, 3))
    a = np.array([box_affine(ex[e], ey[e], ez[e], n, (0, 0, 0), (1, 1, 1), r)
                  for e, r in zip(et, rt)])
    pts = np.stack(phi_np(a[:, 0], a[:, 1], a[:, 2], amp=0.04), 1)
    code, el, rst, d2 = om.findpts(pts)
    assert np.all(code == 0)
    for i in range(P):
        assert np.sqrt(d2[i]) <= 1e-12 * h[el[i]]
        assert _residual(om, el[i], rst[i], pts[i]) <= 1e-12 * h[el[i]]
        if el[i] == et[i]:
            assert np.max(np.abs(rst[i] - rt[i])) <= 1e-11
        else:  # only a face neighbour may claim a point on their shared face
            assert np.min(1 - np.abs(rt[i])) <= 1e-10, (i, rt[i], el[i], et[i])


def test_affine_closed_form_inside_and_border():
    n, lo, hi = (3, 2, 2), np.array([-1.0, 0.5, 2.0]), np.array([2.0, 1.5, 2.6])
    m = w.box_mesh(*n, lo=tuple(lo), hi=tuple(hi), N=3)
    om = oracle.OracleMesh.from_mesh(m)
    _, h = om.bbox()
    rng = np.random.default_rng(12)
    # inside: r = 2 (x - x0) / dx - 1 in the owning element
    pts = lo + (hi - lo) * rng.uniform(0.001, 0.999, (500, 3))
    code, el, rst, d2 = om.findpts(pts)
    assert np.all(code == 0)
    dx = (hi - lo) / np.asarray(n)
    idx = np.floor((pts - lo) / dx).astype(int)
    e_ref = idx[:, 0] + n[0] * (idx[:, 1] + n[1] * idx[:, 2])
    x0 = lo + idx * dx
    r_ref = 2 * (pts - x0) / dx - 1
    interior = np.min(1 - np.abs(r_ref), axis=1) > 1e-9
    assert np.array_equal(el[interior], e_ref[interior])
    assert np.max(np.abs(rst[interior] - r_ref[interior])) <= 1e-12
    # border: points outside a face / edge / corner by 3e-10 h (inside the
    # box margin, beyond the tolerance): closest point is the clamp onto the
    # domain, r has the clamped coordinates at exactly +-1
    hmin = float(h.min())
    outs, refs = [], []
    for _ in range(300):
        q = lo + (hi - lo) * rng.uniform(0.01, 0.99, 3)
        k = rng.integers(1, 4)
        axes = rng.choice(3, k, replace=False)
        for a in axes:
            side = rng.integers(0, 2)
            q[a] = (hi[a] + 3e-10 * hmin) if side else (lo[a] - 3e-10 * hmin)
        outs.append(q)
        refs.append(np.clip(q, lo, hi))
    outs, refs = np.array(outs), np.array(refs)
    code, el, rst, d2 = om.findpts(outs)
    assert np.all(code == 1)
    dref = np.sum((outs - refs) ** 2, axis=1)
    assert np.max(np.abs(d2 - dref) / dref) <= 1e-4
    for i in range(len(outs)):
        x, _ = om.map(el[i], rst[i])
        assert np.max(np.abs(x - refs[i])) <= 1e-14
    # far outside: not found
    far = np.array([[10.0, 1.0, 2.3], [0.0, -3.0, 2.3], [np.nan, 1.0, 2.3]])
    code, el, rst, d2 = om.findpts(far)
    assert np.all(code == 2) and np.all(el == -1) and np.all(np.isinf(d2))
    assert np.all(rst == 0.0)


def test_unit_cube_all_inside():
    m = w.cube_c1()
    om = oracle.OracleMesh.from_mesh(m)
    _, h = om.bbox()
    pts = w.queries_c1(4000, seed=1).numpy()
    code, el, rst, d2 = om.findpts(pts)
    assert np.all(code == 0)
    for i in range(0, 4000, 7):
        assert _residual(om, el[i], rst[i], pts[i]) <= 1e-12 * h[el[i]]


@pytest.mark.parametrize("case", ["annulus", "polymap"])
def test_against_brute_force(case):
    rng = np.random.default_rng(13)
    if case == "annulus":
        m = w.annulus_mesh(2, 6, 2, N=4)
        rho = np.sqrt(rng.uniform(0.15, 1.3, 160))
        th = rng.uniform(0, 2 * np.pi, 160)
        pts = np.stack([rho * np.cos(th), rho * np.sin(th), rng.uniform(-0.05, 1.05, 160)], 1)
    else:
        m, _ = w.poly_map_mesh(2, 2, 2, N=3, amp=0.3)
        pts = rng.uniform(-0.1, 1.25, (160, 3))
    om = oracle.OracleMesh.from_mesh(m)
    _, h = om.bbox()
    code, el, rst, d2 = om.findpts(pts)
    bc, be, br, bd = om.brute(pts, grid=4, only_boxes=False)
    bc2, be2, br2, bd2 = om.brute(pts, grid=4, only_boxes=True)
    assert np.any(code == 0) and np.any(code == 1)
    for i in range(len(pts)):
        if bc[i] == 0:   # some element contains the point: findpts must find one
            assert code[i] == 0, i
            if el[i] != be[i]:
                assert np.min(1 - np.abs(rst[i])) <= 1e-10 and np.min(1 - np.abs(br[i])) <= 1e-10
            assert np.sqrt(d2[i]) <= 1e-12 * h[el[i]]
        elif bc2[i] == 1:  # outside: no false local minimum among box candidates
            assert code[i] == 1, i
            assert d2[i] <= bd2[i] * (1 + 1e-10) + 1e-30, (i, d2[i], bd2[i])
        else:
            assert code[i] == 2



def test_spiral_nearest_node_start():
    """Section 3.1, spiral test: on one N = 15 element wound 1.5 times, Newton
    started at the closest GLL node finds every point of the element, while a
    start at the element's centre is trapped for a large share of them; for
    points between the turns, no element point the brute-force multi-start
    search finds is missed, and the returned distance never undercuts its
    minimum (a returned local minimum may exceed it: the paper claims no
    global minimum off the element)."""
    m = w.spiral_element()
    om = oracle.OracleMesh.from_mesh(m, 1e-12)
    b, h = om.bbox()
    pts, rt = spiral_exact_points(m, 1000, 17)
    code, el, rst, d2 = om.findpts(pts)
    assert np.all(code == 0) and np.all(el == 0)
    assert np.max(np.abs(rst - rt)) <= 1e-10
    assert np.sqrt(d2).max() <= 1e-12 * h[0]
    trapped = sum(np.sqrt(om.newton(0, p, r0=np.zeros(3))[1]) > 1e-12 * h[0] for p in pts[:300])
    assert trapped >= 30, trapped  # the centre start fails on this geometry
    rng = np.random.default_rng(18)
    q = rng.uniform(b[0, 0::2], b[0, 1::2], (300, 3))
    code, el, rst, d2 = om.findpts(q)
    bc, _, _, bd = om.brute(q, grid=4)
    assert np.any(bc == 0) and np.any(bc == 1)
    assert np.array_equal(code == 0, bc == 0)
    assert np.all(d2 >= bd * (1 - 1e-10) - 1e-30)


@pytest.mark.parametrize("seed", [17, 19])
def test_spiral_exact_points_inside_at_paper_tolerance(seed):
    """Section 3.1, spiral test: random points of the element are found to a
    tolerance of 1e-14 (relative to h_e here).  Each point is x^e(r_true),
    built by scipy's barycentric interpolant, so the map's own rounding at
    r_true (a few 1e-16 h_e) is the floor; Newton must not stop short of the
    tolerance, so every point comes back inside with a residual, recomputed
    through the map, within 1e-14 h_e."""
    m = w.spiral_element()
    om = oracle.OracleMesh.from_mesh(m, 1e-14)
    _, h = om.bbox()
    pts, rt = spiral_exact_points(m, 1000, seed)
    code, el, rst, d2 = om.findpts(pts)
    assert np.array_equal(np.bincount(code, minlength=3), [1000, 0, 0])
    assert np.all(el == 0)
    assert np.sqrt(d2).max() <= 1e-14 * h[0]
    for i in range(0, 1000, 5):
        assert _residual(om, 0, rst[i], pts[i]) <= 1e-14 * h[0]
    assert np.max(np.abs(rst - rt)) <= 1e-11
