"""Pins for the two-dimensional oracle (quadrilateral elements; the method
of Section 2.1 on the reference square): affine closed forms for inside and
border points, exact recovery through an analytic polynomial map, brute
force with many Newton starts, agreement with the (separately pinned) 3D
oracle on the same mesh extruded into a thin layer, the session / distance
selection against the exact distance fields, and interpolation."""
import numpy as np

import oracle
import workloads as w


def _affine2(ex, ey, n, lo, hi, r):
    e = np.array([ex, ey], float)
    n, lo, hi = np.asarray(n, float), np.asarray(lo, float), np.asarray(hi, float)
    return lo + (hi - lo) * (e + (np.asarray(r) + 1.0) * 0.5) / n


def test_affine_closed_form_inside_and_border():
    n, lo, hi = (3, 2), (0.0, 0.0), (2.0, 1.0)
    m = w.box2d_mesh(*n, lo, hi, N=4)
    om = oracle.OracleMesh2.from_mesh(m)
    rng = np.random.default_rng(21)
    P = rng.uniform((-0.3, -0.3), (2.3, 1.3), (3000, 2))
    code, el, rs, d2 = om.findpts(P)
    b, h = om.bbox()
    cl = np.clip(P, lo, hi)
    inside = np.all(P == cl, axis=1)
    # points outside every box come back not found; the rest of the outside
    # ones are border points at the distance to the rectangle
    nf = code == 2
    assert np.all(inside[code == 0]) and np.all(~inside[code != 0])
    bor = code == 1
    assert np.allclose(np.sqrt(d2[bor]), np.linalg.norm(P[bor] - cl[bor], axis=1),
                       rtol=1e-12, atol=1e-14)
    assert np.all(np.isinf(d2[nf])) and np.all(el[nf] == -1)
    for i in np.nonzero(code == 0)[0]:
        x = _affine2(el[i] % n[0], el[i] // n[0], n, lo, hi, rs[i])
        assert np.linalg.norm(x - P[i]) <= 1e-12 * h[el[i]]
    # border: the returned (el, r) maps onto the clamped point
    for i in np.nonzero(bor)[0][:300]:
        x = _affine2(el[i] % n[0], el[i] // n[0], n, lo, hi, rs[i])
        assert np.linalg.norm(x - cl[i]) <= 1e-12


def test_exact_recovery_polynomial_map():
    n, N = (4, 3), 3
    m, phi = w.poly_map_mesh2d(*n, N=N, amp=0.04)
    om = oracle.OracleMesh2.from_mesh(m)
    _, h = om.bbox()
    rng = np.random.default_rng(22)
    P = 2000
    et = rng.integers(0, m.E, P)
    rt = rng.uniform(-1, 1, (P, 2))
    a = np.array([_affine2(e % n[0], e // n[0], n, (0, 0), (1, 1), r) for e, r in zip(et, rt)])
    pts = np.stack(phi(a[:, 0], a[:, 1]), 1)
    code, el, rs, d2 = om.findpts(pts)
    assert np.all(code == 0)
    same = el == et
    assert np.max(np.abs(rs[same] - rt[same])) <= 1e-10
    # a different element only on a shared edge
    assert np.all(np.min(1 - np.abs(rt[~same]), axis=1) <= 1e-10)
    assert np.sqrt(d2).max() <= 1e-12 * h.max()


def test_against_brute_force():
    rng = np.random.default_rng(23)
    for m in (w.annulus2d_mesh(3, 10, N=4), w.poly_map_mesh2d(3, 3, N=3, amp=0.05)[0]):
        om = oracle.OracleMesh2.from_mesh(m)
        _, h = om.bbox()
        if m.name.startswith("annulus"):
            rho = np.sqrt(rng.uniform(0.15, 1.3, 400))
            th = rng.uniform(0, 2 * np.pi, 400)
            pts = np.stack([rho * np.cos(th), rho * np.sin(th)], 1)
        else:
            pts = rng.uniform(-0.1, 1.2, (400, 2))
        code, el, rs, d2 = om.findpts(pts)
        bc, be, br, bd = om.brute(pts, grid=5, all_nodes=True, only_boxes=True)
        assert np.any(code == 0) and np.any(code == 1)
        assert np.array_equal(code, bc)
        for i in range(len(pts)):
            if bc[i] == 0 and el[i] != be[i]:
                assert np.min(1 - np.abs(rs[i])) <= 1e-10 and np.min(1 - np.abs(br[i])) <= 1e-10
            if bc[i] == 1:
                assert d2[i] <= bd[i] * (1 + 1e-10) + 1e-30, (i, d2[i], bd[i])


def test_matches_3d_oracle_on_extruded_mesh():
    """The 2D mesh extruded into a layer z = 1e-3 t (same order in t): a
    point (x, y, 0) has the same owner, (r, s), distance and code in both
    oracles (the 3D closest point lies on t = 0)."""
    N = 4
    m2 = w.annulus2d_mesh(3, 12, N=N)
    n1 = N + 1
    zt = w.gll_points(N)
    x3 = np.repeat(m2.x.numpy()[:, None, :, :], n1, axis=1)
    y3 = np.repeat(m2.y.numpy()[:, None, :, :], n1, axis=1)
    z3 = np.broadcast_to(1e-3 * zt[None, :, None, None], x3.shape).copy()
    om2 = oracle.OracleMesh2.from_mesh(m2)
    om3 = oracle.OracleMesh(x3, y3, z3, N)
    rng = np.random.default_rng(24)
    rho = np.sqrt(rng.uniform(0.15, 1.3, 1500))
    th = rng.uniform(0, 2 * np.pi, 1500)
    p2 = np.stack([rho * np.cos(th), rho * np.sin(th)], 1)
    p3 = np.concatenate([p2, np.zeros((len(p2), 1))], 1)
    c2, e2, r2, d2 = om2.findpts(p2)
    c3, e3, r3, d3 = om3.findpts(p3)
    assert np.array_equal(c2, c3)
    assert np.array_equal(e2, e3)
    found, ins = c2 != 2, c2 == 0
    assert np.any(ins) and np.any(c2 == 1)
    assert np.max(np.abs(r2[ins] - r3[ins, :2])) <= 1e-10
    # a border point's r is fixed only to about sqrt(eps) relative (the
    # distance is flat at its minimum); the distance itself agrees closely
    assert np.max(np.abs(r2[found] - r3[found, :2])) <= 1e-6
    assert np.max(np.abs(r3[found, 2])) <= 1e-6
    assert np.allclose(d2[found], d3[found], rtol=1e-9, atol=1e-26)


def test_sessions_and_distance_selection():
    m = w.overlap2d(N=5)
    om = oracle.OracleMesh2.from_mesh(m)
    sess = m.session.numpy()
    rng = np.random.default_rng(25)
    P = rng.uniform(-1.2, 1.2, (3000, 2))
    code, el, rs, d2 = om.findpts(P)
    rho = np.hypot(P[:, 0], P[:, 1])
    in_ring = (rho >= 0.5) & (rho <= 1.0)
    in_box = np.max(np.abs(P), axis=1) >= 0.55
    d_ring = np.minimum(rho - 0.5, 1.0 - rho)
    dx = np.clip(np.abs(P[:, 0]) - 0.55, 0, None)
    dy = np.clip(np.abs(P[:, 1]) - 0.55, 0, None)
    d_box = np.minimum(np.minimum(1.65 - np.abs(P[:, 0]), 1.65 - np.abs(P[:, 1])),
                       np.hypot(dx, dy))
    both = in_ring & in_box
    clear = both & (np.abs(d_ring - d_box) > 0.02)  # well above interpolation error
    assert clear.sum() > 100
    assert np.all(code[both] == 0)
    want = np.where(d_ring > d_box, 1, 0)
    assert np.array_equal(sess[el[clear]], want[clear])
    # session exclusion: a point tagged with its own session is found in the other
    ps = np.zeros(len(P), np.int32)
    c0, e0, _, _ = om.findpts(P, psess=ps)
    assert np.all(sess[e0[c0 != 2]] == 1)
    assert np.all(c0[in_ring] == 0)


def test_interpolation():
    N = 5
    m = w.annulus2d_mesh(2, 8, N=N)
    om = oracle.OracleMesh2.from_mesh(m)
    rng = np.random.default_rng(26)
    E, n1 = m.E, N + 1
    z = w.gll_points(N)
    # per-element reference polynomial of degree N in r and s: exact
    c = rng.normal(size=(E, 3))
    R = z[None, None, :]
    S = z[None, :, None]
    F = c[:, 0, None, None] * R ** N + c[:, 1, None, None] * R * S ** (N - 1) + c[:, 2, None, None]
    P = 500
    el = rng.integers(0, E, P).astype(np.int32)
    rs = rng.uniform(-1, 1, (P, 2))
    code = np.zeros(P, np.int32)
    code[:7] = 2
    out = om.eval(code, el, rs, [F.reshape(-1), m.x.numpy().reshape(-1)])
    ref = c[el, 0] * rs[:, 0] ** N + c[el, 1] * rs[:, 0] * rs[:, 1] ** (N - 1) + c[el, 2]
    assert np.all(np.isnan(out[:, :7]))
    assert np.max(np.abs(out[0, 7:] - ref[7:])) <= 1e-12 * np.abs(ref).max()
    xs = np.array([om.map(e, r)[0][0] for e, r in zip(el, rs)])
    assert np.max(np.abs(out[1, 7:] - xs[7:])) <= 1e-14
