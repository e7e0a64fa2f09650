"""More GPU parity against the CPU oracle (through the C ABI):

* findpts_eval with 4, 5 and 9 fields at orders 7, 9 and 12 -- each order's
  interpolation kernel, the split of a call into launches of at most 8
  fields, and at order 7 (3e5 points) the staged path (grouping by the
  two-level counting sort, values staged in bucket order and moved to the
  output) -- element by element at 1e-13 max|F|, with crowded elements
  spread over several work units and not-found points in the mix;
* the closest-node start at exact near-ties: points midway between two
  nodes on neighbouring turns of the N = 15 spiral (Section 3.1), where the
  start node decides which local minimum Newton settles in;
* mixed precision with three overlapping sessions and the distance
  discriminator, points on interior element faces of the session with the
  larger distance (the binary32 phase leaves face pairs unsolved);
* a loose tolerance (1e-6) on a rotated curved mesh, where the oriented-box
  filter must keep every element that holds a point within tol h_e.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as w
from parity import MIXED_EVAL_REL, compare_eval, compare_locate

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _fp():
    from paper_1811_04891_amd import findpts as fp
    return fp


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.mark.parametrize("N", [7, 9, 12])
@pytest.mark.parametrize("nf", [4, 5, 9])
def test_eval_many_fields(dev, N, nf):
    fp = _fp()
    _say(f"case: findpts_eval N={N} nf={nf}")
    mesh = w.annulus_mesh(2, 8, 2, N=N)
    E = mesh.E
    fields, _ = w.poly_fields(mesh, nf, seed=100 + N + nf)
    rng = np.random.default_rng(200 + N + nf)
    # order 7: above the size where the matrix-core kernel's pass is staged
    P = 300_001 if N <= 7 else 30_001
    # a crowded element (several work units of every kernel), a spread of
    # the rest, ragged counts, and not-found points
    el = np.where(rng.uniform(size=P) < 0.35, 3, rng.integers(0, E, P)).astype(np.int32)
    rst = rng.uniform(-1, 1, (P, 3))
    rst[::17] = np.clip(np.round(rst[::17]), -1, 1)  # corners and faces of [-1,1]^3
    code = np.zeros(P, np.int32)
    nf_idx = rng.choice(P, 300, replace=False)
    code[nf_idx] = 2
    el[nf_idx] = -1
    rst[nf_idx] = 0.0
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, N, tol=TOL, max_points=P)
    out = fp.findpts_eval(h, torch.as_tensor(code).to(dev), torch.as_tensor(el).to(dev),
                          torch.as_tensor(rst).to(dev), [f.to(dev) for f in fields])
    torch.cuda.synchronize()
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    ref = om.eval(code, el, rst, [f.numpy() for f in fields])
    compare_eval(out.cpu().numpy(), ref, [f.numpy() for f in fields], rel=1e-13)
    h.free()


@pytest.mark.parametrize("N", [4, 7, 9])
@pytest.mark.parametrize("nf", [5, 9])
def test_eval_many_fields_mixed(dev, N, nf):
    """Mixed precision: orders up to 7 interpolate in binary32 (binary32
    accumulation, all fields of a launch in one pass), within MIXED_EVAL_REL
    max|F| of the oracle; higher orders interpolate in binary64."""
    fp = _fp()
    _say(f"case: findpts_eval mixed N={N} nf={nf}")
    mesh = w.annulus_mesh(2, 8, 2, N=N)
    fields, _ = w.poly_fields(mesh, nf, seed=300 + N + nf)
    rng = np.random.default_rng(400 + N + nf)
    P = 300_001 if N == 7 else 20_001
    el = np.where(rng.uniform(size=P) < 0.3, 5, rng.integers(0, mesh.E, P)).astype(np.int32)
    rst = rng.uniform(-1, 1, (P, 3))
    code = np.zeros(P, np.int32)
    nf_idx = rng.choice(P, 200, replace=False)
    code[nf_idx], el[nf_idx], rst[nf_idx] = 2, -1, 0.0
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, N, tol=TOL, max_points=P,
                         precision=fp.FP_PREC_MIXED)
    out = fp.findpts_eval(h, torch.as_tensor(code).to(dev), torch.as_tensor(el).to(dev),
                          torch.as_tensor(rst).to(dev), [f.to(dev) for f in fields])
    torch.cuda.synchronize()
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    hf = [f.numpy() for f in fields]
    ref = om.eval(code, el, rst, hf)
    compare_eval(out.cpu().numpy(), ref, hf, rel=MIXED_EVAL_REL if N <= 7 else 1e-13)
    h.free()


def _spiral_turn_midpoints(mesh, draws, seed):
    """Points midway between node a = (i, N, k) (s = +1 face of one turn) and
    node b = (i', 0, k) (s = -1 face of the next turn), i' the r index whose
    angle 1.5 pi (r + 1) is nearest 2 pi further on.  Kept only where a and b
    are the two closest nodes (checked here in numpy), so that the closest
    node is decided by rounding; Newton from a and from b ends in different
    local minima."""
    hd = mesh.host()
    N = mesh.N
    n1 = N + 1
    z = w.gll_points(N)
    th = 1.5 * np.pi * (z + 1)
    X = np.stack([hd[c].reshape(-1) for c in "xyz"], 1)
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(draws):
        i, k = int(rng.integers(0, n1)), int(rng.integers(0, n1))
        if th[i] + 2 * np.pi > th[-1]:
            continue
        ii = int(np.argmin(np.abs(th - (th[i] + 2 * np.pi))))
        ia, ib = i + n1 * (N + n1 * k), ii + n1 * (0 + n1 * k)
        m = 0.5 * (X[ia] + X[ib])
        d = np.sum((X - m) ** 2, 1)
        if set(np.argsort(d)[:2]) == {ia, ib}:
            out.append(m)
    return np.array(out)


def test_spiral_start_node_near_ties(dev):
    """Section 2.1: Newton starts at the closest point of the mapped GLL mesh.
    Points midway between two nodes on neighbouring turns of the spiral are
    outside the element, about equally far from both turns; the start node
    picks the local minimum.  Both sides take the node of smallest squared
    distance (summed in x, y, z order), ties to the smaller index, so code,
    element, distance and r agree with the oracle."""
    fp = _fp()
    _say("case: spiral midway points between turns (start-node near-ties)")
    mesh = w.spiral_element()
    pts = _spiral_turn_midpoints(mesh, 2000, 24)
    assert len(pts) > 300
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, tol=TOL, max_points=1024)
    code, el, rst, d2 = fp.findpts(h, torch.as_tensor(pts).to(dev))
    torch.cuda.synchronize()
    g = (code.cpu().numpy(), el.cpu().numpy(), rst.cpu().numpy(), d2.cpu().numpy())
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    _, hs = om.bbox()
    o = om.findpts(pts)
    st = compare_locate(om, pts, g, o, hs, TOL)
    assert st["border"] == len(pts)
    # the start node is unique here (no tie between local minima is left to
    # either side): dist2 and r of every border point agree
    bor = (o[0] == 1) & (g[0] == 1)
    assert np.all(np.abs(g[3][bor] - o[3][bor]) <= 1e-9 * o[3][bor])
    assert np.max(np.abs(g[2][bor] - o[2][bor])) <= 1e-8
    _say(f"spiral midway ok {st}")
    h.free()


def test_mixed_three_sessions_faces(dev):
    """Three sessions: a long box (session 0, delta 100 everywhere: it always
    wins where it is a candidate), two shorter boxes of 2 x 2 x 1 elements
    (sessions 1 and 2) overlapping it.  Points lie on the interior faces
    between elements of session 0; tagged with session 1 or 2 they must go
    to session 0 (largest delta) and, among its two face elements, to the
    smaller id, as in the oracle, in binary64 and in mixed precision."""
    fp = _fp()
    _say("case: mixed precision, three sessions, points on interior faces")
    m0 = w.box_mesh(4, 2, 2, (0, 0, 0), (3, 1, 1), N=4)
    m1 = w.box_mesh(2, 2, 1, (0, 0, 0), (2, 1, 1), N=4)
    m2 = w.box_mesh(2, 2, 1, (1, 0, 0), (3, 1, 1), N=4)
    ms = [m0, m1, m2]
    x = torch.cat([m.x for m in ms]); y = torch.cat([m.y for m in ms]); z = torch.cat([m.z for m in ms])
    sess = torch.cat([torch.full((m.E,), i, dtype=torch.int32) for i, m in enumerate(ms)])
    delta = torch.cat([torch.full_like(m0.x, 100.0), 2.0 - m1.x, m2.x - 1.0])
    mesh = w.Mesh("three_faces", 4, x, y, z, sess, delta)
    rng = np.random.default_rng(61)
    P = 3000
    pts = rng.uniform((0.05, 0.05, 0.05), (2.95, 0.95, 0.95), (P, 3))
    ax = rng.integers(0, 3, P)
    faces = [np.array([0.75, 1.5, 2.25]), np.array([0.5]), np.array([0.5])]
    for i in range(P):  # snap one coordinate onto an interior face of session 0
        f = faces[ax[i]]
        pts[i, ax[i]] = f[rng.integers(0, len(f))]
    tags = torch.as_tensor(rng.integers(1, 3, P).astype(np.int32))
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    _, hs = om.bbox()
    o = om.findpts(pts, tags.numpy())
    assert np.all(o[0] == 0) and np.all(sess.numpy()[o[1]] == 0)
    md = mesh.to(dev)
    for prec in (fp.FP_PREC_FP64, fp.FP_PREC_MIXED):
        h = fp.findpts_setup(md.x, md.y, md.z, 4, tol=TOL, elem_session=md.session,
                             delta=md.delta, max_points=4096, precision=prec)
        code, el, rst, d2 = fp.findpts(h, torch.as_tensor(pts).to(dev), tags.to(dev))
        torch.cuda.synchronize()
        g = (code.cpu().numpy(), el.cpu().numpy(), rst.cpu().numpy(), d2.cpu().numpy())
        st = compare_locate(om, pts, g, o, hs, TOL)
        # the owner session is decided by delta, never by a face tie
        assert np.all(sess.numpy()[g[1]] == 0)
        # and within session 0 the smaller face element, as in the oracle
        assert np.array_equal(g[1], o[1]), prec
        _say(f"three sessions faces prec={prec} ok {st}")
        h.free()


def _rotation(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * (K @ K)


def _loose_tol_case(tol):
    """An annulus (2 x 10 x 2 elements, N = 5) rotated about a skew axis, and
    points within 0.8 tol h_e of the shared azimuthal faces, on either side:
    inside one element and, by the tolerance, inside its neighbour too."""
    base = w.annulus_mesh(2, 10, 2, N=5)
    R = _rotation([1.0, 2.0, 0.5], 0.7)
    X = torch.stack([base.x, base.y, base.z], -1) @ torch.as_tensor(R.T)
    mesh = w.Mesh("annulus_rot", base.N, X[..., 0].contiguous(), X[..., 1].contiguous(),
                  X[..., 2].contiguous())
    rng = np.random.default_rng(62)
    P = 3000
    hmin = 0.5  # below every element's node extent (0.59 and up) on this mesh
    rho = rng.uniform(0.5, 1.0, P)
    off = rng.uniform(0.05, 0.8, P) * tol * hmin * rng.choice([-1.0, 1.0], P)
    th = 2 * np.pi * rng.integers(0, 10, P) / 10 + off / rho
    q = np.stack([rho * np.cos(th), rho * np.sin(th), rng.uniform(0.02, 0.98, P)], 1)
    return mesh, q @ R.T


def test_loose_tolerance_rotated_mesh(dev):
    """tol = 1e-6 on a curved mesh rotated about a skew axis (Section 2.1:
    the tolerance decides inside).  Points within tol h_e of a shared face
    are inside both elements; the smaller id owns them.  The oriented-box
    first round must keep both elements (its margin covers tol h_e), so the
    owners match the oracle exactly."""
    fp = _fp()
    _say("case: tol 1e-6 on a rotated curved mesh, points near shared faces")
    tol = 1e-6
    mesh, pts = _loose_tol_case(tol)
    om = oracle.OracleMesh.from_mesh(mesh, tol)
    _, hs = om.bbox()
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, tol=tol, max_points=4096)
    code, el, rst, d2 = fp.findpts(h, torch.as_tensor(pts).to(dev))
    torch.cuda.synchronize()
    g = (code.cpu().numpy(), el.cpu().numpy(), rst.cpu().numpy(), d2.cpu().numpy())
    o = om.findpts(pts)
    st = compare_locate(om, pts, g, o, hs, tol)
    assert np.all(o[0] == 0)
    assert np.array_equal(g[1], o[1])
    _say(f"loose tolerance ok {st}")
    h.free()
