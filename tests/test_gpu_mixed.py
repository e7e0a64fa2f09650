"""GPU parity of the mixed-precision location (binary32 Newton on the matrix
cores, binary64 end game and classification) against the binary64 CPU oracle,
under the same rules as the binary64 path: same codes and elements (face
ties and the tolerance band aside), r within 1e-10, and the GPU's own
residual, recomputed by the oracle's map, at most tol * h_e = 1e-12 h_e.
Mixed-precision interpolation accumulates in binary32 and is checked at the
bound MIXED_EVAL_REL of tests/parity.py."""
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


def _run(fp, mesh, pts, dev, precision, max_points=1 << 16, psess=None, fields=(), tol=TOL):
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, tol=tol, elem_session=md.session,
                         delta=md.delta, max_points=max_points, precision=precision)
    ps = None if psess is None else psess.to(dev)
    code, el, rst, d2 = fp.findpts(h, pts.to(dev), ps)
    out = None
    if fields:
        out = fp.findpts_eval(h, code, el, rst, [f.to(dev) for f in fields])
    torch.cuda.synchronize()
    res = (code.cpu().numpy(), el.cpu().numpy(), rst.cpu().numpy(), d2.cpu().numpy())
    return h, res, (None if out is None else out.cpu().numpy())


def test_mixed_c1_unit_cube(dev):
    fp = _fp()
    _say("case: mixed precision, unit cube N=5, 1e4 points")
    mesh = w.cube_c1()
    pts = w.queries_c1()
    f = mesh.x ** 2 + mesh.y * mesh.z + mesh.z ** 3
    h, g, out = _run(fp, mesh, pts, dev, fp.FP_PREC_MIXED, fields=[f])
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    o = om.findpts(pts.numpy())
    _, hs = om.bbox()
    st = compare_locate(om, pts.numpy(), g, o, hs, TOL)
    assert st["inside"] == len(pts)
    compare_eval(out, om.eval(g[0], g[1], g[2], [f.numpy()]), [f.numpy()], rel=MIXED_EVAL_REL)
    pairs, iters, npts, cands = fp.findpts_stats(h)
    assert cands == om.last_stats[0]
    _say(f"mixed c1 ok {st}; iters/pair {iters / pairs:.2f}")


@pytest.fixture(scope="module")
def c2(dev):
    mesh = w.annulus_c2()
    pts = w.queries_c2()
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    return mesh, pts, om


def test_mixed_c2_subset(dev, c2):
    fp = _fp()
    mesh, pts, om = c2
    sub = pts[:60_001]
    _say("case: mixed precision, annulus C2 mesh, 60001-point subset")
    fields, _ = w.poly_fields(mesh, 2, seed=2)
    h, g, out = _run(fp, mesh, sub, dev, fp.FP_PREC_MIXED, max_points=1 << 17, fields=fields)
    o = om.findpts(sub.numpy())
    _, hs = om.bbox()
    st = compare_locate(om, sub.numpy(), g, o, hs, TOL, check_residual_every=3)
    assert st["border"] > 0 and st["notfound"] > 0
    ref = om.eval(g[0], g[1], g[2], [f.numpy() for f in fields])
    compare_eval(out, ref, [f.numpy() for f in fields], rel=MIXED_EVAL_REL)
    _say(f"mixed c2 subset ok {st}")


def test_mixed_vs_fp64_full_size(dev, c2):
    """Benchmark workload at full size, launch configuration of the
    benchmark: mixed and binary64 give the same codes and elements except at
    face ties, r within 1e-10; a seeded sample is checked against the
    oracle, including the residual bound."""
    fp = _fp()
    mesh, pts, om = c2
    _say("case: mixed vs fp64, annulus C2 full 1.01M points")
    _, g64, _ = _run(fp, mesh, pts, dev, fp.FP_PREC_FP64, max_points=1 << 20)
    _, gmx, _ = _run(fp, mesh, pts, dev, fp.FP_PREC_MIXED, max_points=1 << 20)
    c64, e64, r64, d64 = g64
    cmx, emx, rmx, dmx = gmx
    assert np.array_equal(c64, cmx)
    same = e64 == emx
    ties = ~same
    assert np.all(np.min(1 - np.abs(rmx[ties]), axis=1) <= 1e-10), "element differs off a face"
    ins = same & (c64 == 0)
    assert np.max(np.abs(r64[ins] - rmx[ins])) <= 1e-10
    rng = np.random.default_rng(23)
    idx = np.sort(rng.choice(len(pts), 20_000, replace=False))
    o = om.findpts(pts.numpy()[idx])
    _, hs = om.bbox()
    st = compare_locate(om, pts.numpy()[idx], tuple(a[idx] for a in gmx), o, hs, TOL,
                        check_residual_every=2)
    _say(f"mixed full ok: {int(np.sum(ties))} face ties vs fp64; sample {st}")


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_mixed_orders(dev, N):
    fp = _fp()
    _say(f"case: mixed precision, order N={N}")
    if N >= 3:
        mesh = w.annulus_mesh(2, 8, 2, N=N)
    else:
        mesh = w.box_mesh(3, 3, 2, lo=(-1, 0, 0), hi=(2, 1, 0.5), N=N)
    rng = np.random.default_rng(40 + N)
    if N >= 3:
        rho = np.sqrt(rng.uniform(0.2, 1.2, 3000))
        th = rng.uniform(0, 2 * np.pi, 3000)
        pts = np.stack([rho * np.cos(th), rho * np.sin(th), rng.uniform(-0.05, 1.05, 3000)], 1)
    else:
        pts = rng.uniform((-1.1, -0.1, -0.1), (2.1, 1.1, 0.6), (3000, 3))
    pts = torch.as_tensor(pts)
    h, g, _ = _run(fp, mesh, pts, dev, fp.FP_PREC_MIXED)
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    _, hs = om.bbox()
    compare_locate(om, pts.numpy(), g, om.findpts(pts.numpy()), hs, TOL)


@pytest.mark.parametrize("N", [8, 9])
def test_mixed_high_order_many_chunks(dev, N):
    """Orders 8 and 9 (a binary32 launch, then binary64 Newton from its end
    points): 4 curved elements with 3000 points, so each element's pairs span
    several pair chunks of both kernels and many 16-slot rounds."""
    fp = _fp()
    _say(f"case: mixed precision, order N={N}, 4 elements x 750 points")
    mesh = w.annulus_mesh(1, 4, 1, N=N)
    rng = np.random.default_rng(60 + N)
    rho = np.sqrt(rng.uniform(0.2, 1.2, 3000))
    th = rng.uniform(0, 2 * np.pi, 3000)
    pts = np.stack([rho * np.cos(th), rho * np.sin(th), rng.uniform(-0.05, 1.05, 3000)], 1)
    pts = torch.as_tensor(pts)
    h, g, _ = _run(fp, mesh, pts, dev, fp.FP_PREC_MIXED)
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    _, hs = om.bbox()
    compare_locate(om, pts.numpy(), g, om.findpts(pts.numpy()), hs, TOL)


def test_mixed_far_from_origin(dev):
    """A curved mesh translated by 1000.  A binary32 coordinate there rounds
    by up to 3e-5, 1.2e-4 h_e (h_e = 0.25): binary32 arithmetic on the raw
    coordinates could not reach the binary32 phase's target (3e-5 h_e).  In
    binary64 the map itself rounds by a few 1e-13 there, so the tolerance is
    1e-10 (the paper leaves it to the user)."""
    fp = _fp()
    _say("case: mixed precision, mesh translated by 1000, tol 1e-10")
    base = w.cube_c1()
    sh = 1000.0
    tol = 1e-10
    mesh = w.Mesh("cube_shifted", base.N, base.x + sh, base.y - sh, base.z + sh,
                  base.session, base.delta)
    pts = w.queries_c1(3000, seed=5) + torch.tensor([sh, -sh, sh], dtype=torch.float64)
    h, g, _ = _run(fp, mesh, pts, dev, fp.FP_PREC_MIXED, tol=tol)
    om = oracle.OracleMesh.from_mesh(mesh, tol)
    _, hs = om.bbox()
    st = compare_locate(om, pts.numpy(), g, om.findpts(pts.numpy()), hs, tol)
    assert st["inside"] == len(pts)


def test_mixed_exact_recovery(dev):
    fp = _fp()
    _say("case: mixed precision, exact recovery through the analytic map")
    from helpers import box_affine, box_elem_ids, phi_np
    n = (3, 3, 3)
    mesh, _ = w.poly_map_mesh(*n, N=4, amp=0.04)
    ex, ey, ez = box_elem_ids(mesh.E, n)
    rng = np.random.default_rng(32)
    P = 5000
    et = rng.integers(0, mesh.E, P)
    rt = rng.uniform(-1, 1, (P, 3))
    a = np.array([box_affine(ex[e], ey[e], ez[e], n, (0, 0, 0), (1, 1, 1), r)
                  for e, r in zip(et, rt)])
    pts = np.stack(phi_np(a[:, 0], a[:, 1], a[:, 2], amp=0.04), 1)
    h, g, _ = _run(fp, mesh, torch.as_tensor(pts), dev, fp.FP_PREC_MIXED)
    gc, ge, gr, gd = g
    assert np.all(gc == 0)
    same = ge == et
    assert np.max(np.abs(gr[same] - rt[same])) <= 1e-11
    assert np.all(np.min(1 - np.abs(rt[~same]), axis=1) <= 1e-10)


def test_mixed_two_sessions(dev):
    fp = _fp()
    _say("case: mixed precision, two overlapping sessions, interface nodes")
    mesh = w.overlap_c3()
    pts, tags = w.c3_interface_nodes(mesh)
    rng = np.random.default_rng(4)
    idx = torch.as_tensor(np.sort(rng.choice(len(pts), 20_000, replace=False)))
    pts, tags = pts[idx].contiguous(), tags[idx].contiguous()
    h, g, _ = _run(fp, mesh, pts, dev, fp.FP_PREC_MIXED, psess=tags)
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    _, hs = om.bbox()
    st = compare_locate(om, pts.numpy(), g, om.findpts(pts.numpy(), tags.numpy()), hs, TOL,
                        check_residual_every=3)
    _say(f"mixed two sessions ok {st}")
