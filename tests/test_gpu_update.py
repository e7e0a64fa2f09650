"""GPU tests of findpts_update (moving and deforming meshes): after an update
the handle gives the same boxes, hash and located points as a handle set up
from scratch on the new coordinates (bit-identical), matches the oracle, and
grows its hash arrays when the new grid needs more room."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as w
from parity import compare_locate

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


def _moved(mesh, angle, shift, amp):
    """Rigid rotation about z by `angle`, a translation, and a smooth
    deformation of amplitude `amp` (small enough to keep every element
    valid)."""
    c, s = math.cos(angle), math.sin(angle)
    x = c * mesh.x - s * mesh.y + shift[0]
    y = s * mesh.x + c * mesh.y + shift[1]
    z = mesh.z + shift[2] + amp * torch.sin(math.pi * mesh.x) * torch.sin(math.pi * mesh.y)
    return w.Mesh(mesh.name + "_moved", mesh.N, x.contiguous(), y.contiguous(), z.contiguous(),
                  mesh.session, mesh.delta)


def _locate(fp, h, pts, dev):
    code, el, rst, d2 = fp.findpts(h, pts.to(dev))
    torch.cuda.synchronize()
    return code.cpu().numpy(), el.cpu().numpy(), rst.cpu().numpy(), d2.cpu().numpy()


def test_update_equals_fresh_setup(dev):
    fp = _fp()
    _say("case: annulus N=7, five moves, update vs fresh setup")
    mesh = w.annulus_mesh(4, 32, 4, N=7)
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, tol=TOL, max_points=1 << 15)
    rng = np.random.default_rng(7)
    for step in range(5):
        mv = _moved(mesh, 0.05 * (step + 1), (0.01 * step, -0.02 * step, 0.03 * step),
                    0.002 * step)
        mvd = mv.to(dev)
        fp.findpts_update(h, mvd.x, mvd.y, mvd.z)
        fresh = fp.findpts_setup(mvd.x, mvd.y, mvd.z, mesh.N, tol=TOL, max_points=1 << 15)
        b1, s1 = fp.findpts_get_bbox(h)
        b2, s2 = fp.findpts_get_bbox(fresh)
        assert np.array_equal(b1, b2) and np.array_equal(s1, s2)
        nc1, lo1, dx1, m1 = fp.findpts_get_hash(h)
        nc2, lo2, dx2, m2 = fp.findpts_get_hash(fresh)
        assert list(nc1) == list(nc2) and list(m1) == list(m2)
        o1, c1 = fp.findpts_get_cells(h)
        o2, c2 = fp.findpts_get_cells(fresh)
        assert np.array_equal(o1, o2) and np.array_equal(c1, c2)
        # points around the moved annulus, some outside
        rho = np.sqrt(rng.uniform(0.2, 1.2, 20_000))
        th = rng.uniform(0, 2 * np.pi, 20_000)
        p0 = np.stack([rho * np.cos(th), rho * np.sin(th), rng.uniform(-0.05, 1.05, 20_000)], 1)
        c, s = math.cos(0.05 * (step + 1)), math.sin(0.05 * (step + 1))
        pts = np.stack([c * p0[:, 0] - s * p0[:, 1] + 0.01 * step,
                        s * p0[:, 0] + c * p0[:, 1] - 0.02 * step,
                        p0[:, 2] + 0.03 * step], 1)
        pts = torch.as_tensor(pts)
        for prec in (fp.FP_PREC_FP64, fp.FP_PREC_MIXED):
            fp.findpts_set_precision(h, prec)
            fp.findpts_set_precision(fresh, prec)
            g1 = _locate(fp, h, pts, dev)
            g2 = _locate(fp, fresh, pts, dev)
            for a, b in zip(g1, g2):
                assert np.array_equal(a, b)
        fresh.free()
    # the last configuration against the oracle
    om = oracle.OracleMesh.from_mesh(mv, TOL)
    _, hs = om.bbox()
    fp.findpts_set_precision(h, fp.FP_PREC_FP64)
    g = _locate(fp, h, pts, dev)
    st = compare_locate(om, pts.numpy(), g, om.findpts(pts.numpy()), hs, TOL)
    assert st["inside"] > 0 and st["notfound"] > 0
    _say(f"update ok {st}")
    h.free()


def test_update_grows_hash_and_keeps_results(dev):
    fp = _fp()
    _say("case: update to a mesh stretched 3x (more hash cells), then back")
    mesh = w.cube_c1()
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, tol=TOL, max_points=4096)
    foot0 = fp.findpts_footprint(h)
    big = w.Mesh("stretched", mesh.N, (3.0 * mesh.x).contiguous(), mesh.y, mesh.z)
    bd = big.to(dev)
    fp.findpts_update(h, bd.x, bd.y, bd.z)
    fresh = fp.findpts_setup(bd.x, bd.y, bd.z, mesh.N, tol=TOL, max_points=4096)
    pts = torch.as_tensor(np.random.default_rng(3).uniform((0, 0, 0), (3, 1, 1), (5000, 3)))
    for a, b in zip(_locate(fp, h, pts, dev), _locate(fp, fresh, pts, dev)):
        assert np.array_equal(a, b)
    fresh.free()
    assert fp.findpts_footprint(h) >= foot0
    fp.findpts_update(h, md.x, md.y, md.z)
    q = w.queries_c1(3000, seed=4)
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    _, hs = om.bbox()
    g = _locate(fp, h, q, dev)
    st = compare_locate(om, q.numpy(), g, om.findpts(q.numpy()), hs, TOL)
    assert st["inside"] == len(q)
    h.free()


def test_update_errors(dev):
    fp = _fp()
    _say("case: update with non-finite coordinates, then recovery; delta rules")
    mesh = w.cube_c1()
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, tol=TOL, max_points=1024)
    bad = md.x.clone()
    bad.view(-1)[17] = float("nan")
    with pytest.raises(fp.FindptsError) as ei:
        fp.findpts_update(h, bad, md.y, md.z)
    assert ei.value.code == fp.FP_EINVAL
    fp.findpts_update(h, md.x, md.y, md.z)
    q = w.queries_c1(500, seed=8)
    code, _, _, _ = fp.findpts(h, q.to(dev))
    assert int((code == 0).sum()) == 500
    with pytest.raises(fp.FindptsError) as ei:
        fp.findpts_update(h, md.x, md.y, md.z, delta=md.x)
    assert ei.value.code == fp.FP_ESTATE
    h.free()


def test_update_two_sessions_delta(dev):
    fp = _fp()
    _say("case: two sessions, the annulus session moves with its distance field")
    mesh = w.overlap_c3()
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, tol=TOL, elem_session=md.session,
                         delta=md.delta, max_points=1 << 16)
    # move the annulus session (session 1) by 0.02 in x; its delta moves with it
    s1 = (mesh.session == 1)[:, None, None, None].to(torch.float64)
    mv = w.Mesh("c3_moved", mesh.N, (mesh.x + 0.02 * s1).contiguous(), mesh.y, mesh.z,
                mesh.session, mesh.delta)
    mvd = mv.to(dev)
    fp.findpts_update(h, mvd.x, mvd.y, mvd.z, delta=mvd.delta)
    fresh = fp.findpts_setup(mvd.x, mvd.y, mvd.z, mesh.N, tol=TOL, elem_session=mvd.session,
                             delta=mvd.delta, max_points=1 << 16)
    pts, tags = w.queries_c3(n=30_000, seed=12)
    code1, el1, r1, d1 = fp.findpts(h, pts.to(dev), tags.to(dev))
    code2, el2, r2, d2 = fp.findpts(fresh, pts.to(dev), tags.to(dev))
    torch.cuda.synchronize()
    for a, b in ((code1, code2), (el1, el2), (r1, r2), (d1, d2)):
        assert torch.equal(a, b)
    om = oracle.OracleMesh.from_mesh(mv, TOL)
    _, hs = om.bbox()
    g = (code1.cpu().numpy(), el1.cpu().numpy(), r1.cpu().numpy(), d1.cpu().numpy())
    compare_locate(om, pts.numpy(), g, om.findpts(pts.numpy(), tags.numpy()), hs, TOL,
                   check_residual_every=3)
    fresh.free()
    h.free()
