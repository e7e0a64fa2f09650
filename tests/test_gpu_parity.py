"""GPU parity: the HIP findpts / findpts_eval path (through the C ABI)
against the CPU oracle on the same seeded inputs.  Sizes span many element
wavefronts and ragged tails; the full 1.01M-point annulus workload is run in
the same launch configuration as the benchmark and checked on a sample."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as w
from parity import compare_eval, compare_locate

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


def _run(fp, mesh, pts, dev, max_points=1 << 16, psess=None, fields=(), tol=TOL):
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, tol=tol, elem_session=md.session,
                         delta=md.delta, max_points=max_points)
    ps = None if psess is None else psess.to(dev)
    code, el, rst, d2 = fp.findpts(h, pts.to(dev), ps)
    out = None
    if fields:
        out = fp.findpts_eval(h, code, el, rst, [f.to(dev) for f in fields])
    torch.cuda.synchronize()
    res = (code.cpu().numpy(), el.cpu().numpy(), rst.cpu().numpy(), d2.cpu().numpy())
    return h, res, (None if out is None else out.cpu().numpy())


def test_c1_unit_cube_full(dev):
    fp = _fp()
    _say("case: unit cube N=5, 1e4 points, 1 field")
    mesh = w.cube_c1()
    pts = w.queries_c1()
    X = mesh.x
    f = X ** 2 + mesh.y * mesh.z + mesh.z ** 3
    h, g, out = _run(fp, mesh, pts, dev, fields=[f])
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    o = om.findpts(pts.numpy())
    _, hs = om.bbox()
    st = compare_locate(om, pts.numpy(), g, o, hs, TOL)
    assert st["inside"] == len(pts)
    ref = om.eval(g[0], g[1], g[2], [f.numpy()])
    compare_eval(out, ref, [f.numpy()])
    # candidates of the method (hash + box + session) = oracle count (exact)
    pairs, iters, npts, cands = fp.findpts_stats(h)
    assert cands == om.last_stats[0] and npts == len(pts)
    _say(f"c1 ok {st}, gpu pairs/pt {pairs / npts:.3f} iters/pair {iters / pairs:.2f}; "
         f"oracle cands/pt {cands / npts:.3f} iters/cand {om.last_stats[1] / om.last_stats[0]:.2f}")


def test_setup_boxes_and_hash(dev):
    fp = _fp()
    for mesh in (w.cube_c1(), w.annulus_mesh(4, 16, 3, N=7)):
        _say(f"case: setup parity {mesh.name} E={mesh.E}")
        md = mesh.to(dev)
        h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, max_points=16)
        gb, gh = fp.findpts_get_bbox(h)
        om = oracle.OracleMesh.from_mesh(mesh)
        ob, oh = om.bbox()
        assert np.array_equal(gh, oh)  # node extents: exact min/max
        # the two sides sum the Bernstein transform in different orders (and
        # the GPU fuses multiply-adds): a few ulps, far below the 1e-8 h margin
        scale = np.max(np.abs(ob))
        assert np.max(np.abs(gb - ob)) <= 1e-13 * scale
        nc, lo, dx, (ncell, nnz, maxc) = fp.findpts_get_hash(h)
        off, cel = fp.findpts_get_cells(h)
        assert ncell == nc[0] * nc[1] * nc[2] and off[-1] == nnz
        # every cell list = ascending ids of boxes overlapping the cell, computed
        # on the host from the GPU's own boxes and grid
        inv = 1.0 / dx
        def cidx(v, a):
            return np.clip(np.floor((v - lo[a]) * inv[a]).astype(int), 0, nc[a] - 1)
        ref = [[] for _ in range(ncell)]
        for e in range(mesh.E):
            r = [(cidx(gb[e, 2 * a], a), cidx(gb[e, 2 * a + 1], a)) for a in range(3)]
            for k in range(r[2][0], r[2][1] + 1):
                for j in range(r[1][0], r[1][1] + 1):
                    for i in range(r[0][0], r[0][1] + 1):
                        ref[i + nc[0] * (j + nc[1] * k)].append(e)
        for c in range(ncell):
            assert list(cel[off[c]:off[c + 1]]) == ref[c]
        assert maxc == max(len(r) for r in ref)
        h.free()


@pytest.fixture(scope="module")
def c2(dev):
    mesh = w.annulus_c2()
    pts = w.queries_c2()
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    return mesh, pts, om


def test_c2_annulus_subset(dev, c2):
    fp = _fp()
    mesh, pts, om = c2
    sub = pts[:60_001]  # ragged
    _say("case: annulus C2 mesh, 60001-point subset")
    fields, _ = w.poly_fields(mesh, 2, seed=2)
    h, g, out = _run(fp, mesh, sub, dev, max_points=1 << 17, fields=fields)
    o = om.findpts(sub.numpy())
    _, hs = om.bbox()
    st = compare_locate(om, sub.numpy(), g, o, hs, TOL, check_residual_every=7)
    assert st["border"] > 0 and st["notfound"] > 0
    ref = om.eval(g[0], g[1], g[2], [f.numpy() for f in fields])
    compare_eval(out, ref, [f.numpy() for f in fields])
    pairs, _, npts, cands = fp.findpts_stats(h)
    assert cands == om.last_stats[0] and npts == len(sub)
    _say(f"c2 subset ok {st}; pairs solved/pt {pairs / npts:.3f}, method cands/pt {cands / npts:.3f}")


def test_c2_full_size(dev, c2):
    """The benchmark workload at full size (1.01M points, one pass of
    max_points = 2^20, 4 fields), every point's location and every
    interpolated value against the oracle."""
    fp = _fp()
    mesh, pts, om = c2
    _say("case: annulus C2 full 1.01M points, 4 fields, every output")
    md = mesh.to(dev)
    fields, _ = w.poly_fields(md, 4, seed=2)  # built on the device, copied for the oracle
    h, g, out = _run(fp, mesh, pts, dev, max_points=1 << 20, fields=fields)
    o = om.findpts(pts.numpy())
    _, hs = om.bbox()
    st = compare_locate(om, pts.numpy(), g, o, hs, TOL, check_residual_every=50)
    assert st["border"] > 0 and st["notfound"] > 0
    hf = [f.cpu().numpy() for f in fields]
    compare_eval(out, om.eval(g[0], g[1], g[2], hf), hf)
    pairs, _, npts, cands = fp.findpts_stats(h)
    assert cands == om.last_stats[0] and npts == len(pts)
    _say(f"c2 full ok {st}")
    h.free()


def test_chunked_equals_single_pass(dev):
    fp = _fp()
    mesh = w.annulus_mesh(4, 16, 3, N=5)
    pts = w.queries_c2(n_in=20_000, seed=9)
    _say("case: multi-pass (max_points=4099) vs single pass")
    _, g1, _ = _run(fp, mesh, pts, dev, max_points=1 << 16)
    _, g2, _ = _run(fp, mesh, pts, dev, max_points=4099)
    for a, b in zip(g1, g2):
        assert np.array_equal(a, b)


def test_edge_cases(dev):
    fp = _fp()
    mesh = w.cube_c1()
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, max_points=256)
    _say("case: edge cases (empty, NaN, far, ragged sizes)")
    e = torch.empty((0, 3), dtype=torch.float64, device=dev)
    code, el, rst, d2 = fp.findpts(h, e)
    assert code.numel() == 0
    odd = torch.tensor([[np.nan, 0.5, 0.5], [0.5, np.inf, 0.5], [5.0, 0.5, 0.5],
                        [0.5, 0.5, -1e9], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0]],
                       dtype=torch.float64, device=dev)
    code, el, rst, d2 = fp.findpts(h, odd)
    c = code.cpu().numpy()
    assert list(c[:4]) == [2, 2, 2, 2] and list(c[4:]) == [0, 0]
    assert list(el.cpu().numpy()[:4]) == [-1] * 4
    assert np.all(np.isinf(d2.cpu().numpy()[:4]))
    vals = fp.findpts_eval(h, code, el, rst, [md.x])
    v = vals.cpu().numpy()[0]
    assert np.all(np.isnan(v[:4])) and abs(v[4]) <= 1e-15 and abs(v[5] - 1.0) <= 1e-15
    om = oracle.OracleMesh.from_mesh(mesh)
    _, hs = om.bbox()
    for n in (1, 63, 64, 65, 255, 256, 257, 1000):
        pts = w.queries_c1(n, seed=100 + n)
        code, el, rst, d2 = fp.findpts(h, pts.to(dev))
        g = (code.cpu().numpy(), el.cpu().numpy(), rst.cpu().numpy(), d2.cpu().numpy())
        compare_locate(om, pts.numpy(), g, om.findpts(pts.numpy()), hs, TOL)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 8, 9, 10, 11, 12, 13, 14, 15])
def test_orders(dev, N):
    fp = _fp()
    _say(f"case: order N={N}")
    mesh = w.annulus_mesh(2, 8, 2, N=N) if N >= 3 else w.cube_c1(perturb=0.0)
    if N < 3:
        mesh = w.box_mesh(3, 3, 2, lo=(-1, 0, 0), hi=(2, 1, 0.5), N=N)
    rng = np.random.default_rng(N)
    if N >= 3:
        rho = np.sqrt(rng.uniform(0.2, 1.2, 3000))
        th = rng.uniform(0, 2 * np.pi, 3000)
        pts = np.stack([rho * np.cos(th), rho * np.sin(th), rng.uniform(-0.05, 1.05, 3000)], 1)
    else:
        pts = rng.uniform((-1.1, -0.1, -0.1), (2.1, 1.1, 0.6), (3000, 3))
    pts = torch.as_tensor(pts)
    fields, _ = w.ref_poly_fields(mesh, 1, seed=N)
    h, g, out = _run(fp, mesh, pts, dev, fields=fields)
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    o = om.findpts(pts.numpy())
    _, hs = om.bbox()
    compare_locate(om, pts.numpy(), g, o, hs, TOL)
    ref = om.eval(g[0], g[1], g[2], [fields[0].numpy()])
    compare_eval(out, ref, [fields[0].numpy()], rel=1e-12)


def test_exact_recovery(dev):
    fp = _fp()
    _say("case: exact recovery through the analytic polynomial map")
    from helpers import box_affine, box_elem_ids, phi_np
    n = (3, 3, 3)
    mesh, _ = w.poly_map_mesh(*n, N=4, amp=0.04)
    ex, ey, ez = box_elem_ids(mesh.E, n)
    rng = np.random.default_rng(31)
    P = 5000
    et = rng.integers(0, mesh.E, P)
    rt = rng.uniform(-1, 1, (P, 3))
    a = np.array([box_affine(ex[e], ey[e], ez[e], n, (0, 0, 0), (1, 1, 1), r) for e, r in zip(et, rt)])
    pts = np.stack(phi_np(a[:, 0], a[:, 1], a[:, 2], amp=0.04), 1)
    h, g, _ = _run(fp, mesh, torch.as_tensor(pts), dev)
    gc, ge, gr, gd = g
    assert np.all(gc == 0)
    same = ge == et
    assert np.max(np.abs(gr[same] - rt[same])) <= 1e-11
    assert np.all(np.min(1 - np.abs(rt[~same]), axis=1) <= 1e-10)


def test_spiral_n15(dev):
    """The N = 15 spiral stand-in (Section 3.1): exact points x^e(r_true)
    are all found with r_true recovered, points between the turns match the
    oracle (both start Newton at the closest GLL node, so both settle in the
    same local minimum), and evaluating the coordinate fields at the returned
    (el, r) gives the points back.  At the paper's tolerance of 1e-14 (h_e
    relative) every exact point is found inside on both sides, with full
    parity and the GPU's residual, recomputed by the oracle's map, within
    tol h_e."""
    fp = _fp()
    from helpers import spiral_exact_points
    _say("case: spiral element N=15, 1000 exact + 1000 box + 16 far points")
    mesh = w.spiral_element()
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    b, hs = om.bbox()
    ex, rt = spiral_exact_points(mesh, 1000, 19)
    rng = np.random.default_rng(20)
    box = rng.uniform(b[0, 0::2], b[0, 1::2], (1000, 3))
    far = rng.uniform(-1, 1, (16, 3)) * 20.0 + 30.0
    pts = np.concatenate([ex, box, far])
    hd = mesh.host()
    coords = [mesh.x, mesh.y, mesh.z]
    h, g, out = _run(fp, mesh, torch.as_tensor(pts), dev, fields=coords)
    gc, ge, gr, gd = g
    st = compare_locate(om, pts, g, om.findpts(pts), hs, TOL)
    assert np.all(gc[:1000] == 0) and np.all(ge[:1000] == 0)
    assert np.max(np.abs(gr[:1000] - rt)) <= 1e-10
    assert np.all(gc[2000:] == 2)
    ins = gc == 0
    back = out.T[ins]
    assert np.max(np.abs(back - pts[ins])) <= 2 * TOL * hs[0]
    ref = om.eval(g[0], g[1], g[2], [hd[c] for c in "xyz"])
    compare_eval(out, ref, [hd[c] for c in "xyz"], rel=1e-13)
    _say(f"spiral tol 1e-12: {st}")
    tol = 1e-14
    h14, g14, _ = _run(fp, mesh, torch.as_tensor(ex), dev, tol=tol)
    om14 = oracle.OracleMesh.from_mesh(mesh, tol)
    oc = om14.findpts(ex)[0]
    gc, ge, gr, gd = g14
    assert np.array_equal(np.bincount(oc, minlength=3), [1000, 0, 0])
    assert np.array_equal(np.bincount(gc, minlength=3), [1000, 0, 0])
    assert np.all(ge == 0)
    assert np.max(np.abs(gr - rt)) <= 1e-11
    assert np.sqrt(gd).max() <= tol * hs[0]
    st14 = compare_locate(om14, ex, g14, om14.findpts(ex), hs, tol)
    _say(f"spiral tol 1e-14: {st14}")


def test_eval_reference_polynomials(dev):
    fp = _fp()
    _say("case: eval of reference-space polynomials, 3 fields, random (e, r)")
    mesh = w.annulus_mesh(3, 8, 2, N=7)
    fields, coef = w.ref_poly_fields(mesh, 3, seed=4)
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, max_points=5000)
    rng = np.random.default_rng(4)
    P = 4001
    el = torch.as_tensor(rng.integers(0, mesh.E, P).astype(np.int32))
    rst = torch.as_tensor(rng.uniform(-1, 1, (P, 3)))
    code = torch.zeros(P, dtype=torch.int32)
    out = fp.findpts_eval(h, code.to(dev), el.to(dev), rst.to(dev), [f.to(dev) for f in fields])
    out = out.cpu().numpy()
    a = np.arange(8)
    for f in range(3):
        for p in range(0, P, 13):
            c = coef[f, el[p]]
            r = rst[p].numpy()
            ref = np.einsum("cba,c,b,a->", c, r[2] ** a, r[1] ** a, r[0] ** a)
            assert abs(out[f, p] - ref) <= 1e-13 * np.abs(c).sum()


def test_three_sessions_delta(dev):
    fp = _fp()
    _say("case: three sessions with distance discriminator")
    boxes = [((0, 0, 0), (3, 1, 1)), ((0, 0, 0), (2, 1, 1)), ((1, 0, 0), (3, 1, 1))]
    ms = [w.box_mesh(1, 1, 1, lo, hi, N=2) for lo, hi in boxes]
    x = torch.cat([m.x for m in ms]); y = torch.cat([m.y for m in ms]); z = torch.cat([m.z for m in ms])
    delta = torch.cat([torch.full_like(ms[0].x, 100.0), 2.0 - ms[1].x, ms[2].x - 1.0])
    mesh = w.Mesh("three", 2, x, y, z, torch.tensor([0, 1, 2], dtype=torch.int32), delta)
    xs = np.array([0.5, 1.2, 1.4, 1.5, 1.6, 1.9, 2.5])
    pts = torch.as_tensor(np.stack([xs, np.full_like(xs, 0.3), np.full_like(xs, 0.7)], 1))
    for tag, ref in ((0, [1, 1, 1, 1, 2, 2, 2]), (1, [0] * 7), (-1, [0] * 7)):
        ps = torch.full((7,), tag, dtype=torch.int32)
        _, g, _ = _run(fp, mesh, pts, dev, psess=ps)
        assert list(g[0]) == [0] * 7 and list(g[1]) == ref, (tag, g[1])


def test_two_sessions_overlap_subset(dev):
    fp = _fp()
    _say("case: two overlapping sessions (box with hole + annulus), interface nodes")
    mesh = w.overlap_c3()
    pts, tags = w.c3_interface_nodes(mesh)
    rng = np.random.default_rng(3)
    idx = torch.as_tensor(np.sort(rng.choice(len(pts), 30_000, replace=False)))
    pts, tags = pts[idx].contiguous(), tags[idx].contiguous()
    h, g, _ = _run(fp, mesh, pts, dev, psess=tags)
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    o = om.findpts(pts.numpy(), tags.numpy())
    _, hs = om.bbox()
    st = compare_locate(om, pts.numpy(), g, o, hs, TOL, check_residual_every=3)
    sess = mesh.session.numpy()
    found = g[0] != 2
    assert np.all(sess[g[1][found]] != tags.numpy()[found])
    _say(f"two sessions ok {st}")


def _sampled(om, pts, g, idx, hs, psess=None, every=4):
    o = om.findpts(pts[idx], None if psess is None else psess[idx])
    return compare_locate(om, pts[idx], tuple(a[idx] for a in g), o, hs, TOL,
                          check_residual_every=every)


def _invariants(g, E):
    gc, ge, gr, gd = g
    assert np.all((gc >= 0) & (gc <= 2))
    assert np.all((ge >= -1) & (ge < E))
    assert np.all(np.abs(gr) <= 1.0)
    assert np.all((gc == 2) == np.isinf(gd))
    assert np.all((gc == 2) == (ge == -1))


def test_c5_large_box_full_size_sampled(dev):
    """200,000 curved elements of order 7, 2e7 points clustered near spheres,
    in one pass of 2e7 points (the benchmark's launch configuration); a seeded
    sample of 20,000 outputs against the oracle, whole-output invariants, and
    the mixed-precision path against binary64 on every point."""
    fp = _fp()
    _say("case: large box C5, 200,000 elements, 2e7 points, sampled parity")
    mesh = w.big_box_c5()
    pts = w.queries_c5()
    fields, _ = w.poly_fields(mesh.to(dev), 5, seed=5)  # on the device
    h, g, out = _run(fp, mesh, pts, dev, max_points=20_000_000, fields=fields)
    _invariants(g, mesh.E)
    rng = np.random.default_rng(55)
    idx = np.sort(rng.choice(len(pts), 20_000, replace=False))
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    _, hs = om.bbox()
    st = _sampled(om, pts.numpy(), g, idx, hs)
    assert st["inside"] > 0.8 * len(idx) and st["border"] + st["notfound"] > 0
    hf = [f.cpu().numpy() for f in fields]
    compare_eval(out[:, idx], om.eval(g[0][idx], g[1][idx], g[2][idx], hf), hf)
    assert np.array_equal(np.isnan(out[0]), g[0] == 2)
    del hf
    _say(f"c5 fp64 ok {st}")
    fp.findpts_set_precision(h, fp.FP_PREC_MIXED)
    code, el, rst, d2 = fp.findpts(h, pts.to(dev))
    torch.cuda.synchronize()
    gm = (code.cpu().numpy(), el.cpu().numpy(), rst.cpu().numpy(), d2.cpu().numpy())
    _invariants(gm, mesh.E)
    assert np.array_equal(gm[0], g[0])
    ties = gm[1] != g[1]
    assert np.all(np.min(1 - np.abs(gm[2][ties]), axis=1) <= 1e-10)
    st = _sampled(om, pts.numpy(), gm, idx, hs)
    _say(f"c5 mixed ok {st}, {int(ties.sum())} face ties vs fp64")
    h.free()


def test_c3_interface_faces_full_size_sampled(dev):
    """Two overlapping sessions, 1.2e6 points on the interface faces tagged
    with their session, one pass of 2^21 points; sampled parity (distance
    discriminator and session exclusion included) and invariants."""
    fp = _fp()
    _say("case: two sessions C3, 1.2e6 interface-face points, sampled parity")
    mesh = w.overlap_c3()
    pts, tags = w.queries_c3(n=1_200_000)
    fields, _ = w.poly_fields(mesh.to(dev), 5, seed=3)  # on the device
    h, g, out = _run(fp, mesh, pts, dev, max_points=1 << 21, psess=tags, fields=fields)
    _invariants(g, mesh.E)
    sess = mesh.session.numpy()
    found = g[0] != 2
    assert np.all(sess[g[1][found]] != tags.numpy()[found])
    rng = np.random.default_rng(33)
    idx = np.sort(rng.choice(len(pts), 20_000, replace=False))
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    _, hs = om.bbox()
    st = _sampled(om, pts.numpy(), g, idx, hs, psess=tags.numpy())
    hf = [f.cpu().numpy() for f in fields]
    compare_eval(out[:, idx], om.eval(g[0][idx], g[1][idx], g[2][idx], hf), hf)
    _say(f"c3 full ok {st}")
    h.free()


@pytest.mark.parametrize("N,prec", [(7, "fp64"), (7, "mixed"), (4, "fp64"), (9, "fp64"),
                                    (15, "fp64")])
def test_points_at_mesh_nodes(dev, N, prec):
    """Query points that are mesh nodes: Newton ends at its start node (the
    path that takes no matrix evaluation).  Every point is found inside, at
    distance 0, with r equal to a GLL node triple of the returned element,
    as in the oracle."""
    fp = _fp()
    _say(f"case: points at mesh nodes N={N} {prec}")
    mesh = w.annulus_mesh(2, 6, 2, N=N)
    hd = mesh.host()
    rng = np.random.default_rng(70 + N)
    idx = rng.choice(hd["x"].size, 3000, replace=False)
    pts = np.stack([hd["x"].reshape(-1)[idx], hd["y"].reshape(-1)[idx],
                    hd["z"].reshape(-1)[idx]], 1)
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, N, tol=TOL, max_points=4096,
                         precision=fp.FP_PREC_MIXED if prec == "mixed" else fp.FP_PREC_FP64)
    code, el, rst, d2 = fp.findpts(h, torch.as_tensor(pts).to(dev))
    torch.cuda.synchronize()
    g = (code.cpu().numpy(), el.cpu().numpy(), rst.cpu().numpy(), d2.cpu().numpy())
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    _, hs = om.bbox()
    compare_locate(om, pts, g, om.findpts(pts), hs, TOL)
    assert np.all(g[0] == 0)
    z = w.gll_points(N)
    assert np.all(np.min(np.abs(g[2][:, :, None] - z[None, None, :]), axis=2) <= 1e-12)
    h.free()


def test_points_at_mesh_nodes_2d(dev):
    fp = _fp()
    _say("case: 2D points at mesh nodes")
    m = w.annulus2d_mesh(3, 10, N=7)
    hd = m.host()
    rng = np.random.default_rng(77)
    idx = rng.choice(hd["x"].size, 1500, replace=False)
    pts = np.stack([hd["x"].reshape(-1)[idx], hd["y"].reshape(-1)[idx]], 1)
    md = m.to(dev)
    h = fp.findpts2_setup(md.x, md.y, m.N, tol=TOL)
    code, el, rs, d2 = fp.findpts2(h, torch.as_tensor(pts).to(dev))
    torch.cuda.synchronize()
    g = (code.cpu().numpy(), el.cpu().numpy(), rs.cpu().numpy(), d2.cpu().numpy())
    om = oracle.OracleMesh2.from_mesh(m, TOL)
    _, hs = om.bbox()
    compare_locate(om, pts, g, om.findpts(pts), hs, TOL)
    assert np.all(g[0] == 0)
    z = w.gll_points(7)
    assert np.all(np.min(np.abs(g[2][:, :, None] - z[None, None, :]), axis=2) <= 1e-12)
    h.free()
