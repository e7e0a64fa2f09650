"""GPU parity of the two-dimensional path (findpts2 / findpts2_eval through
the C ABI) against the 2D CPU oracle on the same seeded inputs: boxes,
orders 1..15, exact recovery through a polynomial map, two sessions with
the distance discriminator and session exclusion, interpolation, chunked
passes, empty and far-away inputs, and the 1.01M-point ring workload on a
sample."""
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


def _run(fp, m, pts, dev, psess=None, fields=(), max_points=1 << 16, tol=TOL):
    md = m.to(dev)
    h = fp.findpts2_setup(md.x, md.y, m.N, tol=tol, elem_session=md.session, delta=md.delta,
                          max_points=max_points)
    ps = None if psess is None else torch.as_tensor(psess, dtype=torch.int32).to(dev)
    code, el, rs, d2 = fp.findpts2(h, torch.as_tensor(pts).to(dev).contiguous(), ps)
    out = None
    if fields:
        out = fp.findpts2_eval(h, code, el, rs, [f.to(dev).contiguous() for f in fields])
    torch.cuda.synchronize()
    g = (code.cpu().numpy(), el.cpu().numpy(), rs.cpu().numpy(), d2.cpu().numpy())
    return h, g, (None if out is None else out.cpu().numpy())


def _ring_points(rng, n, a=0.15, b=1.3):
    rho = np.sqrt(rng.uniform(a, b, n))
    th = rng.uniform(0, 2 * np.pi, n)
    return np.stack([rho * np.cos(th), rho * np.sin(th)], 1)


def _fields(m, seed):
    rng = np.random.default_rng(seed)
    c = rng.normal(size=6)
    x, y = m.x, m.y
    return [c[0] + c[1] * x + c[2] * y * y + c[3] * x * y ** 3 + c[4] * x ** 5,
            torch.sin(3 * x) * torch.cos(2 * y) + c[5]]


def test_boxes_match_oracle(dev):
    fp = _fp()
    for m in (w.annulus2d_mesh(4, 20, N=7), w.poly_map_mesh2d(5, 4, N=3)[0]):
        _say(f"case: 2D boxes {m.name} E={m.E}")
        md = m.to(dev)
        h = fp.findpts2_setup(md.x, md.y, m.N, max_points=16)
        gb, gh = fp.findpts2_get_bbox(h)
        ob, oh = oracle.OracleMesh2.from_mesh(m).bbox()
        scale = np.abs(ob).max()
        assert np.max(np.abs(gb - ob)) <= 1e-13 * scale
        assert np.max(np.abs(gh - oh)) <= 1e-14 * scale
        h.free()


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_orders_ring(dev, N):
    fp = _fp()
    _say(f"case: 2D ring N={N}")
    m = w.annulus2d_mesh(3, 16, N=N)
    rng = np.random.default_rng(100 + N)
    pts = _ring_points(rng, 4000)
    fl = _fields(m, N)
    h, g, out = _run(fp, m, pts, dev, fields=fl)
    om = oracle.OracleMesh2.from_mesh(m, TOL)
    _, hs = om.bbox()
    st = compare_locate(om, pts, g, om.findpts(pts), hs, TOL)
    assert st["inside"] > 1000 and st["border"] > 100 and st["notfound"] > 100
    fln = [f.numpy() for f in fl]
    compare_eval(out, om.eval(g[0], g[1], g[2], fln), fln, rel=1e-12)
    pairs, iters, cands = fp.findpts2_stats(h)
    assert cands == om.last_stats[0]  # the method's candidate sets (hash + boxes)
    assert pairs <= 2 * cands  # a candidate is solved at most once per round
    _say(f"N={N} ok {st}, pairs/cand {pairs / max(cands, 1):.3f}, "
         f"iters/pair {iters / max(pairs, 1):.2f}")


def test_exact_recovery(dev):
    fp = _fp()
    _say("case: 2D exact recovery through a polynomial map")
    n = (6, 5)
    m, phi = w.poly_map_mesh2d(*n, N=4, amp=0.04)
    rng = np.random.default_rng(31)
    P = 20000
    et = rng.integers(0, m.E, P)
    rt = rng.uniform(-1, 1, (P, 2))
    ex, ey = et % n[0], et // n[0]
    a = np.stack([(ex + (rt[:, 0] + 1) / 2) / n[0], (ey + (rt[:, 1] + 1) / 2) / n[1]], 1)
    pts = np.stack(phi(a[:, 0], a[:, 1]), 1)
    h, g, _ = _run(fp, m, pts, dev)
    gc, ge, gr, gd = g
    assert np.all(gc == 0)
    same = ge == et
    assert np.max(np.abs(gr[same] - rt[same])) <= 1e-11
    assert np.all(np.min(1 - np.abs(rt[~same]), axis=1) <= 1e-10)


def test_two_sessions(dev):
    fp = _fp()
    _say("case: 2D two sessions with the distance field, tagged and untagged points")
    m = w.overlap2d(N=7)
    om = oracle.OracleMesh2.from_mesh(m, TOL)
    _, hs = om.bbox()
    rng = np.random.default_rng(41)
    pts = rng.uniform(-1.8, 1.8, (30000, 2))
    ps = rng.integers(-1, 2, len(pts)).astype(np.int32)
    for tags in (None, ps):
        h, g, _ = _run(fp, m, pts, dev, psess=tags)
        st = compare_locate(om, pts, g, om.findpts(pts, psess=tags), hs, TOL)
        _say(f"sessions {'tagged' if tags is not None else 'untagged'}: {st}")
        h.free()


def test_chunked_edge_cases(dev):
    fp = _fp()
    _say("case: 2D passes of 1000 points = one pass; empty call; far points")
    m = w.annulus2d_mesh(4, 24, N=5)
    rng = np.random.default_rng(51)
    pts = _ring_points(rng, 5003)
    _, g1, _ = _run(fp, m, pts, dev, max_points=1000)
    _, g2, _ = _run(fp, m, pts, dev, max_points=1 << 14)
    for a, b in zip(g1, g2):
        assert np.array_equal(a, b)
    md = m.to(dev)
    h = fp.findpts2_setup(md.x, md.y, m.N)
    e = torch.empty((0, 2), dtype=torch.float64, device=dev)
    code, el, rs, d2 = fp.findpts2(h, e)
    assert code.numel() == 0
    far = torch.tensor([[50.0, 0.0], [0.0, -7.5], [float("nan"), 0.0]], dtype=torch.float64,
                       device=dev)
    code, el, rs, d2 = fp.findpts2(h, far)
    out = fp.findpts2_eval(h, code, el, rs, [md.x])
    torch.cuda.synchronize()
    assert code.tolist() == [2, 2, 2] and el.tolist() == [-1, -1, -1]
    assert torch.all(torch.isinf(d2)) and torch.all(torch.isnan(out))


def test_ring_c6_full_size_sampled(dev):
    fp = _fp()
    _say("case: 2D ring 16,384 elements N=7, 1.01M points, 2 fields, sampled")
    m = w.annulus2d_c6()
    pts = w.queries2d_c6()
    fl = _fields(m, 7)
    h, g, out = _run(fp, m, pts.numpy(), dev, fields=fl, max_points=1 << 20)
    gc, ge, gr, gd = g
    # invariants on all points
    assert set(np.unique(gc)) <= {0, 1, 2}
    assert np.all((ge >= 0) == (gc != 2)) and np.all(ge < m.E)
    assert np.all(np.abs(gr) <= 1.0)
    rho = np.hypot(pts[:, 0].numpy(), pts[:, 1].numpy())
    assert np.all(gc[(rho > 0.5 + 1e-9) & (rho < 1 - 1e-9)] == 0)
    # the oracle on a sample
    idx = np.random.default_rng(61).choice(len(pts), 20000, replace=False)
    om = oracle.OracleMesh2.from_mesh(m, TOL)
    _, hs = om.bbox()
    sp = pts.numpy()[idx]
    st = compare_locate(om, sp, tuple(a[idx] for a in g), om.findpts(sp), hs, TOL)
    fln = [f.numpy() for f in fl]
    compare_eval(out[:, idx], om.eval(gc[idx], ge[idx], gr[idx], fln), fln, rel=1e-12)
    _say(f"c6 sample ok {st}")
