"""GPU tests of the serving layer (fps_*): requests on several resident
meshes of different size and order, run concurrently on the serving streams,
give bit-identical results to the same request run alone through findpts +
findpts_eval; a small HBM budget forces admission to wait; a sample of served
results matches the CPU oracle."""
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


@pytest.fixture(scope="module")
def served(dev):
    """Four meshes (boxes and annuli, N = 9, 7, 7, 7; E from 125 to 1980;
    N = 9 runs the non-matrix-core Newton kernel) with 3 fields each."""
    fp = _fp()
    ms = w.serving_meshes(count=4, e_min=100, e_max=2000, nfields=3, device=dev)
    handles = []
    for m in ms:
        md = m.mesh
        handles.append(fp.findpts_setup(md.x, md.y, md.z, md.N, tol=TOL, max_points=4096))
    torch.cuda.synchronize()
    return ms, handles


def _requests(ms, n, seed, p_max=30_000, p_min=1):
    rq = w.serving_requests(n, len(ms), p_min=p_min, p_max=p_max, nf_max=3, seed=seed)
    rng = np.random.default_rng(seed)
    for r in rq:
        if rng.random() < 0.2:
            r["field_ids"] = []  # findpts only
    return rq


def _alone(fp, h, fields, pts, fids):
    code, el, rst, d2 = fp.findpts(h, pts)
    out = fp.findpts_eval(h, code, el, rst, [fields[i] for i in fids]) if fids else None
    torch.cuda.synchronize()
    return code, el, rst, d2, out


def _same(a, b):
    for x, y in zip(a, b):
        if x is None or y is None:
            assert x is None and y is None
            continue
        assert torch.equal(torch.isnan(x), torch.isnan(y))
        assert torch.equal(torch.nan_to_num(x, nan=0.0), torch.nan_to_num(y, nan=0.0))


def test_serving_alone_vs_mix(dev, served):
    fp = _fp()
    ms, handles = served
    _say("case: 49 requests on 4 meshes, 4 slots, all submitted at once")
    srv = fp.Server(1 << 30, slots=4)
    ids = [srv.add_mesh(h, m.fields) for h, m in zip(handles, ms)]
    rq = _requests(ms, 48, seed=41)
    # a large first request keeps its slot busy while the next ones arrive
    rq.insert(0, {"mesh": 1, "P": 400_000, "field_ids": [0, 1, 2], "seed": 9})
    pts = [w.serving_points(ms[r["mesh"]].kind, r["P"], r["seed"], dev) for r in rq]
    torch.cuda.synchronize()
    reqs = [srv.submit(ids[r["mesh"]], p, r["field_ids"]) for r, p in zip(rq, pts)]
    for q in reqs:
        assert srv.wait(q, 60.0) == fp.FP_OK
    lat = srv.latency()
    _say(f"mix: {lat}")
    assert lat["completed"] == len(rq) and lat["waiting"] == 0 and lat["running"] == 0
    assert 0 < lat["p50_s"] <= lat["p99_s"]
    assert lat["peak_concurrent"] >= 2  # their work overlapped on the device
    for r, p, q in zip(rq, pts, reqs):
        m = ms[r["mesh"]]
        ref = _alone(fp, handles[r["mesh"]], m.fields, p, r["field_ids"])
        _same((q.code, q.el, q.rst, q.dist2, q.out), ref)
    srv.destroy()


def test_serving_matches_oracle(dev, served):
    fp = _fp()
    ms, handles = served
    _say("case: served results vs the CPU oracle, 3 requests")
    srv = fp.Server(1 << 28, slots=2)
    ids = [srv.add_mesh(h, m.fields) for h, m in zip(handles, ms)]
    for k, mi in enumerate((0, 1, 3)):
        m = ms[mi]
        pts = w.serving_points(m.kind, 3001 + k, 77 + k, dev)
        # a few points outside the domain: border and not-found answers
        pts[:20] = pts[:20] * 1.3 + 0.05
        torch.cuda.synchronize()
        q = srv.submit(ids[mi], pts, [0, 2])
        assert srv.wait(q) == fp.FP_OK
        om = oracle.OracleMesh.from_mesh(m.mesh.to("cpu"), TOL)
        _, hs = om.bbox()
        g = (q.code.cpu().numpy(), q.el.cpu().numpy(), q.rst.cpu().numpy(), q.dist2.cpu().numpy())
        compare_locate(om, pts.cpu().numpy(), g, om.findpts(pts.cpu().numpy()), hs, TOL)
        fl = [m.fields[0].cpu().numpy(), m.fields[2].cpu().numpy()]
        compare_eval(q.out.cpu().numpy(), om.eval(g[0], g[1], g[2], fl), fl)
    srv.destroy()


def test_serving_small_budget_waits(dev, served):
    fp = _fp()
    ms, handles = served
    _say("case: HBM budget of about one request workspace: admission waits")
    # the workspace of the largest request alone (one pass), plus a little;
    # requests of 50,000..200,000 points run longer on the GPU than the host
    # takes to submit the next, so their workspaces would overlap in time
    rq = _requests(ms, 24, seed=42, p_max=200_000, p_min=50_000)
    big = max(rq, key=lambda r: r["P"])
    probe = fp.Server(1 << 30, slots=1)
    pid = [probe.add_mesh(h, m.fields) for h, m in zip(handles, ms)]
    p = w.serving_points(ms[big["mesh"]].kind, big["P"], big["seed"], dev)
    torch.cuda.synchronize()
    q = probe.submit(pid[big["mesh"]], p, big["field_ids"])
    probe.wait(q)
    need = probe.latency()["peak_arena_bytes"]
    probe.destroy()
    budget = int(need * 1.2)
    srv = fp.Server(budget, slots=4)
    ids = [srv.add_mesh(h, m.fields) for h, m in zip(handles, ms)]
    pts = [w.serving_points(ms[r["mesh"]].kind, r["P"], r["seed"], dev) for r in rq]
    torch.cuda.synchronize()
    reqs = [srv.submit(ids[r["mesh"]], pp, r["field_ids"]) for r, pp in zip(rq, pts)]
    for qq in reqs:
        assert srv.wait(qq, 60.0) == fp.FP_OK
    lat = srv.latency()
    _say(f"small budget {budget}: {lat}")
    assert lat["completed"] == len(rq)
    assert lat["peak_arena_bytes"] <= budget
    assert lat["waited_admissions"] > 0
    for r, pp, qq in zip(rq, pts, reqs):
        ref = _alone(fp, handles[r["mesh"]], ms[r["mesh"]].fields, pp, r["field_ids"])
        _same((qq.code, qq.el, qq.rst, qq.dist2, qq.out), ref)
    # a request whose smallest pass does not fit is refused at submission
    tiny = fp.Server(4096, slots=1)
    tid = tiny.add_mesh(handles[0], ms[0].fields)
    with pytest.raises(fp.FindptsError) as ei:
        tiny.submit(tid, pts[0], [0])
    assert ei.value.code == fp.FP_ENOMEM
    tiny.destroy()
    srv.destroy()


def test_serving_wait_timeout_and_reset(dev, served):
    fp = _fp()
    ms, handles = served
    _say("case: wait with a zero timeout on a queued request, then complete")
    m = ms[1]
    pts = w.serving_points(m.kind, 200_000, 5, dev)
    torch.cuda.synchronize()
    srv = fp.Server(1 << 30, slots=1)
    mid = srv.add_mesh(handles[1], m.fields)
    a = srv.submit(mid, pts, [0, 1, 2])
    b = srv.submit(mid, pts[:1000].contiguous(), [1])
    # with one slot, b cannot start before a has finished its 200,000 points
    assert srv.wait(b, 0.0) == fp.FP_EBUSY
    assert srv.wait(a) == fp.FP_OK and srv.wait(b) == fp.FP_OK
    with pytest.raises(fp.FindptsError):
        srv.wait(b)  # a ticket is waited for once
    lat = srv.latency(reset=True)
    assert lat["completed"] == 2 and lat["points_per_s"] > 0
    assert srv.latency()["completed"] == 0
    e = srv.submit(mid, pts[:0].contiguous(), [0])  # empty request
    assert srv.wait(e) == fp.FP_OK
    srv.destroy()
