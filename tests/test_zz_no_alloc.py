"""The interpolation entry point that allocates nothing, findpts_eval_noalloc
(its grouping arrays live in the library's per-GPU scratch array), against
findpts_eval on the same handle and inputs, called through the C ABI: two
calls in a row, the second with a smaller input.  The first call is larger
than one pass of the scratch array (about 4.19 million points), so it runs
in two passes.  Outputs are bit-identical to findpts_eval's (same kernels,
each point's value independent of its neighbours) and within 1e-13 max|F| of
the oracle (Section 2.1 interpolation)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as w
from parity import compare_eval

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _same(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(a[~np.isnan(a)],
                                                                       b[~np.isnan(b)])


def test_eval_noalloc_matches_eval():
    from paper_1811_04891_amd import findpts as fp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dev = torch.device("cuda:0")
    mesh = w.annulus_mesh(4, 16, 3, N=7)
    md = mesh.to(dev)
    fields = [f.to(dev) for f in w.poly_fields(mesh, 3, seed=13)[0]]
    hf = [f.cpu().numpy() for f in fields]
    om = oracle.OracleMesh.from_mesh(mesh, 1e-12)
    h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, tol=1e-12, max_points=1 << 17)

    # call 1: 4.5 million (element, r) pairs, 1 % not found: two passes
    _say("case: eval_noalloc, 4.5e6 points, 3 fields, N=7")
    rng = np.random.default_rng(14)
    P = 4_500_000
    el = rng.integers(0, mesh.E, P).astype(np.int32)
    rst = rng.uniform(-1, 1, (P, 3))
    code = np.zeros(P, np.int32)
    nf = rng.choice(P, P // 100, replace=False)
    code[nf], el[nf], rst[nf] = 2, -1, 0.0
    c_d, e_d, r_d = (torch.as_tensor(code).to(dev), torch.as_tensor(el).to(dev),
                     torch.as_tensor(rst).to(dev))
    ref = fp.findpts_eval(h, c_d, e_d, r_d, fields)
    out = torch.full((3, P), -7.0, dtype=torch.float64, device=dev)
    fp.findpts_eval_noalloc(h, c_d, e_d, r_d, fields, out)
    torch.cuda.synchronize()
    assert _same(out, ref)
    sub = slice(0, P, 9)
    compare_eval(out.cpu().numpy()[:, sub], om.eval(code[sub], el[sub], rst[sub], hf), hf)

    # call 2, smaller: located points of the annulus, 2 fields
    _say("case: eval_noalloc, 60001 located points, 2 fields")
    pts = w.queries_c2(n_in=60_000, seed=15)[:60_001].contiguous()
    cd, ed, rd, _ = fp.findpts(h, pts.to(dev))
    ref2 = fp.findpts_eval(h, cd, ed, rd, fields[:2])
    out2 = torch.full((2, pts.shape[0]), -7.0, dtype=torch.float64, device=dev)
    fp.findpts_eval_noalloc(h, cd, ed, rd, fields[:2], out2)
    torch.cuda.synchronize()
    assert _same(out2, ref2)
    g = (cd.cpu().numpy(), ed.cpu().numpy(), rd.cpu().numpy())
    compare_eval(out2.cpu().numpy(), om.eval(*g, hf[:2]), hf[:2])
    assert np.any(g[0] == 2) and np.any(g[0] == 0)
    _say("eval_noalloc ok")
    h.free()
