"""GPU parity of the interface-data calls (mass-flux correction, time
extrapolation) against the oracle, on a box surface with exact quadrature and
on the two-session interface with velocities interpolated by findpts_eval."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as w
from helpers import box_surface
from oracle.interface import extrapolate, flux_correct

pytestmark = pytest.mark.gpu


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


def _t(a, dev, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev)


def test_flux_correct_box_closed_form(dev):
    fp = _fp()
    _say("case: flux correction on a box surface, u = (x, 0, 0)")
    x, wq, n = box_surface((0, 0, 0), (1, 2, 3), N=5)
    u = np.stack([x[0], np.zeros_like(x[0]), np.zeros_like(x[0])])
    for iface in (np.ones(wq.size, bool), n[0] > 0.5):
        g_o, u_o = flux_correct(wq, n, iface, u)
        ug = _t(u, dev)
        work = fp.fp_flux_correct(_t(wq, dev), _t(n, dev), ug,
                                  iface=_t(iface.astype(np.int32), dev, torch.int32))
        torch.cuda.synchronize()
        g = float(work[0].cpu())
        assert abs(g - g_o) <= 1e-14 * abs(g_o)
        assert np.max(np.abs(ug.cpu().numpy() - u_o)) <= 1e-14
    # iface = NULL means every point
    ug = _t(u, dev)
    work = fp.fp_flux_correct(_t(wq, dev), _t(n, dev), ug)
    assert abs(float(work[0].cpu()) + 6.0 / 22.0) <= 1e-14


def test_flux_correct_two_session_interface(dev):
    fp = _fp()
    _say("case: interface velocities interpolated by findpts_eval, then corrected")
    mesh = w.overlap_c3()
    pts, tags, nrm, wts = w.c3_interface_quadrature(mesh)
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, mesh.N, tol=1e-12, elem_session=md.session,
                         delta=md.delta, max_points=1 << 17)
    vel, _ = w.poly_fields(mesh, 3, degree=3, seed=21)
    code, el, rst, d2 = fp.findpts(h, pts.to(dev), tags.to(dev))
    u = fp.findpts_eval(h, code, el, rst, [f.to(dev) for f in vel])
    torch.cuda.synchronize()
    assert int((code == 2).sum()) == 0
    # points of each session contiguous, so that a session is a column slice
    order = torch.argsort(tags, stable=True)
    pts, tags, nrm, wts = pts[order], tags[order], nrm[:, order], wts[order]
    code, el, rst, d2 = fp.findpts(h, pts.to(dev).contiguous(), tags.to(dev))
    u = fp.findpts_eval(h, code, el, rst, [f.to(dev) for f in vel])
    torch.cuda.synchronize()
    n0 = int((tags == 0).sum())
    for tag, sl in ((0, slice(0, n0)), (1, slice(n0, len(tags)))):
        us = u[:3, sl]                    # a strided view of the eval output
        assert us.stride(0) == u.shape[1]
        ns, ws = nrm[:, tags == tag].contiguous(), wts[tags == tag].contiguous()
        u_host = us.cpu().numpy()
        g_o, u_o = flux_correct(ws.numpy(), ns.numpy(), np.ones(ws.numel(), bool), u_host)
        w1 = fp.fp_flux_correct(ws.to(dev), ns.to(dev), us)
        g1 = float(w1[0].cpu())
        # the two sides sum in different orders: the flux, a sum with
        # cancellation, agrees to a few ulps of sum |w u.n| (a sequential sum
        # of P terms is within P eps of it), gamma to that over the area
        abs_flux = float(np.sum(ws.numpy() * np.abs(np.sum(u_host * ns.numpy(), axis=0))))
        area = float(np.sum(ws.numpy()))
        tol_g = 1e-12 * abs_flux / area
        assert abs(g1 - g_o) <= tol_g
        assert np.max(np.abs(us.cpu().numpy() - u_o)) <= tol_g + 1e-15 * np.max(np.abs(u_o))
        flux = float(np.sum(ws.numpy() * np.sum(us.cpu().numpy() * ns.numpy(), axis=0)))
        scale = float(np.sum(ws.numpy() * np.abs(u_host).sum(axis=0)))
        assert abs(flux) <= 1e-13 * scale
        # the same sums give the same bits, also on a contiguous copy
        us2 = _t(u_host, dev)
        w2 = fp.fp_flux_correct(ws.to(dev), ns.to(dev), us2)
        assert float(w2[0].cpu()) == g1
        _say(f"session {tag}: gamma {g1:.6e} (oracle {g_o:.6e})")
    h.free()


@pytest.mark.parametrize("m", [1, 2, 3])
def test_extrapolate(dev, m):
    fp = _fp()
    rng = np.random.default_rng(30 + m)
    hist = [rng.standard_normal(100_003) for _ in range(m)]
    out = fp.fp_extrapolate([_t(a, dev) for a in hist], m)
    ref = extrapolate(hist, m)
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-15 * 4 * np.max(np.abs(ref))
