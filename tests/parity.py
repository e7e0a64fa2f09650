"""Parity rules between the GPU findpts path and the CPU oracle.

For each point (these are readings of points the paper leaves open):
* not found (code 2): both sides say so, el = -1, dist2 = +inf.
* inside (code 0): same code; same element, or, if the elements differ, the
  point lies on a shared face (1 - |r_d| <= 1e-10 on both sides) and both
  residuals pass; |r_gpu - r_oracle|_inf <= R_TOL when the elements agree;
  the GPU's own residual ||x^e(r_gpu) - x*||, recomputed by the oracle's
  map, is <= tol * h_e.
* a code 0 / code 1 flip is accepted only inside the band
  |sqrt(d2) - tol h_e| <= 1e-3 tol h_e.
* border (code 1): dist2 agrees to 1e-9 relative plus eps (2 d + eps), with
  d = sqrt(dist2) and eps = 1e-13 h: each side's binary64 map carries an
  absolute error of order eps, so two distances d may differ by eps and their
  squares by eps (2 d + eps), which exceeds the relative term for points
  closer than about 1e-4 h to the face; if the elements differ, the oracle's
  own Newton on the GPU's element must reach the same distance (a tie between
  local minima).
Integer outputs (code, el) are compared exactly outside these cases.
"""
import numpy as np

R_TOL = 1e-10
FACE_TOL = 1e-10


def compare_locate(om, pts, gpu, ora, h, tol, max_report=5, check_residual_every=1):
    gc, ge, gr, gd = gpu
    oc, oe, orr, od = ora
    pts = np.asarray(pts).reshape(len(gc), -1)  # 3D (x y z) or 2D (x y) points
    bad = []
    n = len(gc)
    # not found
    nf = (oc == 2) | (gc == 2)
    for i in np.nonzero(nf & ~((oc == 2) & (gc == 2)))[0]:
        bad.append((i, "not-found mismatch", gc[i], oc[i]))
    ok2 = (oc == 2) & (gc == 2)
    if np.any(ge[ok2] != -1) or np.any(~np.isinf(gd[ok2])) or np.any(gr[ok2] != 0):
        bad.append((-1, "not-found outputs", None, None))
    # code flips
    flip = (oc != gc) & ~nf
    for i in np.nonzero(flip)[0]:
        e = oe[i]
        band = abs(np.sqrt(od[i]) - tol * h[e]) <= 1e-3 * tol * h[e]
        if not band:
            bad.append((i, "code flip", gc[i], oc[i]))
    # inside
    ins = (oc == 0) & (gc == 0)
    same = ins & (ge == oe)
    if np.any(same):
        dr = np.max(np.abs(gr[same] - orr[same]), axis=1)
        for i in np.nonzero(same)[0][dr > R_TOL]:
            bad.append((i, "rst", np.abs(gr[i] - orr[i]).max(), R_TOL))
    for i in np.nonzero(ins & (ge != oe))[0]:
        on_face = (np.min(1 - np.abs(gr[i])) <= FACE_TOL and
                   np.min(1 - np.abs(orr[i])) <= FACE_TOL)
        if not on_face:
            bad.append((i, "inside element differs off a face", ge[i], oe[i]))
    idx = np.nonzero(gc == 0)[0][::check_residual_every]
    for i in idx:
        x, _ = om.map(ge[i], gr[i])
        res = np.linalg.norm(x - pts[i])
        if not res <= tol * h[ge[i]]:
            bad.append((i, "gpu residual", res, tol * h[ge[i]]))
    # border
    bor = (oc == 1) & (gc == 1)
    for i in np.nonzero(bor)[0]:
        e = oe[i]
        eps = 1e-13 * h[e]
        floor = eps * (2.0 * np.sqrt(od[i]) + eps)
        if abs(gd[i] - od[i]) > 1e-9 * od[i] + floor:
            if ge[i] != oe[i]:
                _, d2o, _ = om.newton(ge[i], pts[i])
                if abs(d2o - od[i]) <= 1e-8 * od[i] + floor:
                    continue
            bad.append((i, "border dist2", gd[i], od[i]))
        elif ge[i] != oe[i]:
            _, d2o, _ = om.newton(ge[i], pts[i])
            if abs(d2o - od[i]) > 1e-8 * od[i] + floor:
                bad.append((i, "border element", ge[i], oe[i]))
    if bad:
        msg = "; ".join(str(b) for b in bad[:max_report])
        raise AssertionError(f"{len(bad)} parity failures of {n}: {msg}")
    return {"n": n, "inside": int(np.sum(gc == 0)), "border": int(np.sum(gc == 1)),
            "notfound": int(np.sum(gc == 2)),
            "elem_face_ties": int(np.sum(ins & (ge != oe))),
            "max_dr": float(np.max(np.abs(gr[same] - orr[same]))) if np.any(same) else 0.0}


# Mixed-precision interpolation (orders up to 7) accumulates in binary32:
# three sum-factorised contractions of n1 <= 8 terms, each within
# gamma_8 sum|terms| <= 8 u Lambda max|input| (u = 2^-24, Lambda = the GLL
# Lebesgue constant, 1.97 at N = 7), plus the binary32 rounding of the nodal
# values and of the basis values: at most (3 * 8 + 4) u Lambda^3 max|F| =
# 1.3e-5 max|F|.
MIXED_EVAL_REL = 2e-5


def compare_eval(gpu_out, ref_out, fields, rel=1e-13):
    """|f_gpu - f_ref| <= rel * max|F| per field; NaN exactly where the
    reference is NaN."""
    g, r = np.asarray(gpu_out), np.asarray(ref_out)
    assert g.shape == r.shape
    nan_r = np.isnan(r)
    assert np.array_equal(np.isnan(g), nan_r), "NaN pattern differs"
    for f in range(g.shape[0]):
        scale = float(np.max(np.abs(np.asarray(fields[f]))))
        err = np.max(np.abs(g[f][~nan_r[f]] - r[f][~nan_r[f]])) if np.any(~nan_r[f]) else 0.0
        assert err <= rel * scale, (f, err, rel * scale)
