"""Benchmark: points located + interpolated per second on one MI355X.

Headline workload (one step = findpts + findpts_eval of every query point):
the large box, 200,000 sine-perturbed hexahedra of order 7 (100 x 50 x 40
on [0,2] x [0,1] x [0,0.8], 68.6 M unique GLL points), 2e7 query points
clustered near 8 random interior spheres (normal offsets N(0, 0.01^2), in
random order; points outside the domain kept), 5 float64 fields given as
random polynomials of total degree 7, in one pass of 2e7 points.  All inputs
are synthetic, seeded, built on the device and resident in HBM before timing
starts.  Both precisions are timed; --precision picks the headline one.

Prints one JSON line.  Besides the throughput it reports:
  roofline      the first-pass Newton (locate) kernel of the headline
                precision: algorithmic flops per launch / its mean duration
                (HIP events the library records on the launch stream) vs
                78.6 TFLOP/s; HBM bytes per launch from the committed
                hardware-counter summary when it was taken on this source
  cpu_baseline  the CPU oracle timed on a bounded sample of the same points
  legs          the other workloads: the annulus (16,384 elements, 1.01e6
                points, 4 fields) in both precisions plus a moving-mesh
                re-setup, the unit cube (64 elements, 1e4 points, 1 field),
                the two overlapping sessions with 1.2e6 interface-face points
                (4 fields) in both precisions, the N = 15 spiral at tol 1e-14,
                the Schwarz interface exchange, the two-dimensional ring, and
                a serving stream on 16 resident meshes (saturated throughput
                and p50/p99 latency at 0.5, 0.8 and 0.95 of it)
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBPS = 8000.0


def locate_flops_per_point(N, c, K):
    """Algorithmic float64 flops of one point's location: per candidate, the
    closest-node scan (7V), K Newton iterations each evaluating the map and
    its Jacobian by sum factorisation (12V + 18 n1^2 + 24 n1) and one final
    map evaluation (6 (V + n1^2 + n1))."""
    n1 = N + 1
    V = n1 ** 3
    return c * (7 * V + K * (12 * V + 18 * n1 ** 2 + 24 * n1) + 6 * (V + n1 ** 2 + n1))


def eval_flops_per_point(N, nf):
    n1 = N + 1
    return nf * 2 * (n1 ** 3 + n1 ** 2 + n1)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fp_locate.hip", "fp_mfma.inc", "fp_newton8.inc", "fp_mixed8.inc",
              "fp_newton_pl.inc", "fp_mfma.h", "fp_basis.h", "fp_internal.h"):
        with open(os.path.join(ROOT, "paper_1811_04891_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_profile(name):
    """Key: value pairs of a committed rocprofv3 counter summary under
    profiles/, if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    return vals


def cpu_baseline(mesh, pts, fields, desc, target_s=10.0, psess=None):
    """The oracle (plain C double, OpenMP over points) on the first n points
    of the workload, n sized from a probe so that the timed call takes about
    target_s on all host threads; also one core on 20,000 of them."""
    import numpy as np

    import oracle
    om = oracle.OracleMesh.from_mesh(mesh, 1e-12)
    nthreads = len(os.sched_getaffinity(0))
    cores = oracle.threads(nthreads)
    p = pts.cpu().numpy()
    ps = None if psess is None else psess.cpu().numpy()
    probe_n = min(len(p), 50_000)
    t = time.perf_counter()
    om.findpts(p[:probe_n], None if ps is None else ps[:probe_n], nthreads=nthreads)
    dt = time.perf_counter() - t
    n = int(min(len(p), max(probe_n, probe_n * target_s / max(dt, 1e-3))))
    sample = p[:n]
    sps = None if ps is None else ps[:n]
    hf = [f.cpu().numpy() for f in fields]
    t = time.perf_counter()
    code, el, rst, _ = om.findpts(sample, sps, nthreads=nthreads)
    om.eval(code, el, rst, hf, nthreads=nthreads)
    t_loc = time.perf_counter() - t
    c = om.last_stats[0] / n
    K = om.last_stats[1] / max(om.last_stats[0], 1)
    n1 = min(n, 20_000)
    t = time.perf_counter()
    c1, e1, r1, _ = om.findpts(sample[:n1], None if sps is None else sps[:n1], nthreads=1)
    om.eval(c1, e1, r1, hf, nthreads=1)
    t1 = time.perf_counter() - t
    oracle.threads(nthreads)
    return {"value": n / t_loc, "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} of the {len(p)} query points of {desc}, findpts + "
                      f"findpts_eval of the {len(fields)} fields (plain C double, OpenMP), "
                      f"{t_loc:.1f} s",
            "method_candidates_per_point": c, "method_newton_iters_per_candidate": K,
            "one_core_points_per_s": n1 / t1}


def serving_bench(fp, w, dev, precision, n_req, n_warm, slots=4, seed=40):
    """Serving stream: 16 resident meshes (E log-uniform in 500..50,000,
    N in {5, 7, 9}, 5 fields each), requests of 1e3..1e6 points (log-uniform)
    with 1..5 fields, Poisson arrivals at 0.5, 0.8 and 0.95 of the saturated
    request rate.  Returns p50/p99 latency per arrival rate."""
    import numpy as np
    import torch

    t0 = time.perf_counter()
    ms = w.serving_meshes(count=16, device=dev)
    handles = []
    for m in ms:
        md = m.mesh
        handles.append(fp.findpts_setup(md.x, md.y, md.z, md.N, tol=1e-12, max_points=4096,
                                        precision=precision))
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(0.8 * free, 64 << 30))
    srv = fp.Server(budget, slots=slots)
    ids = [srv.add_mesh(h, m.fields) for h, m in zip(handles, ms)]
    rq = w.serving_requests(n_warm + n_req, len(ms), seed=seed)
    pts, outs = [], []
    for r in rq:
        p = w.serving_points(ms[r["mesh"]].kind, r["P"], r["seed"], dev)
        P, nf = r["P"], len(r["field_ids"])
        pts.append(p)
        outs.append((torch.empty(P, dtype=torch.int32, device=dev),
                     torch.empty(P, dtype=torch.int32, device=dev),
                     torch.empty((P, 3), dtype=torch.float64, device=dev),
                     torch.empty(P, dtype=torch.float64, device=dev),
                     torch.empty((nf, P), dtype=torch.float64, device=dev)))
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    mean_p = float(np.mean([r["P"] for r in rq[n_warm:]]))
    print(f"# serving: {len(ms)} meshes, E total {sum(m.mesh.E for m in ms)}, "
          f"{len(rq)} requests, mean {mean_p:.0f} points, generated in {gen_s:.1f} s",
          file=sys.stderr, flush=True)

    def run(rate):
        # warm-up requests back to back, then the measured ones at `rate`
        # requests/s (None: all at once)
        for i in range(n_warm):
            srv.wait(srv.submit(ids[rq[i]["mesh"]], pts[i], rq[i]["field_ids"], out=outs[i]))
        srv.latency(reset=True)
        t = time.perf_counter()
        tickets = []
        for i in range(n_warm, len(rq)):
            if rate is not None:
                t += rq[i]["gap"] / rate
                while True:
                    d = t - time.perf_counter()
                    if d <= 0:
                        break
                    time.sleep(min(d, 2e-4) if d > 5e-4 else 0)
            tickets.append(srv.submit(ids[rq[i]["mesh"]], pts[i], rq[i]["field_ids"],
                                      out=outs[i]))
        for q in tickets:
            srv.wait(q)
        return srv.latency(reset=True)

    sat = run(None)
    R = sat["points_per_s"] / mean_p
    levels = []
    for frac in (0.5, 0.8, 0.95):
        lat = run(frac * R)
        levels.append({"rate_frac": frac, "requests_per_s": frac * R,
                       "p50_ms": lat["p50_s"] * 1e3, "p99_ms": lat["p99_s"] * 1e3,
                       "points_per_s": lat["points_per_s"],
                       "peak_concurrent": lat["peak_concurrent"]})
        print(f"# serving at {frac:.2f} R: p50 {lat['p50_s'] * 1e3:.2f} ms, "
              f"p99 {lat['p99_s'] * 1e3:.2f} ms", file=sys.stderr, flush=True)
    srv.destroy()
    for h in handles:
        h.free()
    return {
        "workload": "16 resident meshes (even: sine-perturbed cubes, odd: annuli), E "
                    f"{min(m.mesh.E for m in ms)}..{max(m.mesh.E for m in ms)}, N in {{5,7,9}}, "
                    f"5 fields each; {n_req} measured requests (+{n_warm} warm-up) of "
                    "1e3..1e6 points log-uniform, 1..5 fields, Poisson arrivals",
        "precision": "mixed" if precision == fp.FP_PREC_MIXED else "fp64",
        "slots": slots, "hbm_budget_bytes": budget,
        "mean_points_per_request": mean_p,
        "saturated": {"points_per_s": sat["points_per_s"], "requests_per_s": R,
                      "p50_ms": sat["p50_s"] * 1e3, "p99_ms": sat["p99_s"] * 1e3,
                      "peak_concurrent": sat["peak_concurrent"]},
        "poisson": levels,
    }


def schwarz_bench(fp, w, dev, precision, steps=10, kappa=4):
    """Schwarz interface exchange on the two-session mesh (box with a hole,
    19,360 elements + annulus, 8,000 elements, order 7): the 120,320 interface
    GLL nodes, tagged with their session, are located once; each timestep
    extrapolates the interface data (third order), then runs `kappa`
    subiterations of findpts_eval of 4 fields (u, v, w, p) and the mass-flux
    correction of the velocity on each session's interface."""
    import numpy as np
    import torch

    mesh = w.overlap_c3(device=dev)
    pts, tags, nrm, wts = w.c3_interface_quadrature(mesh)
    order = torch.argsort(tags, stable=True)
    pts, tags = pts[order].contiguous(), tags[order].contiguous()
    nrm, wts = nrm[:, order].contiguous(), wts[order].contiguous()
    P = pts.shape[0]
    n0 = int((tags == 0).sum())
    fields, _ = w.poly_fields(mesh, 4, degree=7, seed=3)
    h = fp.findpts_setup(mesh.x, mesh.y, mesh.z, mesh.N, tol=1e-12, elem_session=mesh.session,
                         delta=mesh.delta, max_points=1 << 17, precision=precision)
    code = torch.empty(P, dtype=torch.int32, device=dev)
    el = torch.empty(P, dtype=torch.int32, device=dev)
    rst = torch.empty((P, 3), dtype=torch.float64, device=dev)
    d2 = torch.empty(P, dtype=torch.float64, device=dev)
    out = torch.empty((4, P), dtype=torch.float64, device=dev)
    hist = [torch.zeros((4, P), dtype=torch.float64, device=dev) for _ in range(3)]
    pred = torch.empty((4, P), dtype=torch.float64, device=dev)
    work = torch.empty(fp.FP_FLUX_WORK, dtype=torch.float64, device=dev)
    ws0, ws1 = wts[:n0].contiguous(), wts[n0:].contiguous()
    stream = torch.cuda.current_stream()

    def locate():
        fp.findpts(h, pts, tags, code, el, rst, d2)

    def subiteration():
        fp.findpts_eval(h, code, el, rst, fields, out)
        fp.fp_flux_correct(ws0, nrm[:, :n0], out[:3, :n0], work=work)
        fp.fp_flux_correct(ws1, nrm[:, n0:], out[:3, n0:], work=work)

    def timestep():
        fp.fp_extrapolate(hist, 3, pred)
        for _ in range(kappa):
            subiteration()
        hist.insert(0, hist.pop())
        hist[0].copy_(out)

    locate()
    for _ in range(2):
        timestep()
    torch.cuda.synchronize()
    res = {}
    for name, fn, reps in (("locate_ms", locate, steps), ("subiteration_ms", subiteration,
                                                           steps * kappa),
                           ("timestep_ms", timestep, steps)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        res[name] = a.elapsed_time(b) / reps
    codes = np.bincount(code.cpu().numpy(), minlength=3).tolist()
    h.free()
    res.update({
        "workload": "two sessions (box with a hole, 19,360 elements; annulus, 8,000; N=7), "
                    f"{P} interface GLL nodes tagged by session, 4 fields; per timestep "
                    f"third-order extrapolation + {kappa} x (findpts_eval + mass-flux "
                    "correction per session)",
        "precision": "mixed" if precision == fp.FP_PREC_MIXED else "fp64",
        "interface_points": P, "kappa": kappa, "codes": codes,
        "interface_points_per_s_eval": P / (res["subiteration_ms"] / 1e3),
    })
    return res


def spiral_bench(fp, w, dev, reps=20):
    """Section 3.1 robustness case: one N = 15 spiral element, 1000 points
    x^e(r) for random r, tol = 1e-14; the points are produced on the device by
    interpolating the coordinate fields at (el 0, r).  Also the same call on
    1e6 such points (the N = 15 Newton throughput)."""
    import numpy as np
    import torch
    mesh = w.spiral_element(device=dev)
    h = fp.findpts_setup(mesh.x, mesh.y, mesh.z, mesh.N, tol=1e-14, max_points=1 << 20)
    out = {"element": "N=15 spiral, 1.5 turns", "tol": 1e-14}
    for P in (1000, 1_000_000):
        g = torch.Generator(device="cpu").manual_seed(21)
        r = (torch.rand((P, 3), generator=g, dtype=torch.float64) * 2 - 1).to(dev)
        zero = torch.zeros(P, dtype=torch.int32, device=dev)
        pts = fp.findpts_eval(h, zero, zero, r, [mesh.x, mesh.y, mesh.z]).t().contiguous()
        for _ in range(3):
            code, el, rst, d2 = fp.findpts(h, pts)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps if P <= 1000 else 5):
            t0 = time.perf_counter()
            code, el, rst, d2 = fp.findpts(h, pts)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        c = np.bincount(code.cpu().numpy(), minlength=3).tolist()
        dr = float((rst - r).abs().max())
        out[f"P{P}"] = {"ms_per_call_median": 1e3 * float(np.median(ts)),
                        "points_per_s": P / float(np.median(ts)), "codes": c,
                        "max_abs_r_error": dr}
    h.free()
    return out


def locate2_flops_per_pair(N, K):
    """Algorithmic binary64 flops of one 2D pair: closest-node scan (5 per
    node) and K + 1 evaluations of the map and Jacobian (two coordinates:
    4 V for the r contraction of value and derivative, 6 n1 for the s
    contractions, plus 20 n1 for the basis and its derivative in r and s)."""
    n1 = N + 1
    V = n1 * n1
    return 5 * V + (K + 1) * (8 * V + 32 * n1)


def twod_bench(fp, w, dev, steps=20, warmup=3, nfields=4):
    """Two-dimensional path on the 16,384-element ring (N = 7, 1.01e6 points,
    4 fields): findpts2 + findpts2_eval per step."""
    import numpy as np
    import torch
    m = w.annulus2d_c6(device=dev)
    pts = w.queries2d_c6(device=dev)
    P = pts.shape[0]
    g = torch.Generator(device="cpu").manual_seed(8)
    fl = [torch.randn((m.E, m.N + 1, m.N + 1), generator=g, dtype=torch.float64).to(dev)
          for _ in range(nfields)]
    t0 = time.perf_counter()
    h = fp.findpts2_setup(m.x, m.y, m.N, tol=1e-12, max_points=1 << 20)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    code = torch.empty(P, dtype=torch.int32, device=dev)
    el = torch.empty(P, dtype=torch.int32, device=dev)
    rs = torch.empty((P, 2), dtype=torch.float64, device=dev)
    d2 = torch.empty(P, dtype=torch.float64, device=dev)
    out = torch.empty((nfields, P), dtype=torch.float64, device=dev)

    def locate():
        fp.findpts2(h, pts, None, code, el, rs, d2)

    def step():
        locate()
        fp.findpts2_eval(h, code, el, rs, fl, out)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    fp.findpts2_stats(h, reset=True)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    pairs, iters, cands = fp.findpts2_stats(h)
    a.record()
    for _ in range(steps):
        locate()
    b.record()
    torch.cuda.synchronize()
    ms_loc = a.elapsed_time(b) / steps
    K = iters / max(pairs, 1)
    flops = locate2_flops_per_pair(m.N, K) * pairs / steps
    codes = np.bincount(code.cpu().numpy(), minlength=3).tolist()
    h.free()
    return {"workload": "ring2d_c6: 16,384 curved quads N=7 (256x64, exact arcs), "
                        f"{P} points (1% outside), {nfields} f64 fields; findpts2 + findpts2_eval",
            "value": P / (ms / 1e3), "unit": "points/s", "ms_per_step": ms,
            "findpts2_ms": ms_loc, "setup_ms": 1e3 * setup_s,
            "pairs_per_point": pairs / steps / P, "newton_iters_per_pair": K,
            "method_candidates_per_point": cands / steps / P,
            "alg_flops_per_findpts2": flops,
            "findpts2_tflops": flops / (ms_loc / 1e3) / 1e12, "codes": codes}




def run_workload(fp, dev, mesh, pts, fields, steps, warmup, max_points, precisions,
                 psess=None, tol=1e-12):
    """findpts + findpts_eval of every point per step, for each precision in
    turn on one handle.  Per precision: ms per step (HIP events around the
    steps on the launch stream), the library's per-kernel timings, device
    counters, and the results of the last step."""
    import torch

    stream = torch.cuda.current_stream()
    P = pts.shape[0]
    nf = len(fields)
    t0 = time.perf_counter()
    h = fp.findpts_setup(mesh.x, mesh.y, mesh.z, mesh.N, tol=tol, elem_session=mesh.session,
                         delta=mesh.delta, max_points=max_points)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    code = torch.empty(P, dtype=torch.int32, device=dev)
    el = torch.empty(P, dtype=torch.int32, device=dev)
    rst = torch.empty((P, 3), dtype=torch.float64, device=dev)
    d2 = torch.empty(P, dtype=torch.float64, device=dev)
    out = torch.empty((nf, P), dtype=torch.float64, device=dev) if nf else None

    def step():
        fp.findpts(h, pts, psess, code, el, rst, d2)
        if nf:
            fp.findpts_eval(h, code, el, rst, fields, out)

    res = {}
    for prec in precisions:
        fp.findpts_set_precision(h, prec)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        fp.findpts_stats(h, reset=True)
        fp.findpts_timing(h, True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(steps):
            step()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        fp.findpts_timing(h, False)
        tim = fp.findpts_timing_read(h)
        counts = fp.findpts_stats(h, first_pass=True)
        res[prec] = {"ms": ms, "tim": tim, "counts": counts, "steps": steps,
                     "res": (code.cpu().numpy(), el.cpu().numpy(), rst.cpu().numpy(),
                             d2.cpu().numpy()),
                     "out": None if out is None else out.cpu().numpy()}
        print(f"# {mesh.name} {'mixed' if prec else 'fp64'}: {ms:.3f} ms/step, "
              f"{P / ms * 1e3:.4g} points/s; kernels {tim}", file=sys.stderr, flush=True)
    return h, setup_s, res, step


def summarize(N, P, nf, r):
    """Throughput, kernel breakdown and the first-pass Newton kernel's
    achieved binary64 rate for one precision of one workload."""
    import numpy as np

    tim = r["tim"]
    pairs, iters, located, cands, pairs1, iters1 = r["counts"]
    per = lambda k: tim[k][0] / max(tim[k][1], 1)
    launches = max(tim["locate_kernel"][1], 1)
    c1 = pairs1 / max(located, 1)
    K1 = iters1 / max(pairs1, 1)
    flops_launch = located / launches * locate_flops_per_point(N, c1, K1)
    return {
        "value": P / (r["ms"] / 1e3), "unit": "points/s", "ms_per_step": r["ms"],
        "breakdown_ms": {"locate_kernel": per("locate_kernel"),
                         "locate_kernel_2nd_pass": per("locate_kernel_2"),
                         "eval_kernel": per("eval_kernel"),
                         "findpts": per("findpts"), "findpts_eval": per("findpts_eval"),
                         "locate_launches_per_step": launches / r["steps"]},
        "pairs_per_point": pairs / max(located, 1),
        "first_pass_pairs_per_point": c1,
        "newton_iters_per_pair": iters / max(pairs, 1),
        "first_pass_newton_iters_per_pair": K1,
        "method_candidates_per_point": cands / max(located, 1),
        "locate_alg_flops_per_launch": flops_launch,
        "locate_tflops": flops_launch / (per("locate_kernel") / 1e3) / 1e12,
        "eval_alg_flops_per_step": P * eval_flops_per_point(N, nf),
        "codes": np.bincount(r["res"][0], minlength=3).tolist(),
    }


def agreement(r64, rmx, nf):
    """Mixed precision against binary64 on the same workload: codes,
    elements (face ties), |dr| and the interpolated values."""
    import numpy as np

    c64, e64, g64, _ = r64["res"]
    cmx, emx, gmx, _ = rmx["res"]
    same = (e64 == emx) & (c64 == cmx)
    ins = same & (c64 == 0)
    rec = {"codes_equal": bool(np.array_equal(c64, cmx)),
           "elements_differ": int(np.sum(e64 != emx)),
           "max_abs_dr": float(np.max(np.abs(g64[ins] - gmx[ins]))) if np.any(ins) else 0.0}
    if nf and r64["out"] is not None:
        o64, omx = r64["out"][:, ins], rmx["out"][:, ins]
        scale = np.maximum(np.max(np.abs(o64), axis=1), 1e-300)[:, None]
        err = np.abs(omx - o64) / scale
        rec["field_err_rel_max"] = float(err.max()) if err.size else 0.0
        rec["field_err_rel_median"] = float(np.median(err)) if err.size else 0.0
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=20_000_000,
                    help="query points of the headline workload")
    ap.add_argument("--max-points", type=int, default=20_000_000,
                    help="points per findpts pass (the handle's workspace)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after timing, run the library's plain copy kernel over this many MiB "
                         "(reference launch for scaling hardware byte counters)")
    ap.add_argument("--serving-requests", type=int, default=1000,
                    help="measured requests of the serving stream (0 = skip it)")
    ap.add_argument("--serving-warmup", type=int, default=50)
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the headline workload (for profiler runs)")
    ap.add_argument("--legs", default="annulus,cube,two_sessions,spiral,schwarz,twod,serving",
                    help="comma-separated secondary legs to run")
    ap.add_argument("--skip-headline", action="store_true",
                    help="run only the secondary legs (no JSON headline line)")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="precision of the headline line (the other one is timed beside it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for {args.gpus}); "
              "several GPUs would each hold the mesh and take a share of the points, "
              "and that sharding is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as w
    from paper_1811_04891_amd import findpts as fp

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    head = fp.FP_PREC_MIXED if args.precision == "mixed" else fp.FP_PREC_FP64
    other = fp.FP_PREC_FP64 if head == fp.FP_PREC_MIXED else fp.FP_PREC_MIXED
    pname = {fp.FP_PREC_FP64: "fp64", fp.FP_PREC_MIXED: "mixed"}

    legs_on = set(args.legs.split(",")) if not args.headline_only else set()
    rec = {}
    if not args.skip_headline:
        rec = headline(args, fp, w, dev, head, other, pname)
    legs = run_legs(args, fp, w, dev, head, legs_on, stream)
    if legs:
        rec["legs"] = legs
        if "serving" in legs:
            mid = legs["serving"]["poisson"][1]
            rec["p50_ms"], rec["p99_ms"] = mid["p50_ms"], mid["p99_ms"]
    if "copy" in legs_on or not args.skip_headline:
        copy_rate(args, fp, dev, stream, rec)
    print(json.dumps(rec), flush=True)
    if args.copy_mib > 0:
        n = args.copy_mib << 20
        src = torch.ones(n // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            fp.fp_copy(src, dst, stream)
        torch.cuda.synchronize()
        print(f"# copy kernel: {n} bytes read, {n} bytes written per launch", file=sys.stderr,
              flush=True)


def headline(args, fp, w, dev, head, other, pname):
    """The large box in both precisions, its roofline and the CPU oracle."""
    import torch

    mesh = w.big_box_c5(device=dev)
    pts = w.queries_c5(n=args.points, device=dev)
    fields, _ = w.poly_fields(mesh, 5, degree=7, seed=5)
    P, N, nf = pts.shape[0], mesh.N, len(fields)
    torch.cuda.synchronize()
    print(f"# setup: E={mesh.E} N={N} points={P} fields={nf}", file=sys.stderr, flush=True)
    h, setup_s, res, _ = run_workload(fp, dev, mesh, pts, fields, args.steps, args.warmup,
                                      args.max_points, (other, head))
    sh, so = summarize(N, P, nf, res[head]), summarize(N, P, nf, res[other])
    h.free()
    prof = read_profile(f"locate_big_box_c5_{pname[head]}_pmc.txt")
    traffic = float(prof["hbm_bytes_per_launch"]) if prof else None
    rec = {
        "metric": "points located+interpolated/sec, FP64 vs mixed; p50/p99 request latency",
        "value": sh["value"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sh["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == fp.FP_PREC_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"big_box_c5: 200,000 curved hexes N=7 (100x50x40, sine-perturbed), "
                        f"{P} query points near 8 random spheres (random order), {nf} f64 "
                        f"fields; findpts+findpts_eval, {args.precision}",
            "E": mesh.E, "N": N, "points": P, "fields": nf, "precision": args.precision,
            "points_per_pass": args.max_points, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "alu",
            "kernel": ("k_newton8 (trust-region Newton, binary64 matrix cores), first pass"
                       if head == fp.FP_PREC_FP64 else
                       "k_mixed8 (binary32 Newton + binary64 refinement), first pass"),
            "achieved": sh["locate_tflops"],
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": sh["locate_tflops"] / PEAK_FP64_TFLOPS,
            "traffic": traffic,
            "alg_flops_per_launch": sh["locate_alg_flops_per_launch"],
            "launch_ms": sh["breakdown_ms"]["locate_kernel"],
            "candidates_per_point": sh["first_pass_pairs_per_point"],
            "newton_iters_per_candidate": sh["first_pass_newton_iters_per_pair"],
        },
        "breakdown_ms": dict(sh["breakdown_ms"], setup_s=setup_s),
        "gpu_counts": {k: sh[k] for k in ("pairs_per_point", "newton_iters_per_pair",
                                          "method_candidates_per_point", "codes")},
        pname[other]: so,
        "fp64_vs_mixed": agreement(res[fp.FP_PREC_FP64], res[fp.FP_PREC_MIXED], nf),
    }
    del res
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(w.Mesh(mesh.name, N, mesh.x, mesh.y, mesh.z), pts,
                                           fields, "the large-box workload", args.cpu_seconds)
    del mesh, pts, fields
    torch.cuda.empty_cache()
    return rec


def run_legs(args, fp, w, dev, head, on, stream):
    """The secondary workloads named in `on`."""
    import numpy as np
    import torch

    legs = {}
    if "annulus" in on:
        # ---- the annulus, both precisions, then a moving-mesh re-setup -------
        m2 = w.annulus_c2(device=dev)
        p2 = w.queries_c2(device=dev)
        f2, _ = w.poly_fields(m2, 4, degree=7, seed=2)
        h2, s2, r2, step2 = run_workload(fp, dev, m2, p2, f2, args.steps, args.warmup, 1 << 20,
                                         (fp.FP_PREC_FP64, fp.FP_PREC_MIXED))
        legs["annulus_c2"] = {
            "workload": "16,384 curved hexes N=7 (64x16x16, exact arcs), 1,010,000 points "
                        "(1% outside), 4 f64 fields",
            "fp64": summarize(7, p2.shape[0], 4, r2[fp.FP_PREC_FP64]),
            "mixed": summarize(7, p2.shape[0], 4, r2[fp.FP_PREC_MIXED]),
            "fp64_vs_mixed": agreement(r2[fp.FP_PREC_FP64], r2[fp.FP_PREC_MIXED], 4),
            "setup_s": s2,
        }
        del r2
        fp.findpts_set_precision(h2, fp.FP_PREC_FP64)
        upd = []
        for k in range(1, 6):
            c, sn = math.cos(0.01 * k), math.sin(0.01 * k)
            xk = (c * m2.x - sn * m2.y).contiguous()
            yk = (sn * m2.x + c * m2.y).contiguous()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fp.findpts_update(h2, xk, yk, m2.z)
            torch.cuda.synchronize()
            upd.append(time.perf_counter() - t0)
        ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ea.record(stream)
        step2()
        eb.record(stream)
        torch.cuda.synchronize()
        legs["annulus_c2"]["moving_mesh"] = {
            "update_ms": 1e3 * float(np.median(upd)), "updates": len(upd),
            "step_ms_after_update": ea.elapsed_time(eb)}
        h2.free()
        del m2, p2, f2

    if "cube" in on:
        # ---- the unit cube -------------------------------------------------
        m1 = w.cube_c1(device=dev)
        p1 = w.queries_c1(device=dev)
        f1 = [(m1.x ** 2 + m1.y * m1.z + m1.z ** 3).contiguous()]
        h1, s1, r1, _ = run_workload(fp, dev, m1, p1, f1, args.steps, args.warmup, 1 << 14,
                                     (fp.FP_PREC_FP64,))
        legs["unit_cube_c1"] = {"workload": "64 perturbed hexes N=5, 10,000 points, 1 field",
                                "fp64": summarize(5, p1.shape[0], 1, r1[fp.FP_PREC_FP64])}
        h1.free()

    if "two_sessions" in on:
        # ---- two sessions, 1.2e6 interface-face points ----------------------
        m3 = w.overlap_c3(device=dev)
        p3, t3 = w.queries_c3(n=1_200_000, device=dev)
        f3, _ = w.poly_fields(m3, 4, degree=7, seed=3)
        h3, s3, r3, _ = run_workload(fp, dev, m3, p3, f3, args.steps, args.warmup, 1 << 21,
                                     (fp.FP_PREC_FP64, fp.FP_PREC_MIXED), psess=t3)
        legs["two_sessions_c3"] = {
            "workload": "box with a hole (19,360 hexes) + annulus (8,000), N=7, 1,200,000 "
                        "interface-face points tagged by session, distance discriminator, "
                        "4 f64 fields",
            "fp64": summarize(7, p3.shape[0], 4, r3[fp.FP_PREC_FP64]),
            "mixed": summarize(7, p3.shape[0], 4, r3[fp.FP_PREC_MIXED]),
            "fp64_vs_mixed": agreement(r3[fp.FP_PREC_FP64], r3[fp.FP_PREC_MIXED], 4),
        }
        h3.free()
        del r3, m3, p3, t3, f3
        torch.cuda.empty_cache()

    if "spiral" in on:
        legs["spiral"] = spiral_bench(fp, w, dev)
        print(f"# spiral: {legs['spiral']}", file=sys.stderr, flush=True)
    if "schwarz" in on:
        legs["schwarz_exchange"] = schwarz_bench(fp, w, dev, head)
        print(f"# schwarz exchange: {legs['schwarz_exchange']}", file=sys.stderr, flush=True)
    if "twod" in on:
        legs["twod"] = twod_bench(fp, w, dev)
        print(f"# 2D: {legs['twod']}", file=sys.stderr, flush=True)
    if "serving" in on and args.serving_requests > 0:
        # the serving stream runs in mixed precision, as its workload specifies
        legs["serving"] = serving_bench(fp, w, dev, fp.FP_PREC_MIXED, args.serving_requests,
                                        args.serving_warmup)
    return legs


def copy_rate(args, fp, dev, stream, rec):
    """The library's plain copy kernel over 1 GiB: the achievable HBM stream
    rate beside the 8 TB/s datasheet figure (not in counter runs, whose only
    copy launches are the --copy-mib reference)."""
    import torch

    nb = 0 if args.copy_mib > 0 else 1 << 30
    if nb:
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            fp.fp_copy(src, dst, stream)
        ca, cb_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ca.record(stream)
        for _ in range(5):
            fp.fp_copy(src, dst, stream)
        cb_.record(stream)
        torch.cuda.synchronize()
        rec["copy_GBps"] = 2 * nb * 5 / (ca.elapsed_time(cb_) / 1e3) / 1e9
        del src, dst

if __name__ == "__main__":
    main()
