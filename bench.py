"""Benchmark: points located + interpolated per second on one MI355X.

Workload (one step = findpts + findpts_eval of every query point): the
cylinder-in-box annulus, 16,384 curved hexahedra of order 7 (64 azimuthal x
16 radial x 16 axial, rho in [0.5, 1], z in [0, 1], nodes at exact polar
positions), 1,010,000 query points (1e6 area-uniform in the annulus plus 1 %
outside it), 4 float64 fields given as random polynomials of total degree 7.
All inputs are synthetic, seeded, and resident in HBM before timing starts.
Both precisions are timed; --precision picks the headline one.

Prints one JSON line.  Besides the throughput it reports:
  roofline      the Newton (locate) kernel, FP64: algorithmic flops per launch
                / its mean duration (HIP events recorded by the library on the
                launch stream) vs 78.6 TFLOP/s; HBM traffic from the committed
                hardware-counter summary when it was taken on this source
  cpu_baseline  the CPU oracle timed on a bounded sample of the same points
  spiral        the N = 15 spiral element at tol 1e-14: 1000 points (the
                paper's robustness case) and 1e6 points
  twod          the two-dimensional path on a 16,384-element ring
  serving       a stream of requests on 16 resident meshes through the
                serving layer: saturated throughput and p50/p99 latency at
                0.5, 0.8 and 0.95 of the saturated request rate
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
PROFILE_PMC = os.path.join(ROOT, "profiles", "locate_annulus_c2_pmc.txt")


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
    for f in ("fp_locate.hip", "fp_mfma.inc", "fp_mfma.h", "fp_basis.h", "fp_internal.h"):
        with open(os.path.join(ROOT, "paper_1811_04891_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per locate launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    if not os.path.exists(PROFILE_PMC):
        return None
    vals = {}
    for line in open(PROFILE_PMC):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(mesh, pts, fields, target_s=10.0):
    import numpy as np

    import oracle
    om = oracle.OracleMesh.from_mesh(mesh, 1e-12)
    nthreads = len(os.sched_getaffinity(0))
    cores = oracle.threads(nthreads)
    p = pts.cpu().numpy()
    # size the sample from a probe large enough to keep every thread busy
    probe_n = min(len(p), 50_000)
    t = time.perf_counter()
    om.findpts(p[:probe_n], nthreads=nthreads)
    dt = time.perf_counter() - t
    n = int(min(len(p), max(probe_n, probe_n * target_s / max(dt, 1e-3))))
    sample = p[:n]
    hf = [f.cpu().numpy() for f in fields]
    t = time.perf_counter()
    code, el, rst, _ = om.findpts(sample, nthreads=nthreads)
    om.eval(code, el, rst, hf, nthreads=nthreads)
    t_loc = time.perf_counter() - t
    c = om.last_stats[0] / n
    K = om.last_stats[1] / max(om.last_stats[0], 1)
    # one core on a 20,000-point slice of the same sample
    n1 = min(n, 20_000)
    t = time.perf_counter()
    c1, e1, r1, _ = om.findpts(sample[:n1], nthreads=1)
    om.eval(c1, e1, r1, hf, nthreads=1)
    t1 = time.perf_counter() - t
    oracle.threads(nthreads)  # restore the thread count for later oracle calls
    return {"n": n, "seconds": t_loc, "cores": cores, "c": c, "K": K, "om": om,
            "sample_code": code, "one_core": n1 / t1}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=1_000_000,
                    help="in-annulus points (1 %% more are placed outside)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after timing, run the library's plain copy kernel over this many MiB "
                         "(reference launch for scaling hardware byte counters)")
    ap.add_argument("--serving-requests", type=int, default=1000,
                    help="measured requests of the serving stream (0 = skip it)")
    ap.add_argument("--serving-warmup", type=int, default=50)
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the moving-mesh, spiral and Schwarz-exchange sections (for "
                         "profiler runs of the headline kernels)")
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
    mesh_cpu = w.annulus_c2()
    mesh = mesh_cpu.to(dev)
    pts = w.queries_c2(n_in=args.points).to(dev)
    P = pts.shape[0]
    fields, _ = w.poly_fields(mesh, 4, degree=7, seed=2)
    N = mesh.N
    print(f"# setup: E={mesh.E} N={N} points={P} fields=4", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    h = fp.findpts_setup(mesh.x, mesh.y, mesh.z, N, tol=1e-12, max_points=1 << 20)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    code = torch.empty(P, dtype=torch.int32, device=dev)
    el = torch.empty(P, dtype=torch.int32, device=dev)
    rst = torch.empty((P, 3), dtype=torch.float64, device=dev)
    d2 = torch.empty(P, dtype=torch.float64, device=dev)
    out = torch.empty((4, P), dtype=torch.float64, device=dev)

    def step():
        fp.findpts(h, pts, None, code, el, rst, d2)
        fp.findpts_eval(h, code, el, rst, fields, out)

    def timed(prec):
        fp.findpts_set_precision(h, prec)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        fp.findpts_stats(h, reset=True)
        fp.findpts_timing(h, True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            step()
        ev1.record(stream)
        torch.cuda.synchronize()
        total_ms = ev0.elapsed_time(ev1)
        fp.findpts_timing(h, False)
        tim = fp.findpts_timing_read(h)
        counts = fp.findpts_stats(h)
        ms = total_ms / args.steps
        res = (code.cpu().numpy(), el.cpu().numpy(), rst.cpu().numpy(), d2.cpu().numpy())
        print(f"# {'mixed' if prec else 'fp64'}: {ms:.3f} ms/step, {P / ms * 1e3:.4g} points/s; "
              f"kernels {tim}", file=sys.stderr, flush=True)
        return ms, tim, counts, res

    head = fp.FP_PREC_MIXED if args.precision == "mixed" else fp.FP_PREC_FP64
    other = fp.FP_PREC_FP64 if head == fp.FP_PREC_MIXED else fp.FP_PREC_MIXED
    ms_o, tim_o, counts_o, res_o = timed(other)
    ms_per_step, tim, (pairs, iters, located, cands), res_h = timed(head)
    value = P / (ms_per_step / 1e3)
    codes = np.bincount(res_h[0], minlength=3)
    # agreement of the two precisions on this workload
    res64, resmx = (res_h, res_o) if head == fp.FP_PREC_FP64 else (res_o, res_h)
    same_el = res64[1] == resmx[1]
    agree = {
        "codes_equal": bool(np.array_equal(res64[0], resmx[0])),
        "elements_differ": int(np.sum(~same_el)),
        "max_abs_dr": float(np.max(np.abs(res64[2][same_el] - resmx[2][same_el]))),
    }

    cb = None
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cb = cpu_baseline(mesh_cpu, pts, fields, args.cpu_seconds)
    # algorithmic flops of the launches timed: the (point, element) pairs the
    # kernel solves and their Newton iterations, as counted on the device
    # (the method's own candidate count, measured by the oracle, is larger:
    # the oriented-box filter removes most non-owner candidates)
    c_gpu = pairs / max(located, 1)
    K_gpu = iters / max(pairs, 1)
    c_alg, K_alg = c_gpu, K_gpu
    loc_ms = tim["locate_kernel"][0] / max(tim["locate_kernel"][1], 1)
    ev_ms = tim["eval_kernel"][0] / max(tim["eval_kernel"][1], 1)
    alg_flops = P * locate_flops_per_point(N, c_alg, K_alg)
    achieved = alg_flops / (loc_ms / 1e3) / 1e12
    traffic = read_traffic()
    rec = {
        "metric": "points located+interpolated/sec, FP64 vs mixed; p50/p99 request latency",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == fp.FP_PREC_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "annulus_c2: 16,384 curved hexes N=7 (64x16x16, exact arcs), "
                        f"{P} query points (1% outside), 4 f64 fields; findpts+findpts_eval, "
                        f"{args.precision}",
            "E": mesh.E, "N": N, "points": P, "fields": 4, "precision": args.precision,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_locate_mfma (trust-region Newton on FP64 matrix cores)",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": traffic,
            "alg_flops_per_launch": alg_flops,
            "launch_ms": loc_ms,
            "candidates_per_point": c_alg,
            "newton_iters_per_candidate": K_alg,
        },
        "breakdown_ms": {
            "locate_kernel": loc_ms,
            "eval_kernel": ev_ms,
            "findpts": tim["findpts"][0] / max(tim["findpts"][1], 1),
            "findpts_eval": tim["findpts_eval"][0] / max(tim["findpts_eval"][1], 1),
            "setup_s": setup_s,
        },
        "gpu_counts": {"pairs_per_point": c_gpu, "newton_iters_per_pair": K_gpu,
                       "method_candidates_per_point": cands / max(located, 1),
                       "codes": codes.tolist()},
    }
    # moving mesh: re-setup on the device after each rigid rotation (0.01 rad)
    # of the annulus, then findpts + findpts_eval on the moved mesh
    import math
    upd = []
    for k in range(1, 1 if args.headline_only else 6):
        c, sn = math.cos(0.01 * k), math.sin(0.01 * k)
        xk = (c * mesh.x - sn * mesh.y).contiguous()
        yk = (sn * mesh.x + c * mesh.y).contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fp.findpts_update(h, xk, yk, mesh.z)
        torch.cuda.synchronize()
        upd.append(time.perf_counter() - t0)
    fp.findpts_set_precision(h, head)
    if upd:
        ev2a, ev2b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev2a.record(stream)
        step()
        ev2b.record(stream)
        torch.cuda.synchronize()
        moved_codes = np.bincount(code.cpu().numpy(), minlength=3).tolist()
        rec["moving_mesh"] = {
            "update_ms": 1e3 * float(np.median(upd)), "updates": len(upd),
            "setup_ms": 1e3 * setup_s, "step_ms_after_update": ev2a.elapsed_time(ev2b),
            "codes_after_update": moved_codes,
        }
    oname = "mixed" if other == fp.FP_PREC_MIXED else "fp64"
    rec[oname] = {
        "value": P / (ms_o / 1e3), "ms_per_step": ms_o,
        "locate_kernel_ms": tim_o["locate_kernel"][0] / max(tim_o["locate_kernel"][1], 1),
        "newton_iters_per_pair": counts_o[1] / max(counts_o[0], 1),
    }
    rec["fp64_vs_mixed"] = agree
    if cb:
        rec["cpu_baseline"] = {
            "value": cb["n"] / cb["seconds"],
            "unit": "points/s",
            "cores": cb["cores"],
            "kind": "oracle",
            "sample": f"first {cb['n']} of the same {P} query points, findpts + "
                      f"findpts_eval of the 4 fields (plain C double, OpenMP), "
                      f"{cb['seconds']:.1f} s",
            "method_candidates_per_point": cb["c"],
            "method_newton_iters_per_candidate": cb["K"],
            "one_core_points_per_s": cb["one_core"],
        }
    h.free()
    # the library's plain copy kernel over 1 GiB: the achievable HBM stream rate
    # beside the 8 TB/s datasheet figure (not in counter runs, whose only copy
    # launches are the --copy-mib reference)
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
    if not args.headline_only:
        rec["spiral"] = spiral_bench(fp, w, dev)
        print(f"# spiral: {rec['spiral']}", file=sys.stderr, flush=True)
        rec["schwarz_exchange"] = schwarz_bench(fp, w, dev, head)
        print(f"# schwarz exchange: {rec['schwarz_exchange']}", file=sys.stderr, flush=True)
        rec["twod"] = twod_bench(fp, w, dev)
        print(f"# 2D: {rec['twod']}", file=sys.stderr, flush=True)
    if args.serving_requests > 0:
        sv = serving_bench(fp, w, dev, head, args.serving_requests, args.serving_warmup)
        rec["serving"] = sv
        mid = sv["poisson"][1]
        rec["p50_ms"], rec["p99_ms"] = mid["p50_ms"], mid["p99_ms"]
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


if __name__ == "__main__":
    main()
