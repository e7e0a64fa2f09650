// findpts: candidate lookup, (point, element) pair grouping, trust-region
// Newton per pair with one element per wavefront, owner selection.
//
// Section 2.1 of the paper: hash table -> elementwise bounding boxes ->
// trust-region Newton on ||x^e(r) - x*||^2 started from the closest mapped
// GLL node -> inside / border / not found; session-id exclusion; among
// several sessions the largest distance-to-boundary wins.
//
// Pipeline per pass of at most max_points points, all on the caller's stream:
//   k_cand     per point: hash cell, box + session test, candidate list
//              (ascending element ids) and each pair's rank in its element
//   scan       pair counts per element -> element offsets
//   k_scatter  pair slots grouped by element
//   k_locate   one 64-lane wavefront per element; lanes = pairs of that
//              element; node data read once per wave through scalar loads
//   k_select   per point: classification and owner rule, caller's order
#include <cmath>

#include "fp_basis.h"
#include "fp_internal.h"

namespace fp {

struct LocArgs {
    const double *geom;
    const double *esize;
    const double *bbox;
    const double *delta;
    const int *esess;
    const int *cell_off;
    const int *cell_el;
    Grid g;
    const double *pts;
    const int *psess;
    int npts;
    int MC;
    double tol;
    int *ncand;
    int *cand_el;
    int *cand_pos;
    int *elem_cnt;
    const int *elem_off;
    int *order;
    double *res;
    double *res_dl;
    int *res_in;
    unsigned long long *stats;
};

__device__ __forceinline__ int cell_of(const Grid &g, int a, double x)
{
    double u = (x - g.lo[a]) * g.inv[a];
    int i = (int)floor(u);
    return i < 0 ? 0 : (i >= g.nc[a] ? g.nc[a] - 1 : i);
}

__global__ __launch_bounds__(256) void k_cand(LocArgs a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.npts) return;
    const double x0 = a.pts[3 * (long long)p], x1 = a.pts[3 * (long long)p + 1],
                 x2 = a.pts[3 * (long long)p + 2];
    const int ps = a.psess ? a.psess[p] : -1;
    int n = 0;
    const Grid &g = a.g;
    // NaN fails every comparison, so non-finite points find nothing
    if (x0 >= g.lo[0] && x0 <= g.hi[0] && x1 >= g.lo[1] && x1 <= g.hi[1] && x2 >= g.lo[2] &&
        x2 <= g.hi[2]) {
        const long long c = cell_of(g, 0, x0) +
                            (long long)g.nc[0] * (cell_of(g, 1, x1) +
                                                  (long long)g.nc[1] * cell_of(g, 2, x2));
        const int qb = a.cell_off[c], qe = a.cell_off[c + 1];
        int *ce = a.cand_el + (long long)p * a.MC;
        int *cp = a.cand_pos + (long long)p * a.MC;
        for (int q = qb; q < qe; ++q) {
            const int e = a.cell_el[q];
            const double *b = a.bbox + 6 * (long long)e;
            if (x0 < b[0] || x0 > b[1] || x1 < b[2] || x1 > b[3] || x2 < b[4] || x2 > b[5])
                continue;
            if (ps >= 0 && a.esess && a.esess[e] == ps) continue;
            ce[n] = e;
            cp[n] = atomicAdd(&a.elem_cnt[e], 1);
            ++n;
        }
    }
    a.ncand[p] = n;
}

__global__ __launch_bounds__(256) void k_scatter(LocArgs a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.npts) return;
    const int n = a.ncand[p];
    const long long s0 = (long long)p * a.MC;
    for (int k = 0; k < n; ++k) {
        const int e = a.cand_el[s0 + k];
        a.order[a.elem_off[e] + a.cand_pos[s0 + k]] = (int)(s0 + k);
    }
}

// Solve the 3x3 system A d = b by Cramer's rule; false if det is 0 or the
// result is not finite.
__device__ __forceinline__ bool solve3(const double (&A)[9], const double (&b)[3],
                                       double (&d)[3])
{
    const double c00 = A[4] * A[8] - A[5] * A[7];
    const double c01 = A[5] * A[6] - A[3] * A[8];
    const double c02 = A[3] * A[7] - A[4] * A[6];
    const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    const double c10 = A[2] * A[7] - A[1] * A[8];
    const double c11 = A[0] * A[8] - A[2] * A[6];
    const double c12 = A[1] * A[6] - A[0] * A[7];
    const double c20 = A[1] * A[5] - A[2] * A[4];
    const double c21 = A[2] * A[3] - A[0] * A[5];
    const double c22 = A[0] * A[4] - A[1] * A[3];
    const double inv = 1.0 / det;
    d[0] = (c00 * b[0] + c10 * b[1] + c20 * b[2]) * inv;
    d[1] = (c01 * b[0] + c11 * b[1] + c21 * b[2]) * inv;
    d[2] = (c02 * b[0] + c12 * b[1] + c22 * b[2]) * inv;
    return det != 0.0 && isfinite(d[0]) && isfinite(d[1]) && isfinite(d[2]);
}

// Trust-region Newton constants (stop tests, radius rules).
constexpr double kResidStop = 1e-13;  // phi <= (kResidStop h_e)^2
constexpr double kStepStop = 1e-13;   // accepted step with |s|_inf below this
constexpr double kStepTiny = 1e-15;   // no progress possible
constexpr int kMaxIter = 50;

template <int N1>
__global__ __launch_bounds__(kWave) void k_locate(LocArgs a, const double *__restrict__ basis)
{
    constexpr int V = N1 * N1 * N1;
    const BasisPtr<double> B{as_const(basis)};
    const int e = blockIdx.x;
    const int beg = a.elem_off[e], end = a.elem_off[e + 1];
    if (beg >= end) return;
    cptr<double> X = as_const(a.geom + (long long)e * 3 * V);
    const double he = a.esize[e];
    const double rstop = (kResidStop * he) * (kResidStop * he);
    unsigned long long my_iters = 0;

    for (int base = beg; base < end; base += kWave) {
        const int q = base + (int)threadIdx.x;
        const bool act = q < end;
        const int slot = act ? a.order[q] : 0;
        const int p = slot / a.MC;
        double xs[3] = {0.0, 0.0, 0.0};
        if (act) {
            xs[0] = a.pts[3 * (long long)p];
            xs[1] = a.pts[3 * (long long)p + 1];
            xs[2] = a.pts[3 * (long long)p + 2];
        }
        // closest mapped GLL node (ties: smallest node index)
        double best = INFINITY;
        int bq = 0;
#pragma unroll 8
        for (int n = 0; n < V; ++n) {
            const double dx = X[n] - xs[0], dy = X[V + n] - xs[1], dz = X[2 * V + n] - xs[2];
            const double d = fma(dz, dz, fma(dy, dy, dx * dx));
            if (d < best) {
                best = d;
                bq = n;
            }
        }
        double rt[3];
        {
            const int i0 = bq % N1, i1 = (bq / N1) % N1, i2 = bq / (N1 * N1);
            rt[0] = rt[1] = rt[2] = 0.0;
#pragma unroll
            for (int i = 0; i < N1; ++i) {
                const double zi = B.z(i);
                rt[0] = (i == i0) ? zi : rt[0];
                rt[1] = (i == i1) ? zi : rt[1];
                rt[2] = (i == i2) ? zi : rt[2];
            }
        }

        // projected trust-region Gauss-Newton: a coordinate on a bound of
        // [-1,1]^3 whose descent direction points outward is held; the
        // trust radius is measured in the max norm
        double r[3] = {0, 0, 0}, F[3] = {0, 0, 0}, J[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        double phi = INFINITY, D = 1.0, pred = 0.0, ns = 0.0;
        bool limited = false, have = false;
        int it = 0;
        bool done = !act;
        while (!done) {
            double xt[3], Jt[9];
            geo_eval<N1>(X, B, rt, xt, Jt);
            const double Ft[3] = {xt[0] - xs[0], xt[1] - xs[1], xt[2] - xs[2]};
            const double phit = fma(Ft[2], Ft[2], fma(Ft[1], Ft[1], Ft[0] * Ft[0]));
            bool acc = true, stop = false;
            if (have) {
                const double rho = (phi - phit) / pred;
                acc = rho >= 0.01;
                if (rho > 0.75 && limited)
                    D = fmin(2.0 * D, 2.0);
                else if (rho < 0.25)
                    D = 0.25 * ns;
                if (acc && ns <= kStepStop) stop = true;
            }
            // branch-free update: the trial Jacobian is consumed on every path,
            // so its half of the contraction is not sunk into a branch away
            // from the pipelined node loads
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                r[d] = acc ? rt[d] : r[d];
                F[d] = acc ? Ft[d] : F[d];
            }
#pragma unroll
            for (int d = 0; d < 9; ++d) J[d] = acc ? Jt[d] : J[d];
            phi = acc ? phit : phi;
            have = true;
            if (!stop && (phi <= rstop || it >= kMaxIter)) stop = true;
            if (!stop) {
                ++it;
                double g[3];
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    g[d] = fma(J[6 + d], F[2], fma(J[3 + d], F[1], J[d] * F[0]));
                double m[3];
                int nf = 0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const bool held = (r[d] >= 1.0 && g[d] < 0.0) || (r[d] <= -1.0 && g[d] > 0.0);
                    m[d] = held ? 0.0 : 1.0;
                    nf += held ? 0 : 1;
                }
                if (nf == 0) {
                    stop = true;
                } else {
                    double dl[3];
                    bool ok;
                    if (nf == 3) {
                        const double b[3] = {-F[0], -F[1], -F[2]};
                        ok = solve3(J, b, dl);
                    } else {
                        // reduced normal equations: (M J^T J M + I - M) d = -M g
                        double A[9], b[3];
#pragma unroll
                        for (int u = 0; u < 3; ++u) {
#pragma unroll
                            for (int v = 0; v < 3; ++v) {
                                const double jtj =
                                    fma(J[6 + u], J[6 + v], fma(J[3 + u], J[3 + v], J[u] * J[v]));
                                A[3 * u + v] = m[u] * m[v] * jtj + ((u == v) ? 1.0 - m[u] : 0.0);
                            }
                            b[u] = -m[u] * g[u];
                        }
                        ok = solve3(A, b, dl);
                    }
                    if (!ok) {
#pragma unroll
                        for (int d = 0; d < 3; ++d) dl[d] = -m[d] * g[d];
                    }
                    const double nd = fmax(fabs(dl[0]), fmax(fabs(dl[1]), fabs(dl[2])));
                    if (!(nd > 0.0) || !isfinite(nd)) {
                        stop = true;
                    } else {
                        limited = nd > D;
                        const double sc = limited ? D / nd : 1.0;
                        double s[3];
                        ns = 0.0;
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const double v = fmin(1.0, fmax(-1.0, r[d] + dl[d] * sc));
                            rt[d] = v;
                            s[d] = v - r[d];
                            ns = fmax(ns, fabs(s[d]));
                        }
                        double q2 = 0.0;
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const double t =
                                fma(J[3 * c + 2], s[2], fma(J[3 * c + 1], s[1], fma(J[3 * c], s[0], F[c])));
                            q2 = fma(t, t, q2);
                        }
                        pred = phi - q2;
                        if (ns <= kStepTiny || !(pred > 0.0)) stop = true;
                    }
                }
            }
            done = stop;
        }
        if (act) {
            my_iters += (unsigned long long)it;
            double *o = a.res + 4 * (long long)slot;
            o[0] = r[0];
            o[1] = r[1];
            o[2] = r[2];
            o[3] = phi;
            const bool inside = sqrt(phi) <= a.tol * he;
            a.res_in[slot] = inside ? 1 : 0;
            if (a.res_dl) {
                double dl = 0.0;
                if (inside) {
                    double hr[N1], hs[N1], ht[N1];
                    lagrange<N1>(B, r[0], hr);
                    lagrange<N1>(B, r[1], hs);
                    lagrange<N1>(B, r[2], ht);
                    dl = field_value<N1>(as_const(a.delta + (long long)e * V), hr, hs, ht);
                }
                a.res_dl[slot] = dl;
            }
        }
    }
    // wave totals -> counters
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) my_iters += __shfl_xor(my_iters, o, kWave);
    if (threadIdx.x == 0) {
        atomicAdd(&a.stats[0], (unsigned long long)(end - beg));
        atomicAdd(&a.stats[1], my_iters);
    }
}

// Owner selection per point (candidates are in ascending element order).
__global__ __launch_bounds__(256) void k_select(LocArgs a, int *__restrict__ code,
                                                int *__restrict__ el, double *__restrict__ rst,
                                                double *__restrict__ dist2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.npts) return;
    const int n = a.ncand[p];
    const long long s0 = (long long)p * a.MC;
    int w = -1, c = 2;
    bool anyin = false;
    for (int k = 0; k < n; ++k) anyin |= a.res_in[s0 + k] != 0;
    if (anyin) {
        c = 0;
        if (a.res_dl) {
            // best delta of each session among its inside candidates; the
            // largest wins (ties: smaller session), then the smallest element
            int bs = 0;
            double bd = -INFINITY;
            bool hv = false;
            for (int k = 0; k < n; ++k) {
                if (!a.res_in[s0 + k]) continue;
                const int sk = a.esess ? a.esess[a.cand_el[s0 + k]] : 0;
                double sd = -INFINITY;
                for (int u = 0; u < n; ++u) {
                    if (!a.res_in[s0 + u]) continue;
                    const int su = a.esess ? a.esess[a.cand_el[s0 + u]] : 0;
                    if (su == sk) sd = fmax(sd, a.res_dl[s0 + u]);
                }
                if (!hv || sd > bd || (sd == bd && sk < bs)) {
                    hv = true;
                    bd = sd;
                    bs = sk;
                }
            }
            for (int k = 0; k < n && w < 0; ++k) {
                if (!a.res_in[s0 + k]) continue;
                const int sk = a.esess ? a.esess[a.cand_el[s0 + k]] : 0;
                if (sk == bs) w = k;
            }
        } else {
            for (int k = 0; k < n && w < 0; ++k)
                if (a.res_in[s0 + k]) w = k;
        }
    } else if (n > 0) {
        c = 1;
        w = 0;
        for (int k = 1; k < n; ++k) {
            const double dk = a.res[4 * (s0 + k) + 3], dw = a.res[4 * (s0 + w) + 3];
            const bool tie = fabs(dk - dw) <= 1e-14 * fmax(dk, dw);
            if (!tie && dk < dw) w = k;  // ties keep the earlier (smaller) id
        }
    }
    code[p] = c;
    if (w < 0) {
        el[p] = -1;
        rst[3 * (long long)p] = rst[3 * (long long)p + 1] = rst[3 * (long long)p + 2] = 0.0;
        dist2[p] = INFINITY;
    } else {
        const double *o = a.res + 4 * (s0 + w);
        el[p] = a.cand_el[s0 + w];
        rst[3 * (long long)p] = o[0];
        rst[3 * (long long)p + 1] = o[1];
        rst[3 * (long long)p + 2] = o[2];
        dist2[p] = o[3];
    }
    atomicAdd(&a.stats[2], 1ULL);
}

#define FP_DISPATCH_N1(n1, MACRO) \
    switch (n1) {                 \
        case 2: MACRO(2); break;  \
        case 3: MACRO(3); break;  \
        case 4: MACRO(4); break;  \
        case 5: MACRO(5); break;  \
        case 6: MACRO(6); break;  \
        case 7: MACRO(7); break;  \
        case 8: MACRO(8); break;  \
        case 9: MACRO(9); break;  \
        case 10: MACRO(10); break; \
        case 11: MACRO(11); break; \
        case 12: MACRO(12); break; \
        case 13: MACRO(13); break; \
        case 14: MACRO(14); break; \
        case 15: MACRO(15); break; \
        case 16: MACRO(16); break; \
        default: return hipErrorInvalidValue; \
    }

static hipError_t launch_locate_kernel(const fp_handle *h, const LocArgs &a, hipStream_t s)
{
#define FP_LAUNCH_LOCATE(N1) k_locate<N1><<<h->E, kWave, 0, s>>>(a, h->d_basis)
    FP_DISPATCH_N1(h->n1, FP_LAUNCH_LOCATE);
#undef FP_LAUNCH_LOCATE
    return hipGetLastError();
}

}  // namespace fp

using namespace fp;

static void record(fp_handle *h, int phase, hipEvent_t a, hipEvent_t b)
{
    h->timed.push_back(TimedPair{phase, a, b});
}

extern "C" int findpts(fp_handle *h, int npts, const double *pts, const int *pt_session,
                       int *code, int *el, double *rst, double *dist2, void *stream)
{
    if (!h) {
        set_error("findpts: NULL handle");
        return FP_EINVAL;
    }
    if (npts < 0) {
        set_error("findpts: npts < 0");
        return FP_EINVAL;
    }
    if (npts == 0) return FP_OK;
    if (!pts || !code || !el || !rst || !dist2) {
        set_error("findpts: NULL argument");
        return FP_EINVAL;
    }
    if (h->precision != FP_PREC_FP64) {
        set_error("findpts: mixed precision is not available in this build");
        return FP_ESTATE;
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    FP_HIP(hipGetDevice(&dev));
    if (dev != h->device) FP_HIP(hipSetDevice(h->device));
    for (int start = 0; start < npts; start += h->max_points) {
        const int n = (npts - start < h->max_points) ? npts - start : h->max_points;
        LocArgs a{};
        a.geom = h->geom;
        a.esize = h->esize;
        a.bbox = h->bbox;
        a.delta = h->delta;
        a.esess = h->esess;
        a.cell_off = h->cell_off;
        a.cell_el = h->cell_el;
        a.g = h->grid;
        a.pts = pts + 3 * (long long)start;
        a.psess = pt_session ? pt_session + start : nullptr;
        a.npts = n;
        a.MC = h->MC;
        a.tol = h->tol;
        a.ncand = h->ncand;
        a.cand_el = h->cand_el;
        a.cand_pos = h->cand_pos;
        a.elem_cnt = h->elem_cnt;
        a.elem_off = h->elem_off;
        a.order = h->order;
        a.res = h->res;
        a.res_dl = h->delta ? h->res_dl : nullptr;
        a.res_in = h->res_in;
        a.stats = h->stats;

        hipEvent_t t0 = nullptr, t1 = nullptr, l0 = nullptr, l1 = nullptr;
        if (h->timing) {
            t0 = pool_event(h);
            t1 = pool_event(h);
            l0 = pool_event(h);
            l1 = pool_event(h);
            FP_HIP(hipEventRecord(t0, s));
        }
        const int pb = (n + 255) / 256;
        FP_HIP(fill_int(h->elem_cnt, 0, (long long)h->E + 1, s));
        k_cand<<<pb, 256, 0, s>>>(a);
        FP_HIP(hipGetLastError());
        FP_HIP(scan_exclusive(h->elem_cnt, h->elem_off, h->E, h->scan_tmp, s));
        k_scatter<<<pb, 256, 0, s>>>(a);
        FP_HIP(hipGetLastError());
        if (h->timing) FP_HIP(hipEventRecord(l0, s));
        FP_HIP(launch_locate_kernel(h, a, s));
        if (h->timing) FP_HIP(hipEventRecord(l1, s));
        k_select<<<pb, 256, 0, s>>>(a, code + start, el + start, rst + 3 * (long long)start,
                                   dist2 + start);
        FP_HIP(hipGetLastError());
        if (h->timing) {
            FP_HIP(hipEventRecord(t1, s));
            record(h, 0, l0, l1);
            record(h, 2, t0, t1);
        }
    }
    return FP_OK;
}
