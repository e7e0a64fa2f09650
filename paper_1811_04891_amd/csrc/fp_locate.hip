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
//   k_locate_mfma  (orders 1..7) one wavefront per work unit (a run of one
//              element's pairs), element block in LDS, map and Jacobian of 16
//              pairs at a time on the matrix cores (fp_mfma.inc)
//   k_locate   (orders 8..15) one wavefront per work unit of 64 pairs,
//              lanes = pairs, node rows through scalar loads
//   k_select   per point: classification and owner rule, caller's order
#include <algorithm>
#include <cmath>

#include "fp_basis.h"
#include "fp_internal.h"
#include "fp_mfma.h"

namespace fp {

struct LocArgs {
    const double *geom;
    const double *esize;
    const float *obb;    // non-null: also test the oriented box (first pass)
    const double *erec;  // per element, 16 doubles: axis-aligned box, oriented box
    int *redo;           // first pass writes 1 for tasks left without an inside
                         // candidate and with a partial candidate set, else 0
    const int *only;     // non-null (second pass): tasks with only[t] != 0
    int *gate;           // first pass: cleared by k_cand, set by k_select when any
                         // task is flagged; second pass: every kernel returns at
                         // once while it is zero
    const double *delta;
    const int *esess;
    const int *cell_off;
    const float4 *cell_box;  // per cell entry: binary32 outward box, element id
    Grid g;
    const double *pts;
    const int *psess;
    int npts;
    int M;  // candidate slots are candidate-major: slot(t, k) = k * M + t
    double tol;
    int *ncand;
    int *cand_el;
    int *cand_pos;
    int *elem_cnt;
    const int *elem_off;
    int E;
    int *order;
    double *res;
    double *res_dl;
    int *res_in;
    unsigned *cand_part;  // per k_cand block: the method's candidates (first pass)
    unsigned *iter_part;  // per block: Newton iterations of its pairs
    int pair_max;         // second pass, orders 1..7: up to this many pairs run on
                          // k_newton_pair (one wavefront per pair), else 0
};

__device__ __forceinline__ int cell_of(const Grid &g, int a, double x)
{
    double u = (x - g.lo[a]) * g.inv[a];
    int i = (int)floor(u);
    return i < 0 ? 0 : (i >= g.nc[a] ? g.nc[a] - 1 : i);
}

__device__ __forceinline__ bool task_on(const LocArgs &a, int t)
{
    return t < a.npts && (!a.only || a.only[t] != 0);
}

// res_in of a pair: 0 = solved, not inside; 1 = inside; kUnsolved = left by the
// mixed-precision first pass to the binary64 second pass
constexpr int kUnsolved = 2;
// res_in kOutside: the mixed-precision first pass found the point clearly
// outside the element (binary32 residual far above its rounding level on a
// face of [-1,1]^3): never inside; solved in binary64 only if the point has no
// inside candidate (its distance is then needed)
constexpr int kOutside = 3;

// ncand[t] = candidate count | (1 << kFullBit) when the list is the method's
// whole candidate set (no second pass needed for that point)
constexpr int kFullBit = 30;
constexpr int kCountMask = (1 << kFullBit) - 1;

// Candidates of one point: hash cell, then the closed axis-aligned box and
// the session exclusion (the method's candidate set), then, in the first
// pass, the oriented box.  The oriented box holds the whole element, so it
// never drops an element that contains the point; points left without an
// inside candidate get, in the second pass, the candidates the first pass
// dropped, appended after its own (whose results stay; a pair the binary32
// phase left unsolved is solved again in its slot).  cand_pos = -1 marks a
// slot that keeps its first-pass result.
__global__ __launch_bounds__(256) void k_cand(LocArgs a)
{
    if (a.only && !*a.gate) return;  // second pass with nothing flagged
    if (a.obb && blockIdx.x == 0 && threadIdx.x == 0) *a.gate = 0;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int naabb = 0, n = 0, n1st = 0;
    if (t < a.npts && a.only && !a.only[t]) {
        a.ncand[t] = 0;
    } else if (t < a.npts) {
        const int p = t;
        const double x0 = a.pts[3 * (long long)p], x1 = a.pts[3 * (long long)p + 1],
                     x2 = a.pts[3 * (long long)p + 2];
        const int ps = a.psess ? a.psess[p] : -1;
        int full = a.obb ? 0 : 1;
        bool take = true;
        if (a.only) {  // second pass: the first pass's candidates stay in their slots
            n1st = a.ncand[t] & kCountMask;
            n = n1st;
            // a first-pass list that is already the whole set (taken without
            // the oriented-box filter, or left intact by it) gets nothing
            // appended: only its unsolved slots are solved again
            take = (a.ncand[t] >> kFullBit) == 0;
        }
        const Grid &g = a.g;
        // NaN fails every comparison, so non-finite points find nothing
        if (take && x0 >= g.lo[0] && x0 <= g.hi[0] && x1 >= g.lo[1] && x1 <= g.hi[1] &&
            x2 >= g.lo[2] && x2 <= g.hi[2]) {
            const long long c = cell_of(g, 0, x0) +
                                (long long)g.nc[0] * (cell_of(g, 1, x1) +
                                                      (long long)g.nc[1] * cell_of(g, 2, x2));
            const int qb = a.cell_off[c], qe = a.cell_off[c + 1];
            // rounding is monotonic: x in [lo, hi] implies (float)x in the
            // outward-rounded binary32 box
            const float xf0 = (float)x0, xf1 = (float)x1, xf2 = (float)x2;
            int *ce = a.cand_el + t;
            // pass 0: oriented-box filter (first pass only); pass 1: every
            // candidate, taken when the filter left none (the point then
            // has its full candidate set and needs no second pass)
            for (int pass = a.obb ? 0 : 1; pass < 2 && (n == 0 || a.only); ++pass) {
                for (int q = qb; q < qe; ++q) {
                    // binary32 box (outward-rounded: a superset), then the
                    // exact binary64 box of the method
                    const float4 lo = a.cell_box[2 * (long long)q], hi = a.cell_box[2 * (long long)q + 1];
                    if (xf0 < lo.x || xf0 > hi.x || xf1 < lo.y || xf1 > hi.y || xf2 < lo.z ||
                        xf2 > hi.z)
                        continue;
                    const int e = __float_as_int(lo.w);
                    const double *b = a.erec + 16 * (long long)e;  // one line: both boxes
                    if (x0 < b[0] || x0 > b[1] || x1 < b[2] || x1 > b[3] || x2 < b[4] || x2 > b[5])
                        continue;
                    if (ps >= 0 && a.esess && a.esess[e] == ps) continue;
                    if (pass == 0 || a.only) {
                        ++naabb;
                        const float *o = (const float *)(b + 6);
                        const double d0 = x0 - (double)o[9], d1 = x1 - (double)o[10],
                                     d2 = x2 - (double)o[11];
                        bool in = true;
#pragma unroll
                        for (int ax = 0; ax < 3; ++ax) {
                            const double u = fma((double)o[3 * ax + 2], d2,
                                                 fma((double)o[3 * ax + 1], d1,
                                                     (double)o[3 * ax] * d0));
                            in = in && u >= (double)o[12 + ax] && u <= (double)o[15 + ax];
                        }
                        if (in == (a.only != nullptr)) continue;  // second pass: the dropped
                    }
                    ce[(long long)n * a.M] = e;
                    // a slot appended by the second pass is new: no state of
                    // an earlier call may read as a pair to resume
                    if (a.only) a.res_in[(long long)n * a.M + t] = 0;
                    ++n;
                }
                // the method's whole set: taken in pass 1, or left intact by
                // the oriented-box filter
                if (pass == 1 || naabb == 0 || n == naabb) full = 1;
                if (pass == 0 && naabb == 0) break;     // nothing to take
            }
        }
        a.ncand[t] = n | (full << kFullBit);
    }
    // each pair's rank in its element, from converged code so that lanes
    // sharing an element (a crowded element) share one atomic add
    int nmax = n;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nmax = max(nmax, __shfl_xor(nmax, o, kWave));
    for (int k = 0; k < nmax; ++k) {
        const long long s = (long long)k * a.M + t;
        // a first-pass slot is solved again only if it was left unsolved
        const bool act =
            k < n && (k >= n1st || a.res_in[s] == kUnsolved || a.res_in[s] == kOutside);
        const int e = act ? a.cand_el[s] : -1;
        const int r = wave_rank(a.elem_cnt, e, act);
        if (k < n) a.cand_pos[s] = act ? r : -1;
    }
    if (a.obb) {  // the method's candidates of this block (first pass covers every point)
        __shared__ unsigned wsum[256 / kWave];
        unsigned v = (unsigned)naabb;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned b = 0;
            for (int i = 0; i < 256 / kWave; ++i) b += wsum[i];
            a.cand_part[blockIdx.x] = b;
        }
    }
}

__global__ __launch_bounds__(256) void k_scatter(LocArgs a)
{
    if (a.only && !*a.gate) return;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.npts) return;
    const int n = a.ncand[p] & kCountMask;  // 0 for tasks the pass skips
    for (int k = 0; k < n; ++k) {
        const long long s = (long long)k * a.M + p;
        const int r = a.cand_pos[s];
        if (r >= 0) a.order[a.elem_off[a.cand_el[s]] + r] = (int)s;
    }
}

// 1 / x from the hardware reciprocal and two Newton-Raphson refinements
// (within an ulp or two of the quotient, no scaling for denormals: the
// trust-region step it scales does not need a correctly rounded quotient).
__device__ __forceinline__ double rcp64(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(fma(-x, y, 1.0), y, y);
    return fma(fma(-x, y, 1.0), y, y);
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
    const double inv = rcp64(det);
    d[0] = (c00 * b[0] + c10 * b[1] + c20 * b[2]) * inv;
    d[1] = (c01 * b[0] + c11 * b[1] + c21 * b[2]) * inv;
    d[2] = (c02 * b[0] + c12 * b[1] + c22 * b[2]) * inv;
    return det != 0.0 && isfinite(d[0]) && isfinite(d[1]) && isfinite(d[2]);
}

// Trust-region Newton constants (stop tests, radius rules).
constexpr double kResidStop = 1e-13;  // residual stop: at most kResidStop h_e
constexpr double kStepStop = 1e-13;   // accepted step with |s|_inf below this
constexpr double kStepTiny = 1e-15;   // no progress possible
constexpr int kMaxIter = 50;

// Squared residual at which Newton stops: a tenth of the inside tolerance,
// at most kResidStop, relative to h_e (a point the tolerance accepts is never
// left short of it).
__device__ __forceinline__ double resid_stop(double tol, double he)
{
    const double c = fmin(0.1 * tol, kResidStop) * he;
    return c * c;
}

// Projected trust-region Gauss-Newton on phi(r) = ||x(r) - x*||^2 over
// [-1,1]^3.  A coordinate on a bound whose descent direction points outward
// is held; the step solves J d = -F when every coordinate is free, else the
// reduced normal equations on the free ones (steepest descent if singular);
// it is scaled to the trust radius (max norm) and projected on the cube.
// rho = actual / predicted decrease; accept if rho >= 0.01; radius doubled
// (up to 2) when rho > 0.75 and the radius limited the step, set to |s|/4
// when rho < 0.25.  Stop: phi <= (min(1e-13, tol/10) h_e)^2, an accepted
// step with |s| <= 1e-13 (quadratic convergence: the point it reaches is at
// the map's rounding level), no possible progress, or 50 iterations.
struct TRNewton {
    double r[3], F[3], J[9], phi, D, pred, ns;
    double rt[3];  // next trial point
    double step_stop = kStepStop;
    int max_it = kMaxIter;
    bool limited, have;
    int it;

    __device__ __forceinline__ void start(const double (&r0)[3])
    {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            rt[d] = r0[d];
            r[d] = 0.0;
            F[d] = 0.0;
        }
#pragma unroll
        for (int d = 0; d < 9; ++d) J[d] = 0.0;
        phi = INFINITY;
        D = 1.0;
        pred = 0.0;
        ns = 0.0;
        limited = false;
        have = false;
        it = 0;
    }

    // Consume the map and Jacobian evaluated at rt; returns true when done,
    // otherwise leaves the next trial point in rt.
    __device__ __forceinline__ bool update(const double (&xt)[3], const double (&Jt)[9],
                                           const double (&xs)[3], double rstop)
    {
        return accept(xt, Jt, xs, rstop) || step();
    }

    // The two halves of update.  accept: take or reject the trial point rt
    // (model ratio, radius) and test the stop rules; true when done.
    __device__ __forceinline__ bool accept(const double (&xt)[3], const double (&Jt)[9],
                                           const double (&xs)[3], double rstop)
    {
        const double Ft[3] = {xt[0] - xs[0], xt[1] - xs[1], xt[2] - xs[2]};
        const double phit = fma(Ft[2], Ft[2], fma(Ft[1], Ft[1], Ft[0] * Ft[0]));
        bool acc = true, stop = false;
        if (have) {
            // rho = (phi - phit) / pred against 0.01, 0.75 and 0.25, with
            // pred > 0 (a step is only tried when its predicted decrease is)
            const double ared = phi - phit;
            acc = ared >= 0.01 * pred;
            if (ared > 0.75 * pred && limited)
                D = fmin(2.0 * D, 2.0);
            else if (ared < 0.25 * pred)
                D = 0.25 * ns;
            if (acc && ns <= step_stop) stop = true;
        }
        // branch-free update: the trial Jacobian is consumed on every path,
        // so its half of the contraction is not sunk into a branch away from
        // the pipelined node loads
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            r[d] = acc ? rt[d] : r[d];
            F[d] = acc ? Ft[d] : F[d];
        }
#pragma unroll
        for (int d = 0; d < 9; ++d) J[d] = acc ? Jt[d] : J[d];
        phi = acc ? phit : phi;
        have = true;
        return stop || phi <= rstop || it >= max_it;
    }

    // step: the next trial point rt from the accepted state; true when no
    // step can be taken (the pair is then done).
    __device__ __forceinline__ bool step()
    {
        ++it;
        double g[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) g[d] = fma(J[6 + d], F[2], fma(J[3 + d], F[1], J[d] * F[0]));
        double m[3];
        int nf = 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const bool held = (r[d] >= 1.0 && g[d] < 0.0) || (r[d] <= -1.0 && g[d] > 0.0);
            m[d] = held ? 0.0 : 1.0;
            nf += held ? 0 : 1;
        }
        if (nf == 0) return true;
        // one solve for both cases (lanes of a wavefront differ in nf): J d = -F
        // when all coordinates are free, else the reduced normal equations
        // (M J^T J M + I - M) d = -M g; a wavefront whose lanes are all free
        // (the usual case) skips forming the second
        double A[9], b[3], dl[3];
        if (__all(nf == 3)) {
#pragma unroll
            for (int u = 0; u < 3; ++u) {
#pragma unroll
                for (int v = 0; v < 3; ++v) A[3 * u + v] = J[3 * u + v];
                b[u] = -F[u];
            }
        } else {
#pragma unroll
            for (int u = 0; u < 3; ++u) {
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    const double jtj =
                        fma(J[6 + u], J[6 + v], fma(J[3 + u], J[3 + v], J[u] * J[v]));
                    const double red = m[u] * m[v] * jtj + ((u == v) ? 1.0 - m[u] : 0.0);
                    A[3 * u + v] = (nf == 3) ? J[3 * u + v] : red;
                }
                b[u] = (nf == 3) ? -F[u] : -m[u] * g[u];
            }
        }
        const bool ok = solve3(A, b, dl);
        if (!ok) {
#pragma unroll
            for (int d = 0; d < 3; ++d) dl[d] = -m[d] * g[d];
        }
        const double nd = fmax(fabs(dl[0]), fmax(fabs(dl[1]), fabs(dl[2])));
        if (!(nd > 0.0) || !isfinite(nd)) return true;
        limited = nd > D;
        const double sc = limited ? D * rcp64(nd) : 1.0;
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
        return ns <= kStepTiny || !(pred > 0.0);
    }
};

// Squared distance of a node from the point as the closest-node rule defines
// it: the squares of the x, y and z differences summed in that order, each
// operation rounded on its own (no fused multiply-add), so that near-ties are
// decided the same way whatever the scan's arithmetic.
__device__ __forceinline__ double node_dist2(double t0, double t1, double t2)
{
#pragma clang fp contract(off)
    return (t0 * t0 + t1 * t1) + t2 * t2;
}

// Reference coordinates of GLL node n (i + n1 (j + n1 k)).
template <int N1>
__device__ __forceinline__ void node_rst(BasisPtr<double> B, int n, double (&r)[3])
{
    const int i0 = n % N1, i1 = (n / N1) % N1, i2 = n / (N1 * N1);
    r[0] = r[1] = r[2] = 0.0;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
        const double zi = B.z(i);
        r[0] = (i == i0) ? zi : r[0];
        r[1] = (i == i1) ? zi : r[1];
        r[2] = (i == i2) ? zi : r[2];
    }
}

// Store one candidate's result (and the distance field if inside).
template <int N1>
__device__ __forceinline__ void store_pair(const LocArgs &a, BasisPtr<double> B, int slot, int e,
                                           const TRNewton &t, double he)
{
    constexpr int V = N1 * N1 * N1;
    double *o = a.res + 4 * (long long)slot;
    o[0] = t.r[0];
    o[1] = t.r[1];
    o[2] = t.r[2];
    o[3] = t.phi;
    const bool inside = sqrt(t.phi) <= a.tol * he;
    a.res_in[slot] = inside ? 1 : 0;
    if (a.res_dl) {
        double dl = 0.0;
        if (inside) {
            double hr[N1], hs[N1], ht[N1];
            lagrange<N1>(B, t.r[0], hr);
            lagrange<N1>(B, t.r[1], hs);
            lagrange<N1>(B, t.r[2], ht);
            dl = field_value_v<N1>(a.delta + (long long)e * V, hr, hs, ht);
        }
        a.res_dl[slot] = dl;
    }
}

// One 64-lane wavefront per work unit (up to 64 pairs of one element), lanes
// over its pairs, node rows from the scalar cache (orders 8 and above, whose
// matrix-core fragments would not fit in registers).
constexpr int kUnitScalar = 64;

// Map and Jacobian at GLL node nd of an element in global memory: the value
// is the node itself, each derivative a one-dimensional sum along its line
// (D = h_b'(z_a) at a n1 + b).
template <int N1>
__device__ __forceinline__ void node_geo_g(const double *__restrict__ X,
                                           const double *__restrict__ D, int nd,
                                           double (&x)[3], double (&J)[9])
{
    constexpr int V = N1 * N1 * N1;
    const int i0 = nd % N1, j0 = (nd / N1) % N1, k0 = nd / (N1 * N1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double *Xc = X + c * V;
        double dr = 0.0, ds = 0.0, dt = 0.0;
#pragma unroll
        for (int m = 0; m < N1; ++m) {
            dr = fma(Xc[nd - i0 + m], D[i0 * N1 + m], dr);
            ds = fma(Xc[nd + N1 * (m - j0)], D[j0 * N1 + m], ds);
            dt = fma(Xc[nd + N1 * N1 * (m - k0)], D[k0 * N1 + m], dt);
        }
        x[c] = Xc[nd];
        J[3 * c] = dr;
        J[3 * c + 1] = ds;
        J[3 * c + 2] = dt;
    }
}

template <int N1>
__global__ __launch_bounds__(kWave) void k_locate(LocArgs a, const double *__restrict__ basis,
                                                  const double *__restrict__ dnode)
{
    if (a.only && !*a.gate) return;
    constexpr int V = N1 * N1 * N1;
    const BasisPtr<double> B{as_const(basis)};
    unsigned long long my_iters = 0;
    const UnitList units(a.elem_off, a.E, 1, a.E, kUnitScalar);
    for (long long u = xcd_unit(blockIdx.x, gridDim.x); u < units.end; u += gridDim.x) {
        Unit U;
        if (!units.at(u, U)) continue;
        const int e = U.seg;
        cptr<double> X = as_const(a.geom + (long long)e * 3 * V);
        const double he = a.esize[e];
        const double rstop = resid_stop(a.tol, he);
        const int q = U.beg + (int)threadIdx.x;
        const bool act = q < U.end;
        const int slot = act ? a.order[q] : 0;
        const int p = slot % a.M;
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
            const double d = node_dist2(X[n] - xs[0], X[V + n] - xs[1], X[2 * V + n] - xs[2]);
            if (d < best) {
                best = d;
                bq = n;
            }
        }
        double r0[3];
        node_rst<N1>(B, bq, r0);
        TRNewton t;
        t.start(r0);
        // the first Newton step from the node's own value and line sums
        bool done = !act;
        if (act) {
            double xn[3], Jn[9];
            node_geo_g<N1>(a.geom + (long long)e * 3 * V, dnode, bq, xn, Jn);
            done = t.update(xn, Jn, xs, rstop);
        }
        while (!done) {
            double xt[3], Jt[9];
            geo_eval<N1>(X, B, t.rt, xt, Jt);
            done = t.update(xt, Jt, xs, rstop);
        }
        if (act) {
            my_iters += (unsigned long long)t.it;
            store_pair<N1>(a, B, slot, e, t, he);
        }
    }
    // wave totals -> counters
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) my_iters += __shfl_xor(my_iters, o, kWave);
    if (threadIdx.x == 0) a.iter_part[blockIdx.x] = (unsigned)my_iters;
}

#include "fp_mfma.inc"
#include "fp_newton8.inc"
#include "fp_mixed8.inc"
#include "fp_newton_pl.inc"
#include "fp_pair.inc"

constexpr int kStatsBlocks = 32;

// Fold one pass's partial counts into the handle's counters: a few blocks,
// each adding its share with one atomic per counter.
__global__ __launch_bounds__(1024) void k_stats(const unsigned *cand_part, int nb,
                                                const unsigned *iter_part, int ni, int E,
                                                const int *elem_off, long long located,
                                                int first, const int *gate,
                                                unsigned long long *stats)
{
    if (gate && !*gate) return;
    __shared__ unsigned long long sc[1024 / kWave], si[1024 / kWave];
    unsigned long long c = 0, it = 0;
    const int stride = blockDim.x * gridDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += stride) c += cand_part[i];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ni; i += stride) it += iter_part[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o, kWave);
        it += __shfl_xor(it, o, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sc[threadIdx.x / kWave] = c;
        si[threadIdx.x / kWave] = it;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long C = 0, I = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
            C += sc[w];
            I += si[w];
        }
        const unsigned long long pairs = blockIdx.x == 0 ? (unsigned long long)elem_off[E] : 0ull;
        if (pairs) atomicAdd(&stats[0], pairs);
        if (I) atomicAdd(&stats[1], I);
        if (first) {
            if (pairs) atomicAdd(&stats[4], pairs);
            if (I) atomicAdd(&stats[5], I);
        }
        if (located && blockIdx.x == 0) atomicAdd(&stats[2], (unsigned long long)located);
        if (C) atomicAdd(&stats[3], C);
    }
}

// Owner selection per point; ownership and ties go by explicit element ids
// (the second pass appends the candidates the first dropped, unsorted).
__global__ __launch_bounds__(256) void k_select(LocArgs a, int *__restrict__ code,
                                                int *__restrict__ el, double *__restrict__ rst,
                                                double *__restrict__ dist2)
{
    if (a.only && !*a.gate) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (!task_on(a, t)) return;
    const int p = t;
    const int nv = a.ncand[t];
    const int n = nv & kCountMask;
    const bool full = (nv >> kFullBit) != 0;
    auto S =[&](int k) { return (long long)k * a.M + t; };
    int w = -1, c = 2;
    bool anyin = false, unsolved = false, outside = false;
    for (int k = 0; k < n; ++k) {
        const int in = a.res_in[S(k)];
        anyin |= in == 1;
        unsolved |= in == kUnsolved;
        outside |= in == kOutside;
    }
    if (anyin) {
        c = 0;
        if (a.res_dl) {
            // best delta of each session among its inside candidates; the
            // largest wins (ties: smaller session), then the smallest element
            int bs = 0;
            double bd = -INFINITY;
            bool hv = false;
            for (int k = 0; k < n; ++k) {
                if (a.res_in[S(k)] != 1) continue;
                const int sk = a.esess ? a.esess[a.cand_el[S(k)]] : 0;
                double sd = -INFINITY;
                for (int u = 0; u < n; ++u) {
                    if (a.res_in[S(u)] != 1) continue;
                    const int su = a.esess ? a.esess[a.cand_el[S(u)]] : 0;
                    if (su == sk) sd = fmax(sd, a.res_dl[S(u)]);
                }
                if (!hv || sd > bd || (sd == bd && sk < bs)) {
                    hv = true;
                    bd = sd;
                    bs = sk;
                }
            }
            for (int k = 0; k < n; ++k) {
                if (a.res_in[S(k)] != 1) continue;
                const int sk = a.esess ? a.esess[a.cand_el[S(k)]] : 0;
                if (sk == bs && (w < 0 || a.cand_el[S(k)] < a.cand_el[S(w)])) w = k;
            }
        } else {
            for (int k = 0; k < n; ++k)
                if (a.res_in[S(k)] == 1 && (w < 0 || a.cand_el[S(k)] < a.cand_el[S(w)])) w = k;
        }
    } else if (unsolved || outside) {
        c = 1;  // provisional: the second pass decides
    } else if (n > 0) {
        c = 1;
        w = 0;
        for (int k = 1; k < n; ++k) {
            const double dk = a.res[4 * (S(k)) + 3], dw = a.res[4 * (S(w)) + 3];
            const bool tie = fabs(dk - dw) <= 1e-14 * fmax(dk, dw);
            // ties go to the smaller element id (the second pass appends the
            // candidates the first dropped, so the list is not sorted)
            if ((!tie && dk < dw) || (tie && a.cand_el[S(k)] < a.cand_el[S(w)])) w = k;
        }
    }
    code[p] = c;
    if (w < 0) {
        el[p] = -1;
        rst[3 * (long long)p] = rst[3 * (long long)p + 1] = rst[3 * (long long)p + 2] = 0.0;
        dist2[p] = INFINITY;
    } else {
        const double *o = a.res + 4 * (S(w));
        el[p] = a.cand_el[S(w)];
        rst[3 * (long long)p] = o[0];
        rst[3 * (long long)p + 1] = o[1];
        rst[3 * (long long)p + 2] = o[2];
        dist2[p] = o[3];
    }
    if (a.obb) {
        bool redo = c != 0 && (!full || unsolved || outside);
        if (c == 0 && unsolved) {
            // a pair the binary32 phase left unsolved may be inside too: with
            // the distance field it may belong to a session with a larger
            // delta, without it a smaller element id wins; the second pass
            // solves it in binary64 and selects again
            for (int k = 0; k < n; ++k)
                if (a.res_in[S(k)] == kUnsolved &&
                    (a.res_dl || a.cand_el[S(k)] < a.cand_el[S(w)]))
                    redo = true;
        }
        a.redo[t] = redo ? 1 : 0;
        // open the second pass (one store per wavefront with a flagged task)
        const unsigned long long b = __ballot(redo);
        if (b != 0ull && (int)(threadIdx.x & (kWave - 1)) == __ffsll((long long)b) - 1) *a.gate = 1;
    }
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

// Launches the order's Newton kernel over the work units of the pass's pairs
// (n points); *nblk receives the grid size (one iteration partial per block).
static hipError_t launch_locate_kernel(const fp_handle *h, const LocArgs &a, int n,
                                       hipStream_t s, int *nblk)
{
#define FP_GRID(K) (a.only ? std::min(unit_grid(h->E, n, (K)), kSecondPassGrid) \
                           : unit_grid(h->E, n, (K)))
#define FP_LAUNCH_LOCATE(N1)                                      \
    do {                                                          \
        *nblk = FP_GRID(kUnitScalar);                             \
        k_locate<N1><<<*nblk, kWave, 0, s>>>(a, h->d_basis, h->d_dnode); \
    } while (0)
// mixed precision: first pass only (the second pass is binary64).  At order 5
// the binary64 kernel (two wavefronts per SIMD) is faster than the binary32
// design of orders <= 6, so a mixed-precision handle locates in binary64 there.
constexpr int kBinary64Only = 6;
// mixed precision: first pass only (the second pass is binary64)
#define FP_LAUNCH_MFMA(N1)                                                           \
    do {                                                                             \
        if (h->precision == FP_PREC_MIXED && a.obb && N1 == kN8) {                   \
            *nblk = FP_GRID(kUnitMixed);                                             \
            k_mixed8<<<*nblk, kWave, 0, s>>>(a, h->d_basis, h->d_basis32, h->d_dnode); \
        } else if (h->precision == FP_PREC_MIXED && a.obb && N1 != kBinary64Only) {  \
            *nblk = FP_GRID(kUnitMixed);                                             \
            k_locate_mixed<N1><<<*nblk, kWave, 0, s>>>(a, h->d_basis, h->d_basis32,  \
                                                        h->d_dnode);                 \
        } else if (N1 == kN8) {                                                      \
            *nblk = FP_GRID(kUnitMfma);                                              \
            k_newton8<<<*nblk, kWave, 0, s>>>(a, h->d_basis, h->d_dnode);            \
        } else {                                                                     \
            *nblk = FP_GRID(kUnitMfma);                                              \
            k_locate_mfma<N1><<<*nblk, kWave, 0, s>>>(a, h->d_basis, h->d_dnode);     \
        }                                                                            \
        if (a.only && a.pair_max > 0)                                                \
            k_newton_pair<N1><<<*nblk, kWave, 0, s>>>(a, h->d_basis);                 \
    } while (0)
// orders 8 and 9: matrix cores, one plane per lane; mixed precision (first
// pass): a binary32 phase, then binary64 Newton from its end points
#define FP_LAUNCH_PL(N1)                                                              \
    do {                                                                              \
        *nblk = FP_GRID(kUnitPl);                                                     \
        if (h->precision == FP_PREC_MIXED && a.obb) {                                 \
            k_mixed_pl<N1><<<*nblk, 2 * kWave, 0, s>>>(a, h->d_basis32, h->d_dnode); \
            k_newton_pl<N1, true><<<*nblk, 2 * kWave, 0, s>>>(a, h->d_basis, h->d_basis32, \
                                                             h->d_dnode);             \
        } else                                                                        \
            k_newton_pl<N1, false><<<*nblk, 2 * kWave, 0, s>>>(a, h->d_basis, h->d_basis32, \
                                                              h->d_dnode);            \
    } while (0)
    switch (h->n1) {
        case 2: FP_LAUNCH_MFMA(2); break;
        case 3: FP_LAUNCH_MFMA(3); break;
        case 4: FP_LAUNCH_MFMA(4); break;
        case 5: FP_LAUNCH_MFMA(5); break;
        case 6: FP_LAUNCH_MFMA(6); break;
        case 7: FP_LAUNCH_MFMA(7); break;
        case 8: FP_LAUNCH_MFMA(8); break;
        case 9: FP_LAUNCH_PL(9); break;
        case 10: FP_LAUNCH_PL(10); break;
        case 11: FP_LAUNCH_LOCATE(11); break;
        case 12: FP_LAUNCH_LOCATE(12); break;
        case 13: FP_LAUNCH_LOCATE(13); break;
        case 14: FP_LAUNCH_LOCATE(14); break;
        case 15: FP_LAUNCH_LOCATE(15); break;
        case 16: FP_LAUNCH_LOCATE(16); break;
        default: return hipErrorInvalidValue;
    }
#undef FP_LAUNCH_LOCATE
#undef FP_LAUNCH_MFMA
#undef FP_LAUNCH_PL
#undef FP_GRID
    return hipGetLastError();
}

}  // namespace fp

using namespace fp;

static void record(fp_handle *h, int phase, hipEvent_t a, hipEvent_t b)
{
    h->timed.push_back(TimedPair{phase, a, b});
}

namespace fp {

int run_findpts(fp_handle *h, const Work &w, int npts, const double *pts, const int *pt_session,
                int *code, int *el, double *rst, double *dist2, hipStream_t s, bool timed)
{
    for (int start = 0; start < npts; start += w.M) {
        const int n = (npts - start < w.M) ? npts - start : w.M;
        LocArgs a{};
        a.geom = h->geom;
        a.esize = h->esize;
        a.erec = h->erec;
        a.delta = h->delta;
        a.esess = h->esess;
        a.cell_off = h->cell_off;
        a.cell_box = h->cell_box;
        a.g = h->grid;
        a.pts = pts + 3 * (long long)start;
        a.psess = pt_session ? pt_session + start : nullptr;
        a.npts = n;
        a.M = w.M;
        a.tol = h->tol;
        a.ncand = w.ncand;
        a.cand_el = w.cand_el;
        a.cand_pos = w.cand_pos;
        a.elem_cnt = w.elem_cnt;
        a.elem_off = w.elem_off;
        a.E = h->E;
        a.order = w.order;
        a.res = w.res;
        a.res_dl = h->delta ? w.res_dl : nullptr;
        a.res_in = w.res_in;
        a.cand_part = w.cand_part;
        a.iter_part = w.iter_part;
        a.gate = w.gate;

        hipEvent_t t0 = nullptr, t1 = nullptr, l0 = nullptr, l1 = nullptr;
        if (timed) {
            t0 = pool_event(h);
            t1 = pool_event(h);
            l0 = pool_event(h);
            l1 = pool_event(h);
            FP_HIP(hipEventRecord(t0, s));
        }
        const int pb = (n + 255) / 256;
        int *co = code + start, *eo = el + start;
        double *ro = rst + 3 * (long long)start, *dO = dist2 + start;
        // first pass: oriented-box candidates; tasks without an inside
        // candidate (and with a partial candidate set) are flagged for the
        // second pass
        a.obb = h->obb;
        a.redo = w.redo;
        FP_HIP(fill_int(w.elem_cnt, 0, (long long)h->E + 1, s));
        k_cand<<<pb, 256, 0, s>>>(a);
        FP_HIP(hipGetLastError());
        FP_HIP(scan_exclusive(w.elem_cnt, w.elem_off, h->E, w.scan_tmp, s));
        k_scatter<<<pb, 256, 0, s>>>(a);
        FP_HIP(hipGetLastError());
        if (timed) FP_HIP(hipEventRecord(l0, s));
        int nblk = 0;
        FP_HIP(launch_locate_kernel(h, a, n, s, &nblk));
        if (timed) FP_HIP(hipEventRecord(l1, s));
        k_select<<<pb, 256, 0, s>>>(a, co, eo, ro, dO);
        FP_HIP(hipGetLastError());
        k_stats<<<kStatsBlocks, 1024, 0, s>>>(w.cand_part, pb, w.iter_part, nblk, h->E,
                                              w.elem_off, n, 1, nullptr, h->stats);
        FP_HIP(hipGetLastError());
        // second pass over the flagged tasks with the axis-aligned candidates
        // only (other tasks get no candidates and keep their result)
        a.obb = nullptr;
        a.redo = nullptr;
        a.only = w.redo;
        a.pair_max = h->n1 <= kN8 ? kPairMax : 0;
        FP_HIP(fill_int_gated(w.elem_cnt, 0, (long long)h->E + 1, w.gate, s));
        k_cand<<<pb, 256, 0, s>>>(a);
        FP_HIP(hipGetLastError());
        FP_HIP(scan_exclusive(w.elem_cnt, w.elem_off, h->E, w.scan_tmp, s, w.gate));
        k_scatter<<<pb, 256, 0, s>>>(a);
        FP_HIP(hipGetLastError());
        hipEvent_t m0 = nullptr, m1 = nullptr;
        if (timed) {
            m0 = pool_event(h);
            m1 = pool_event(h);
            FP_HIP(hipEventRecord(m0, s));
        }
        FP_HIP(launch_locate_kernel(h, a, n, s, &nblk));
        if (timed) {
            FP_HIP(hipEventRecord(m1, s));
            record(h, 4, m0, m1);
        }
        k_select<<<pb, 256, 0, s>>>(a, co, eo, ro, dO);
        FP_HIP(hipGetLastError());
        k_stats<<<kStatsBlocks, 1024, 0, s>>>(w.cand_part, 0, w.iter_part, nblk, h->E,
                                              w.elem_off, 0, 0, w.gate, h->stats);
        FP_HIP(hipGetLastError());
        if (timed) {
            FP_HIP(hipEventRecord(t1, s));
            record(h, 0, l0, l1);
            record(h, 2, t0, t1);
        }
    }
    return FP_OK;
}

}  // namespace fp

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
    int dev = 0;
    FP_HIP(hipGetDevice(&dev));
    if (dev != h->device) FP_HIP(hipSetDevice(h->device));
    return run_findpts(h, h->work, npts, pts, pt_session, code, el, rst, dist2,
                       (hipStream_t)stream, h->timing);
}
