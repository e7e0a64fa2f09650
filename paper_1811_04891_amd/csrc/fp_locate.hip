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
    const double *obb;   // non-null: also test the oriented box (first pass)
    const int *idx;      // non-null: task t is point idx[t] (second pass)
    const int *dcount;   // non-null: number of tasks, read on the device
    int *redo;           // first pass: points without an inside candidate
    int *redo_n;
    const double *delta;
    const int *esess;
    const int *cell_off;
    const int *cell_el;
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

__device__ __forceinline__ int task_count(const LocArgs &a)
{
    return a.dcount ? *a.dcount : a.npts;
}

// ncand[t] = candidate count | (1 << kFullBit) when the list is the method's
// whole candidate set (no second pass needed for that point)
constexpr int kFullBit = 30;
constexpr int kCountMask = (1 << kFullBit) - 1;

// Candidates of one point: hash cell, then the closed axis-aligned box and
// the session exclusion (the method's candidate set), then, in the first
// pass, the oriented box.  The oriented box holds the whole element, so it
// never drops an element that contains the point; points left without an
// inside candidate are redone with the axis-aligned set alone.
__global__ __launch_bounds__(256) void k_cand(LocArgs a)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int naabb = 0;
    if (t < task_count(a)) {
        const int p = a.idx ? a.idx[t] : t;
        const double x0 = a.pts[3 * (long long)p], x1 = a.pts[3 * (long long)p + 1],
                     x2 = a.pts[3 * (long long)p + 2];
        const int ps = a.psess ? a.psess[p] : -1;
        int n = 0, full = a.obb ? 0 : 1;
        const Grid &g = a.g;
        // NaN fails every comparison, so non-finite points find nothing
        if (x0 >= g.lo[0] && x0 <= g.hi[0] && x1 >= g.lo[1] && x1 <= g.hi[1] &&
            x2 >= g.lo[2] && x2 <= g.hi[2]) {
            const long long c = cell_of(g, 0, x0) +
                                (long long)g.nc[0] * (cell_of(g, 1, x1) +
                                                      (long long)g.nc[1] * cell_of(g, 2, x2));
            const int qb = a.cell_off[c], qe = a.cell_off[c + 1];
            int *ce = a.cand_el + t;
            int *cp = a.cand_pos + t;
            // pass 0: oriented-box filter (first pass only); pass 1: every
            // candidate, taken when the filter left none (the point then
            // has its full candidate set and needs no second pass)
            for (int pass = a.obb ? 0 : 1; pass < 2 && n == 0; ++pass) {
                for (int q = qb; q < qe; ++q) {
                    const int e = a.cell_el[q];
                    const double *b = a.bbox + 6 * (long long)e;
                    if (x0 < b[0] || x0 > b[1] || x1 < b[2] || x1 > b[3] || x2 < b[4] || x2 > b[5])
                        continue;
                    if (ps >= 0 && a.esess && a.esess[e] == ps) continue;
                    if (pass == 0) {
                        ++naabb;
                        const double *o = a.obb + 18 * (long long)e;
                        const double d0 = x0 - o[9], d1 = x1 - o[10], d2 = x2 - o[11];
                        bool in = true;
#pragma unroll
                        for (int ax = 0; ax < 3; ++ax) {
                            const double u =
                                fma(o[3 * ax + 2], d2, fma(o[3 * ax + 1], d1, o[3 * ax] * d0));
                            in = in && u >= o[12 + ax] && u <= o[15 + ax];
                        }
                        if (!in) continue;
                    }
                    ce[(long long)n * a.M] = e;
                    cp[(long long)n * a.M] = atomicAdd(&a.elem_cnt[e], 1);
                    ++n;
                }
                if (pass == 1 || naabb == 0) full = 1;  // the method's whole set
                if (pass == 0 && naabb == 0) break;     // nothing to take
            }
        }
        a.ncand[t] = n | (full << kFullBit);
    }
    if (a.obb) {  // count the method's candidates (first pass covers every point)
        unsigned long long v = (unsigned long long)naabb;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && v) atomicAdd(&a.stats[3], v);
    }
}

__global__ __launch_bounds__(256) void k_scatter(LocArgs a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= task_count(a)) return;
    const int n = a.ncand[p] & kCountMask;
    for (int k = 0; k < n; ++k) {
        const long long s = (long long)k * a.M + p;
        const int e = a.cand_el[s];
        a.order[a.elem_off[e] + a.cand_pos[s]] = (int)s;
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

// Projected trust-region Gauss-Newton on phi(r) = ||x(r) - x*||^2 over
// [-1,1]^3.  A coordinate on a bound whose descent direction points outward
// is held; the step solves J d = -F when every coordinate is free, else the
// reduced normal equations on the free ones (steepest descent if singular);
// it is scaled to the trust radius (max norm) and projected on the cube.
// rho = actual / predicted decrease; accept if rho >= 0.01; radius doubled
// (up to 2) when rho > 0.75 and the radius limited the step, set to |s|/4
// when rho < 0.25.  Stop: phi <= (1e-13 h_e)^2, an accepted step with
// |s| <= 1e-13, no possible progress, or 50 iterations.
struct TRNewton {
    double r[3], F[3], J[9], phi, D, pred, ns;
    double rt[3];  // next trial point
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
        if (stop || phi <= rstop || it >= kMaxIter) return true;
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
                    const double jtj = fma(J[6 + u], J[6 + v], fma(J[3 + u], J[3 + v], J[u] * J[v]));
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
        if (!(nd > 0.0) || !isfinite(nd)) return true;
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
        return ns <= kStepTiny || !(pred > 0.0);
    }
};

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

// One 64-lane wavefront per element, node rows from the scalar cache (used
// for orders above 9, whose element block does not fit the LDS budget).
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
        const int tk = slot % a.M;
        const int p = a.idx ? a.idx[tk] : tk;
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
        double r0[3];
        node_rst<N1>(B, bq, r0);
        TRNewton t;
        t.start(r0);
        bool done = !act;
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
    if (threadIdx.x == 0) {
        atomicAdd(&a.stats[0], (unsigned long long)(end - beg));
        atomicAdd(&a.stats[1], my_iters);
    }
}

// Element groups staged in LDS.  A 256-thread block owns G consecutive
// elements and every (point, element) pair of them (contiguous in the
// element-grouped order).  After staging the G element blocks (each padded
// by 16 bytes so that lanes reading different elements hit different LDS
// banks), the block first finds every pair's closest node (full-width
// scans), then runs Newton with lane refill: a lane that finishes its pair
// takes the next unstarted pair of the group, so lanes stay busy while
// iteration counts differ.
constexpr int kGrpThreads = 256;

template <int N1>
struct Group {
    static constexpr int V = N1 * N1 * N1;
    static constexpr int stride = 3 * V + 2;  // doubles per staged element
    static constexpr int G = (3 * V * 8 <= 6 * 1024) ? 8 : (3 * V * 8 <= 12 * 1024 ? 4 : 2);
    static constexpr int lds_bytes = G * stride * 8;
};

template <int N1>
__global__ __launch_bounds__(kGrpThreads) void k_locate_grp(LocArgs a,
                                                          const double *__restrict__ basis,
                                                          int E)
{
    using Gr = Group<N1>;
    constexpr int V = Gr::V, G = Gr::G, S = Gr::stride;
    __shared__ double sX[G * S];
    __shared__ int next;
    const BasisPtr<double> B{as_const(basis)};
    const int e0 = blockIdx.x * G;
    const int ne = min(G, E - e0);
    const int pb = a.elem_off[e0], pe = a.elem_off[e0 + ne];
    const int count = pe - pb;
    if (count <= 0) return;  // uniform across the block
    // stage the elements that have pairs (others are never read)
    for (int g = 0; g < ne; ++g) {
        if (a.elem_off[e0 + g + 1] == a.elem_off[e0 + g]) continue;
        const double2 *src = (const double2 *)(a.geom + (long long)(e0 + g) * 3 * V);
        double *dst = sX + g * S;
        for (int q = threadIdx.x; q < 3 * V / 2; q += kGrpThreads) {
            const double2 v = src[q];
            dst[2 * q] = v.x;
            dst[2 * q + 1] = v.y;
        }
        if ((3 * V) & 1) {
            if (threadIdx.x == 0) dst[3 * V - 1] = a.geom[(long long)(e0 + g) * 3 * V + 3 * V - 1];
        }
    }
    if (threadIdx.x == 0) next = kGrpThreads;
    __syncthreads();

    // closest node of every pair (stored in cand_pos, free after the scatter)
    for (int u = threadIdx.x; u < count; u += kGrpThreads) {
        const int slot = a.order[pb + u];
        const int tk = slot % a.M;
        const int p = a.idx ? a.idx[tk] : tk;
        const int g = a.cand_el[slot] - e0;
        const double x0 = a.pts[3 * (long long)p], x1 = a.pts[3 * (long long)p + 1],
                     x2 = a.pts[3 * (long long)p + 2];
        lptr<double> X = (lptr<double>)(sX + g * S);
        double best = INFINITY;
        int bq = 0;
#pragma unroll 8
        for (int n = 0; n < V; ++n) {
            const double dx = X[n] - x0, dy = X[V + n] - x1, dz = X[2 * V + n] - x2;
            const double d = fma(dz, dz, fma(dy, dy, dx * dx));
            if (d < best) {
                best = d;
                bq = n;
            }
        }
        a.cand_pos[slot] = bq;
    }
    __syncthreads();

    // Newton with lane refill
    unsigned long long my_iters = 0;
    int u = threadIdx.x;
    int slot = 0, g = 0;
    double xs[3] = {0.0, 0.0, 0.0}, he = 0.0, rstop = 0.0;
    TRNewton t;
    auto begin_pair = [&](int uu) {
        slot = a.order[pb + uu];
        const int tk = slot % a.M;
        const int p = a.idx ? a.idx[tk] : tk;
        g = a.cand_el[slot] - e0;
        xs[0] = a.pts[3 * (long long)p];
        xs[1] = a.pts[3 * (long long)p + 1];
        xs[2] = a.pts[3 * (long long)p + 2];
        he = a.esize[e0 + g];
        rstop = (kResidStop * he) * (kResidStop * he);
        double r0[3];
        node_rst<N1>(B, a.cand_pos[slot], r0);
        t.start(r0);
    };
    if (u < count) begin_pair(u);
    while (u < count) {
        double xt[3], Jt[9];
        geo_eval_lds<N1>((lptr<double>)(sX + g * S), B, t.rt, xt, Jt);
        if (t.update(xt, Jt, xs, rstop)) {
            my_iters += (unsigned long long)t.it;
            store_pair<N1>(a, B, slot, e0 + g, t, he);
            u = atomicAdd(&next, 1);
            if (u < count) begin_pair(u);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) my_iters += __shfl_xor(my_iters, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicAdd(&a.stats[1], my_iters);
        if (threadIdx.x == 0) atomicAdd(&a.stats[0], (unsigned long long)count);
    }
}

// ---------------------------------------------------------------------------
// Matrix-core Newton.  For the pairs of one element the first contraction of
// the element map, a(c,k,j; point) = sum_i X_c[k][j][i] h_i(r_point), is a
// dense product (element rows x basis values of 16 points), done with the
// 16x16x4 MFMA.  One wavefront per element: 16 pair slots, slot n owning the
// 4 lanes n + 16 g (g = 0..3) -- the lanes that hold column n of the B
// operand and of the result.  The element's A fragments stay in registers
// for all its pairs.  Lane g holds, for each plane (c, k) of an M block,
// the rows j = g + 4 w; it contracts them with h_j(s), then with h_k(t), and
// the 4 lanes of a slot add their partial sums by a butterfly, which gives
// bit-identical totals in all 4 lanes (IEEE addition commutes), so the 4
// copies of the slot's Newton state stay in step.
// ---------------------------------------------------------------------------
typedef double dx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dx4 mfma16(double a, double b, dx4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// f64 16x16x4 result layout: row i, column j at lane j + 16 (i % 4),
// component i / 4.
__device__ __forceinline__ int mrow(int g, int v) { return 4 * v + g; }

template <int N1>
struct MShape {
    static constexpr int JP = N1 <= 4 ? 4 : (N1 <= 8 ? 8 : 16);  // padded rows per plane
    static constexpr int PPB = 16 / JP;                           // planes per M block
    static constexpr int NPL = 3 * N1;                            // planes (c, k)
    static constexpr int MB = (NPL + PPB - 1) / PPB;              // M blocks
    static constexpr int KB = (N1 + 3) / 4;                       // K blocks (over i)
    static constexpr int EPP = JP / 4;                            // rows per plane and lane
    static constexpr int V = N1 * N1 * N1;
    static constexpr int SB = (V + 15) / 16;                      // node blocks (start scan)
};

// A fragments of one element: A[mb][kb] at lane l = row + 16 q holds
// X_c[k][j][i] for i = 4 kb + q and the (c, k, j) of row `row` of block mb.
template <int N1>
__device__ __forceinline__ void load_afrag(lptr<double> X, int lane,
                                           double (&A)[MShape<N1>::MB][MShape<N1>::KB])
{
    using S = MShape<N1>;
    const int row = lane & 15, q = lane >> 4;
    const int gr = row % 4, vr = row / 4;  // inverse of mrow
    const int p = vr / S::EPP, jj = gr + 4 * (vr % S::EPP);
#pragma unroll
    for (int mb = 0; mb < S::MB; ++mb) {
        const int P = mb * S::PPB + p;
        const int c = P / N1, k = P % N1;
#pragma unroll
        for (int kb = 0; kb < S::KB; ++kb) {
            const int i = 4 * kb + q;
            const bool ok = P < S::NPL && jj < N1 && i < N1;
            A[mb][kb] = ok ? X[c * S::V + N1 * (jj + N1 * k) + i] : 0.0;
        }
    }
}

// Basis values one lane needs for its slot's trial point.
template <int N1>
struct LaneBasis {
    double hrl[MShape<N1>::KB], drl[MShape<N1>::KB];   // h_i(r), i = 4 kb + g
    double hsl[MShape<N1>::EPP], dsl[MShape<N1>::EPP]; // h_j(s), j = g + 4 w
    double ht[N1], dt[N1];
};

template <int N1>
__device__ __forceinline__ void lane_basis(BasisPtr<double> B, const double (&r)[3], int g,
                                           LaneBasis<N1> &L)
{
    using S = MShape<N1>;
    double h[N1], d[N1];
    lagrange_d<N1>(B, r[0], h, d);
#pragma unroll
    for (int kb = 0; kb < S::KB; ++kb) {
        double hv = 0.0, dv = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = 4 * kb + q;
            if (i < N1) {
                hv = (g == q) ? h[i] : hv;
                dv = (g == q) ? d[i] : dv;
            }
        }
        L.hrl[kb] = hv;
        L.drl[kb] = dv;
    }
    lagrange_d<N1>(B, r[1], h, d);
#pragma unroll
    for (int w = 0; w < S::EPP; ++w) {
        double hv = 0.0, dv = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = q + 4 * w;
            if (j < N1) {
                hv = (g == q) ? h[j] : hv;
                dv = (g == q) ? d[j] : dv;
            }
        }
        L.hsl[w] = hv;
        L.dsl[w] = dv;
    }
    lagrange_d<N1>(B, r[2], L.ht, L.dt);
}

__device__ __forceinline__ double xor_add(double v, int m)
{
    return v + __shfl_xor(v, m, kWave);
}

// Map and Jacobian at the slots' trial points (all 64 lanes take part).
template <int N1>
__device__ __forceinline__ void mfma_geo(const double (&A)[MShape<N1>::MB][MShape<N1>::KB],
                                         const LaneBasis<N1> &L, double (&x)[3], double (&J)[9])
{
    using S = MShape<N1>;
    double v[3] = {0, 0, 0}, vr[3] = {0, 0, 0}, vs[3] = {0, 0, 0}, vt[3] = {0, 0, 0};
#pragma unroll
    for (int mb = 0; mb < S::MB; ++mb) {
        dx4 ch = {0, 0, 0, 0}, cd = {0, 0, 0, 0};
#pragma unroll
        for (int kb = 0; kb < S::KB; ++kb) {
            ch = mfma16(A[mb][kb], L.hrl[kb], ch);
            cd = mfma16(A[mb][kb], L.drl[kb], cd);
        }
#pragma unroll
        for (int p = 0; p < S::PPB; ++p) {
            const int P = mb * S::PPB + p;
            if (P < S::NPL) {
                const int c = P / N1, k = P % N1;
                double sa = 0.0, sd = 0.0, sb = 0.0;
#pragma unroll
                for (int w = 0; w < S::EPP; ++w) {
                    const double ah = ch[p * S::EPP + w], ad = cd[p * S::EPP + w];
                    sa = fma(ah, L.hsl[w], sa);
                    sd = fma(ah, L.dsl[w], sd);
                    sb = fma(ad, L.hsl[w], sb);
                }
                v[c] = fma(sa, L.ht[k], v[c]);
                vt[c] = fma(sa, L.dt[k], vt[c]);
                vs[c] = fma(sd, L.ht[k], vs[c]);
                vr[c] = fma(sb, L.ht[k], vr[c]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = xor_add(xor_add(v[c], 16), 32);
        J[3 * c + 0] = xor_add(xor_add(vr[c], 16), 32);
        J[3 * c + 1] = xor_add(xor_add(vs[c], 16), 32);
        J[3 * c + 2] = xor_add(xor_add(vt[c], 16), 32);
    }
}

// Closest node of the 16 slots' points: C = |X|^2 - 2 X . x* over the nodes
// (rows) by MFMA; smallest value, ties to the smaller node index.
template <int N1>
__device__ __forceinline__ int mfma_start(lptr<double> X, int lane, const double (&xs)[3])
{
    using S = MShape<N1>;
    constexpr int V = S::V;
    const int g = lane >> 4, row = lane & 15;
    const double b = (g < 3) ? -2.0 * xs[g] : 1.0;
    double best = INFINITY;
    int bn = 0;
#pragma unroll 4
    for (int mb = 0; mb < S::SB; ++mb) {
        const int node = 16 * mb + row;
        double a;
        if (node < V) {
            if (g < 3) {
                a = X[g * V + node];
            } else {
                const double x0 = X[node], x1 = X[V + node], x2 = X[2 * V + node];
                a = fma(x2, x2, fma(x1, x1, x0 * x0));
            }
        } else {
            a = (g < 3) ? 0.0 : 1e300;  // padding rows never win
        }
        dx4 c = {0, 0, 0, 0};
        c = mfma16(a, b, c);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int nd = 16 * mb + mrow(g, v);
            if (c[v] < best) {  // nodes increase with mb and v within a lane
                best = c[v];
                bn = nd;
            }
        }
    }
#pragma unroll
    for (int m = 16; m <= 32; m <<= 1) {
        const double ob = __shfl_xor(best, m, kWave);
        const int on = __shfl_xor(bn, m, kWave);
        if (ob < best || (ob == best && on < bn)) {
            best = ob;
            bn = on;
        }
    }
    return bn;
}

constexpr int kMfmaChunk = 256;  // pairs staged in LDS at a time

// One wavefront per element.  LDS holds the element block (one coalesced
// load) and, per chunk of pairs, each pair's slot, point and start node, so
// that refilling a slot reads LDS only.
template <int N1>
__global__ __launch_bounds__(kWave) void k_locate_mfma(LocArgs a, const double *__restrict__ basis)
{
    using S = MShape<N1>;
    constexpr int V = S::V;
    __shared__ double sX[3 * V];
    __shared__ double sP[3 * kMfmaChunk];
    __shared__ int sS[kMfmaChunk], sn[kMfmaChunk];
    const BasisPtr<double> B{as_const(basis)};
    const int e = blockIdx.x;
    const int beg = a.elem_off[e], end = a.elem_off[e + 1];
    if (beg >= end) return;
    const int lane = threadIdx.x, n = lane & 15, g = lane >> 4;
    {
        const double2 *src = (const double2 *)(a.geom + (long long)e * 3 * V);
        for (int q = lane; q < 3 * V / 2; q += kWave) {
            const double2 v = src[q];
            sX[2 * q] = v.x;
            sX[2 * q + 1] = v.y;
        }
        if ((3 * V) & 1) {
            if (lane == 0) sX[3 * V - 1] = a.geom[(long long)e * 3 * V + 3 * V - 1];
        }
    }
    __syncthreads();
    const lptr<double> X = (lptr<double>)sX;
    double A[S::MB][S::KB];
    load_afrag<N1>(X, lane, A);
    const double he = a.esize[e];
    const double rstop = (kResidStop * he) * (kResidStop * he);
    unsigned long long my_iters = 0;

    for (int c0 = beg; c0 < end; c0 += kMfmaChunk) {
        const int cnt = min(kMfmaChunk, end - c0);
        for (int u = lane; u < cnt; u += kWave) {
            const int slot = a.order[c0 + u];
            const int tk = slot % a.M;
            const int p = a.idx ? a.idx[tk] : tk;
            sS[u] = slot;
            sP[3 * u] = a.pts[3 * (long long)p];
            sP[3 * u + 1] = a.pts[3 * (long long)p + 1];
            sP[3 * u + 2] = a.pts[3 * (long long)p + 2];
        }
        __syncthreads();
        // start nodes, 16 pairs per MFMA batch
        for (int b0 = 0; b0 < cnt; b0 += 16) {
            const int u = b0 + n;
            double xs[3] = {0.0, 0.0, 0.0};
            if (u < cnt) {
                xs[0] = sP[3 * u];
                xs[1] = sP[3 * u + 1];
                xs[2] = sP[3 * u + 2];
            }
            const int bn = mfma_start<N1>(X, lane, xs);
            if (u < cnt && g == 0) sn[u] = bn;
        }
        __syncthreads();

        // Newton with slot refill
        int u = n, next = 16;
        int slot = 0;
        double xs[3] = {0.0, 0.0, 0.0};
        TRNewton t;
        {
            const double r0[3] = {0.0, 0.0, 0.0};
            t.start(r0);
        }
        auto begin_pair = [&](int uu) {
            slot = sS[uu];
            xs[0] = sP[3 * uu];
            xs[1] = sP[3 * uu + 1];
            xs[2] = sP[3 * uu + 2];
            double r0[3];
            node_rst<N1>(B, sn[uu], r0);
            t.start(r0);
        };
        bool active = u < cnt;
        if (active) begin_pair(u);
        while (__ballot(active) != 0) {
            LaneBasis<N1> L;
            lane_basis<N1>(B, t.rt, g, L);
            double xt[3], Jt[9];
            mfma_geo<N1>(A, L, xt, Jt);
            bool done = false;
            if (active) {
                done = t.update(xt, Jt, xs, rstop);
                if (done && g == 0) {
                    my_iters += (unsigned long long)t.it;
                    store_pair<N1>(a, B, slot, e, t, he);
                }
            }
            // finished slots take the next pairs, in slot order
            const unsigned long long fin = __ballot(done && g == 0) & 0xFFFFull;
            if (fin) {
                const int rank = __popcll(fin & ((1ull << n) - 1ull));
                if (done) {
                    u = next + rank;
                    active = u < cnt;
                    if (active) begin_pair(u);
                }
                next += __popcll(fin);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) my_iters += __shfl_xor(my_iters, o, kWave);
    if (lane == 0) {
        atomicAdd(&a.stats[0], (unsigned long long)(end - beg));
        atomicAdd(&a.stats[1], my_iters);
    }
}

// Owner selection per point (candidates are in ascending element order).
__global__ __launch_bounds__(256) void k_select(LocArgs a, int *__restrict__ code,
                                                int *__restrict__ el, double *__restrict__ rst,
                                                double *__restrict__ dist2)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = t < task_count(a);
    if (a.obb) {  // first pass covers every point once: count them
        unsigned long long v = live ? 1ULL : 0ULL;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0 && v) atomicAdd(&a.stats[2], v);
    }
    if (!live) return;
    const int p = a.idx ? a.idx[t] : t;
    const int nv = a.ncand[t];
    const int n = nv & kCountMask;
    const bool full = (nv >> kFullBit) != 0;
    auto S =[&](int k) { return (long long)k * a.M + t; };
    int w = -1, c = 2;
    bool anyin = false;
    for (int k = 0; k < n; ++k) anyin |= a.res_in[S(k)] != 0;
    if (anyin) {
        c = 0;
        if (a.res_dl) {
            // best delta of each session among its inside candidates; the
            // largest wins (ties: smaller session), then the smallest element
            int bs = 0;
            double bd = -INFINITY;
            bool hv = false;
            for (int k = 0; k < n; ++k) {
                if (!a.res_in[S(k)]) continue;
                const int sk = a.esess ? a.esess[a.cand_el[S(k)]] : 0;
                double sd = -INFINITY;
                for (int u = 0; u < n; ++u) {
                    if (!a.res_in[S(u)]) continue;
                    const int su = a.esess ? a.esess[a.cand_el[S(u)]] : 0;
                    if (su == sk) sd = fmax(sd, a.res_dl[S(u)]);
                }
                if (!hv || sd > bd || (sd == bd && sk < bs)) {
                    hv = true;
                    bd = sd;
                    bs = sk;
                }
            }
            for (int k = 0; k < n && w < 0; ++k) {
                if (!a.res_in[S(k)]) continue;
                const int sk = a.esess ? a.esess[a.cand_el[S(k)]] : 0;
                if (sk == bs) w = k;
            }
        } else {
            for (int k = 0; k < n && w < 0; ++k)
                if (a.res_in[S(k)]) w = k;
        }
    } else if (n > 0) {
        c = 1;
        w = 0;
        for (int k = 1; k < n; ++k) {
            const double dk = a.res[4 * (S(k)) + 3], dw = a.res[4 * (S(w)) + 3];
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
        const double *o = a.res + 4 * (S(w));
        el[p] = a.cand_el[S(w)];
        rst[3 * (long long)p] = o[0];
        rst[3 * (long long)p + 1] = o[1];
        rst[3 * (long long)p + 2] = o[2];
        dist2[p] = o[3];
    }
    if (a.obb && c != 0 && !full) a.redo[atomicAdd(a.redo_n, 1)] = p;
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
#define FP_LAUNCH_GRP(N1)                                                                 \
    k_locate_grp<N1><<<(h->E + Group<N1>::G - 1) / Group<N1>::G, kGrpThreads, 0, s>>>(a, \
                                                                              h->d_basis, h->E)
#define FP_LAUNCH_LOCATE(N1) k_locate<N1><<<h->E, kWave, 0, s>>>(a, h->d_basis)
#define FP_LAUNCH_MFMA(N1) k_locate_mfma<N1><<<h->E, kWave, 0, s>>>(a, h->d_basis)
    switch (h->n1) {
        case 2: FP_LAUNCH_MFMA(2); break;
        case 3: FP_LAUNCH_MFMA(3); break;
        case 4: FP_LAUNCH_MFMA(4); break;
        case 5: FP_LAUNCH_MFMA(5); break;
        case 6: FP_LAUNCH_MFMA(6); break;
        case 7: FP_LAUNCH_MFMA(7); break;
        case 8: FP_LAUNCH_MFMA(8); break;
        case 9: FP_LAUNCH_GRP(9); break;
        case 10: FP_LAUNCH_GRP(10); break;
        case 11: FP_LAUNCH_LOCATE(11); break;
        case 12: FP_LAUNCH_LOCATE(12); break;
        case 13: FP_LAUNCH_LOCATE(13); break;
        case 14: FP_LAUNCH_LOCATE(14); break;
        case 15: FP_LAUNCH_LOCATE(15); break;
        case 16: FP_LAUNCH_LOCATE(16); break;
        default: return hipErrorInvalidValue;
    }
#undef FP_LAUNCH_GRP
#undef FP_LAUNCH_LOCATE
#undef FP_LAUNCH_MFMA
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
        a.M = h->max_points;
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
        int *co = code + start, *eo = el + start;
        double *ro = rst + 3 * (long long)start, *dO = dist2 + start;
        // first pass: oriented-box candidates; points without an inside
        // candidate go to the redo list
        a.obb = h->obb;
        a.redo = h->redo;
        a.redo_n = h->redo_n;
        FP_HIP(fill_int(h->redo_n, 0, 1, s));
        FP_HIP(fill_int(h->elem_cnt, 0, (long long)h->E + 1, s));
        k_cand<<<pb, 256, 0, s>>>(a);
        FP_HIP(hipGetLastError());
        FP_HIP(scan_exclusive(h->elem_cnt, h->elem_off, h->E, h->scan_tmp, s));
        k_scatter<<<pb, 256, 0, s>>>(a);
        FP_HIP(hipGetLastError());
        if (h->timing) FP_HIP(hipEventRecord(l0, s));
        FP_HIP(launch_locate_kernel(h, a, s));
        if (h->timing) FP_HIP(hipEventRecord(l1, s));
        k_select<<<pb, 256, 0, s>>>(a, co, eo, ro, dO);
        FP_HIP(hipGetLastError());
        // second pass over the redo list with the axis-aligned candidates
        // only (sized on the device: kernels past the count return at once)
        a.obb = nullptr;
        a.idx = h->redo;
        a.dcount = h->redo_n;
        FP_HIP(fill_int(h->elem_cnt, 0, (long long)h->E + 1, s));
        k_cand<<<pb, 256, 0, s>>>(a);
        FP_HIP(hipGetLastError());
        FP_HIP(scan_exclusive(h->elem_cnt, h->elem_off, h->E, h->scan_tmp, s));
        k_scatter<<<pb, 256, 0, s>>>(a);
        FP_HIP(hipGetLastError());
        FP_HIP(launch_locate_kernel(h, a, s));
        k_select<<<pb, 256, 0, s>>>(a, co, eo, ro, dO);
        FP_HIP(hipGetLastError());
        if (h->timing) {
            FP_HIP(hipEventRecord(t1, s));
            record(h, 0, l0, l1);
            record(h, 2, t0, t1);
        }
    }
    return FP_OK;
}
