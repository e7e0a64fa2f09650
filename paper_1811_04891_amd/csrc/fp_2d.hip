// findpts / findpts_eval in two dimensions: meshes of curved quadrilateral
// spectral elements (the method of Section 2.1 on the reference square
// [-1,1]^2; the paper's Figs. 1 and 6 are two-dimensional overlapping
// meshes).
//
// Setup: packed element blocks (E x 2 x n1^2), Bernstein-hull boxes and h_e
// (one wavefront per element), a uniform hash grid of about 4 E cells with
// ascending element lists, and an oriented box per element.  findpts2, per
// pass of at most max_points points, in two rounds like the 3D path (first
// the candidates whose oriented box holds the point; then, for points left
// without an inside candidate whose list the oriented boxes cut, the whole
// axis-aligned set):
//   k2_cand     per point: cell, box and session test (and the oriented box
//               in the first round), candidate list and each pair's rank in
//               its element
//   scan        pair counts per element -> offsets; k2_scatter groups pairs
//   k2_locate   one wavefront per work unit (up to 64 pairs of one element):
//               closest mapped node (node rows by scalar loads), trust-region
//               Newton on [-1,1]^2 with the 3D rules
//   k2_select   inside / border / not found, smallest inside id, distance
//               discriminator across sessions
// findpts2_eval groups points by element the same way (k2_eval, one
// wavefront per work unit, field rows by scalar loads).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "fp_basis.h"
#include "fp_internal.h"

struct fp2_handle {
    int device = 0;
    int E = 0, N = 0, n1 = 0, V = 0;
    double tol = 0.0;
    int M = 0;   // points per pass
    int MC = 1;  // longest cell list: candidate slots per point

    double *geom = nullptr;   // E x 2 x V
    double *esize = nullptr;  // E
    double *bbox = nullptr;   // E x 4: xmin xmax ymin ymax
    float *obb = nullptr;     // E x 10 binary32: frame Q (2 x 2, rows = axes), centre (2),
                              // rotated lo (2), rotated hi (2)
    int *esess = nullptr;     // E or null
    double *delta = nullptr;  // E x V or null
    double glo[2] = {0, 0}, ghi[2] = {0, 0}, ginv[2] = {0, 0};
    int nc[2] = {1, 1};
    long long ncell = 0;
    int nnz = 0;
    int *cell_off = nullptr, *cell_el = nullptr;

    // workspace
    int *ncand = nullptr, *cand_el = nullptr, *cand_pos = nullptr;
    int *elem_cnt = nullptr, *elem_off = nullptr, *order = nullptr;
    double *res = nullptr;  // M x MC x 3: r, s, d2
    int *res_in = nullptr;
    double *res_dl = nullptr;
    unsigned *iter_part = nullptr;
    unsigned *cand_part = nullptr;  // per k2_cand block: axis-aligned candidates
    int *redo = nullptr;            // M: second-round flag per point
    int *ev_pos = nullptr, *ev_order = nullptr;
    int *scan_tmp = nullptr;
    int *d_flag = nullptr;
    double *d_g = nullptr;
    double *d_binv = nullptr;
    double *d_basis = nullptr;
    double *d_dnode = nullptr;  // n1 x n1: h_b'(z_a)
    unsigned long long *stats = nullptr;  // pairs solved, Newton iterations, method candidates
    fp::Basis basis{};

    std::vector<void *> allocs;
    size_t bytes = 0;
};

namespace fp {
namespace {

constexpr int kUnit2 = 64;

__device__ __forceinline__ double wave_min2(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ double wave_max2(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

__global__ __launch_bounds__(256) void k2_pack(const double *__restrict__ x,
                                               const double *__restrict__ y, long long EV, int V,
                                               double *__restrict__ geom, int *__restrict__ bad)
{
    int flag = 0;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < EV;
         q += (long long)gridDim.x * blockDim.x) {
        const long long e = q / V, i = q - e * V;
        const double a = x[q], b = y[q];
        flag |= !(isfinite(a) && isfinite(b));
        geom[2 * e * V + i] = a;
        geom[(2 * e + 1) * V + i] = b;
    }
    if (flag) atomicOr(bad, 1);
}

// One wavefront per element: Bernstein coefficients of x and y (the inverse
// nodal-Bernstein matrix along r, then s, in LDS), their range, the node
// extents (h_e) and the margin 1e-8 h_e + 1e-14 max|x|.
__global__ __launch_bounds__(kWave) void k2_bbox(const double *__restrict__ geom, int n1,
                                                 const double *__restrict__ binv,
                                                 double *__restrict__ bbox,
                                                 double *__restrict__ esize)
{
    __shared__ double A[kMaxN1 * kMaxN1], Bc[kMaxN1 * kMaxN1], Bi[kMaxN1 * kMaxN1];
    const int e = blockIdx.x, t = threadIdx.x, V = n1 * n1;
    for (int q = t; q < V; q += kWave) Bi[q] = binv[q];
    double lo[2], hi[2], he = 0.0, amax = 0.0;
    for (int c = 0; c < 2; ++c) {
        const double *X = geom + ((long long)e * 2 + c) * V;
        double mn = INFINITY, mx = -INFINITY;
        for (int q = t; q < V; q += kWave) {
            const double v = X[q];
            A[q] = v;
            mn = fmin(mn, v);
            mx = fmax(mx, v);
            amax = fmax(amax, fabs(v));
        }
        mn = wave_min2(mn);
        mx = wave_max2(mx);
        he = fmax(he, mx - mn);
        __syncthreads();
        for (int q = t; q < V; q += kWave) {  // along r
            const int i = q % n1, j = q / n1;
            double s = 0.0;
            for (int l = 0; l < n1; ++l) s = fma(Bi[i * n1 + l], A[j * n1 + l], s);
            Bc[q] = s;
        }
        __syncthreads();
        double cmn = INFINITY, cmx = -INFINITY;
        for (int q = t; q < V; q += kWave) {  // along s
            const int i = q % n1, j = q / n1;
            double s = 0.0;
            for (int l = 0; l < n1; ++l) s = fma(Bi[j * n1 + l], Bc[i + n1 * l], s);
            cmn = fmin(cmn, s);
            cmx = fmax(cmx, s);
        }
        lo[c] = wave_min2(cmn);
        hi[c] = wave_max2(cmx);
        __syncthreads();
    }
    amax = wave_max2(amax);
    if (t == 0) {
        const double m = 1e-8 * he + 1e-14 * amax;
        for (int c = 0; c < 2; ++c) {
            bbox[4 * e + 2 * c] = lo[c] - m;
            bbox[4 * e + 2 * c + 1] = hi[c] + m;
        }
        esize[e] = he;
    }
}

// Oriented box of each element (one wavefront per element): frame from the
// mean edge vectors along r and s (Gram-Schmidt; identity if degenerate),
// rounded to binary32 with the centre before the Bernstein hull of the
// rotated coordinates u = Q (x - centre) is taken, so the box holds the
// element for the stored frame; same margin as the axis-aligned box, bounds
// rounded outward.
__global__ __launch_bounds__(kWave) void k2_obb(const double *__restrict__ geom, int n1,
                                                const double *__restrict__ binv,
                                                const double *__restrict__ bbox,
                                                const double *__restrict__ esize,
                                                double tol, float *__restrict__ obb)
{
    __shared__ double A[kMaxN1 * kMaxN1], Bc[kMaxN1 * kMaxN1], Bi[kMaxN1 * kMaxN1];
    const int e = blockIdx.x, t = threadIdx.x, V = n1 * n1;
    for (int q = t; q < V; q += kWave) Bi[q] = binv[q];
    const double *X = geom + (long long)e * 2 * V;
    double ed[2][2];
    for (int c = 0; c < 2; ++c) {
        double sr = 0.0, ss = 0.0;
        for (int q = t; q < n1; q += kWave) {
            sr += X[c * V + n1 - 1 + n1 * q] - X[c * V + n1 * q];
            ss += X[c * V + q + n1 * (n1 - 1)] - X[c * V + q];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            sr += __shfl_xor(sr, o, kWave);
            ss += __shfl_xor(ss, o, kWave);
        }
        ed[0][c] = sr;
        ed[1][c] = ss;
    }
    double Q[2][2];
    bool ok = true;
    for (int a = 0; a < 2; ++a) {
        double v[2] = {ed[a][0], ed[a][1]};
        if (a == 1) {
            const double d = v[0] * Q[0][0] + v[1] * Q[0][1];
            v[0] -= d * Q[0][0];
            v[1] -= d * Q[0][1];
        }
        const double nv = sqrt(v[0] * v[0] + v[1] * v[1]);
        const double ne = sqrt(ed[a][0] * ed[a][0] + ed[a][1] * ed[a][1]);
        ok = ok && isfinite(nv) && nv > 1e-6 * ne && ne > 0.0;
        Q[a][0] = ok ? v[0] / nv : 0.0;
        Q[a][1] = ok ? v[1] / nv : 0.0;
    }
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) Q[a][c] = (double)(float)(ok ? Q[a][c] : (a == c ? 1.0 : 0.0));
    const double *bb = bbox + 4 * (long long)e;
    const double ctr[2] = {(double)(float)(0.5 * (bb[0] + bb[1])),
                           (double)(float)(0.5 * (bb[2] + bb[3]))};
    double lo[2], hi[2], amax = 0.0;
    for (int a = 0; a < 2; ++a) {
        for (int q = t; q < V; q += kWave) {
            const double u = Q[a][0] * (X[q] - ctr[0]) + Q[a][1] * (X[V + q] - ctr[1]);
            A[q] = u;
            amax = fmax(amax, fabs(u));
        }
        __syncthreads();
        for (int q = t; q < V; q += kWave) {  // along r
            const int i = q % n1, j = q / n1;
            double sum = 0.0;
            for (int l = 0; l < n1; ++l) sum = fma(Bi[i * n1 + l], A[j * n1 + l], sum);
            Bc[q] = sum;
        }
        __syncthreads();
        double cmn = INFINITY, cmx = -INFINITY;
        for (int q = t; q < V; q += kWave) {  // along s
            const int i = q % n1, j = q / n1;
            double sum = 0.0;
            for (int l = 0; l < n1; ++l) sum = fma(Bi[j * n1 + l], Bc[i + n1 * l], sum);
            cmn = fmin(cmn, sum);
            cmx = fmax(cmx, sum);
        }
        lo[a] = wave_min2(cmn);
        hi[a] = wave_max2(cmx);
        __syncthreads();
    }
    amax = wave_max2(amax);
    if (t == 0) {
        const double cabs = fmax(fabs(ctr[0]), fabs(ctr[1]));
        // the axis-aligned box's margin, or the inside tolerance when that is
        // larger (a point within tol h_e of the element may be inside; the
        // rounded frame's rows have norm 1 to within 1e-7)
        const double m = fmax(1e-8, (1.0 + 1e-6) * tol) * esize[e] + 1e-14 * (amax + cabs);
        float *o = obb + 10 * (long long)e;
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < 2; ++c) o[2 * a + c] = (float)Q[a][c];  // exact
        for (int c = 0; c < 2; ++c) {
            o[4 + c] = (float)ctr[c];  // exact
            const double l = lo[c] - m, u = hi[c] + m;
            float lf = (float)l, uf = (float)u;
            if ((double)lf > l) lf = nextafterf(lf, -INFINITY);
            if ((double)uf < u) uf = nextafterf(uf, INFINITY);
            o[6 + c] = lf;
            o[8 + c] = uf;
        }
    }
}

__global__ __launch_bounds__(256) void k2_gbox(const double *__restrict__ bbox, int E,
                                               double *__restrict__ out)
{
    __shared__ double red[4][256 / kWave];
    double v[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (int e = threadIdx.x; e < E; e += blockDim.x)
        for (int a = 0; a < 2; ++a) {
            v[2 * a] = fmin(v[2 * a], bbox[4 * e + 2 * a]);
            v[2 * a + 1] = fmax(v[2 * a + 1], bbox[4 * e + 2 * a + 1]);
        }
    const int w = threadIdx.x / kWave;
    for (int a = 0; a < 2; ++a) {
        const double mn = wave_min2(v[2 * a]), mx = wave_max2(v[2 * a + 1]);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            red[2 * a][w] = mn;
            red[2 * a + 1][w] = mx;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int a = 0; a < 2; ++a) {
            double mn = red[2 * a][0], mx = red[2 * a + 1][0];
            for (int q = 1; q < (int)(blockDim.x / kWave); ++q) {
                mn = fmin(mn, red[2 * a][q]);
                mx = fmax(mx, red[2 * a + 1][q]);
            }
            out[2 * a] = mn;
            out[2 * a + 1] = mx;
        }
}

struct Grid2 {
    double lo[2], hi[2], inv[2];
    int nc[2];
};

__device__ __forceinline__ int cell2(const Grid2 &g, int a, double x)
{
    const double u = (x - g.lo[a]) * g.inv[a];
    int i = (u >= 0.0) ? (int)fmin(u, (double)(g.nc[a] - 1)) : 0;
    return i < 0 ? 0 : (i >= g.nc[a] ? g.nc[a] - 1 : i);
}

// mode 0: count entries per cell; mode 1: write element ids.
__global__ __launch_bounds__(256) void k2_hash_pass(const double *__restrict__ bbox, int E,
                                                    Grid2 g, int mode, int *__restrict__ cnt,
                                                    const int *__restrict__ off,
                                                    int *__restrict__ cell_el)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const double *b = bbox + 4 * (long long)e;
    const int i0 = cell2(g, 0, b[0]), i1 = cell2(g, 0, b[1]);
    const int j0 = cell2(g, 1, b[2]), j1 = cell2(g, 1, b[3]);
    for (int j = j0; j <= j1; ++j)
        for (int i = i0; i <= i1; ++i) {
            const long long c = i + (long long)g.nc[0] * j;
            const int pos = atomicAdd(&cnt[c], 1);
            if (mode == 1) cell_el[off[c] + pos] = e;
        }
}

// Sort each cell list ascending (insertion sort; lists are short) and find
// the longest list.
__global__ __launch_bounds__(256) void k2_hash_sort(const int *__restrict__ off,
                                                    int *__restrict__ cell_el, long long ncell,
                                                    int *__restrict__ maxlen)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int b = off[c], n = off[c + 1] - b;
    int *L = cell_el + b;
    for (int i = 1; i < n; ++i) {
        const int v = L[i];
        int j = i - 1;
        while (j >= 0 && L[j] > v) {
            L[j + 1] = L[j];
            --j;
        }
        L[j + 1] = v;
    }
    atomicMax(maxlen, n);
}

constexpr int kFull2 = 30;  // ncand bit: the list is the method's whole set
constexpr int kCount2 = (1 << kFull2) - 1;

struct Loc2 {
    const float *obb;  // non-null: first round (oriented boxes)
    int *redo;         // first round writes the second-round flags
    const int *only;   // non-null: second round, points with only[t] != 0
    unsigned *cand_part;
    const double *geom, *esize, *bbox, *delta, *pts;
    const int *esess, *cell_off, *cell_el, *psess;
    Grid2 g;
    int npts, M, MC, E;
    double tol;
    int *ncand, *cand_el, *cand_pos, *elem_cnt;
    const int *elem_off;
    int *order;
    double *res;
    int *res_in;
    double *res_dl;
    unsigned *iter_part;
};

// Candidates of each point: hash cell, then the closed box, then session
// exclusion; ascending element ids (the cell lists are sorted).  First
// round: only those whose oriented box holds the point, or every one if none
// does (then, or when the filter dropped nothing, the list is the whole set).
__global__ __launch_bounds__(256) void k2_cand(Loc2 a)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool skip = t >= a.npts || (a.only && !a.only[t]);
    const double x = skip ? NAN : a.pts[2 * (long long)t];
    const double y = skip ? NAN : a.pts[2 * (long long)t + 1];
    int n = 0, naabb = 0, full = a.obb ? 0 : 1;
    if (x >= a.g.lo[0] && x <= a.g.hi[0] && y >= a.g.lo[1] && y <= a.g.hi[1]) {
        const long long c = cell2(a.g, 0, x) + (long long)a.g.nc[0] * cell2(a.g, 1, y);
        const int ps = a.psess ? a.psess[t] : -1;
        for (int pass = a.obb ? 0 : 1; pass < 2 && n == 0; ++pass) {
            for (int q = a.cell_off[c]; q < a.cell_off[c + 1] && n < a.MC; ++q) {
                const int e = a.cell_el[q];
                const double *b = a.bbox + 4 * (long long)e;
                if (!(x >= b[0] && x <= b[1] && y >= b[2] && y <= b[3])) continue;
                if (ps >= 0 && a.esess && a.esess[e] == ps) continue;
                if (pass == 0) {
                    ++naabb;
                    const float *o = a.obb + 10 * (long long)e;
                    const double d0 = x - (double)o[4], d1 = y - (double)o[5];
                    const double u0 = fma((double)o[1], d1, (double)o[0] * d0);
                    const double u1 = fma((double)o[3], d1, (double)o[2] * d0);
                    if (!(u0 >= (double)o[6] && u0 <= (double)o[8] && u1 >= (double)o[7] &&
                          u1 <= (double)o[9]))
                        continue;
                }
                a.cand_el[(long long)n * a.M + t] = e;
                ++n;
            }
            if (pass == 1 || naabb == 0 || n == naabb) full = 1;
            if (pass == 0 && naabb == 0) break;
        }
    }
    // ranks in the elements from converged code (shared atomics for lanes
    // on the same element)
    int nmax = n;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nmax = max(nmax, __shfl_xor(nmax, o, kWave));
    for (int k = 0; k < nmax; ++k) {
        const bool act = k < n;
        const long long s = (long long)k * a.M + t;
        const int e = act ? a.cand_el[s] : -1;
        const int r = wave_rank(a.elem_cnt, e, act);
        if (act) a.cand_pos[s] = r;
    }
    if (t < a.npts) a.ncand[t] = n | (full << kFull2);
    if (a.obb) {  // the method's candidates of this block (the first round sees every point)
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

__global__ __launch_bounds__(256) void k2_scatter(Loc2 a)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.npts) return;
    const int n = a.ncand[t] & kCount2;
    for (int k = 0; k < n; ++k) {
        const long long s = (long long)k * a.M + t;
        a.order[a.elem_off[a.cand_el[s]] + a.cand_pos[s]] = (int)s;
    }
}

// x_c(r, s) and J[c][d] = dx_c/dr_d for both coordinates, sum-factorised:
// r first (value and derivative), then s.
template <int N1>
__device__ __forceinline__ void geo2(cptr<double> X, BasisPtr<double> B, const double (&r)[2],
                                     double (&x)[2], double (&J)[4])
{
    constexpr int V = N1 * N1;
    FP_PIN_SGPR(X);
    double hr[N1], dr[N1], hs[N1], ds[N1];
    lagrange_d<N1>(B, r[0], hr, dr);
    lagrange_d<N1>(B, r[1], hs, ds);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        double v = 0.0, vr = 0.0, vs = 0.0;
#pragma unroll
        for (int j = 0; j < N1; ++j) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int i = 0; i < N1; ++i) {
                const double xv = X[c * V + N1 * j + i];
                a = fma(xv, hr[i], a);
                b = fma(xv, dr[i], b);
            }
            v = fma(a, hs[j], v);
            vs = fma(a, ds[j], vs);
            vr = fma(b, hs[j], vr);
        }
        x[c] = v;
        J[2 * c] = vr;
        J[2 * c + 1] = vs;
        // the Jacobian is complete here: otherwise its half of the
        // contraction is sunk past the trust-region acceptance branch, and
        // the element rows it reads are held (spilled) across that branch
        FP_KEEP(x[c]);
        FP_KEEP(J[2 * c]);
        FP_KEEP(J[2 * c + 1]);
    }
}

constexpr double kResidStop2 = 1e-13;
constexpr double kStepStop2 = 1e-13;
constexpr double kStepTiny2 = 1e-15;
constexpr int kMaxIter2 = 50;

// The projected trust-region Gauss-Newton of the 3D path on [-1,1]^2: a
// coordinate on a bound whose descent direction points outward is held; the
// step solves J d = -F with both coordinates free, else the reduced normal
// equation on the free one (steepest descent if singular); scaled to the
// trust radius (max norm) and projected.  Accept if rho >= 0.01; radius x2
// (up to 2) if rho > 0.75 and limited, |s|/4 if rho < 0.25.  Stop: phi <=
// (min(1e-13, tol/10) h_e)^2, an accepted step with |s| <= 1e-13, no
// possible progress, or 50 iterations.
struct TR2 {
    double r[2], F[2], J[4], phi, D, pred, ns;
    double rt[2];
    bool limited, have;
    int it;

    __device__ __forceinline__ void start(const double (&r0)[2])
    {
        rt[0] = r0[0];
        rt[1] = r0[1];
        r[0] = r[1] = F[0] = F[1] = 0.0;
        J[0] = J[1] = J[2] = J[3] = 0.0;
        phi = INFINITY;
        D = 1.0;
        pred = ns = 0.0;
        limited = have = false;
        it = 0;
    }

    __device__ __forceinline__ bool update(const double (&xt)[2], const double (&Jt)[4],
                                           const double (&xs)[2], double rstop)
    {
        const double Ft[2] = {xt[0] - xs[0], xt[1] - xs[1]};
        const double phit = fma(Ft[1], Ft[1], Ft[0] * Ft[0]);
        bool acc = true, stop = false;
        if (have) {
            const double rho = (phi - phit) / pred;
            acc = rho >= 0.01;
            if (rho > 0.75 && limited)
                D = fmin(2.0 * D, 2.0);
            else if (rho < 0.25)
                D = 0.25 * ns;
            if (acc && ns <= kStepStop2) stop = true;
        }
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            r[d] = acc ? rt[d] : r[d];
            F[d] = acc ? Ft[d] : F[d];
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) J[d] = acc ? Jt[d] : J[d];
        phi = acc ? phit : phi;
        have = true;
        if (stop || phi <= rstop || it >= kMaxIter2) return true;
        ++it;
        double g[2], m[2];
        int nf = 0;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            g[d] = fma(J[2 + d], F[1], J[d] * F[0]);
            const bool held = (r[d] >= 1.0 && g[d] < 0.0) || (r[d] <= -1.0 && g[d] > 0.0);
            m[d] = held ? 0.0 : 1.0;
            nf += held ? 0 : 1;
        }
        if (nf == 0) return true;
        // both free: J d = -F; else (M J^T J M + I - M) d = -M g
        double A[4], b[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const double jtj = fma(J[2 + u], J[2 + v], J[u] * J[v]);
                const double red = m[u] * m[v] * jtj + ((u == v) ? 1.0 - m[u] : 0.0);
                A[2 * u + v] = (nf == 2) ? J[2 * u + v] : red;
            }
            b[u] = (nf == 2) ? -F[u] : -m[u] * g[u];
        }
        const double det = A[0] * A[3] - A[1] * A[2];
        double dl[2] = {(b[0] * A[3] - A[1] * b[1]) / det, (A[0] * b[1] - b[0] * A[2]) / det};
        if (!(det != 0.0 && isfinite(dl[0]) && isfinite(dl[1]))) {
            dl[0] = -m[0] * g[0];
            dl[1] = -m[1] * g[1];
        }
        const double nd = fmax(fabs(dl[0]), fabs(dl[1]));
        if (!(nd > 0.0) || !isfinite(nd)) return true;
        limited = nd > D;
        const double sc = limited ? D / nd : 1.0;
        double s[2];
        ns = 0.0;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const double v = fmin(1.0, fmax(-1.0, r[d] + dl[d] * sc));
            rt[d] = v;
            s[d] = v - r[d];
            ns = fmax(ns, fabs(s[d]));
        }
        double q2 = 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const double t = fma(J[2 * c + 1], s[1], fma(J[2 * c], s[0], F[c]));
            q2 = fma(t, t, q2);
        }
        pred = phi - q2;
        return ns <= kStepTiny2 || !(pred > 0.0);
    }
};

// One wavefront per work unit (up to 64 pairs of one element), one lane per
// pair: closest mapped GLL node (ties: smallest node index), then Newton.
template <int N1>
__global__ __launch_bounds__(kWave) void k2_locate(Loc2 a, const double *__restrict__ basis,
                                                   const double *__restrict__ dnode)
{
    constexpr int V = N1 * N1;
    const BasisPtr<double> B{as_const(basis)};
    unsigned long long my_iters = 0;
    const UnitList units(a.elem_off, a.E, 1, a.E, kUnit2);
    for (long long u = xcd_unit(blockIdx.x, gridDim.x); u < units.end; u += gridDim.x) {
        Unit U;
        if (!units.at(u, U)) continue;
        const int e = U.seg;
        cptr<double> X = as_const(a.geom + (long long)e * 2 * V);
        const double he = a.esize[e];
        const double cstop = fmin(0.1 * a.tol, kResidStop2) * he;
        const double rstop = cstop * cstop;
        const int q = U.beg + (int)threadIdx.x;
        const bool act = q < U.end;
        const int slot = act ? a.order[q] : 0;
        const int p = slot % a.M;
        double xs[2] = {0.0, 0.0};
        if (act) {
            xs[0] = a.pts[2 * (long long)p];
            xs[1] = a.pts[2 * (long long)p + 1];
        }
        double best = INFINITY;
        int bq = 0;
#pragma unroll 8
        for (int n = 0; n < V; ++n) {
            const double dx = X[n] - xs[0], dy = X[V + n] - xs[1];
            const double d = fma(dy, dy, dx * dx);
            if (d < best) {
                best = d;
                bq = n;
            }
        }
        const double r0[2] = {B.z(bq % N1), B.z(bq / N1)};
        TR2 t;
        t.start(r0);
        // the first Newton step from the node's value and line sums
        // (D = h_b'(z_a) at a n1 + b)
        bool done = !act;
        if (act) {
            const double *Xg = a.geom + (long long)e * 2 * V;
            const int i0 = bq % N1, j0 = bq / N1;
            double xn[2], Jn[4];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double dr = 0.0, ds = 0.0;
#pragma unroll
                for (int m = 0; m < N1; ++m) {
                    dr = fma(Xg[c * V + bq - i0 + m], dnode[i0 * N1 + m], dr);
                    ds = fma(Xg[c * V + bq + N1 * (m - j0)], dnode[j0 * N1 + m], ds);
                }
                xn[c] = Xg[c * V + bq];
                Jn[2 * c] = dr;
                Jn[2 * c + 1] = ds;
            }
            done = t.update(xn, Jn, xs, rstop);
        }
        while (!done) {
            double xt[2], Jt[4];
            geo2<N1>(X, B, t.rt, xt, Jt);
            done = t.update(xt, Jt, xs, rstop);
        }
        if (act) {
            my_iters += (unsigned long long)t.it;
            double *o = a.res + 3 * (long long)slot;
            o[0] = t.r[0];
            o[1] = t.r[1];
            o[2] = t.phi;
            const bool inside = sqrt(t.phi) <= a.tol * he;
            a.res_in[slot] = inside ? 1 : 0;
            if (a.res_dl) {
                double dl = 0.0;
                if (inside) {
                    double hr[N1], hs[N1];
                    lagrange<N1>(B, t.r[0], hr);
                    lagrange<N1>(B, t.r[1], hs);
                    const double *D = a.delta + (long long)e * V;
#pragma unroll
                    for (int j = 0; j < N1; ++j) {
                        double s = 0.0;
#pragma unroll
                        for (int i = 0; i < N1; ++i) s = fma(D[N1 * j + i], hr[i], s);
                        dl = fma(s, hs[j], dl);
                    }
                }
                a.res_dl[slot] = dl;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) my_iters += __shfl_xor(my_iters, o, kWave);
    if (threadIdx.x == 0) a.iter_part[blockIdx.x] = (unsigned)my_iters;
}

// Owner selection per point (candidates in ascending element order): an
// inside candidate wins (with a distance field: the session whose best
// inside value is largest, ties to the smaller session, then the smallest
// element of it; else the smallest element); otherwise the smallest distance
// (ties within 1e-14 relative keep the smaller id); no candidate: not found.
__global__ __launch_bounds__(256) void k2_select(Loc2 a, int *__restrict__ code,
                                                 int *__restrict__ el, double *__restrict__ rs,
                                                 double *__restrict__ dist2)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.npts || (a.only && !a.only[t])) return;  // second round: flagged points
    const int nv = a.ncand[t];
    const int n = nv & kCount2;
    const bool full = (nv >> kFull2) != 0;
    auto S = [&](int k) { return (long long)k * a.M + t; };
    int w = -1, c = 2;
    bool anyin = false;
    for (int k = 0; k < n; ++k) anyin |= a.res_in[S(k)] == 1;
    if (anyin) {
        c = 0;
        if (a.res_dl) {
            int bs = 0;
            double bd = -INFINITY;
            bool hv = false;
            for (int k = 0; k < n; ++k) {
                if (a.res_in[S(k)] != 1) continue;
                const int sk = a.esess ? a.esess[a.cand_el[S(k)]] : 0;
                double sd = -INFINITY;
                for (int v = 0; v < n; ++v) {
                    if (a.res_in[S(v)] != 1) continue;
                    const int sv = a.esess ? a.esess[a.cand_el[S(v)]] : 0;
                    if (sv == sk) sd = fmax(sd, a.res_dl[S(v)]);
                }
                if (!hv || sd > bd || (sd == bd && sk < bs)) {
                    hv = true;
                    bd = sd;
                    bs = sk;
                }
            }
            for (int k = 0; k < n && w < 0; ++k) {
                if (a.res_in[S(k)] != 1) continue;
                const int sk = a.esess ? a.esess[a.cand_el[S(k)]] : 0;
                if (sk == bs) w = k;
            }
        } else {
            for (int k = 0; k < n && w < 0; ++k)
                if (a.res_in[S(k)] == 1) w = k;
        }
    } else if (n > 0) {
        c = 1;
        w = 0;
        for (int k = 1; k < n; ++k) {
            const double dk = a.res[3 * S(k) + 2], dw = a.res[3 * S(w) + 2];
            const bool tie = fabs(dk - dw) <= 1e-14 * fmax(dk, dw);
            if (!tie && dk < dw) w = k;
        }
    }
    code[t] = c;
    if (w < 0) {
        el[t] = -1;
        rs[2 * (long long)t] = rs[2 * (long long)t + 1] = 0.0;
        dist2[t] = INFINITY;
    } else {
        const double *o = a.res + 3 * S(w);
        el[t] = a.cand_el[S(w)];
        rs[2 * (long long)t] = o[0];
        rs[2 * (long long)t + 1] = o[1];
        dist2[t] = o[2];
    }
    if (a.obb) a.redo[t] = (c != 0 && !full) ? 1 : 0;
}

__global__ __launch_bounds__(1024) void k2_stats(const unsigned *iter_part, int ni,
                                                 const unsigned *cand_part, int nb, int E,
                                                 const int *elem_off, unsigned long long *stats)
{
    __shared__ unsigned long long si[1024 / kWave], sc[1024 / kWave];
    unsigned long long it = 0, c = 0;
    for (int i = threadIdx.x; i < ni; i += blockDim.x) it += iter_part[i];
    for (int i = threadIdx.x; i < nb; i += blockDim.x) c += cand_part[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        it += __shfl_xor(it, o, kWave);
        c += __shfl_xor(c, o, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        si[threadIdx.x / kWave] = it;
        sc[threadIdx.x / kWave] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long I = 0, Cn = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
            I += si[w];
            Cn += sc[w];
        }
        atomicAdd(&stats[0], (unsigned long long)elem_off[E]);
        atomicAdd(&stats[1], I);
        if (Cn) atomicAdd(&stats[2], Cn);
    }
}

// ---- interpolation -------------------------------------------------------
struct Ev2 {
    const int *code, *el;
    const double *rs;
    int npts, E;
    int *cnt;
    const int *off;
    int *pos, *order;
    double *out;      // this launch's first field
    long long ostride;
    int nf;
    double *out_all;  // the call's first field (NaN fill of every field)
    int nf_all;
    const double *f[kMaxEvalFields];
};

__global__ __launch_bounds__(256) void k2_ev_count(Ev2 a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int e = p < a.npts ? a.el[p] : -1;
    const bool ok = p < a.npts && a.code[p] != FP_NOT_FOUND && e >= 0 && e < a.E;
    const int r = wave_rank(a.cnt, e, ok);  // converged: every lane of the wave
    if (p >= a.npts) return;
    if (ok) {
        a.pos[p] = r;
    } else {
        a.pos[p] = -1;
        for (int f = 0; f < a.nf_all; ++f) a.out_all[f * a.ostride + p] = NAN;
    }
}

__global__ __launch_bounds__(256) void k2_ev_scatter(Ev2 a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.npts) return;
    const int k = a.pos[p];
    if (k >= 0) a.order[a.off[a.el[p]] + k] = p;
}

constexpr int kUnitEval2 = 256;

// One wavefront per work unit (up to 256 points of one element, 64 at a
// time), field rows by scalar loads: f = sum_j h_j(s) sum_i h_i(r) F[j][i].
template <int N1>
__global__ __launch_bounds__(kWave) void k2_eval(Ev2 a, const double *__restrict__ basis)
{
    constexpr int V = N1 * N1;
    const BasisPtr<double> B{as_const(basis)};
    const UnitList units(a.off, a.E, 1, a.E, kUnitEval2);
    for (long long u = xcd_unit(blockIdx.x, gridDim.x); u < units.end; u += gridDim.x) {
        Unit U;
        if (!units.at(u, U)) continue;
        const int e = U.seg;
        for (int base = U.beg; base < U.end; base += kWave) {
            const int q = base + (int)threadIdx.x;
            const bool act = q < U.end;
            const int p = act ? a.order[q] : 0;
            const double r0 = act ? a.rs[2 * (long long)p] : 0.0;
            const double r1 = act ? a.rs[2 * (long long)p + 1] : 0.0;
            double hr[N1], hs[N1];
            lagrange<N1>(B, r0, hr);
            lagrange<N1>(B, r1, hs);
            for (int f = 0; f < a.nf; ++f) {
                cptr<double> F = as_const(a.f[f] + (long long)e * V);
                double v = 0.0;
#pragma unroll
                for (int j = 0; j < N1; ++j) {
                    double s = 0.0;
#pragma unroll
                    for (int i = 0; i < N1; ++i) s = fma(F[N1 * j + i], hr[i], s);
                    v = fma(s, hs[j], v);
                }
                if (act) a.out[f * a.ostride + p] = v;
            }
        }
    }
}

#define FP2_SWITCH(MACRO)            \
    switch (h->n1) {                 \
        case 2: MACRO(2); break;     \
        case 3: MACRO(3); break;     \
        case 4: MACRO(4); break;     \
        case 5: MACRO(5); break;     \
        case 6: MACRO(6); break;     \
        case 7: MACRO(7); break;     \
        case 8: MACRO(8); break;     \
        case 9: MACRO(9); break;     \
        case 10: MACRO(10); break;   \
        case 11: MACRO(11); break;   \
        case 12: MACRO(12); break;   \
        case 13: MACRO(13); break;   \
        case 14: MACRO(14); break;   \
        case 15: MACRO(15); break;   \
        case 16: MACRO(16); break;   \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_locate2(const fp2_handle *h, const Loc2 &a, int nblk, hipStream_t s)
{
#define FP2_LOC(N1) k2_locate<N1><<<nblk, kWave, 0, s>>>(a, h->d_basis, h->d_dnode)
    FP2_SWITCH(FP2_LOC)
#undef FP2_LOC
    return hipGetLastError();
}

hipError_t launch_eval2(const fp2_handle *h, const Ev2 &a, int nblk, hipStream_t s)
{
#define FP2_EV(N1) k2_eval<N1><<<nblk, kWave, 0, s>>>(a, h->d_basis)
    FP2_SWITCH(FP2_EV)
#undef FP2_EV
    return hipGetLastError();
}

template <class T>
hipError_t dalloc2(fp2_handle *h, T **p, size_t count)
{
    const size_t b = sizeof(T) * (count ? count : 1);
    const hipError_t e = hipMalloc((void **)p, b);
    if (e == hipSuccess) {
        h->bytes += b;
        h->allocs.push_back((void *)*p);
    } else {
        *p = nullptr;
    }
    return e;
}

void release2(fp2_handle *h)
{
    if (!h) return;
    (void)hipDeviceSynchronize();
    for (void *p : h->allocs) (void)hipFree(p);
    delete h;
}

}  // namespace
}  // namespace fp

using namespace fp;

#define FP2_HIP(call)                               \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) {                     \
            int rc_ = fp::hip_fail(e_, #call);      \
            release2(h);                            \
            return rc_;                             \
        }                                           \
    } while (0)

extern "C" int findpts2_setup(fp2_handle **out, const double *x, const double *y, int E, int N,
                              double tol, const int *elem_session, const double *delta,
                              int max_points, void *stream)
{
    if (!out || !x || !y) {
        set_error("findpts2_setup: NULL argument");
        return FP_EINVAL;
    }
    *out = nullptr;
    if (N < 1 || N > kMaxN1 - 1) {
        set_error("findpts2_setup: N must be in [1, 15]");
        return FP_ERANGE;
    }
    if (E < 1 || max_points < 1 || !(tol > 0.0 && tol < 1.0)) {
        set_error("findpts2_setup: need E >= 1, max_points >= 1, 0 < tol < 1");
        return FP_EINVAL;
    }
    const int n1 = N + 1, V = n1 * n1;
    const long long EV = (long long)E * V;
    if (EV * 2 > (1LL << 40)) {
        set_error("findpts2_setup: mesh too large");
        return FP_ERANGE;
    }
    hipStream_t s = (hipStream_t)stream;
    fp2_handle *h = new fp2_handle();
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        set_error("findpts2_setup: no HIP device");
        return FP_EHIP;
    }
    h->E = E;
    h->N = N;
    h->n1 = n1;
    h->V = V;
    h->tol = tol;
    h->M = max_points;
    h->basis = make_basis(N);
    FP2_HIP(dalloc2(h, &h->geom, 2 * (size_t)EV));
    FP2_HIP(dalloc2(h, &h->esize, (size_t)E));
    FP2_HIP(dalloc2(h, &h->bbox, 4 * (size_t)E));
    FP2_HIP(dalloc2(h, &h->obb, 10 * (size_t)E));
    FP2_HIP(dalloc2(h, &h->d_flag, 1));
    FP2_HIP(dalloc2(h, &h->d_g, 4));
    FP2_HIP(dalloc2(h, &h->d_binv, (size_t)n1 * n1));
    FP2_HIP(dalloc2(h, &h->d_basis, 2 * kMaxN1));
    FP2_HIP(dalloc2(h, &h->d_dnode, (size_t)n1 * n1));
    FP2_HIP(dalloc2(h, &h->stats, 3));
    const std::vector<double> binv = bernstein_to_nodal_inverse(N, h->basis.z);
    const std::vector<double> dnode = node_derivatives(h->basis, N);
    FP2_HIP(hipMemcpyAsync(h->d_basis, &h->basis, sizeof(Basis), hipMemcpyHostToDevice, s));
    FP2_HIP(hipMemcpyAsync(h->d_dnode, dnode.data(), sizeof(double) * n1 * n1,
                           hipMemcpyHostToDevice, s));
    FP2_HIP(hipMemcpyAsync(h->d_binv, binv.data(), sizeof(double) * n1 * n1,
                           hipMemcpyHostToDevice, s));
    FP2_HIP(hipMemsetAsync(h->stats, 0, 3 * sizeof(unsigned long long), s));
    if (elem_session) {
        FP2_HIP(dalloc2(h, &h->esess, (size_t)E));
        FP2_HIP(hipMemcpyAsync(h->esess, elem_session, sizeof(int) * E, hipMemcpyDeviceToDevice, s));
    }
    if (delta) {
        FP2_HIP(dalloc2(h, &h->delta, (size_t)EV));
        FP2_HIP(hipMemcpyAsync(h->delta, delta, sizeof(double) * EV, hipMemcpyDeviceToDevice, s));
    }
    FP2_HIP(hipMemsetAsync(h->d_flag, 0, sizeof(int), s));
    {
        const long long blocks = std::min<long long>((EV + 255) / 256, 256LL * 64);
        k2_pack<<<(int)blocks, 256, 0, s>>>(x, y, EV, V, h->geom, h->d_flag);
        FP2_HIP(hipGetLastError());
    }
    k2_bbox<<<E, kWave, 0, s>>>(h->geom, n1, h->d_binv, h->bbox, h->esize);
    FP2_HIP(hipGetLastError());
    k2_obb<<<E, kWave, 0, s>>>(h->geom, n1, h->d_binv, h->bbox, h->esize, h->tol, h->obb);
    FP2_HIP(hipGetLastError());
    k2_gbox<<<1, 256, 0, s>>>(h->bbox, E, h->d_g);
    FP2_HIP(hipGetLastError());
    double gb[4];
    int bad = 0;
    FP2_HIP(hipMemcpyAsync(gb, h->d_g, sizeof gb, hipMemcpyDeviceToHost, s));
    FP2_HIP(hipMemcpyAsync(&bad, h->d_flag, sizeof bad, hipMemcpyDeviceToHost, s));
    FP2_HIP(hipStreamSynchronize(s));
    if (bad) {
        release2(h);
        set_error("findpts2_setup: non-finite node coordinates");
        return FP_EINVAL;
    }
    // hash grid: about 4 E cells (two per element and axis)
    Grid2 g{};
    double ext[2], area = 1.0;
    for (int a = 0; a < 2; ++a) {
        g.lo[a] = gb[2 * a];
        g.hi[a] = gb[2 * a + 1];
        ext[a] = g.hi[a] - g.lo[a];
        if (!(ext[a] > 0.0)) ext[a] = 1e-300;
        area *= ext[a];
    }
    const double dens = std::sqrt(4.0 * (double)E / area);
    for (int a = 0; a < 2; ++a) {
        double n = std::floor(ext[a] * dens + 0.5);
        n = std::min(std::max(n, 1.0), 16384.0);
        g.nc[a] = (int)n;
        g.inv[a] = g.nc[a] / ext[a];
        h->glo[a] = g.lo[a];
        h->ghi[a] = g.hi[a];
        h->ginv[a] = g.inv[a];
        h->nc[a] = g.nc[a];
    }
    h->ncell = (long long)g.nc[0] * g.nc[1];
    int *cnt = nullptr;
    FP2_HIP(dalloc2(h, &cnt, (size_t)h->ncell + 1));
    FP2_HIP(dalloc2(h, &h->cell_off, (size_t)h->ncell + 1));
    const int stn = std::max(scan_tmp_size(h->ncell), scan_tmp_size((long long)E + 1));
    FP2_HIP(dalloc2(h, &h->scan_tmp, (size_t)stn));
    FP2_HIP(fill_int(cnt, 0, h->ncell + 1, s));
    const int eb = (E + 255) / 256;
    k2_hash_pass<<<eb, 256, 0, s>>>(h->bbox, E, g, 0, cnt, nullptr, nullptr);
    FP2_HIP(hipGetLastError());
    FP2_HIP(scan_exclusive(cnt, h->cell_off, (int)h->ncell, h->scan_tmp, s));
    int nnz = 0;
    FP2_HIP(hipMemcpyAsync(&nnz, h->cell_off + h->ncell, sizeof(int), hipMemcpyDeviceToHost, s));
    FP2_HIP(hipStreamSynchronize(s));
    h->nnz = nnz;
    FP2_HIP(dalloc2(h, &h->cell_el, (size_t)nnz));
    FP2_HIP(fill_int(cnt, 0, h->ncell, s));
    k2_hash_pass<<<eb, 256, 0, s>>>(h->bbox, E, g, 1, cnt, h->cell_off, h->cell_el);
    FP2_HIP(hipGetLastError());
    FP2_HIP(hipMemsetAsync(h->d_flag, 0, sizeof(int), s));
    k2_hash_sort<<<(int)((h->ncell + 255) / 256), 256, 0, s>>>(h->cell_off, h->cell_el, h->ncell,
                                                               h->d_flag);
    FP2_HIP(hipGetLastError());
    int maxlen = 0;
    FP2_HIP(hipMemcpyAsync(&maxlen, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    FP2_HIP(hipStreamSynchronize(s));
    h->MC = std::max(1, maxlen);
    // workspace for max_points points per pass
    const size_t M = (size_t)h->M, MC = (size_t)h->MC;
    FP2_HIP(dalloc2(h, &h->ncand, M));
    FP2_HIP(dalloc2(h, &h->cand_el, M * MC));
    FP2_HIP(dalloc2(h, &h->cand_pos, M * MC));
    FP2_HIP(dalloc2(h, &h->elem_cnt, (size_t)E + 1));
    FP2_HIP(dalloc2(h, &h->elem_off, (size_t)E + 1));
    FP2_HIP(dalloc2(h, &h->order, M * MC));
    FP2_HIP(dalloc2(h, &h->res, 3 * M * MC));
    FP2_HIP(dalloc2(h, &h->res_in, M * MC));
    if (delta) FP2_HIP(dalloc2(h, &h->res_dl, M * MC));
    FP2_HIP(dalloc2(h, &h->iter_part, (size_t)unit_grid(E, (long long)M, kUnit2)));
    FP2_HIP(dalloc2(h, &h->ev_pos, M));
    FP2_HIP(dalloc2(h, &h->redo, M));
    FP2_HIP(dalloc2(h, &h->cand_part, (M + 255) / 256));
    FP2_HIP(dalloc2(h, &h->ev_order, M));
    FP2_HIP(hipStreamSynchronize(s));
    *out = h;
    return FP_OK;
}

extern "C" int findpts2(fp2_handle *h, int npts, const double *pts, const int *pt_session,
                        int *code, int *el, double *rs, double *dist2, void *stream)
{
    if (!h) {
        set_error("findpts2: NULL handle");
        return FP_EINVAL;
    }
    if (npts < 0) {
        set_error("findpts2: npts < 0");
        return FP_EINVAL;
    }
    if (npts == 0) return FP_OK;
    if (!pts || !code || !el || !rs || !dist2) {
        set_error("findpts2: NULL argument");
        return FP_EINVAL;
    }
    int dev = 0;
    FP_HIP(hipGetDevice(&dev));
    if (dev != h->device) FP_HIP(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    for (int start = 0; start < npts; start += h->M) {
        const int n = (npts - start < h->M) ? npts - start : h->M;
        Loc2 a{};
        a.geom = h->geom;
        a.esize = h->esize;
        a.bbox = h->bbox;
        a.delta = h->delta;
        a.pts = pts + 2 * (long long)start;
        a.esess = h->esess;
        a.cell_off = h->cell_off;
        a.cell_el = h->cell_el;
        a.psess = pt_session ? pt_session + start : nullptr;
        for (int d = 0; d < 2; ++d) {
            a.g.lo[d] = h->glo[d];
            a.g.hi[d] = h->ghi[d];
            a.g.inv[d] = h->ginv[d];
            a.g.nc[d] = h->nc[d];
        }
        a.npts = n;
        a.M = h->M;
        a.MC = h->MC;
        a.E = h->E;
        a.tol = h->tol;
        a.ncand = h->ncand;
        a.cand_el = h->cand_el;
        a.cand_pos = h->cand_pos;
        a.elem_cnt = h->elem_cnt;
        a.elem_off = h->elem_off;
        a.order = h->order;
        a.res = h->res;
        a.res_in = h->res_in;
        a.res_dl = h->res_dl;
        a.iter_part = h->iter_part;
        a.cand_part = h->cand_part;
        const int pb = (n + 255) / 256;
        for (int round = 0; round < 2; ++round) {
            a.obb = round == 0 ? h->obb : nullptr;
            a.redo = round == 0 ? h->redo : nullptr;
            a.only = round == 0 ? nullptr : h->redo;
            FP_HIP(fill_int(h->elem_cnt, 0, (long long)h->E + 1, s));
            k2_cand<<<pb, 256, 0, s>>>(a);
            FP_HIP(hipGetLastError());
            FP_HIP(scan_exclusive(h->elem_cnt, h->elem_off, h->E, h->scan_tmp, s));
            k2_scatter<<<pb, 256, 0, s>>>(a);
            FP_HIP(hipGetLastError());
            const int nblk = unit_grid(h->E, n, kUnit2);
            FP_HIP(launch_locate2(h, a, nblk, s));
            k2_select<<<pb, 256, 0, s>>>(a, code + start, el + start, rs + 2 * (long long)start,
                                         dist2 + start);
            FP_HIP(hipGetLastError());
            k2_stats<<<1, 1024, 0, s>>>(h->iter_part, nblk, h->cand_part, round == 0 ? pb : 0,
                                        h->E, h->elem_off, h->stats);
            FP_HIP(hipGetLastError());
        }
    }
    return FP_OK;
}

extern "C" int findpts2_eval(fp2_handle *h, int npts, const int *code, const int *el,
                             const double *rs, int nfields, const double *const *h_fields,
                             double *out, void *stream)
{
    if (!h) {
        set_error("findpts2_eval: NULL handle");
        return FP_EINVAL;
    }
    if (npts < 0 || nfields < 1) {
        set_error("findpts2_eval: npts < 0 or nfields < 1");
        return FP_EINVAL;
    }
    if (npts == 0) return FP_OK;
    if (!code || !el || !rs || !h_fields || !out) {
        set_error("findpts2_eval: NULL argument");
        return FP_EINVAL;
    }
    for (int f = 0; f < nfields; ++f)
        if (!h_fields[f]) {
            set_error("findpts2_eval: NULL field pointer");
            return FP_EINVAL;
        }
    int dev = 0;
    FP_HIP(hipGetDevice(&dev));
    if (dev != h->device) FP_HIP(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    for (int start = 0; start < npts; start += h->M) {
        const int n = (npts - start < h->M) ? npts - start : h->M;
        const int pb = (n + 255) / 256;
        for (int f0 = 0; f0 < nfields; f0 += kMaxEvalFields) {
            const int nf = std::min(kMaxEvalFields, nfields - f0);
            Ev2 a{};
            a.code = code + start;
            a.el = el + start;
            a.rs = rs + 2 * (long long)start;
            a.npts = n;
            a.E = h->E;
            a.cnt = h->elem_cnt;
            a.off = h->elem_off;
            a.pos = h->ev_pos;
            a.order = h->ev_order;
            a.out = out + (long long)f0 * npts + start;
            a.ostride = npts;
            a.nf = nf;
            a.out_all = out + start;
            a.nf_all = nfields;
            for (int f = 0; f < nf; ++f) a.f[f] = h_fields[f0 + f];
            if (f0 == 0) {
                FP_HIP(fill_int(h->elem_cnt, 0, (long long)h->E + 1, s));
                k2_ev_count<<<pb, 256, 0, s>>>(a);
                FP_HIP(hipGetLastError());
                FP_HIP(scan_exclusive(h->elem_cnt, h->elem_off, h->E, h->scan_tmp, s));
                k2_ev_scatter<<<pb, 256, 0, s>>>(a);
                FP_HIP(hipGetLastError());
            }
            FP_HIP(launch_eval2(h, a, unit_grid(h->E, n, kUnitEval2), s));
        }
    }
    return FP_OK;
}

extern "C" int findpts2_stats(fp2_handle *h, long long *h_counts, int reset)
{
    if (!h || !h_counts) {
        set_error("findpts2_stats: NULL argument");
        return FP_EINVAL;
    }
    unsigned long long v[3];
    FP_HIP(hipMemcpy(v, h->stats, sizeof v, hipMemcpyDeviceToHost));
    for (int i = 0; i < 3; ++i) h_counts[i] = (long long)v[i];
    if (reset) FP_HIP(hipMemset(h->stats, 0, sizeof v));
    return FP_OK;
}

extern "C" int findpts2_get_bbox(fp2_handle *h, double *h_bbox, double *h_size)
{
    if (!h || !h_bbox || !h_size) {
        set_error("findpts2_get_bbox: NULL argument");
        return FP_EINVAL;
    }
    FP_HIP(hipMemcpy(h_bbox, h->bbox, sizeof(double) * 4 * h->E, hipMemcpyDeviceToHost));
    FP_HIP(hipMemcpy(h_size, h->esize, sizeof(double) * h->E, hipMemcpyDeviceToHost));
    return FP_OK;
}

extern "C" int findpts2_free(fp2_handle *h)
{
    release2(h);
    return FP_OK;
}
