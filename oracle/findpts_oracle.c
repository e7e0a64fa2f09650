/*
 * findpts_oracle.c -- plain, slow, double-precision CPU reference ("oracle")
 * for point location (findpts) and interpolation (findpts_eval) on meshes of
 * curved isoparametric hexahedral spectral elements, and (second part, or2_*)
 * on meshes of curved quadrilateral elements in two dimensions.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant generator with the HIP library.
 *
 * What it follows (the paper is Mittal, Dutta & Fischer, "Nonconforming
 * Schwarz-spectral element methods for incompressible flow"):
 *   - Section 2 (SEM): geometry and fields are tensor-product polynomials of
 *     order N on GLL nodes of the reference cube [-1,1]^3, isoparametric map.
 *   - Section 2.1 (Interpolation): findpts returns (e, r, s, t) and a code
 *     (inside an element / on a border / not found); it filters candidates
 *     with a hash table, then elementwise bounding boxes, then minimises
 *     ||x^e(r) - x*||^2 by trust-region Newton started from the closest
 *     mapped GLL node; findpts_eval interpolates a scalar field at (e, r).
 *     Session ids exclude a point's own subdomain; among several other
 *     subdomains the one maximising its distance-to-boundary field wins.
 * Where the paper is silent, this file takes these readings:
 *   bounding box   = hull of the tensor Bernstein coefficients + margin,
 *   hash           = uniform grid of about E cells (result-invariant),
 *   start node tie = smallest linear node index,
 *   trust region   = projected Gauss-Newton with an active set for the
 *                    bounds [-1,1]^3 (Nocedal & Wright 2006, Alg. 4.1;
 *                    Bertsekas 1982), constants below,
 *   tolerance      = relative to the element size h_e,
 *   ties           = smallest element id; delta compared across sessions.
 *
 * Parity is pinned (tests/test_oracle_*.py) by closed forms (GLL nodes and
 * weights, affine maps), polynomial exactness of the basis and of
 * interpolation, exact recovery of points generated as x^e(r_true) through
 * an analytic polynomial map, brute force over all elements with many
 * Newton starts, finite-difference Jacobians and an analytic three-session
 * distance test.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (see build.py).
 * No fused multiply-add contraction, no fast-math: IEEE binary64 throughout.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXN1 16 /* N <= 15 */

/* ---------------------------------------------------------------------------
 * Legendre polynomial P_n and its first two derivatives at x, by the
 * three-term recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1} and its
 * derivatives P'_{n+1} = P'_{n-1} + (2n+1) P_n, P''_{n+1} = P''_{n-1} +
 * (2n+1) P'_n.
 * ------------------------------------------------------------------------- */
static void legendre(int n, double x, double *p, double *dp, double *d2p)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0, s0 = 0.0, s1 = 0.0;
    if (n == 0) { *p = 1.0; *dp = 0.0; *d2p = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * p1;
        double s2 = s0 + (2.0 * k + 1.0) * d1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2; s0 = s1; s1 = s2;
    }
    *p = p1; *dp = d1; *d2p = s1;
}

/* GLL nodes and weights (Section 2: nodal bases on the GLL points).
 * Nodes: -1, +1 and the N-1 roots of P_N', found by Newton's method on P_N'
 * from the Chebyshev-Gauss-Lobatto guesses -cos(pi i / N); symmetrised, with
 * the middle node exactly 0 for even N.  Weights w_i = 2 / (N (N+1) P_N(z_i)^2).
 * Returns 0, or -1 if N is out of range. */
int or_gll(int N, double *z, double *w)
{
    if (N < 1 || N > OR_MAXN1 - 1) return -1;
    z[0] = -1.0; z[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            double p, dp, d2p;
            legendre(N, x, &p, &dp, &d2p);
            double dx = dp / d2p;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        z[i] = x;
    }
    for (int i = 0; i < (N + 1) / 2; ++i) {
        double a = 0.5 * (z[N - i] - z[i]);
        z[i] = -a; z[N - i] = a;
    }
    if (N % 2 == 0) z[N / 2] = 0.0;
    for (int i = 0; i <= N; ++i) {
        double p, dp, d2p;
        legendre(N, z[i], &p, &dp, &d2p);
        w[i] = 2.0 / (N * (N + 1.0) * p * p);
    }
    return 0;
}

/* Lagrange basis on the nodes z[0..N] in product form:
 *   h_i(r)  = prod_{m != i} (r - z_m) / (z_i - z_m)
 *   h_i'(r) = sum_{l != i} 1/(z_i - z_l) prod_{m != i,l} (r - z_m)/(z_i - z_m)
 * Exact Kronecker property at the nodes (no division by r - z_m). */
static void lagrange(int N, const double *z, double r, double *h, double *dh)
{
    for (int i = 0; i <= N; ++i) {
        double hi = 1.0, dhi = 0.0;
        for (int m = 0; m <= N; ++m)
            if (m != i) hi *= (r - z[m]) / (z[i] - z[m]);
        for (int l = 0; l <= N; ++l) {
            if (l == i) continue;
            double t = 1.0 / (z[i] - z[l]);
            for (int m = 0; m <= N; ++m)
                if (m != i && m != l) t *= (r - z[m]) / (z[i] - z[m]);
            dhi += t;
        }
        h[i] = hi;
        if (dh) dh[i] = dhi;
    }
}

/* Exposed for the basis pins. */
int or_lagrange(int N, double r, double *h, double *dh)
{
    double z[OR_MAXN1], w[OR_MAXN1];
    if (or_gll(N, z, w)) return -1;
    lagrange(N, z, r, h, dh);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Mesh state.
 * ------------------------------------------------------------------------- */
typedef struct {
    int E, N, n1, V;
    double tol;
    const double *X[3];    /* borrowed: x, y, z, each E*V, r index fastest */
    const int *esess;      /* borrowed or NULL                              */
    const double *delta;   /* borrowed or NULL                              */
    double z[OR_MAXN1], w[OR_MAXN1];
    double *bbox;          /* E*6: xmin xmax ymin ymax zmin zmax            */
    double *h;             /* E: element size                               */
    double lo[3], hi[3], dx[3];
    int nc[3];
    int *cell_off, *cell_el;
} or_mesh;

static inline const double *elem(const or_mesh *m, int c, int e)
{
    return m->X[c] + (size_t)e * m->V;
}

/* Isoparametric map (Section 2): x_c(r) = sum_ijk X_c[ijk] h_i(r) h_j(s) h_k(t)
 * and its Jacobian J[c][d] = d x_c / d r_d, as plain triple sums. */
static void emap(const or_mesh *m, int e, const double r[3], double x[3],
                 double J[9])
{
    int n1 = m->n1;
    double hr[OR_MAXN1], hs[OR_MAXN1], ht[OR_MAXN1];
    double dr[OR_MAXN1], ds[OR_MAXN1], dt[OR_MAXN1];
    lagrange(m->N, m->z, r[0], hr, dr);
    lagrange(m->N, m->z, r[1], hs, ds);
    lagrange(m->N, m->z, r[2], ht, dt);
    for (int c = 0; c < 3; ++c) {
        const double *Xc = elem(m, c, e);
        double v = 0, vr = 0, vs = 0, vt = 0;
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    double X = Xc[i + n1 * (j + n1 * k)];
                    v  += X * hr[i] * hs[j] * ht[k];
                    vr += X * dr[i] * hs[j] * ht[k];
                    vs += X * hr[i] * ds[j] * ht[k];
                    vt += X * hr[i] * hs[j] * dt[k];
                }
        x[c] = v;
        if (J) { J[3 * c] = vr; J[3 * c + 1] = vs; J[3 * c + 2] = vt; }
    }
}

/* Scalar field interpolation (findpts_eval, Section 2.1):
 * f(r) = sum_k h_k(t) sum_j h_j(s) sum_i h_i(r) F[ijk]. */
static double interp(const or_mesh *m, const double *F, const double r[3])
{
    int n1 = m->n1;
    double hr[OR_MAXN1], hs[OR_MAXN1], ht[OR_MAXN1];
    lagrange(m->N, m->z, r[0], hr, NULL);
    lagrange(m->N, m->z, r[1], hs, NULL);
    lagrange(m->N, m->z, r[2], ht, NULL);
    double f = 0.0;
    for (int k = 0; k < n1; ++k) {
        double fs = 0.0;
        for (int j = 0; j < n1; ++j) {
            double fr = 0.0;
            for (int i = 0; i < n1; ++i) fr += hr[i] * F[i + n1 * (j + n1 * k)];
            fs += hs[j] * fr;
        }
        f += ht[k] * fs;
    }
    return f;
}

/* ---------------------------------------------------------------------------
 * Element bounding boxes (Section 2.1: "elementwise bounding boxes").
 * Reading: convert each coordinate's nodal values to tensor Bernstein
 * coefficients on [-1,1]; by the convex-hull property of the Bernstein form
 * the element lies inside [min coef, max coef] per axis.  Expand by
 * 1e-8 h_e + 1e-14 max|x|, h_e = largest per-axis extent of the element's
 * nodes.
 * ------------------------------------------------------------------------- */
static double binom(int n, int k)
{
    double b = 1.0;
    for (int i = 1; i <= k; ++i) b = b * (n - k + i) / i;
    return b;
}

/* Inverse of B[i][k] = b_k(z_i), b_k(x) = C(N,k) ((1+x)/2)^k ((1-x)/2)^(N-k),
 * by Gauss-Jordan elimination with partial pivoting. */
static void bernstein_inverse(int N, const double *z, double *Binv)
{
    int n = N + 1;
    double A[OR_MAXN1][2 * OR_MAXN1];
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < n; ++k) {
            double u = 0.5 * (1.0 + z[i]), v = 0.5 * (1.0 - z[i]);
            A[i][k] = binom(N, k) * pow(u, k) * pow(v, N - k);
            A[i][n + k] = (i == k) ? 1.0 : 0.0;
        }
    }
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int i = c + 1; i < n; ++i)
            if (fabs(A[i][c]) > fabs(A[p][c])) p = i;
        if (p != c)
            for (int k = 0; k < 2 * n; ++k) {
                double t = A[c][k]; A[c][k] = A[p][k]; A[p][k] = t;
            }
        double d = A[c][c];
        for (int k = 0; k < 2 * n; ++k) A[c][k] /= d;
        for (int i = 0; i < n; ++i) {
            if (i == c) continue;
            double f = A[i][c];
            for (int k = 0; k < 2 * n; ++k) A[i][k] -= f * A[c][k];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) Binv[i * n + k] = A[i][n + k];
}

int or_bernstein_inverse(int N, double *Binv)
{
    double z[OR_MAXN1], w[OR_MAXN1];
    if (or_gll(N, z, w)) return -1;
    bernstein_inverse(N, z, Binv);
    return 0;
}

static void element_bbox(const or_mesh *m, const double *Binv, int e)
{
    int n1 = m->n1, V = m->V;
    double *a = malloc(sizeof(double) * V), *b = malloc(sizeof(double) * V);
    double he = 0.0, xmax = 0.0;
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
        const double *Xc = elem(m, c, e);
        double mn = Xc[0], mx = Xc[0];
        for (int q = 0; q < V; ++q) {
            if (Xc[q] < mn) mn = Xc[q];
            if (Xc[q] > mx) mx = Xc[q];
            if (fabs(Xc[q]) > xmax) xmax = fabs(Xc[q]);
        }
        if (mx - mn > he) he = mx - mn;
        /* coefficients: apply Binv along i, then j, then k */
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    double s = 0.0;
                    for (int l = 0; l < n1; ++l)
                        s += Binv[i * n1 + l] * Xc[l + n1 * (j + n1 * k)];
                    a[i + n1 * (j + n1 * k)] = s;
                }
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    double s = 0.0;
                    for (int l = 0; l < n1; ++l)
                        s += Binv[j * n1 + l] * a[i + n1 * (l + n1 * k)];
                    b[i + n1 * (j + n1 * k)] = s;
                }
        for (int k = 0; k < n1; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n1; ++i) {
                    double s = 0.0;
                    for (int l = 0; l < n1; ++l)
                        s += Binv[k * n1 + l] * b[i + n1 * (j + n1 * l)];
                    a[i + n1 * (j + n1 * k)] = s;
                }
        lo[c] = a[0]; hi[c] = a[0];
        for (int q = 0; q < V; ++q) {
            if (a[q] < lo[c]) lo[c] = a[q];
            if (a[q] > hi[c]) hi[c] = a[q];
        }
    }
    double marg = 1e-8 * he + 1e-14 * xmax;
    for (int c = 0; c < 3; ++c) {
        m->bbox[6 * e + 2 * c] = lo[c] - marg;
        m->bbox[6 * e + 2 * c + 1] = hi[c] + marg;
    }
    m->h[e] = he;
    free(a); free(b);
}

/* ---------------------------------------------------------------------------
 * Hash grid (Section 2.1: "a hash table to identify ... potential owners").
 * Reading: a uniform grid over the union of the element boxes with about E
 * cells, n_a = max(1, round(ext_a (E / vol)^(1/3))); each cell lists, in
 * ascending order, the elements whose closed box overlaps it.  The candidate
 * set {e in cell(x*) : x* in box_e} equals {e : x* in box_e} for any grid.
 * ------------------------------------------------------------------------- */
static int cell_of(const or_mesh *m, int a, double x)
{
    double u = (x - m->lo[a]) / m->dx[a];
    int i = (int)floor(u);
    if (i < 0) i = 0;
    if (i > m->nc[a] - 1) i = m->nc[a] - 1;
    return i;
}

static void build_hash(or_mesh *m)
{
    int E = m->E;
    for (int a = 0; a < 3; ++a) { m->lo[a] = m->bbox[2 * a]; m->hi[a] = m->bbox[2 * a + 1]; }
    for (int e = 1; e < E; ++e)
        for (int a = 0; a < 3; ++a) {
            if (m->bbox[6 * e + 2 * a] < m->lo[a]) m->lo[a] = m->bbox[6 * e + 2 * a];
            if (m->bbox[6 * e + 2 * a + 1] > m->hi[a]) m->hi[a] = m->bbox[6 * e + 2 * a + 1];
        }
    double ext[3], vol = 1.0;
    for (int a = 0; a < 3; ++a) {
        ext[a] = m->hi[a] - m->lo[a];
        if (!(ext[a] > 0.0)) ext[a] = 1e-300;
        vol *= ext[a];
    }
    double dens = cbrt((double)E / vol);
    for (int a = 0; a < 3; ++a) {
        double n = floor(ext[a] * dens + 0.5);
        if (n < 1.0) n = 1.0;
        if (n > 4096.0) n = 4096.0;
        m->nc[a] = (int)n;
        m->dx[a] = ext[a] / m->nc[a];
    }
    long ncell = (long)m->nc[0] * m->nc[1] * m->nc[2];
    int *cnt = calloc(ncell + 1, sizeof(int));
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            m->cell_off = malloc(sizeof(int) * (ncell + 1));
            m->cell_off[0] = 0;
            for (long c = 0; c < ncell; ++c) m->cell_off[c + 1] = m->cell_off[c] + cnt[c];
            m->cell_el = malloc(sizeof(int) * (m->cell_off[ncell] + 1));
            memset(cnt, 0, sizeof(int) * ncell);
        }
        for (int e = 0; e < E; ++e) {  /* ascending e keeps each list sorted */
            const double *b = m->bbox + 6 * e;
            int i0 = cell_of(m, 0, b[0]), i1 = cell_of(m, 0, b[1]);
            int j0 = cell_of(m, 1, b[2]), j1 = cell_of(m, 1, b[3]);
            int k0 = cell_of(m, 2, b[4]), k1 = cell_of(m, 2, b[5]);
            for (int k = k0; k <= k1; ++k)
                for (int j = j0; j <= j1; ++j)
                    for (int i = i0; i <= i1; ++i) {
                        long c = i + (long)m->nc[0] * (j + (long)m->nc[1] * k);
                        if (pass == 1) m->cell_el[m->cell_off[c] + cnt[c]] = e;
                        cnt[c]++;
                    }
        }
    }
    free(cnt);
}

or_mesh *or_setup(int E, int N, const double *x, const double *y,
                  const double *z, double tol, const int *esess,
                  const double *delta)
{
    if (E < 1 || N < 1 || N > OR_MAXN1 - 1) return NULL;
    or_mesh *m = calloc(1, sizeof(or_mesh));
    m->E = E; m->N = N; m->n1 = N + 1; m->V = m->n1 * m->n1 * m->n1;
    m->tol = tol;
    m->X[0] = x; m->X[1] = y; m->X[2] = z;
    m->esess = esess; m->delta = delta;
    or_gll(N, m->z, m->w);
    m->bbox = malloc(sizeof(double) * 6 * E);
    m->h = malloc(sizeof(double) * E);
    double Binv[OR_MAXN1 * OR_MAXN1];
    bernstein_inverse(N, m->z, Binv);
#pragma omp parallel for schedule(dynamic, 64)
    for (int e = 0; e < E; ++e) element_bbox(m, Binv, e);
    build_hash(m);
    return m;
}

void or_free(or_mesh *m)
{
    if (!m) return;
    free(m->bbox); free(m->h); free(m->cell_off); free(m->cell_el); free(m);
}

void or_get_bbox(const or_mesh *m, double *bbox, double *h)
{
    memcpy(bbox, m->bbox, sizeof(double) * 6 * m->E);
    memcpy(h, m->h, sizeof(double) * m->E);
}

void or_get_hash(const or_mesh *m, int *nc, double *lo, double *dx, int *nnz)
{
    for (int a = 0; a < 3; ++a) { nc[a] = m->nc[a]; lo[a] = m->lo[a]; dx[a] = m->dx[a]; }
    *nnz = m->cell_off[(long)m->nc[0] * m->nc[1] * m->nc[2]];
}

void or_map(const or_mesh *m, int e, const double *r, double *x, double *J)
{
    emap(m, e, r, x, J);
}

static int in_box(const double *b, const double *p)
{
    return p[0] >= b[0] && p[0] <= b[1] && p[1] >= b[2] && p[1] <= b[3] &&
           p[2] >= b[4] && p[2] <= b[5];
}

/* Candidates of x* (Section 2.1 hash + bounding-box filter + session
 * exclusion): ascending element ids.  Returns the count (written up to max),
 * 0 if x* lies outside the hash box. */
int or_candidates(const or_mesh *m, const double *p, int psess, int *out, int max)
{
    for (int a = 0; a < 3; ++a)
        if (!(p[a] >= m->lo[a] && p[a] <= m->hi[a])) return 0;
    long c = cell_of(m, 0, p[0]) +
             (long)m->nc[0] * (cell_of(m, 1, p[1]) + (long)m->nc[1] * cell_of(m, 2, p[2]));
    int n = 0;
    for (int q = m->cell_off[c]; q < m->cell_off[c + 1]; ++q) {
        int e = m->cell_el[q];
        if (!in_box(m->bbox + 6 * e, p)) continue;
        if (psess >= 0 && m->esess && m->esess[e] == psess) continue;
        if (n < max) out[n] = e;
        n++;
    }
    return n;
}

/* ---------------------------------------------------------------------------
 * Trust-region Newton (Section 2.1): minimise phi(r) = ||x^e(r) - x*||^2 over
 * r in [-1,1]^3, starting at the closest mapped GLL node of element e.
 * Reading: projected Gauss-Newton with an active set.
 *   g = J^T F.  Coordinate d is held if it sits on a bound and -g points out.
 *   Step: all free -> solve J d = -F; else (J_f^T J_f) d_f = -J_f^T F.
 *   If the solve fails, d_f = -g_f (steepest descent).  Scale d to the
 *   trust radius D (max norm), then project r + d onto the cube: s = r' - r.
 *   pred = phi - ||F + J s||^2, ared = phi - phi(r'), rho = ared / pred.
 *   Accept if rho >= 0.01.  D <- min(2D, 2) if rho > 0.75 and the radius
 *   limited the step; D <- |s|/4 if rho < 0.25.
 *   Stop: phi <= (c h_e)^2 with c = min(1e-13, tol / 10), so that a point
 *   the tolerance accepts is never left short of it; an accepted step with
 *   |s| <= 1e-13 (Newton converges quadratically, so the point it reaches is
 *   at the rounding level of the map); |s| <= 1e-15 or pred <= 0 (no
 *   progress possible); 50 iterations.
 * ------------------------------------------------------------------------- */
#define OR_MAXIT 50

/* Squared residual at which Newton stops, for tolerance tol and element
 * size he: a tenth of the inside tolerance, at most 1e-13 h_e. */
static double resid_stop(double tol, double he)
{
    double c = 0.1 * tol < 1e-13 ? 0.1 * tol : 1e-13;
    return (c * he) * (c * he);
}

/* Solve A x = b (n <= 3) by Gaussian elimination with partial pivoting.
 * Returns 0 on success, -1 on a zero pivot or a non-finite result. */
static int solve_small(int n, double A[3][3], const double *b, double *x)
{
    double M[3][4];
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) M[i][j] = A[i][j];
        M[i][n] = b[i];
    }
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int i = c + 1; i < n; ++i)
            if (fabs(M[i][c]) > fabs(M[p][c])) p = i;
        if (M[p][c] == 0.0) return -1;
        if (p != c)
            for (int j = 0; j <= n; ++j) { double t = M[c][j]; M[c][j] = M[p][j]; M[p][j] = t; }
        for (int i = c + 1; i < n; ++i) {
            double f = M[i][c] / M[c][c];
            for (int j = c; j <= n; ++j) M[i][j] -= f * M[c][j];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = M[i][n];
        for (int j = i + 1; j < n; ++j) s -= M[i][j] * x[j];
        x[i] = s / M[i][i];
        if (!isfinite(x[i])) return -1;
    }
    return 0;
}

static void start_node(const or_mesh *m, int e, const double *p, double r[3])
{
    int n1 = m->n1, best = 0;
    double bd = INFINITY;
    for (int q = 0; q < m->V; ++q) {
        double d = 0.0;
        for (int c = 0; c < 3; ++c) {
            double t = elem(m, c, e)[q] - p[c];
            d += t * t;
        }
        if (d < bd) { bd = d; best = q; }   /* strict: smallest index wins ties */
    }
    r[0] = m->z[best % n1];
    r[1] = m->z[(best / n1) % n1];
    r[2] = m->z[best / (n1 * n1)];
}

static double resid(const or_mesh *m, int e, const double *p, const double r[3],
                    double F[3], double J[9])
{
    double x[3];
    emap(m, e, r, x, J);
    double phi = 0.0;
    for (int c = 0; c < 3; ++c) { F[c] = x[c] - p[c]; phi += F[c] * F[c]; }
    return phi;
}

/* Newton from the given start r (in/out).  Returns the iteration count and
 * writes phi at the returned r. */
static int tr_newton(const or_mesh *m, int e, const double *p, double r[3],
                     double *phi_out)
{
    double he = m->h[e], stop = resid_stop(m->tol, he);
    double F[3], J[9], D = 1.0;
    double phi = resid(m, e, p, r, F, J);
    int it = 0;
    while (it < OR_MAXIT) {
        if (phi <= stop) break;
        ++it;
        double g[3];
        for (int d = 0; d < 3; ++d)
            g[d] = J[d] * F[0] + J[3 + d] * F[1] + J[6 + d] * F[2];
        int fr[3], nf = 0;
        for (int d = 0; d < 3; ++d) {
            int held = (r[d] >= 1.0 && g[d] < 0.0) || (r[d] <= -1.0 && g[d] > 0.0);
            if (!held) fr[nf++] = d;
        }
        if (nf == 0) break;
        double dl[3] = {0.0, 0.0, 0.0};
        int bad;
        if (nf == 3) {
            double A[3][3], b[3];
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) A[i][j] = J[3 * i + j];
                b[i] = -F[i];
            }
            bad = solve_small(3, A, b, dl);
        } else {
            double A[3][3], b[3], xs[3];
            for (int a = 0; a < nf; ++a) {
                int da = fr[a];
                for (int bb = 0; bb < nf; ++bb) {
                    int db = fr[bb];
                    A[a][bb] = J[da] * J[db] + J[3 + da] * J[3 + db] + J[6 + da] * J[6 + db];
                }
                b[a] = -g[da];
            }
            bad = solve_small(nf, A, b, xs);
            if (!bad) for (int a = 0; a < nf; ++a) dl[fr[a]] = xs[a];
        }
        if (bad) {
            for (int d = 0; d < 3; ++d) dl[d] = 0.0;
            for (int a = 0; a < nf; ++a) dl[fr[a]] = -g[fr[a]];
        }
        double nd = 0.0;
        for (int d = 0; d < 3; ++d) if (fabs(dl[d]) > nd) nd = fabs(dl[d]);
        if (!(nd > 0.0) || !isfinite(nd)) break;
        int limited = 0;
        if (nd > D) {
            double sc = D / nd;
            for (int d = 0; d < 3; ++d) dl[d] *= sc;
            limited = 1;
        }
        double rn[3], s[3], ns = 0.0;
        for (int d = 0; d < 3; ++d) {
            double v = r[d] + dl[d];
            if (v > 1.0) v = 1.0;
            if (v < -1.0) v = -1.0;
            rn[d] = v;
            s[d] = v - r[d];
            if (fabs(s[d]) > ns) ns = fabs(s[d]);
        }
        if (ns <= 1e-15) break;
        double pred = phi;
        {
            double q = 0.0;
            for (int c = 0; c < 3; ++c) {
                double t = F[c] + J[3 * c] * s[0] + J[3 * c + 1] * s[1] + J[3 * c + 2] * s[2];
                q += t * t;
            }
            pred -= q;
        }
        if (!(pred > 0.0)) break;
        double Fn[3], Jn[9];
        double phin = resid(m, e, p, rn, Fn, Jn);
        double rho = (phi - phin) / pred;
        int acc = rho >= 0.01;
        if (acc) {
            for (int d = 0; d < 3; ++d) { r[d] = rn[d]; F[d] = Fn[d]; }
            for (int q = 0; q < 9; ++q) J[q] = Jn[q];
            phi = phin;
        }
        if (rho > 0.75 && limited) { D = 2.0 * D; if (D > 2.0) D = 2.0; }
        else if (rho < 0.25) D = 0.25 * ns;
        if (acc && ns <= 1e-13) break;
    }
    *phi_out = phi;
    return it;
}

/* One candidate: nearest-GLL start then trust-region Newton; returns
 * iterations, writes r and the squared distance. */
int or_newton(const or_mesh *m, int e, const double *p, double *r, double *d2)
{
    start_node(m, e, p, r);
    return tr_newton(m, e, p, r, d2);
}

/* Newton from a caller-given start (brute-force multi-start tests). */
int or_newton_from(const or_mesh *m, int e, const double *p, double *r, double *d2)
{
    return tr_newton(m, e, p, r, d2);
}

/* Distance-to-boundary field at (e, r) (Section 2.1 discriminator). */
static double delta_at(const or_mesh *m, int e, const double *r)
{
    return interp(m, m->delta + (size_t)e * m->V, r);
}

/* ---------------------------------------------------------------------------
 * Classification and selection (Section 2.1):
 *   candidate is INSIDE if sqrt(d2) <= tol * h_e.
 *   If some candidate is INSIDE: with a delta field, for each session among
 *   the INSIDE candidates take the largest delta(e, r); the session with the
 *   largest value wins (ties: smaller session id) and within it the smallest
 *   INSIDE element id; without delta, the smallest INSIDE element id.
 *   code 0.
 *   Else if candidates exist: smallest d2 (|difference| <= 1e-14 d2 counts as
 *   a tie, smaller id wins); code 1.  Else code 2, el = -1, rst = 0,
 *   dist2 = +inf.
 * ------------------------------------------------------------------------- */
typedef struct { int e; double r[3], d2; int inside; double dl; int sess; } cand_t;

static void select_cands(int has_delta, int dim, const cand_t *cs, int nc, int *code,
                         int *el, double *rst, double *dist2)
{
    int w = -1, anyin = 0;
    for (int q = 0; q < nc; ++q) if (cs[q].inside) { anyin = 1; break; }
    if (anyin) {
        if (has_delta) {
            int bs = 0; double bd = -INFINITY; int have = 0;
            for (int q = 0; q < nc; ++q) {
                if (!cs[q].inside) continue;
                /* best delta of this candidate's session */
                double sd = -INFINITY;
                for (int u = 0; u < nc; ++u)
                    if (cs[u].inside && cs[u].sess == cs[q].sess && cs[u].dl > sd) sd = cs[u].dl;
                if (!have || sd > bd || (sd == bd && cs[q].sess < bs)) {
                    have = 1; bd = sd; bs = cs[q].sess;
                }
            }
            for (int q = 0; q < nc; ++q)
                if (cs[q].inside && cs[q].sess == bs && (w < 0 || cs[q].e < cs[w].e)) w = q;
        } else {
            for (int q = 0; q < nc; ++q)
                if (cs[q].inside && (w < 0 || cs[q].e < cs[w].e)) w = q;
        }
        *code = 0;
    } else if (nc > 0) {
        for (int q = 0; q < nc; ++q) {
            if (w < 0) { w = q; continue; }
            double a = cs[q].d2, b = cs[w].d2;
            int tie = fabs(a - b) <= 1e-14 * (a > b ? a : b);
            if ((!tie && a < b) || (tie && cs[q].e < cs[w].e)) w = q;
        }
        *code = 1;
    }
    if (w < 0) {
        *code = 2; *el = -1;
        for (int d = 0; d < dim; ++d) rst[d] = 0.0;
        *dist2 = INFINITY;
        return;
    }
    *el = cs[w].e;
    for (int d = 0; d < dim; ++d) rst[d] = cs[w].r[d];
    *dist2 = cs[w].d2;
}

static void select_point(const or_mesh *m, const cand_t *cs, int nc, int *code,
                         int *el, double *rst, double *dist2)
{
    select_cands(m->delta != NULL, 3, cs, nc, code, el, rst, dist2);
}

static void fill_cand(const or_mesh *m, cand_t *c, int e, const double *p,
                      const double *r, double d2)
{
    c->e = e;
    for (int d = 0; d < 3; ++d) c->r[d] = r[d];
    double F[3];
    c->d2 = resid(m, e, p, c->r, F, NULL);   /* recomputed at the returned r */
    (void)d2;
    c->inside = sqrt(c->d2) <= m->tol * m->h[e];
    c->sess = m->esess ? m->esess[e] : 0;
    c->dl = (m->delta && c->inside) ? delta_at(m, e, c->r) : 0.0;
}

/* findpts over npts points (xyz interleaved).  psess may be NULL.  stats
 * (may be NULL) receives [total candidates, total Newton iterations]. */
void or_findpts(const or_mesh *m, int npts, const double *pts, const int *psess,
                int *code, int *el, double *rst, double *dist2, long long *stats,
                int nthreads)
{
    long long tc = 0, ti = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel reduction(+ : tc, ti)
    {
        int *ids = malloc(sizeof(int) * (m->E > 0 ? m->E : 1));
        cand_t *cs = malloc(sizeof(cand_t) * (m->E > 0 ? m->E : 1));
#pragma omp for schedule(dynamic, 1024)
        for (int p = 0; p < npts; ++p) {
            const double *x = pts + 3 * (size_t)p;
            int nc = or_candidates(m, x, psess ? psess[p] : -1, ids, m->E);
            for (int q = 0; q < nc; ++q) {
                double r[3], d2;
                ti += or_newton(m, ids[q], x, r, &d2);
                fill_cand(m, &cs[q], ids[q], x, r, d2);
            }
            tc += nc;
            select_point(m, cs, nc, code + p, el + p, rst + 3 * (size_t)p, dist2 + p);
        }
        free(ids); free(cs);
    }
    if (stats) { stats[0] = tc; stats[1] = ti; }
}

/* Brute force (test mode): every element is a candidate unless only_boxes is
 * set (then only elements whose box holds x*, without the hash); each
 * candidate is solved from the nearest GLL node, from every GLL node and
 * from a g^3 grid of starts on [-1,1]^3 (g >= 2), keeping the smallest
 * distance.  Same selection rule. */
void or_brute(const or_mesh *m, int npts, const double *pts, const int *psess,
              int g, int all_nodes, int only_boxes, int *code, int *el,
              double *rst, double *dist2, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        cand_t *cs = malloc(sizeof(cand_t) * m->E);
#pragma omp for schedule(dynamic, 1)
        for (int p = 0; p < npts; ++p) {
            const double *x = pts + 3 * (size_t)p;
            int nc = 0;
            for (int e = 0; e < m->E; ++e) {
                if (psess && psess[p] >= 0 && m->esess && m->esess[e] == psess[p]) continue;
                if (only_boxes && !in_box(m->bbox + 6 * e, x)) continue;
                double br[3], bd = INFINITY, r[3], d2;
                or_newton(m, e, x, r, &d2);
                bd = d2; br[0] = r[0]; br[1] = r[1]; br[2] = r[2];
                int nstart = (all_nodes ? m->V : 0) + g * g * g;
                for (int q = 0; q < nstart; ++q) {
                    if (q < (all_nodes ? m->V : 0)) {
                        r[0] = m->z[q % m->n1]; r[1] = m->z[(q / m->n1) % m->n1];
                        r[2] = m->z[q / (m->n1 * m->n1)];
                    } else {
                        int u = q - (all_nodes ? m->V : 0);
                        r[0] = -1.0 + 2.0 * (u % g) / (g - 1);
                        r[1] = -1.0 + 2.0 * ((u / g) % g) / (g - 1);
                        r[2] = -1.0 + 2.0 * (u / (g * g)) / (g - 1);
                    }
                    tr_newton(m, e, x, r, &d2);
                    if (d2 < bd) { bd = d2; br[0] = r[0]; br[1] = r[1]; br[2] = r[2]; }
                }
                fill_cand(m, &cs[nc], e, x, br, bd);
                nc++;
            }
            select_point(m, cs, nc, code + p, el + p, rst + 3 * (size_t)p, dist2 + p);
        }
        free(cs);
    }
}

/* findpts_eval (Section 2.1): interpolate nf fields (each E*V) at the located
 * points; code 2 gives NaN.  out is field-major: out[f*npts + p]. */
void or_eval(const or_mesh *m, int npts, const int *code, const int *el,
             const double *rst, int nf, const double *const *fields, double *out,
             int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1024)
    for (int p = 0; p < npts; ++p) {
        for (int f = 0; f < nf; ++f) {
            double v = NAN;
            if (code[p] != 2 && el[p] >= 0 && el[p] < m->E)
                v = interp(m, fields[f] + (size_t)el[p] * m->V, rst + 3 * (size_t)p);
            out[(size_t)f * npts + p] = v;
        }
    }
}

/* ===========================================================================
 * Two dimensions: meshes of curved quadrilateral spectral elements.
 *
 * The paper's method and its 2D figures (Figs. 1 and 6) carry over with the
 * reference square [-1,1]^2: x_c(r, s) = sum_ij X_c[i + n1 j] h_i(r) h_j(s)
 * for c = x, y; boxes, hash, closest-node start, trust-region Newton,
 * classification, selection and interpolation follow the 3D readings above
 * with two coordinates (hash: about E cells, n_a = round(ext_a (E/area)^(1/2))).
 * Everything below is written out again for two dimensions; only the 1D
 * helpers (GLL, Lagrange, Bernstein inverse, small solve) and the selection
 * rule are shared with the 3D code.
 * ========================================================================= */
typedef struct {
    int E, N, n1, V;
    double tol;
    const double *X[2];    /* borrowed: x, y, each E*V, r index fastest */
    const int *esess;
    const double *delta;
    double z[OR_MAXN1], w[OR_MAXN1];
    double *bbox;          /* E*4: xmin xmax ymin ymax */
    double *h;
    double lo[2], hi[2], dx[2];
    int nc[2];
    int *cell_off, *cell_el;
} or2_mesh;

static inline const double *elem2(const or2_mesh *m, int c, int e)
{
    return m->X[c] + (size_t)e * m->V;
}

static void emap2(const or2_mesh *m, int e, const double r[2], double x[2], double J[4])
{
    int n1 = m->n1;
    double hr[OR_MAXN1], hs[OR_MAXN1], dr[OR_MAXN1], ds[OR_MAXN1];
    lagrange(m->N, m->z, r[0], hr, dr);
    lagrange(m->N, m->z, r[1], hs, ds);
    for (int c = 0; c < 2; ++c) {
        const double *Xc = elem2(m, c, e);
        double v = 0, vr = 0, vs = 0;
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                double X = Xc[i + n1 * j];
                v  += X * hr[i] * hs[j];
                vr += X * dr[i] * hs[j];
                vs += X * hr[i] * ds[j];
            }
        x[c] = v;
        if (J) { J[2 * c] = vr; J[2 * c + 1] = vs; }
    }
}

static double interp2(const or2_mesh *m, const double *F, const double r[2])
{
    int n1 = m->n1;
    double hr[OR_MAXN1], hs[OR_MAXN1];
    lagrange(m->N, m->z, r[0], hr, NULL);
    lagrange(m->N, m->z, r[1], hs, NULL);
    double f = 0.0;
    for (int j = 0; j < n1; ++j) {
        double fr = 0.0;
        for (int i = 0; i < n1; ++i) fr += hr[i] * F[i + n1 * j];
        f += hs[j] * fr;
    }
    return f;
}

static void element_bbox2(const or2_mesh *m, const double *Binv, int e)
{
    int n1 = m->n1, V = m->V;
    double *a = malloc(sizeof(double) * V), *b = malloc(sizeof(double) * V);
    double he = 0.0, xmax = 0.0, lo[2], hi[2];
    for (int c = 0; c < 2; ++c) {
        const double *Xc = elem2(m, c, e);
        double mn = Xc[0], mx = Xc[0];
        for (int q = 0; q < V; ++q) {
            if (Xc[q] < mn) mn = Xc[q];
            if (Xc[q] > mx) mx = Xc[q];
            if (fabs(Xc[q]) > xmax) xmax = fabs(Xc[q]);
        }
        if (mx - mn > he) he = mx - mn;
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                double t = 0.0;
                for (int l = 0; l < n1; ++l) t += Binv[i * n1 + l] * Xc[l + n1 * j];
                a[i + n1 * j] = t;
            }
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                double t = 0.0;
                for (int l = 0; l < n1; ++l) t += Binv[j * n1 + l] * a[i + n1 * l];
                b[i + n1 * j] = t;
            }
        lo[c] = b[0]; hi[c] = b[0];
        for (int q = 0; q < V; ++q) {
            if (b[q] < lo[c]) lo[c] = b[q];
            if (b[q] > hi[c]) hi[c] = b[q];
        }
    }
    double marg = 1e-8 * he + 1e-14 * xmax;
    for (int c = 0; c < 2; ++c) {
        m->bbox[4 * e + 2 * c] = lo[c] - marg;
        m->bbox[4 * e + 2 * c + 1] = hi[c] + marg;
    }
    m->h[e] = he;
    free(a); free(b);
}

static int cell_of2(const or2_mesh *m, int a, double x)
{
    double u = (x - m->lo[a]) / m->dx[a];
    int i = (int)floor(u);
    if (i < 0) i = 0;
    if (i > m->nc[a] - 1) i = m->nc[a] - 1;
    return i;
}

static void build_hash2(or2_mesh *m)
{
    int E = m->E;
    for (int a = 0; a < 2; ++a) { m->lo[a] = m->bbox[2 * a]; m->hi[a] = m->bbox[2 * a + 1]; }
    for (int e = 1; e < E; ++e)
        for (int a = 0; a < 2; ++a) {
            if (m->bbox[4 * e + 2 * a] < m->lo[a]) m->lo[a] = m->bbox[4 * e + 2 * a];
            if (m->bbox[4 * e + 2 * a + 1] > m->hi[a]) m->hi[a] = m->bbox[4 * e + 2 * a + 1];
        }
    double ext[2], area = 1.0;
    for (int a = 0; a < 2; ++a) {
        ext[a] = m->hi[a] - m->lo[a];
        if (!(ext[a] > 0.0)) ext[a] = 1e-300;
        area *= ext[a];
    }
    double dens = sqrt((double)E / area);
    for (int a = 0; a < 2; ++a) {
        double n = floor(ext[a] * dens + 0.5);
        if (n < 1.0) n = 1.0;
        if (n > 65536.0) n = 65536.0;
        m->nc[a] = (int)n;
        m->dx[a] = ext[a] / m->nc[a];
    }
    long ncell = (long)m->nc[0] * m->nc[1];
    int *cnt = calloc(ncell + 1, sizeof(int));
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            m->cell_off = malloc(sizeof(int) * (ncell + 1));
            m->cell_off[0] = 0;
            for (long c = 0; c < ncell; ++c) m->cell_off[c + 1] = m->cell_off[c] + cnt[c];
            m->cell_el = malloc(sizeof(int) * (m->cell_off[ncell] + 1));
            memset(cnt, 0, sizeof(int) * ncell);
        }
        for (int e = 0; e < E; ++e) {
            const double *b = m->bbox + 4 * e;
            int i0 = cell_of2(m, 0, b[0]), i1 = cell_of2(m, 0, b[1]);
            int j0 = cell_of2(m, 1, b[2]), j1 = cell_of2(m, 1, b[3]);
            for (int j = j0; j <= j1; ++j)
                for (int i = i0; i <= i1; ++i) {
                    long c = i + (long)m->nc[0] * j;
                    if (pass == 1) m->cell_el[m->cell_off[c] + cnt[c]] = e;
                    cnt[c]++;
                }
        }
    }
    free(cnt);
}

or2_mesh *or2_setup(int E, int N, const double *x, const double *y, double tol,
                    const int *esess, const double *delta)
{
    if (E < 1 || N < 1 || N > OR_MAXN1 - 1) return NULL;
    or2_mesh *m = calloc(1, sizeof(or2_mesh));
    m->E = E; m->N = N; m->n1 = N + 1; m->V = m->n1 * m->n1;
    m->tol = tol;
    m->X[0] = x; m->X[1] = y;
    m->esess = esess; m->delta = delta;
    or_gll(N, m->z, m->w);
    m->bbox = malloc(sizeof(double) * 4 * E);
    m->h = malloc(sizeof(double) * E);
    double Binv[OR_MAXN1 * OR_MAXN1];
    bernstein_inverse(N, m->z, Binv);
#pragma omp parallel for schedule(dynamic, 64)
    for (int e = 0; e < E; ++e) element_bbox2(m, Binv, e);
    build_hash2(m);
    return m;
}

void or2_free(or2_mesh *m)
{
    if (!m) return;
    free(m->bbox); free(m->h); free(m->cell_off); free(m->cell_el); free(m);
}

void or2_get_bbox(const or2_mesh *m, double *bbox, double *h)
{
    memcpy(bbox, m->bbox, sizeof(double) * 4 * m->E);
    memcpy(h, m->h, sizeof(double) * m->E);
}

void or2_map(const or2_mesh *m, int e, const double *r, double *x, double *J)
{
    emap2(m, e, r, x, J);
}

static int in_box2(const double *b, const double *p)
{
    return p[0] >= b[0] && p[0] <= b[1] && p[1] >= b[2] && p[1] <= b[3];
}

int or2_candidates(const or2_mesh *m, const double *p, int psess, int *out, int max)
{
    for (int a = 0; a < 2; ++a)
        if (!(p[a] >= m->lo[a] && p[a] <= m->hi[a])) return 0;
    long c = cell_of2(m, 0, p[0]) + (long)m->nc[0] * cell_of2(m, 1, p[1]);
    int n = 0;
    for (int q = m->cell_off[c]; q < m->cell_off[c + 1]; ++q) {
        int e = m->cell_el[q];
        if (!in_box2(m->bbox + 4 * e, p)) continue;
        if (psess >= 0 && m->esess && m->esess[e] == psess) continue;
        if (n < max) out[n] = e;
        n++;
    }
    return n;
}

static void start_node2(const or2_mesh *m, int e, const double *p, double r[2])
{
    int n1 = m->n1, best = 0;
    double bd = INFINITY;
    for (int q = 0; q < m->V; ++q) {
        double d = 0.0;
        for (int c = 0; c < 2; ++c) {
            double t = elem2(m, c, e)[q] - p[c];
            d += t * t;
        }
        if (d < bd) { bd = d; best = q; }
    }
    r[0] = m->z[best % n1];
    r[1] = m->z[best / n1];
}

static double resid2(const or2_mesh *m, int e, const double *p, const double r[2],
                     double F[2], double J[4])
{
    double x[2];
    emap2(m, e, r, x, J);
    double phi = 0.0;
    for (int c = 0; c < 2; ++c) { F[c] = x[c] - p[c]; phi += F[c] * F[c]; }
    return phi;
}

/* The 3D trust-region rules (constants, active set, radius updates, stops)
 * on [-1,1]^2. */
static int tr_newton2(const or2_mesh *m, int e, const double *p, double r[2],
                      double *phi_out)
{
    double he = m->h[e], stop = resid_stop(m->tol, he);
    double F[2], J[4], D = 1.0;
    double phi = resid2(m, e, p, r, F, J);
    int it = 0;
    while (it < OR_MAXIT) {
        if (phi <= stop) break;
        ++it;
        double g[2];
        for (int d = 0; d < 2; ++d) g[d] = J[d] * F[0] + J[2 + d] * F[1];
        int fr[2], nf = 0;
        for (int d = 0; d < 2; ++d) {
            int held = (r[d] >= 1.0 && g[d] < 0.0) || (r[d] <= -1.0 && g[d] > 0.0);
            if (!held) fr[nf++] = d;
        }
        if (nf == 0) break;
        double dl[2] = {0.0, 0.0};
        int bad;
        if (nf == 2) {
            double A[3][3], b[3];
            for (int i = 0; i < 2; ++i) {
                for (int j = 0; j < 2; ++j) A[i][j] = J[2 * i + j];
                b[i] = -F[i];
            }
            bad = solve_small(2, A, b, dl);
        } else {
            int da = fr[0];
            double a = J[da] * J[da] + J[2 + da] * J[2 + da];
            bad = !(a != 0.0);
            if (!bad) {
                dl[da] = -g[da] / a;
                if (!isfinite(dl[da])) bad = 1;
            }
        }
        if (bad) {
            dl[0] = dl[1] = 0.0;
            for (int a = 0; a < nf; ++a) dl[fr[a]] = -g[fr[a]];
        }
        double nd = fabs(dl[0]) > fabs(dl[1]) ? fabs(dl[0]) : fabs(dl[1]);
        if (!(nd > 0.0) || !isfinite(nd)) break;
        int limited = 0;
        if (nd > D) {
            double sc = D / nd;
            dl[0] *= sc; dl[1] *= sc;
            limited = 1;
        }
        double rn[2], s[2], ns = 0.0;
        for (int d = 0; d < 2; ++d) {
            double v = r[d] + dl[d];
            if (v > 1.0) v = 1.0;
            if (v < -1.0) v = -1.0;
            rn[d] = v;
            s[d] = v - r[d];
            if (fabs(s[d]) > ns) ns = fabs(s[d]);
        }
        if (ns <= 1e-15) break;
        double pred = phi;
        for (int c = 0; c < 2; ++c) {
            double t = F[c] + J[2 * c] * s[0] + J[2 * c + 1] * s[1];
            pred -= t * t;
        }
        if (!(pred > 0.0)) break;
        double Fn[2], Jn[4];
        double phin = resid2(m, e, p, rn, Fn, Jn);
        double rho = (phi - phin) / pred;
        int acc = rho >= 0.01;
        if (acc) {
            for (int d = 0; d < 2; ++d) { r[d] = rn[d]; F[d] = Fn[d]; }
            for (int q = 0; q < 4; ++q) J[q] = Jn[q];
            phi = phin;
        }
        if (rho > 0.75 && limited) { D = 2.0 * D; if (D > 2.0) D = 2.0; }
        else if (rho < 0.25) D = 0.25 * ns;
        if (acc && ns <= 1e-13) break;
    }
    *phi_out = phi;
    return it;
}

int or2_newton(const or2_mesh *m, int e, const double *p, double *r, double *d2)
{
    start_node2(m, e, p, r);
    return tr_newton2(m, e, p, r, d2);
}

int or2_newton_from(const or2_mesh *m, int e, const double *p, double *r, double *d2)
{
    return tr_newton2(m, e, p, r, d2);
}

static void fill_cand2(const or2_mesh *m, cand_t *c, int e, const double *p, const double *r)
{
    c->e = e;
    c->r[0] = r[0]; c->r[1] = r[1]; c->r[2] = 0.0;
    double F[2];
    c->d2 = resid2(m, e, p, c->r, F, NULL);
    c->inside = sqrt(c->d2) <= m->tol * m->h[e];
    c->sess = m->esess ? m->esess[e] : 0;
    c->dl = (m->delta && c->inside) ? interp2(m, m->delta + (size_t)e * m->V, c->r) : 0.0;
}

/* findpts in 2D: pts (x, y interleaved), rst receives (r, s) per point. */
void or2_findpts(const or2_mesh *m, int npts, const double *pts, const int *psess,
                 int *code, int *el, double *rst, double *dist2, long long *stats,
                 int nthreads)
{
    long long tc = 0, ti = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel reduction(+ : tc, ti)
    {
        int *ids = malloc(sizeof(int) * m->E);
        cand_t *cs = malloc(sizeof(cand_t) * m->E);
#pragma omp for schedule(dynamic, 1024)
        for (int p = 0; p < npts; ++p) {
            const double *x = pts + 2 * (size_t)p;
            int nc = or2_candidates(m, x, psess ? psess[p] : -1, ids, m->E);
            for (int q = 0; q < nc; ++q) {
                double r[2], d2;
                ti += or2_newton(m, ids[q], x, r, &d2);
                fill_cand2(m, &cs[q], ids[q], x, r);
            }
            tc += nc;
            select_cands(m->delta != NULL, 2, cs, nc, code + p, el + p, rst + 2 * (size_t)p,
                         dist2 + p);
        }
        free(ids); free(cs);
    }
    if (stats) { stats[0] = tc; stats[1] = ti; }
}

/* Brute force in 2D: all elements (or those whose box holds the point),
 * starts at the closest node, every node (all_nodes) and a g x g grid. */
void or2_brute(const or2_mesh *m, int npts, const double *pts, const int *psess,
               int g, int all_nodes, int only_boxes, int *code, int *el,
               double *rst, double *dist2, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        cand_t *cs = malloc(sizeof(cand_t) * m->E);
#pragma omp for schedule(dynamic, 1)
        for (int p = 0; p < npts; ++p) {
            const double *x = pts + 2 * (size_t)p;
            int nc = 0;
            for (int e = 0; e < m->E; ++e) {
                if (psess && psess[p] >= 0 && m->esess && m->esess[e] == psess[p]) continue;
                if (only_boxes && !in_box2(m->bbox + 4 * e, x)) continue;
                double br[2], bd, r[2], d2;
                or2_newton(m, e, x, r, &d2);
                bd = d2; br[0] = r[0]; br[1] = r[1];
                int nn = all_nodes ? m->V : 0;
                for (int q = 0; q < nn + g * g; ++q) {
                    if (q < nn) {
                        r[0] = m->z[q % m->n1]; r[1] = m->z[q / m->n1];
                    } else {
                        int u = q - nn;
                        r[0] = -1.0 + 2.0 * (u % g) / (g - 1);
                        r[1] = -1.0 + 2.0 * (u / g) / (g - 1);
                    }
                    tr_newton2(m, e, x, r, &d2);
                    if (d2 < bd) { bd = d2; br[0] = r[0]; br[1] = r[1]; }
                }
                fill_cand2(m, &cs[nc], e, x, br);
                nc++;
            }
            select_cands(m->delta != NULL, 2, cs, nc, code + p, el + p, rst + 2 * (size_t)p,
                         dist2 + p);
        }
        free(cs);
    }
}

void or2_eval(const or2_mesh *m, int npts, const int *code, const int *el, const double *rs,
              int nf, const double *const *fields, double *out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1024)
    for (int p = 0; p < npts; ++p) {
        for (int f = 0; f < nf; ++f) {
            double v = NAN;
            if (code[p] != 2 && el[p] >= 0 && el[p] < m->E)
                v = interp2(m, fields[f] + (size_t)el[p] * m->V, rs + 2 * (size_t)p);
            out[(size_t)f * npts + p] = v;
        }
    }
}

/* Number of threads an OpenMP region would use (for reporting). */
int or_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
#else
    (void)nthreads;
    return 1;
#endif
}
