// findpts_setup and handle management: mesh copy, element boxes (Bernstein
// hull), hash grid, workspace.  Section 2.1 of the paper: a hash table finds
// the potential owners of x*, then elementwise bounding boxes filter them.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fp_internal.h"

namespace fp {

// ---------------------------------------------------------------------------
// Host-side basis tables (GLL nodes, barycentric weights, Bernstein inverse).
// ---------------------------------------------------------------------------

// Legendre P_n(x) and P_n'(x) by the three-term recurrence.
static void legendre_pd(int n, double x, double &p, double &dp)
{
    double pm = 1.0, pc = x;  // P_0, P_1
    if (n == 0) { p = 1.0; dp = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double pn = ((2 * k + 1) * x * pc - k * pm) / (k + 1);
        pm = pc;
        pc = pn;
    }
    p = pc;
    // (1 - x^2) P_n' = n (P_{n-1} - x P_n); endpoints are not needed here
    dp = n * (pm - x * pc) / (1.0 - x * x);
}

// GLL nodes: +-1 and the roots of P_N'.  Roots of P_N' are the interior
// extrema of P_N; Newton's method is applied to q(x) = (1 - x^2) P_N'(x),
// whose derivative is -N (N + 1) P_N(x), starting from the Chebyshev-Gauss-
// Lobatto points; nodes are then symmetrised.
static void gll_nodes(int N, double *z)
{
    z[0] = -1.0;
    z[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -std::cos(M_PI * i / N);
        for (int it = 0; it < 60; ++it) {
            double p, dp;
            legendre_pd(N, x, p, dp);
            double q = (1.0 - x * x) * dp;
            double dq = -N * (N + 1.0) * p;
            double step = q / dq;
            x -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        z[i] = x;
    }
    for (int i = 0; i < (N + 1) / 2; ++i) {
        double a = 0.5 * (z[N - i] - z[i]);
        z[i] = -a;
        z[N - i] = a;
    }
    if (N % 2 == 0) z[N / 2] = 0.0;
}

Basis make_basis(int N)
{
    Basis b{};
    gll_nodes(N, b.z);
    for (int i = 0; i <= N; ++i) {
        long double d = 1.0L;
        for (int m = 0; m <= N; ++m)
            if (m != i) d *= (long double)b.z[i] - (long double)b.z[m];
        b.wb[i] = (double)(1.0L / d);
    }
    return b;
}

std::vector<double> node_derivatives(const Basis &b, int N)
{
    const int n = N + 1;
    std::vector<double> D((size_t)n * n, 0.0);
    for (int a = 0; a < n; ++a) {
        long double diag = 0.0L;
        for (int c = 0; c < n; ++c) {
            if (c == a) continue;
            const long double v = ((long double)b.wb[c] / (long double)b.wb[a]) /
                                  ((long double)b.z[a] - (long double)b.z[c]);
            D[(size_t)a * n + c] = (double)v;
            diag -= v;
        }
        D[(size_t)a * n + a] = (double)diag;
    }
    return D;
}

// Inverse of M[i][k] = C(N,k) u_i^k (1-u_i)^(N-k), u_i = (1 + z_i)/2: maps
// nodal values to tensor-Bernstein coefficients.  Gauss-Jordan in long
// double on the host.
std::vector<double> bernstein_to_nodal_inverse(int N, const double *z)
{
    const int n = N + 1;
    std::vector<long double> A(n * 2 * n, 0.0L);
    for (int i = 0; i < n; ++i) {
        long double u = 0.5L * (1.0L + z[i]), v = 1.0L - u;
        long double c = 1.0L;  // C(N, k)
        for (int k = 0; k < n; ++k) {
            if (k > 0) c = c * (N - k + 1) / k;
            A[i * 2 * n + k] = c * std::pow(u, (long double)k) * std::pow(v, (long double)(N - k));
        }
        A[i * 2 * n + n + i] = 1.0L;
    }
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (std::fabs(A[i * 2 * n + c]) > std::fabs(A[piv * 2 * n + c])) piv = i;
        if (piv != c)
            for (int k = 0; k < 2 * n; ++k) std::swap(A[c * 2 * n + k], A[piv * 2 * n + k]);
        long double d = A[c * 2 * n + c];
        for (int k = 0; k < 2 * n; ++k) A[c * 2 * n + k] /= d;
        for (int i = 0; i < n; ++i) {
            if (i == c) continue;
            long double f = A[i * 2 * n + c];
            if (f == 0.0L) continue;
            for (int k = 0; k < 2 * n; ++k) A[i * 2 * n + k] -= f * A[c * 2 * n + k];
        }
    }
    std::vector<double> out(n * n);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) out[i * n + k] = (double)A[i * 2 * n + n + k];
    return out;
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------

// Copy x, y, z (each E*V) into the element-blocked E x 3 x V layout (and the
// binary32 copy), flagging non-finite values.
__global__ __launch_bounds__(256) void k_pack(const double *__restrict__ x,
                                              const double *__restrict__ y,
                                              const double *__restrict__ z, long long EV,
                                              int V, double *__restrict__ geom,
                                              float *__restrict__ geom32,
                                              int *__restrict__ bad)
{
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    int flag = 0;
    for (; t < EV; t += stride) {
        long long e = t / V, q = t - e * V;
        double v0 = x[t], v1 = y[t], v2 = z[t];
        flag |= !(isfinite(v0) && isfinite(v1) && isfinite(v2));
        double *g = geom + e * 3 * V + q;
        g[0] = v0;
        g[V] = v1;
        g[2 * V] = v2;
        if (geom32) {
            float *g32 = geom32 + e * 3 * V + q;
            g32[0] = (float)v0;
            g32[V] = (float)v1;
            g32[2 * V] = (float)v2;
        }
    }
    if (flag) atomicOr(bad, 1);
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// One wave per element: Bernstein coefficients of each coordinate (the
// inverse nodal-Bernstein matrix applied along r, s, t in LDS), their min and
// max, the node extents (h_e) and the margin 1e-8 h_e + 1e-14 max|x|.
__global__ __launch_bounds__(kWave) void k_bbox(const double *__restrict__ geom, int n1,
                                                const double *__restrict__ binv,
                                                double *__restrict__ bbox,
                                                double *__restrict__ esize)
{
    extern __shared__ double sh[];
    const int V = n1 * n1 * n1;
    double *A = sh, *B = sh + V;
    __shared__ double Bi[kMaxN1 * kMaxN1];
    const int e = blockIdx.x, t = threadIdx.x;
    for (int q = t; q < n1 * n1; q += kWave) Bi[q] = binv[q];
    double lo[3], hi[3], he = 0.0, amax = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double *X = geom + ((long long)e * 3 + c) * V;
        double mn = INFINITY, mx = -INFINITY;
        for (int q = t; q < V; q += kWave) {
            double v = X[q];
            A[q] = v;
            mn = fmin(mn, v);
            mx = fmax(mx, v);
            amax = fmax(amax, fabs(v));
        }
        mn = wave_min(mn);
        mx = wave_max(mx);
        he = fmax(he, mx - mn);
        __syncthreads();
        for (int q = t; q < V; q += kWave) {  // along r
            int i = q % n1, rest = q - i;
            double s = 0.0;
            for (int l = 0; l < n1; ++l) s = fma(Bi[i * n1 + l], A[rest + l], s);
            B[q] = s;
        }
        __syncthreads();
        for (int q = t; q < V; q += kWave) {  // along s
            int i = q % n1, j = (q / n1) % n1, k = q / (n1 * n1);
            double s = 0.0;
            for (int l = 0; l < n1; ++l) s = fma(Bi[j * n1 + l], B[i + n1 * (l + n1 * k)], s);
            A[q] = s;
        }
        __syncthreads();
        double cmn = INFINITY, cmx = -INFINITY;
        for (int q = t; q < V; q += kWave) {  // along t
            int ij = q % (n1 * n1), k = q / (n1 * n1);
            double s = 0.0;
            for (int l = 0; l < n1; ++l) s = fma(Bi[k * n1 + l], A[ij + n1 * n1 * l], s);
            cmn = fmin(cmn, s);
            cmx = fmax(cmx, s);
        }
        lo[c] = wave_min(cmn);
        hi[c] = wave_max(cmx);
        __syncthreads();
    }
    amax = wave_max(amax);
    if (t == 0) {
        const double m = 1e-8 * he + 1e-14 * amax;
        for (int c = 0; c < 3; ++c) {
            bbox[6 * e + 2 * c] = lo[c] - m;
            bbox[6 * e + 2 * c + 1] = hi[c] + m;
        }
        esize[e] = he;
    }
}

// Oriented box of each element (one wave per element).  Frame: Gram-Schmidt
// of the mean edge vectors along r, s, t (identity if they are degenerate).
// The rotated coordinates u = Q (x - centre) are linear in x, so the
// Bernstein coefficients of their nodal values bound the element in that
// frame exactly as the axis-aligned box does; any Q (orthonormal or not)
// keeps this rigorous.  Margin: the axis-aligned box's, or tol h_e if larger.  The record
// is binary32 (72 bytes, half the binary64 one, for the candidate lookup's
// memory traffic): Q and the centre are rounded first and the bounds are
// computed for the rounded frame, then rounded outward.
__global__ __launch_bounds__(kWave) void k_obb(const double *__restrict__ geom, int n1,
                                               const double *__restrict__ binv,
                                               const double *__restrict__ bbox,
                                               const double *__restrict__ esize,
                                               double tol, float *__restrict__ obb)
{
    extern __shared__ double sh[];
    const int V = n1 * n1 * n1;
    double *A = sh, *B = sh + V;
    __shared__ double Bi[kMaxN1 * kMaxN1];
    const int e = blockIdx.x, t = threadIdx.x;
    for (int q = t; q < n1 * n1; q += kWave) Bi[q] = binv[q];
    const double *X = geom + (long long)e * 3 * V;
    // mean edge vectors (lane-parallel sums over the n1^2 node lines)
    double ed[3][3];
    for (int c = 0; c < 3; ++c) {
        double sr = 0.0, ss = 0.0, st = 0.0;
        for (int q = t; q < n1 * n1; q += kWave) {
            const int a = q % n1, b = q / n1;
            const double *Xc = X + c * V;
            sr += Xc[n1 - 1 + n1 * (a + n1 * b)] - Xc[n1 * (a + n1 * b)];
            ss += Xc[a + n1 * (n1 - 1 + n1 * b)] - Xc[a + n1 * n1 * b];
            st += Xc[a + n1 * (b + n1 * (n1 - 1))] - Xc[a + n1 * b];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            sr += __shfl_xor(sr, o, kWave);
            ss += __shfl_xor(ss, o, kWave);
            st += __shfl_xor(st, o, kWave);
        }
        ed[0][c] = sr;
        ed[1][c] = ss;
        ed[2][c] = st;
    }
    double Q[3][3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        double v[3] = {ed[a][0], ed[a][1], ed[a][2]};
        for (int b = 0; b < a; ++b) {
            const double d = v[0] * Q[b][0] + v[1] * Q[b][1] + v[2] * Q[b][2];
            for (int c = 0; c < 3; ++c) v[c] -= d * Q[b][c];
        }
        const double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        const double ne = sqrt(ed[a][0] * ed[a][0] + ed[a][1] * ed[a][1] + ed[a][2] * ed[a][2]);
        ok = ok && isfinite(nv) && nv > 1e-6 * ne && ne > 0.0;
        for (int c = 0; c < 3; ++c) Q[a][c] = ok ? v[c] / nv : 0.0;
    }
    if (!ok)
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) Q[a][c] = (a == c) ? 1.0 : 0.0;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) Q[a][c] = (double)(float)Q[a][c];
    const double *bb = bbox + 6 * (long long)e;
    const double ctr[3] = {(double)(float)(0.5 * (bb[0] + bb[1])),
                           (double)(float)(0.5 * (bb[2] + bb[3])),
                           (double)(float)(0.5 * (bb[4] + bb[5]))};
    double lo[3], hi[3], amax = 0.0;
    for (int a = 0; a < 3; ++a) {
        for (int q = t; q < V; q += kWave) {
            const double u = Q[a][0] * (X[q] - ctr[0]) + Q[a][1] * (X[V + q] - ctr[1]) +
                             Q[a][2] * (X[2 * V + q] - ctr[2]);
            A[q] = u;
            amax = fmax(amax, fabs(u));
        }
        __syncthreads();
        for (int q = t; q < V; q += kWave) {  // along r
            int i = q % n1, rest = q - i;
            double s = 0.0;
            for (int l = 0; l < n1; ++l) s = fma(Bi[i * n1 + l], A[rest + l], s);
            B[q] = s;
        }
        __syncthreads();
        for (int q = t; q < V; q += kWave) {  // along s
            int i = q % n1, j = (q / n1) % n1, k = q / (n1 * n1);
            double s = 0.0;
            for (int l = 0; l < n1; ++l) s = fma(Bi[j * n1 + l], B[i + n1 * (l + n1 * k)], s);
            A[q] = s;
        }
        __syncthreads();
        double cmn = INFINITY, cmx = -INFINITY;
        for (int q = t; q < V; q += kWave) {  // along t
            int ij = q % (n1 * n1), k = q / (n1 * n1);
            double s = 0.0;
            for (int l = 0; l < n1; ++l) s = fma(Bi[k * n1 + l], A[ij + n1 * n1 * l], s);
            cmn = fmin(cmn, s);
            cmx = fmax(cmx, s);
        }
        lo[a] = wave_min(cmn);
        hi[a] = wave_max(cmx);
        __syncthreads();
    }
    amax = wave_max(amax);
    if (t == 0) {
        const double cabs = fmax(fabs(ctr[0]), fmax(fabs(ctr[1]), fabs(ctr[2])));
        // the axis-aligned box's margin, or the inside tolerance when that is
        // larger (a point within tol h_e of the element may be inside; the
        // rounded frame's rows have norm 1 to within 1e-7)
        const double m = fmax(1e-8, (1.0 + 1e-6) * tol) * esize[e] + 1e-14 * (amax + cabs);
        float *o = obb + 18 * (long long)e;
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) o[3 * a + c] = (float)Q[a][c];  // exact
        for (int c = 0; c < 3; ++c) {
            o[9 + c] = (float)ctr[c];  // exact
            const double l = lo[c] - m, u = hi[c] + m;
            float lf = (float)l, uf = (float)u;
            if ((double)lf > l) lf = nextafterf(lf, -INFINITY);
            if ((double)uf < u) uf = nextafterf(uf, INFINITY);
            o[12 + c] = lf;
            o[15 + c] = uf;
        }
    }
}

// Union of the element boxes (one block).
__global__ __launch_bounds__(256) void k_gbox(const double *__restrict__ bbox, int E,
                                              double *__restrict__ out)
{
    __shared__ double red[6][256 / kWave];
    double v[6] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (int e = threadIdx.x; e < E; e += blockDim.x)
        for (int a = 0; a < 3; ++a) {
            v[2 * a] = fmin(v[2 * a], bbox[6 * e + 2 * a]);
            v[2 * a + 1] = fmax(v[2 * a + 1], bbox[6 * e + 2 * a + 1]);
        }
    const int w = threadIdx.x / kWave;
    for (int a = 0; a < 3; ++a) {
        double mn = wave_min(v[2 * a]), mx = wave_max(v[2 * a + 1]);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            red[2 * a][w] = mn;
            red[2 * a + 1][w] = mx;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) {
            double mn = red[2 * a][0], mx = red[2 * a + 1][0];
            for (int q = 1; q < (int)(blockDim.x / kWave); ++q) {
                mn = fmin(mn, red[2 * a][q]);
                mx = fmax(mx, red[2 * a + 1][q]);
            }
            out[2 * a] = mn;
            out[2 * a + 1] = mx;
        }
    }
}

__device__ __forceinline__ int cell_axis(const Grid &g, int a, double x)
{
    double u = (x - g.lo[a]) * g.inv[a];
    int i = (int)floor(u);
    return i < 0 ? 0 : (i >= g.nc[a] ? g.nc[a] - 1 : i);
}

// mode 0: count entries per cell; mode 1: write element ids.
__global__ __launch_bounds__(256) void k_hash_pass(const double *__restrict__ bbox, int E,
                                                   Grid g, int mode, int *__restrict__ cnt,
                                                   const int *__restrict__ off,
                                                   int *__restrict__ cell_el)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const double *b = bbox + 6 * e;
    int i0 = cell_axis(g, 0, b[0]), i1 = cell_axis(g, 0, b[1]);
    int j0 = cell_axis(g, 1, b[2]), j1 = cell_axis(g, 1, b[3]);
    int k0 = cell_axis(g, 2, b[4]), k1 = cell_axis(g, 2, b[5]);
    for (int k = k0; k <= k1; ++k)
        for (int j = j0; j <= j1; ++j)
            for (int i = i0; i <= i1; ++i) {
                long long c = i + (long long)g.nc[0] * (j + (long long)g.nc[1] * k);
                int pos = atomicAdd(&cnt[c], 1);
                if (mode == 1) cell_el[off[c] + pos] = e;
            }
}

// Sort each cell list ascending (insertion sort; lists are short) and find
// the longest list.
__global__ __launch_bounds__(256) void k_hash_sort(const int *__restrict__ off,
                                                   int *__restrict__ cell_el, long long ncell,
                                                   int *__restrict__ maxlen)
{
    long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int b = off[c], n = off[c + 1] - b;
    int *L = cell_el + b;
    for (int i = 1; i < n; ++i) {
        int v = L[i], j = i - 1;
        while (j >= 0 && L[j] > v) {
            L[j + 1] = L[j];
            --j;
        }
        L[j + 1] = v;
    }
    atomicMax(maxlen, n);
}

// One 128-byte record per element for the candidate lookup: the binary64
// axis-aligned box and the binary32 oriented box share a cache line.
__global__ __launch_bounds__(256) void k_erec(const double *__restrict__ bbox,
                                              const float *__restrict__ obb, int E,
                                              double *__restrict__ erec)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double *r = erec + 16 * (long long)e;
    for (int i = 0; i < 6; ++i) r[i] = bbox[6 * (long long)e + i];
    float *o = (float *)(r + 6);
    for (int i = 0; i < 18; ++i) o[i] = obb[18 * (long long)e + i];
    r[15] = 0.0;
}

// Per cell-list entry, the element's box in binary32 rounded outward (never
// smaller than the binary64 box) with the element id in the spare slot: the
// candidate lookup streams a cell's entries contiguously and tests the exact
// binary64 box only for the survivors.
__global__ __launch_bounds__(256) void k_cellbox(const double *__restrict__ bbox,
                                                 const int *__restrict__ cell_el, long long nnz,
                                                 float4 *__restrict__ cell_box)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnz) return;
    const int e = cell_el[q];
    const double *b = bbox + 6 * (long long)e;
    float lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float l = (float)b[2 * a], u = (float)b[2 * a + 1];
        if ((double)l > b[2 * a]) l = nextafterf(l, -INFINITY);
        if ((double)u < b[2 * a + 1]) u = nextafterf(u, INFINITY);
        lo[a] = l;
        hi[a] = u;
    }
    cell_box[2 * q] = make_float4(lo[0], lo[1], lo[2], __int_as_float(e));
    cell_box[2 * q + 1] = make_float4(hi[0], hi[1], hi[2], 0.0f);
}

}  // namespace fp

// ---------------------------------------------------------------------------
// Workspace layout.
// ---------------------------------------------------------------------------
namespace fp {

namespace {
struct Layout {
    size_t off = 0;
    char *base = nullptr;
    template <class T>
    T *take(size_t count)
    {
        T *p = base ? (T *)(base + off) : nullptr;
        off += ((sizeof(T) * (count ? count : 1) + 255) / 256) * 256;
        return p;
    }
};

void lay_out(Layout &L, Work &w, int E, int MC, int M, bool delta)
{
    const size_t m = (size_t)M, mc = (size_t)MC, e1 = (size_t)E + 1;
    w.M = M;
    w.MC = MC;
    w.E = E;
    w.ncand = L.take<int>(m);
    w.cand_el = L.take<int>(m * mc);
    w.cand_pos = L.take<int>(m * mc);
    w.elem_cnt = L.take<int>(e1);
    w.elem_off = L.take<int>(e1);
    w.order = L.take<int>(m * mc);
    w.res = L.take<double>(m * mc * 4);
    w.res_dl = delta ? L.take<double>(m * mc) : nullptr;
    w.res_in = L.take<int>(m * mc);
    w.redo = L.take<int>(m);
    w.gate = L.take<int>(1);
    w.scan_tmp = L.take<int>((size_t)scan_tmp_size((long long)E + 1));
    w.cand_part = L.take<unsigned>((m + 255) / 256);
    w.iter_part = L.take<unsigned>((size_t)unit_grid(E, M, kUnitMin));
    w.ev_cnt = L.take<int>(e1);
    w.ev_off = L.take<int>(e1);
    w.ev_pos = L.take<int>(m);
    w.ev_order = L.take<int>(m);
    w.ev_slot = L.take<int>(m);
    w.ev_sink = L.take<double>(kEvSink);
}
}  // namespace

size_t work_bytes(int E, int MC, int M, bool delta)
{
    Layout L;
    Work w;
    lay_out(L, w, E, MC, M, delta);
    return L.off;
}

void work_carve(Work &w, char *base, int E, int MC, int M, bool delta)
{
    Layout L;
    L.base = base;
    lay_out(L, w, E, MC, M, delta);
}

}  // namespace fp

// ---------------------------------------------------------------------------
// Handle lifetime.
// ---------------------------------------------------------------------------
using namespace fp;

static void release(fp_handle *h)
{
    void *ptrs[] = {h->d_basis, h->d_basis32, h->geom, h->geom32, h->esize, h->bbox, h->obb,
                    h->esess, h->delta, h->cell_off, h->cell_cnt, h->cell_el, h->cell_box,
                    h->work_mem, h->scan_tmp, h->stats, h->d_flag, h->d_g, h->d_binv,
                    h->d_dnode, h->erec};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &t : h->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto ev : h->event_pool) (void)hipEventDestroy(ev);
    delete h;
}

template <class T>
static hipError_t dalloc(fp_handle *h, T **p, size_t count)
{
    size_t b = sizeof(T) * (count ? count : 1);
    hipError_t e = hipMalloc((void **)p, b);
    if (e == hipSuccess) h->bytes += b;
    return e;
}

#define FP_HIP_H(call)                              \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) {                     \
            int rc_ = fp::hip_fail(e_, #call);      \
            release(h);                             \
            return rc_;                             \
        }                                           \
    } while (0)

// Geometry products of the current node coordinates: packed copies, element
// boxes and sizes, oriented boxes, hash grid (with the per-entry binary32
// boxes) and the longest cell list.  Device arrays keep their allocation when
// large enough (an update of a moving mesh allocates only when its hash needs
// more room than before).  Synchronises `s` three times (global box, entry
// count, longest list).
static int build_geometry(fp_handle *h, const double *x, const double *y, const double *z,
                          hipStream_t s, const char *who)
{
    const int E = h->E;
    const long long V = h->V, EV = (long long)E * V;
    const int n1 = h->n1;
    FP_HIP(hipMemsetAsync(h->d_flag, 0, sizeof(int), s));
    {
        long long blocks = std::min<long long>((EV + 255) / 256, 256LL * 64);
        k_pack<<<(int)blocks, 256, 0, s>>>(x, y, z, EV, (int)V, h->geom, h->geom32, h->d_flag);
        FP_HIP(hipGetLastError());
    }
    k_bbox<<<E, kWave, 2 * V * sizeof(double), s>>>(h->geom, n1, h->d_binv, h->bbox, h->esize);
    FP_HIP(hipGetLastError());
    k_obb<<<E, kWave, 2 * V * sizeof(double), s>>>(h->geom, n1, h->d_binv, h->bbox, h->esize,
                                                    h->tol, h->obb);
    FP_HIP(hipGetLastError());
    k_erec<<<(E + 255) / 256, 256, 0, s>>>(h->bbox, h->obb, E, h->erec);
    FP_HIP(hipGetLastError());
    k_gbox<<<1, 256, 0, s>>>(h->bbox, E, h->d_g);
    FP_HIP(hipGetLastError());
    double gb[6];
    int bad = 0;
    FP_HIP(hipMemcpyAsync(gb, h->d_g, sizeof gb, hipMemcpyDeviceToHost, s));
    FP_HIP(hipMemcpyAsync(&bad, h->d_flag, sizeof bad, hipMemcpyDeviceToHost, s));
    FP_HIP(hipStreamSynchronize(s));
    if (bad) {
        set_error(std::string(who) + ": non-finite node coordinates");
        return FP_EINVAL;
    }

    // hash grid: about 8 E cells (two per element and axis, so each cell
    // lists few elements), cell aspect following the extents
    Grid g{};
    double ext[3], vol = 1.0;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = gb[2 * a];
        g.hi[a] = gb[2 * a + 1];
        ext[a] = g.hi[a] - g.lo[a];
        if (!(ext[a] > 0.0)) ext[a] = 1e-300;
        vol *= ext[a];
    }
    const double dens = std::cbrt(8.0 * (double)E / vol);
    for (int a = 0; a < 3; ++a) {
        double n = std::floor(ext[a] * dens + 0.5);
        n = std::min(std::max(n, 1.0), 1024.0);
        g.nc[a] = (int)n;
        g.inv[a] = g.nc[a] / ext[a];
    }
    h->grid = g;
    h->ncell = (long long)g.nc[0] * g.nc[1] * g.nc[2];
    if (h->ncell + 1 > h->cell_cap) {
        (void)hipFree(h->cell_off);
        (void)hipFree(h->cell_cnt);
        (void)hipFree(h->scan_tmp);
        h->bytes -= sizeof(int) * (2 * (size_t)h->cell_cap + (size_t)h->scan_tmp_n);
        h->cell_off = h->cell_cnt = h->scan_tmp = nullptr;
        h->cell_cap = h->ncell + 1;
        FP_HIP(dalloc(h, &h->cell_off, h->cell_cap));
        FP_HIP(dalloc(h, &h->cell_cnt, h->cell_cap));
        h->scan_tmp_n = std::max(scan_tmp_size(h->ncell), scan_tmp_size((long long)E + 1));
        FP_HIP(dalloc(h, &h->scan_tmp, h->scan_tmp_n));
    }
    int *cnt = h->cell_cnt;
    FP_HIP(fill_int(cnt, 0, h->ncell + 1, s));
    const int eb = (E + 255) / 256;
    k_hash_pass<<<eb, 256, 0, s>>>(h->bbox, E, g, 0, cnt, nullptr, nullptr);
    FP_HIP(hipGetLastError());
    FP_HIP(scan_exclusive(cnt, h->cell_off, (int)h->ncell, h->scan_tmp, s));
    int nnz = 0;
    FP_HIP(hipMemcpyAsync(&nnz, h->cell_off + h->ncell, sizeof(int), hipMemcpyDeviceToHost, s));
    FP_HIP(hipStreamSynchronize(s));
    h->nnz = nnz;
    if (nnz > h->nnz_cap || !h->cell_el) {
        (void)hipFree(h->cell_el);
        (void)hipFree(h->cell_box);
        h->bytes -= (sizeof(int) + 2 * sizeof(float4)) * (size_t)h->nnz_cap;
        h->cell_el = nullptr;
        h->cell_box = nullptr;
        h->nnz_cap = nnz;
        FP_HIP(dalloc(h, &h->cell_el, (size_t)nnz));
        FP_HIP(dalloc(h, &h->cell_box, 2 * (size_t)nnz));
    }
    FP_HIP(fill_int(cnt, 0, h->ncell, s));
    k_hash_pass<<<eb, 256, 0, s>>>(h->bbox, E, g, 1, cnt, h->cell_off, h->cell_el);
    FP_HIP(hipGetLastError());
    FP_HIP(hipMemsetAsync(h->d_flag, 0, sizeof(int), s));
    k_hash_sort<<<(int)((h->ncell + 255) / 256), 256, 0, s>>>(h->cell_off, h->cell_el, h->ncell,
                                                              h->d_flag);
    FP_HIP(hipGetLastError());
    int maxlen = 0;
    FP_HIP(hipMemcpyAsync(&maxlen, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    FP_HIP(hipStreamSynchronize(s));
    h->max_cell = maxlen;
    if (nnz > 0) {
        k_cellbox<<<(int)((nnz + 255) / 256), 256, 0, s>>>(h->bbox, h->cell_el, nnz, h->cell_box);
        FP_HIP(hipGetLastError());
    }
    h->MC = std::max(1, maxlen);
    return FP_OK;
}

// The handle's own workspace, (re)carved when the longest cell list outgrew
// it.  A quarter of headroom on the candidate slots lets a moving mesh whose
// longest list changes by a little keep its workspace (a new allocation is
// also touched for the first time by the next call, which costs tens of ms
// for a workspace of a gigabyte).
static int ensure_workspace(fp_handle *h, const char *who)
{
    if (h->work_mem && h->MC <= h->work.MC) return FP_OK;
    int mc_cap = h->MC + (h->MC + 3) / 4;
    if ((double)h->max_points * (double)mc_cap >= 2147483647.0) mc_cap = h->MC;
    if ((double)h->max_points * (double)mc_cap >= 2147483647.0) {
        set_error(std::string(who) +
                  ": max_points x longest cell list exceeds 2^31; lower max_points");
        return FP_ERANGE;
    }
    if (h->work_mem) {
        FP_HIP(hipDeviceSynchronize());  // calls in flight may still use it
        (void)hipFree(h->work_mem);
        h->bytes -= h->work_bytes;
        h->work_mem = nullptr;
    }
    h->work_bytes = work_bytes(h->E, mc_cap, h->max_points, h->delta != nullptr);
    FP_HIP(hipMalloc(&h->work_mem, h->work_bytes));
    h->bytes += h->work_bytes;
    work_carve(h->work, (char *)h->work_mem, h->E, mc_cap, h->max_points, h->delta != nullptr);
    return FP_OK;
}

extern "C" int findpts_setup(fp_handle **out, const double *x, const double *y,
                             const double *z, int E, int N, double tol,
                             const int *elem_session, const double *delta,
                             int max_points, int precision, void *stream)
{
    if (!out || !x || !y || !z) {
        set_error("findpts_setup: NULL argument");
        return FP_EINVAL;
    }
    *out = nullptr;
    if (N < 1 || N > kMaxN1 - 1) {
        set_error("findpts_setup: N must be in [1, 15]");
        return FP_ERANGE;
    }
    if (E < 1 || max_points < 1 || !(tol > 0.0 && tol < 1.0) ||
        (precision != FP_PREC_FP64 && precision != FP_PREC_MIXED)) {
        set_error("findpts_setup: need E >= 1, max_points >= 1, 0 < tol < 1, known precision");
        return FP_EINVAL;
    }
    const long long n1 = N + 1, V = n1 * n1 * n1;
    if ((long long)E * V * 3 > (1LL << 40)) {
        set_error("findpts_setup: mesh too large");
        return FP_ERANGE;
    }
    hipStream_t s = (hipStream_t)stream;
    fp_handle *h = new fp_handle();
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        set_error("findpts_setup: no HIP device");
        return FP_EHIP;
    }
    {
        // resolve this device's interpolation scratch array at set-up, so
        // that findpts_eval_noalloc never resolves it inside a capture
        char *sp = nullptr;
        const int rc = scratch_ptr(h->device, &sp);
        if (rc != FP_OK) {
            delete h;
            return rc;
        }
    }
    h->E = E;
    h->N = N;
    h->n1 = (int)n1;
    h->V = (int)V;
    h->tol = tol;
    h->precision = precision;
    h->max_points = max_points;
    h->basis = make_basis(N);
    for (int i = 0; i < kMaxN1; ++i) {
        h->basis32.z[i] = (float)h->basis.z[i];
        h->basis32.wb[i] = (float)h->basis.wb[i];
    }
    const long long EV = (long long)E * V;

    // mesh-size arrays (kept for the handle's lifetime)
    FP_HIP_H(dalloc(h, &h->geom, 3 * EV));
    FP_HIP_H(dalloc(h, &h->geom32, 3 * EV));  // kept for either precision
    FP_HIP_H(dalloc(h, &h->esize, E));
    FP_HIP_H(dalloc(h, &h->bbox, 6 * (size_t)E));
    FP_HIP_H(dalloc(h, &h->obb, 18 * (size_t)E));
    FP_HIP_H(dalloc(h, &h->erec, 16 * (size_t)E));
    FP_HIP_H(dalloc(h, &h->stats, kStats));
    FP_HIP_H(dalloc(h, &h->d_basis, 2 * kMaxN1));
    FP_HIP_H(dalloc(h, &h->d_basis32, 2 * kMaxN1));
    FP_HIP_H(dalloc(h, &h->d_flag, 1));
    FP_HIP_H(dalloc(h, &h->d_g, 6));
    FP_HIP_H(dalloc(h, &h->d_binv, (size_t)(n1 * n1)));
    FP_HIP_H(dalloc(h, &h->d_dnode, (size_t)(n1 * n1)));
    FP_HIP_H(hipMemcpyAsync(h->d_basis, &h->basis, sizeof(Basis), hipMemcpyHostToDevice, s));
    FP_HIP_H(hipMemcpyAsync(h->d_basis32, &h->basis32, sizeof(Basis32), hipMemcpyHostToDevice, s));
    FP_HIP_H(hipMemsetAsync(h->stats, 0, kStats * sizeof(unsigned long long), s));
    {
        const std::vector<double> binv = bernstein_to_nodal_inverse(N, h->basis.z);
        const std::vector<double> dnode = node_derivatives(h->basis, N);
        FP_HIP_H(hipMemcpyAsync(h->d_binv, binv.data(), sizeof(double) * n1 * n1,
                                hipMemcpyHostToDevice, s));
        FP_HIP_H(hipMemcpyAsync(h->d_dnode, dnode.data(), sizeof(double) * n1 * n1,
                                hipMemcpyHostToDevice, s));
        FP_HIP_H(hipStreamSynchronize(s));  // the host vectors go out of scope
    }
    if (elem_session) {
        FP_HIP_H(dalloc(h, &h->esess, E));
        FP_HIP_H(hipMemcpyAsync(h->esess, elem_session, sizeof(int) * E,
                                hipMemcpyDeviceToDevice, s));
    }
    if (delta) {
        FP_HIP_H(dalloc(h, &h->delta, EV));
        FP_HIP_H(hipMemcpyAsync(h->delta, delta, sizeof(double) * EV,
                                hipMemcpyDeviceToDevice, s));
    }
    int rc = build_geometry(h, x, y, z, s, "findpts_setup");
    if (rc == FP_OK) rc = ensure_workspace(h, "findpts_setup");
    if (rc != FP_OK) {
        release(h);
        return rc;
    }
    FP_HIP_H(hipStreamSynchronize(s));
    *out = h;
    return FP_OK;
}

extern "C" int findpts_update(fp_handle *h, const double *x, const double *y, const double *z,
                              const double *delta, void *stream)
{
    if (!h || !x || !y || !z) {
        set_error("findpts_update: NULL argument");
        return FP_EINVAL;
    }
    if (delta && !h->delta) {
        set_error("findpts_update: the handle was set up without a distance field");
        return FP_ESTATE;
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    FP_HIP(hipGetDevice(&dev));
    if (dev != h->device) FP_HIP(hipSetDevice(h->device));
    if (delta)
        FP_HIP(hipMemcpyAsync(h->delta, delta, sizeof(double) * (size_t)h->E * h->V,
                              hipMemcpyDeviceToDevice, s));
    int rc = build_geometry(h, x, y, z, s, "findpts_update");
    if (rc == FP_OK) rc = ensure_workspace(h, "findpts_update");
    return rc;
}

extern "C" int findpts_free(fp_handle *h)
{
    if (!h) return FP_OK;
    (void)hipDeviceSynchronize();
    release(h);
    return FP_OK;
}

extern "C" int findpts_set_precision(fp_handle *h, int precision)
{
    if (!h || (precision != FP_PREC_FP64 && precision != FP_PREC_MIXED)) {
        set_error("findpts_set_precision: bad handle or precision");
        return FP_EINVAL;
    }
    h->precision = precision;
    return FP_OK;
}

extern "C" int findpts_stats(fp_handle *h, long long *h_counts, int reset)
{
    if (!h || !h_counts) {
        set_error("findpts_stats: NULL argument");
        return FP_EINVAL;
    }
    unsigned long long v[kStats];
    FP_HIP(hipDeviceSynchronize());
    FP_HIP(hipMemcpy(v, h->stats, sizeof v, hipMemcpyDeviceToHost));
    for (int i = 0; i < kStats; ++i) h_counts[i] = (long long)v[i];
    if (reset) FP_HIP(hipMemset(h->stats, 0, sizeof v));
    return FP_OK;
}

extern "C" int findpts_get_bbox(fp_handle *h, double *h_bbox, double *h_size)
{
    if (!h || !h_bbox || !h_size) {
        set_error("findpts_get_bbox: NULL argument");
        return FP_EINVAL;
    }
    FP_HIP(hipDeviceSynchronize());
    FP_HIP(hipMemcpy(h_bbox, h->bbox, sizeof(double) * 6 * h->E, hipMemcpyDeviceToHost));
    FP_HIP(hipMemcpy(h_size, h->esize, sizeof(double) * h->E, hipMemcpyDeviceToHost));
    return FP_OK;
}

extern "C" int findpts_get_hash(fp_handle *h, int *h_nc, double *h_lo, double *h_dx,
                                long long *h_meta)
{
    if (!h || !h_nc || !h_lo || !h_dx || !h_meta) {
        set_error("findpts_get_hash: NULL argument");
        return FP_EINVAL;
    }
    for (int a = 0; a < 3; ++a) {
        h_nc[a] = h->grid.nc[a];
        h_lo[a] = h->grid.lo[a];
        h_dx[a] = 1.0 / h->grid.inv[a];
    }
    h_meta[0] = h->ncell;
    h_meta[1] = h->nnz;
    h_meta[2] = h->max_cell;
    return FP_OK;
}

extern "C" int findpts_get_cells(fp_handle *h, int *h_cell_off, int *h_cell_el)
{
    if (!h || !h_cell_off || !h_cell_el) {
        set_error("findpts_get_cells: NULL argument");
        return FP_EINVAL;
    }
    FP_HIP(hipDeviceSynchronize());
    FP_HIP(hipMemcpy(h_cell_off, h->cell_off, sizeof(int) * (h->ncell + 1),
                     hipMemcpyDeviceToHost));
    FP_HIP(hipMemcpy(h_cell_el, h->cell_el, sizeof(int) * (h->nnz ? h->nnz : 0),
                     hipMemcpyDeviceToHost));
    return FP_OK;
}

extern "C" int findpts_footprint(const fp_handle *h, size_t *h_bytes)
{
    if (!h || !h_bytes) {
        set_error("findpts_footprint: NULL argument");
        return FP_EINVAL;
    }
    *h_bytes = h->bytes;
    return FP_OK;
}

// ---------------------------------------------------------------------------
// Timing with events on the call's stream.
// ---------------------------------------------------------------------------
namespace fp {
hipEvent_t pool_event(fp_handle *h)
{
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace fp

extern "C" int findpts_timing(fp_handle *h, int enable)
{
    if (!h) {
        set_error("findpts_timing: NULL handle");
        return FP_EINVAL;
    }
    h->timing = enable != 0;
    return FP_OK;
}

extern "C" int findpts_timing_read(fp_handle *h, double *h_ms, long long *h_n)
{
    if (!h || !h_ms || !h_n) {
        set_error("findpts_timing_read: NULL argument");
        return FP_EINVAL;
    }
    for (int i = 0; i < kTimedPhases; ++i) {
        h_ms[i] = 0.0;
        h_n[i] = 0;
    }
    for (auto &t : h->timed) {
        FP_HIP(hipEventSynchronize(t.b));
        float ms = 0.0f;
        FP_HIP(hipEventElapsedTime(&ms, t.a, t.b));
        if (t.phase >= 0 && t.phase < kTimedPhases) {
            h_ms[t.phase] += ms;
            h_n[t.phase] += 1;
        }
        h->event_pool.push_back(t.a);
        h->event_pool.push_back(t.b);
    }
    h->timed.clear();
    return FP_OK;
}
