// Interface data around findpts_eval: the mass-flux correction of the
// interpolated boundary velocity (Section 2.2, Eqs. 1-3) and the m-th order
// time extrapolation of interface data (Section 2).
//
// The flux correction needs two sums over the boundary points of a
// subdomain: F = sum_p w_p (u_p . n_p) over all points, A = sum of
// w_p (n_p . n_p) over the interpolated ones.  They are formed in binary64
// with a fixed grid and a fixed reduction tree (bit-reproducible from run to
// run), gamma = -F / A, and u_p += gamma n_p on the interpolated points.
#include <cmath>

#include "fp_internal.h"

namespace fp {

constexpr int kFluxBlocks = 256;
constexpr int kFluxThreads = 256;
static_assert(2 * kFluxBlocks + 1 <= FP_FLUX_WORK, "flux workspace");

__global__ __launch_bounds__(kFluxThreads) void k_flux_partial(
    int npts, const double *__restrict__ w, const double *__restrict__ n, long long ldn,
    const int *__restrict__ iface, const double *__restrict__ u, long long ldu,
    double *__restrict__ part)
{
    __shared__ double sf[kFluxThreads], sa[kFluxThreads];
    double f = 0.0, ar = 0.0;
    for (long long p = (long long)blockIdx.x * kFluxThreads + threadIdx.x; p < npts;
         p += (long long)kFluxBlocks * kFluxThreads) {
        const double n0 = n[p], n1 = n[ldn + p], n2 = n[2 * ldn + p];
        const double un = fma(u[2 * ldu + p], n2, fma(u[ldu + p], n1, u[p] * n0));
        f = fma(w[p], un, f);
        if (!iface || iface[p]) ar = fma(w[p], fma(n2, n2, fma(n1, n1, n0 * n0)), ar);
    }
    sf[threadIdx.x] = f;
    sa[threadIdx.x] = ar;
    __syncthreads();
    for (int o = kFluxThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sf[threadIdx.x] += sf[threadIdx.x + o];
            sa[threadIdx.x] += sa[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[1 + blockIdx.x] = sf[0];
        part[1 + kFluxBlocks + blockIdx.x] = sa[0];
    }
}

__global__ __launch_bounds__(kFluxBlocks) void k_flux_gamma(double *__restrict__ work)
{
    __shared__ double sf[kFluxBlocks], sa[kFluxBlocks];
    sf[threadIdx.x] = work[1 + threadIdx.x];
    sa[threadIdx.x] = work[1 + kFluxBlocks + threadIdx.x];
    __syncthreads();
    for (int o = kFluxBlocks / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sf[threadIdx.x] += sf[threadIdx.x + o];
            sa[threadIdx.x] += sa[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) work[0] = sa[0] > 0.0 ? -sf[0] / sa[0] : 0.0;
}

__global__ __launch_bounds__(256) void k_flux_apply(int npts, const double *__restrict__ n,
                                                    long long ldn, const int *__restrict__ iface,
                                                    double *__restrict__ u, long long ldu,
                                                    const double *__restrict__ work)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts || (iface && !iface[p])) return;
    const double g = work[0];
    u[p] = fma(g, n[p], u[p]);
    u[ldu + p] = fma(g, n[ldn + p], u[ldu + p]);
    u[2 * ldu + p] = fma(g, n[2 * ldn + p], u[2 * ldu + p]);
}

struct ExtArgs {
    const double *h[3];
    double c[3];
    int order;
};

__global__ __launch_bounds__(256) void k_extrapolate(long long n, ExtArgs a,
                                                     double *__restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = a.c[0] * a.h[0][i];
    if (a.order > 1) v = fma(a.c[1], a.h[1][i], v);
    if (a.order > 2) v = fma(a.c[2], a.h[2][i], v);
    out[i] = v;
}

}  // namespace fp

using namespace fp;

extern "C" int fp_flux_correct(int npts, const double *w, const double *n, long long ldn,
                               const int *iface, double *u, long long ldu, double *work,
                               void *stream)
{
    if (npts < 0 || (npts > 0 && (!w || !n || !u)) || !work || ldn < npts || ldu < npts) {
        set_error("fp_flux_correct: NULL argument, npts < 0 or a stride below npts");
        return FP_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    k_flux_partial<<<kFluxBlocks, kFluxThreads, 0, s>>>(npts, w, n, ldn, iface, u, ldu, work);
    FP_HIP(hipGetLastError());
    k_flux_gamma<<<1, kFluxBlocks, 0, s>>>(work);
    FP_HIP(hipGetLastError());
    if (npts > 0) {
        k_flux_apply<<<(npts + 255) / 256, 256, 0, s>>>(npts, n, ldn, iface, u, ldu, work);
        FP_HIP(hipGetLastError());
    }
    return FP_OK;
}

extern "C" int fp_extrapolate(long long n, int order, const double *const *h_hist, double *out,
                              void *stream)
{
    if (n < 0 || order < 1 || order > 3 || (n > 0 && (!h_hist || !out))) {
        set_error("fp_extrapolate: need n >= 0, 1 <= order <= 3, non-NULL arrays");
        return FP_EINVAL;
    }
    if (n == 0) return FP_OK;
    // weights of the degree order-1 polynomial through the last `order` values
    static const double kW[3][3] = {{1.0, 0.0, 0.0}, {2.0, -1.0, 0.0}, {3.0, -3.0, 1.0}};
    ExtArgs a{};
    for (int q = 0; q < order; ++q) {
        if (!h_hist[q]) {
            set_error("fp_extrapolate: NULL history array");
            return FP_EINVAL;
        }
        a.h[q] = h_hist[q];
        a.c[q] = kW[order - 1][q];
    }
    a.order = order;
    k_extrapolate<<<(int)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(n, a, out);
    FP_HIP(hipGetLastError());
    return FP_OK;
}
