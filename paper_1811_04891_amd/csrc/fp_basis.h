// Device-side tensor-product Lagrange basis on GLL nodes and the
// sum-factorised element map (geometry and Jacobian) for one lane.
//
// The element data pointers are wave-uniform (one element per wavefront), so
// their loads compile to scalar loads and every multiply-add takes the node
// value as a scalar operand; the lane-varying part is only the basis values.
#pragma once

#include "fp_internal.h"

namespace fp {

// h_i(r) = wb_i prod_{m != i} (r - z_m) and h_i'(r), by prefix and suffix
// products (O(n1) per evaluation, no division, exact zeros at other nodes).
// The basis table (z[16] then wb[16]) is read from device memory through the
// scalar cache each time instead of being held in scalar registers.
template <class T>
struct BasisPtr {
    const __attribute__((address_space(4))) T *p;
    __device__ __forceinline__ T z(int i) const { return p[i]; }
    __device__ __forceinline__ T wb(int i) const { return p[kMaxN1 + i]; }
};

template <int N1, class T>
__device__ __forceinline__ void lagrange_d(BasisPtr<T> B, T r, T (&h)[N1], T (&d)[N1])
{
    asm volatile("" : "+s"(B.p));
    T t[N1], pl[N1], dpl[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) t[i] = r - B.z(i);
    pl[0] = T(1);
    dpl[0] = T(0);
#pragma unroll
    for (int i = 1; i < N1; ++i) {
        dpl[i] = dpl[i - 1] * t[i - 1] + pl[i - 1];
        pl[i] = pl[i - 1] * t[i - 1];
    }
    T pr = T(1), dpr = T(0);
#pragma unroll
    for (int i = N1 - 1; i >= 0; --i) {
        h[i] = B.wb(i) * (pl[i] * pr);
        d[i] = B.wb(i) * (dpl[i] * pr + pl[i] * dpr);
        dpr = dpr * t[i] + pr;
        pr = pr * t[i];
    }
}

template <int N1, class T>
__device__ __forceinline__ void lagrange(BasisPtr<T> B, T r, T (&h)[N1])
{
    asm volatile("" : "+s"(B.p));
    T t[N1], pl[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) t[i] = r - B.z(i);
    pl[0] = T(1);
#pragma unroll
    for (int i = 1; i < N1; ++i) pl[i] = pl[i - 1] * t[i - 1];
    T pr = T(1);
#pragma unroll
    for (int i = N1 - 1; i >= 0; --i) {
        h[i] = B.wb(i) * (pl[i] * pr);
        pr = pr * t[i];
    }
}

// Keep a wave-uniform pointer in scalar registers and opaque to loop-
// invariant code motion: without this the compiler hoists all 3V element
// loads out of the Newton loop into vector registers and spills them.
#define FP_PIN_SGPR(p) asm volatile("" : "+s"(p))
#define FP_KEEP(v) asm volatile("" ::"v"(v))

// Element data is read through the constant address space: it is not written
// while a kernel runs, and uniform loads from it are always scalar loads.
template <class T>
using cptr = const __attribute__((address_space(4))) T *;

template <class T>
__device__ __forceinline__ cptr<T> as_const(const T *p)
{
    return (cptr<T>)p;
}

// Loops over the s and t directions are unrolled up to N = 9; beyond that
// they stay rolled (the basis arrays then live in private memory).
template <int N1>
struct Unroll {
    static constexpr int jk = (N1 <= 10) ? N1 : 1;
};

// Element data staged in LDS, read through the LDS address space.
template <class T>
using lptr = const __attribute__((address_space(3))) T *;

// Software-pipelined walk over the node rows of an element, expanded at
// compile time.  Item n is the row (j, k) = (n / C % N1, n / (C N1)) of
// array c = n % C (C = 3 coordinates, or 1 field), N1 values along r.  Rows
// are loaded kPrefetch items ahead (into scalar registers from the scalar
// cache, or into vector registers from LDS); scheduling fences keep the
// compiler from hoisting every load to the top, which would overflow the
// register file.
constexpr int kPrefetch = 2;

template <int N1, int C, int n, class P, class T, class Acc>
__device__ __forceinline__ void walk_rows(P X, T (&buf)[kPrefetch + 1][N1], Acc &acc)
{
    constexpr int V = N1 * N1 * N1;
    constexpr int NI = C * N1 * N1;
    if constexpr (n < NI) {
        if constexpr (n == 0) {
#pragma unroll
            for (int q = 0; q < kPrefetch && q < NI; ++q)
#pragma unroll
                for (int i = 0; i < N1; ++i) buf[q][i] = X[(q % C) * V + (q / C) * N1 + i];
        }
        constexpr int m = n + kPrefetch;
        if constexpr (m < NI) {
#pragma unroll
            for (int i = 0; i < N1; ++i)
                buf[m % (kPrefetch + 1)][i] = X[(m % C) * V + (m / C) * N1 + i];
        }
        __builtin_amdgcn_sched_barrier(0);
        acc.template step<n % C, (n / C) % N1, n / (C * N1)>(buf[n % (kPrefetch + 1)]);
        __builtin_amdgcn_sched_barrier(0);
        walk_rows<N1, C, n + 1>(X, buf, acc);
    }
}

// Accumulators of the geometry contraction: r first (value and derivative),
// then s, then t.
template <int N1, class T>
struct GeoAcc {
    T hr[N1], dr[N1], hs[N1], ds[N1], ht[N1], dt[N1];
    T v[3], vr[3], vs[3], vt[3], ca[3], cb[3], cc[3];
    template <int c, int j, int k>
    __device__ __forceinline__ void step(const T (&row)[N1])
    {
        T a = T(0), b = T(0);
#pragma unroll
        for (int i = 0; i < N1; ++i) {
            a = fma(row[i], hr[i], a);
            b = fma(row[i], dr[i], b);
        }
        if constexpr (j == 0) {
            ca[c] = a * hs[0];
            cb[c] = a * ds[0];
            cc[c] = b * hs[0];
        } else {
            ca[c] = fma(a, hs[j], ca[c]);
            cb[c] = fma(a, ds[j], cb[c]);
            cc[c] = fma(b, hs[j], cc[c]);
        }
        if constexpr (j == N1 - 1) {
            if constexpr (k == 0) {
                v[c] = ca[c] * ht[0];
                vt[c] = ca[c] * dt[0];
                vs[c] = cb[c] * ht[0];
                vr[c] = cc[c] * ht[0];
            } else {
                v[c] = fma(ca[c], ht[k], v[c]);
                vt[c] = fma(ca[c], dt[k], vt[c]);
                vs[c] = fma(cb[c], ht[k], vs[c]);
                vr[c] = fma(cc[c], ht[k], vr[c]);
            }
        }
    }
};

// Geometry and Jacobian with the element block in LDS (per-lane base: lanes
// of one wavefront may work on different elements of a staged group).
template <int N1, class T>
__device__ __forceinline__ void geo_eval_lds(lptr<T> X, BasisPtr<T> B, const T (&r)[3],
                                             T (&x)[3], T (&J)[9])
{
    static_assert(N1 <= 10, "LDS path is unrolled");
    GeoAcc<N1, T> A;
    lagrange_d<N1>(B, r[0], A.hr, A.dr);
    lagrange_d<N1>(B, r[1], A.hs, A.ds);
    lagrange_d<N1>(B, r[2], A.ht, A.dt);
    T buf[kPrefetch + 1][N1];
    walk_rows<N1, 3, 0>(X, buf, A);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = A.v[c];
        J[3 * c + 0] = A.vr[c];
        J[3 * c + 1] = A.vs[c];
        J[3 * c + 2] = A.vt[c];
        FP_KEEP(x[c]);
        FP_KEEP(J[3 * c + 0]);
        FP_KEEP(J[3 * c + 1]);
        FP_KEEP(J[3 * c + 2]);
    }
}

// x_c(r) and J[c][d] = dx_c/dr_d for the three coordinates of one element,
// X = element block (3 x V, r index fastest), sum-factorised: contraction
// over r first (value and r-derivative), then s, then t.
template <int N1, class T>
__device__ __forceinline__ void geo_eval(cptr<T> X, BasisPtr<T> B, const T (&r)[3],
                                         T (&x)[3], T (&J)[9])
{
    FP_PIN_SGPR(X);
    GeoAcc<N1, T> A;
    lagrange_d<N1>(B, r[0], A.hr, A.dr);
    lagrange_d<N1>(B, r[1], A.hs, A.ds);
    lagrange_d<N1>(B, r[2], A.ht, A.dt);
    if constexpr (N1 <= 10) {
        T buf[kPrefetch + 1][N1];
        walk_rows<N1, 3, 0>(X, buf, A);
    } else {
        constexpr int V = N1 * N1 * N1;
#pragma unroll 1
        for (int k = 0; k < N1; ++k) {
            T ca[3] = {T(0), T(0), T(0)}, cb[3] = {T(0), T(0), T(0)}, cc[3] = {T(0), T(0), T(0)};
#pragma unroll 1
            for (int j = 0; j < N1; ++j) {
                const int row = N1 * (j + N1 * k);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    T a = T(0), b = T(0);
#pragma unroll
                    for (int i = 0; i < N1; ++i) {
                        const T xv = X[c * V + row + i];
                        a = fma(xv, A.hr[i], a);
                        b = fma(xv, A.dr[i], b);
                    }
                    ca[c] = fma(a, A.hs[j], ca[c]);
                    cb[c] = fma(a, A.ds[j], cb[c]);
                    cc[c] = fma(b, A.hs[j], cc[c]);
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T v0 = (k == 0) ? T(0) : A.v[c], t0 = (k == 0) ? T(0) : A.vt[c];
                const T s0 = (k == 0) ? T(0) : A.vs[c], r0 = (k == 0) ? T(0) : A.vr[c];
                A.v[c] = fma(ca[c], A.ht[k], v0);
                A.vt[c] = fma(ca[c], A.dt[k], t0);
                A.vs[c] = fma(cb[c], A.ht[k], s0);
                A.vr[c] = fma(cc[c], A.ht[k], r0);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = A.v[c];
        J[3 * c + 0] = A.vr[c];
        J[3 * c + 1] = A.vs[c];
        J[3 * c + 2] = A.vt[c];
        // Consume the results here: otherwise the compiler sinks the parts
        // only some paths need (the Jacobian) into a branch, away from the
        // pipelined node loads, and must keep every node row alive until then.
        FP_KEEP(x[c]);
        FP_KEEP(J[3 * c + 0]);
        FP_KEEP(J[3 * c + 1]);
        FP_KEEP(J[3 * c + 2]);
    }
}

// Geometry only (no Jacobian).
template <int N1, class T>
__device__ __forceinline__ void geo_value(cptr<T> X, BasisPtr<T> B,
                                          const T (&r)[3], T (&x)[3])
{
    constexpr int V = N1 * N1 * N1;
    FP_PIN_SGPR(X);
    T hr[N1], hs[N1], ht[N1];
    lagrange<N1>(B, r[0], hr);
    lagrange<N1>(B, r[1], hs);
    lagrange<N1>(B, r[2], ht);
    T v[3] = {T(0), T(0), T(0)};
#pragma unroll Unroll<N1>::jk
    for (int k = 0; k < N1; ++k) {
        T ca[3] = {T(0), T(0), T(0)};
#pragma unroll Unroll<N1>::jk
        for (int j = 0; j < N1; ++j) {
            T a[3] = {T(0), T(0), T(0)};
            const int row = N1 * (j + N1 * k);
            FP_PIN_SGPR(X);
#pragma unroll
            for (int i = 0; i < N1; ++i)
#pragma unroll
                for (int c = 0; c < 3; ++c) a[c] = fma(X[c * V + row + i], hr[i], a[c]);
#pragma unroll
            for (int c = 0; c < 3; ++c) ca[c] = fma(a[c], hs[j], ca[c]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = fma(ca[c], ht[k], v[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = v[c];
}

// Scalar field value at r with lane-varying element data (vector loads).
template <int N1>
__device__ __forceinline__ double field_value_v(const double *__restrict__ F,
                                                const double (&hr)[N1], const double (&hs)[N1],
                                                const double (&ht)[N1])
{
    double v = 0.0;
#pragma unroll 1
    for (int k = 0; k < N1; ++k) {
        double cs = 0.0;
#pragma unroll 1
        for (int j = 0; j < N1; ++j) {
            double a = 0.0;
            const double *row = F + N1 * (j + N1 * k);
#pragma unroll
            for (int i = 0; i < N1; ++i) a = fma(row[i], hr[i], a);
            cs = fma(a, hs[j], cs);
        }
        v = fma(cs, ht[k], v);
    }
    return v;
}

// Scalar field value at r given the basis values.
template <int N1>
__device__ __forceinline__ double field_value(cptr<double> F,
                                              const double (&hr)[N1], const double (&hs)[N1],
                                              const double (&ht)[N1])
{
    double v = 0.0;
#pragma unroll Unroll<N1>::jk
    for (int k = 0; k < N1; ++k) {
        double cs = 0.0;
#pragma unroll Unroll<N1>::jk
        for (int j = 0; j < N1; ++j) {
            double a = 0.0;
            const int row = N1 * (j + N1 * k);
            FP_PIN_SGPR(F);
#pragma unroll
            for (int i = 0; i < N1; ++i) a = fma(F[row + i], hr[i], a);
            cs = fma(a, hs[j], cs);
        }
        v = fma(cs, ht[k], v);
    }
    return v;
}

}  // namespace fp
