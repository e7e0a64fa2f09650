// Matrix-core building blocks shared by the Newton and interpolation
// kernels: the 16x16x4 MFMA in binary64 and binary32 with their register
// layouts, the row blocking of an element's node data, the basis values of
// one lane's own rows, and the sum over the 4 lanes that share a column.
#pragma once

#include "fp_basis.h"

namespace fp {

typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));

template <class T>
struct MF;

template <>
struct MF<double> {
    typedef dx4 acc;
    static __device__ __forceinline__ acc mma(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // result row i, column j at lane j + 16 (i % 4), component i / 4
    static __device__ __forceinline__ int row(int g, int v) { return 4 * v + g; }
    static __device__ __forceinline__ int grp(int row) { return row % 4; }
    static __device__ __forceinline__ int comp(int row) { return row / 4; }
};

template <>
struct MF<float> {
    typedef fx4 acc;
    static __device__ __forceinline__ acc mma(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // result row i, column j at lane j + 16 (i / 4), component i % 4
    static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
    static __device__ __forceinline__ int grp(int row) { return row / 4; }
    static __device__ __forceinline__ int comp(int row) { return row % 4; }
};

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

// A lane's own node order: position p holds node (p + g) mod N1, so that the
// indices the lane needs for its slot, i = 4 m + g, sit at the fixed positions
// 4 m (weight 0 past the last node).  Loaded once per kernel.
template <int N1, class T = double>
struct LaneNodes {
    T z[N1];
    T w[MShape<N1>::KB];
};

template <int N1, class T = double>
__device__ __forceinline__ void lane_nodes(BasisPtr<double> B, int g, LaneNodes<N1, T> &Z)
{
#pragma unroll
    for (int p = 0; p < N1; ++p) Z.z[p] = (T)B.z((p + g) % N1);
#pragma unroll
    for (int m = 0; m < MShape<N1>::KB; ++m) {
        const int i = 4 * m + g;
        Z.w[m] = i < N1 ? (T)B.wb(i) : T(0);
    }
}

// h_i(r) and h_i'(r) for the lane's indices i = 4 m + g: the product of
// (r - z) over the other nodes, taken in the lane's node order (prefix times
// suffix products), so no lane computes the basis functions it does not use.
template <int N1, class T = double>
__device__ __forceinline__ void lagrange_d_lane(const LaneNodes<N1, T> &Z, T r,
                                                T (&h)[MShape<N1>::KB],
                                                T (&d)[MShape<N1>::KB])
{
    T t[N1], pl[N1], dpl[N1], pr[N1], dpr[N1];
#pragma unroll
    for (int p = 0; p < N1; ++p) t[p] = r - Z.z[p];
    pl[0] = T(1);
    dpl[0] = T(0);
#pragma unroll
    for (int p = 1; p < N1; ++p) {
        dpl[p] = dpl[p - 1] * t[p - 1] + pl[p - 1];
        pl[p] = pl[p - 1] * t[p - 1];
    }
    pr[N1 - 1] = T(1);
    dpr[N1 - 1] = T(0);
#pragma unroll
    for (int p = N1 - 2; p >= 0; --p) {
        dpr[p] = dpr[p + 1] * t[p + 1] + pr[p + 1];
        pr[p] = pr[p + 1] * t[p + 1];
    }
#pragma unroll
    for (int m = 0; m < MShape<N1>::KB; ++m) {
        const int p = 4 * m;
        h[m] = Z.w[m] * (pl[p] * pr[p]);
        d[m] = Z.w[m] * (dpl[p] * pr[p] + pl[p] * dpr[p]);
    }
}

// h_i(r) alone for the lane's indices i = 4 m + g (as lagrange_d_lane).
template <int N1, class T = double>
__device__ __forceinline__ void lagrange_lane(const LaneNodes<N1, T> &Z, T r,
                                              T (&h)[MShape<N1>::KB])
{
    T t[N1], pl[N1], pr[N1];
#pragma unroll
    for (int p = 0; p < N1; ++p) t[p] = r - Z.z[p];
    pl[0] = T(1);
#pragma unroll
    for (int p = 1; p < N1; ++p) pl[p] = pl[p - 1] * t[p - 1];
    pr[N1 - 1] = T(1);
#pragma unroll
    for (int p = N1 - 2; p >= 0; --p) pr[p] = pr[p + 1] * t[p + 1];
#pragma unroll
    for (int m = 0; m < MShape<N1>::KB; ++m) h[m] = Z.w[m] * (pl[4 * m] * pr[4 * m]);
}

// Sum over the 4 lanes n + 16 g of a slot, by two lane swaps (no LDS):
// v_permlane16_swap exchanges the odd 16-lane rows of its first operand with
// the even rows of its second, v_permlane32_swap the upper half of the first
// with the lower half of the second.  With the same value in both operands
// the two results are (lower partner, upper partner) in every lane, so the
// sum is formed in the same order in all 4 lanes: bit-identical totals.
__device__ __forceinline__ unsigned lo32(double v) { return (unsigned)__double_as_longlong(v); }
__device__ __forceinline__ unsigned hi32(double v)
{
    return (unsigned)((unsigned long long)__double_as_longlong(v) >> 32);
}
__device__ __forceinline__ double mk64(unsigned lo, unsigned hi)
{
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int ROWS>
__device__ __forceinline__ double swap_add(double v)
{
    const unsigned l = lo32(v), h = hi32(v);
    if constexpr (ROWS == 16) {
        const auto a = __builtin_amdgcn_permlane16_swap(l, l, false, false);
        const auto b = __builtin_amdgcn_permlane16_swap(h, h, false, false);
        return mk64(a[0], b[0]) + mk64(a[1], b[1]);
    } else {
        const auto a = __builtin_amdgcn_permlane32_swap(l, l, false, false);
        const auto b = __builtin_amdgcn_permlane32_swap(h, h, false, false);
        return mk64(a[0], b[0]) + mk64(a[1], b[1]);
    }
}

template <int ROWS>
__device__ __forceinline__ float swap_add(float v)
{
    const unsigned l = __float_as_uint(v);
    if constexpr (ROWS == 16) {
        const auto a = __builtin_amdgcn_permlane16_swap(l, l, false, false);
        return __uint_as_float(a[0]) + __uint_as_float(a[1]);
    } else {
        const auto a = __builtin_amdgcn_permlane32_swap(l, l, false, false);
        return __uint_as_float(a[0]) + __uint_as_float(a[1]);
    }
}

template <class T>
__device__ __forceinline__ T slot_sum(T v)
{
    return swap_add<32>(swap_add<16>(v));
}

// Lane swaps of two different binary64 values (results in the order the
// builtins return them: first operand, second operand).
template <int ROWS>
__device__ __forceinline__ void swap2(double x, double y, double &xo, double &yo)
{
    if constexpr (ROWS == 16) {
        const auto l = __builtin_amdgcn_permlane16_swap(lo32(x), lo32(y), false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi32(x), hi32(y), false, false);
        xo = mk64(l[0], h[0]);
        yo = mk64(l[1], h[1]);
    } else {
        const auto l = __builtin_amdgcn_permlane32_swap(lo32(x), lo32(y), false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi32(x), hi32(y), false, false);
        xo = mk64(l[0], h[0]);
        yo = mk64(l[1], h[1]);
    }
}

template <int ROWS>
__device__ __forceinline__ void swap2(float x, float y, float &xo, float &yo)
{
    const auto r = (ROWS == 16)
                       ? __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y),
                                                          false, false)
                       : __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y),
                                                          false, false);
    xo = __uint_as_float(r[0]);
    yo = __uint_as_float(r[1]);
}

// slot_sum of four values at once.  Swapping two different values leaves
// the pair sums of the first in the even 16-lane rows and of the second in
// the odd rows, so after the two reduction rounds row r holds the total of
// value r, each formed once and in slot_sum's order; two broadcast rounds
// then give every lane all four totals (bit-identical in the 4 lanes of a
// slot), with half the lane swaps of four slot_sum calls.
template <class T>
__device__ __forceinline__ void slot_sum4(T &a, T &b, T &c, T &d)
{
    T x, y;
    swap2<16>(a, b, x, y);
    const T sab = x + y;
    swap2<16>(c, d, x, y);
    const T scd = x + y;
    swap2<32>(sab, scd, x, y);
    const T t = x + y;  // row r: total of value r
    T p, q;
    swap2<32>(t, t, p, q);   // p = (a, b, a, b), q = (c, d, c, d) by rows
    swap2<16>(p, p, a, b);
    swap2<16>(q, q, c, d);
}

}  // namespace fp
