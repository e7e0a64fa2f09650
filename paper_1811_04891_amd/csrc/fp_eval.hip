// findpts_eval: tensor-product Lagrange interpolation of nodal fields at
// located points (Section 2.1 of the paper).  Points are grouped by element
// (the two-level counting sort of fp_group.h for large passes, atomic
// per-element counters otherwise) so that a wavefront reads an element's
// field values once for a run of its points (a work unit; an element with
// many points is spread over several units).  In large passes at orders
// <= 7 the values go to a staging array in the grouping's order first and
// k_ev_unstage moves them to the caller's output with consecutive stores.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "fp_basis.h"
#include "fp_group.h"
#include "fp_internal.h"
#include "fp_mfma.h"

namespace fp {

struct FieldPtrs {
    const double *f[kMaxEvalFields];
};

struct EvArgs {
    const int *code;
    const int *el;
    const double *rst;
    int npts;
    int E;
    int *cnt;
    const int *off;
    int *pos;
    int *order;
    double *out;   // field-major, stride npts_total
    long long ostride;
    int nf;
    double *out_all;  // first field of the call, for NaN fill
    int nf_all;
    double *sink;     // kEvSink doubles that nothing reads
    double *stage;     // non-null: k_eval_mfma writes the value of field f of the
                       // point at list position u to stage[slot[u] * nf + f], and
                       // k_ev_unstage moves it to out (else it writes out directly)
    const int *slot;   // stage row of each list position (order when not staged)
};

// Grouping key of a point: its element, or -1 when it was not found.
struct EvKey {
    const int *code, *el;
    int E;
    __device__ __forceinline__ int operator()(int p) const
    {
        const int e = el[p];
        return (code[p] != FP_NOT_FOUND && e >= 0 && e < E) ? e : -1;
    }
};

// Count points per element; not-found points get NaN right away.
__global__ __launch_bounds__(256) void k_ev_count(EvArgs a)
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

__global__ __launch_bounds__(256) void k_ev_scatter(EvArgs a)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.npts) return;
    const int k = a.pos[p];
    if (k >= 0) a.order[a.off[a.el[p]] + k] = p;
}

// Staged values to the caller's field-major output: each point reads its nf
// values (its stage row is its index in the grouping's bucket order, so the
// rows of a grouping tile's points lie in a few runs) and the stores of
// consecutive points are consecutive.  Points that were not found get NaN.
// One instance per field count: the row's NF loads are issued together
// before any store (the stores could alias the stage for all the compiler
// knows, so loads and stores taken in turn would wait on each load).
template <int NF>
__global__ __launch_bounds__(256) void k_ev_unstage(EvArgs a)
{
    // the blocks of one grouping tile run on one die, whose L2 then holds
    // the tile's runs of stage rows
    const int p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (p >= a.npts) return;
    const int j = a.pos[p];
    double v[NF];
    if (j < 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) v[f] = NAN;
    } else {
        const double *src = a.stage + (long long)j * NF;
#pragma unroll
        for (int f = 0; f < NF; ++f) v[f] = src[f];
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) a.out[f * a.ostride + p] = v[f];
}

static void launch_unstage(const EvArgs &a, int nblk, hipStream_t s)
{
    switch (a.nf) {
        case 1: k_ev_unstage<1><<<nblk, 256, 0, s>>>(a); break;
        case 2: k_ev_unstage<2><<<nblk, 256, 0, s>>>(a); break;
        case 3: k_ev_unstage<3><<<nblk, 256, 0, s>>>(a); break;
        case 4: k_ev_unstage<4><<<nblk, 256, 0, s>>>(a); break;
        case 5: k_ev_unstage<5><<<nblk, 256, 0, s>>>(a); break;
        case 6: k_ev_unstage<6><<<nblk, 256, 0, s>>>(a); break;
        case 7: k_ev_unstage<7><<<nblk, 256, 0, s>>>(a); break;
        default: k_ev_unstage<8><<<nblk, 256, 0, s>>>(a); break;
    }
}

// One wavefront per work unit: up to kUnitEval points of one element, 64 at a
// time, field rows through scalar loads.
constexpr int kUnitEval = 256;

template <int N1>
__global__ __launch_bounds__(kWave) void k_eval(EvArgs a, FieldPtrs F, const double *__restrict__ basis)
{
    constexpr int V = N1 * N1 * N1;
    const BasisPtr<double> B{as_const(basis)};
    const UnitList units(a.off, a.E, 1, a.E, kUnitEval);
    for (long long unit = xcd_unit(blockIdx.x, gridDim.x); unit < units.end; unit += gridDim.x) {
        Unit U;
        if (!units.at(unit, U)) continue;
        const int e = U.seg, beg = U.beg, end = U.end;
        for (int base = beg; base < end; base += kWave) {
            const int q = base + (int)threadIdx.x;
            const bool act = q < end;
            const int p = act ? a.order[q] : 0;
            double r0 = 0.0, r1 = 0.0, r2 = 0.0;
            if (act) {
                r0 = a.rst[3 * (long long)p];
                r1 = a.rst[3 * (long long)p + 1];
                r2 = a.rst[3 * (long long)p + 2];
            }
            double hr[N1], hs[N1], ht[N1];
            lagrange<N1>(B, r0, hr);
            lagrange<N1>(B, r1, hs);
            lagrange<N1>(B, r2, ht);
            for (int f = 0; f < a.nf; ++f) {
                const double v = field_value<N1>(as_const(F.f[f] + (long long)e * V), hr, hs, ht);
                if (act) a.out[f * a.ostride + p] = v;
            }
        }
    }
}

// Field rows of one staged element: value-only contraction, r then s then t.
template <int N1>
struct FieldAcc {
    double hr[N1], hs[N1], ht[N1];
    double v, cs;
    template <int c, int j, int k>
    __device__ __forceinline__ void step(const double (&row)[N1])
    {
        double a = 0.0;
#pragma unroll
        for (int i = 0; i < N1; ++i) a = fma(row[i], hr[i], a);
        cs = (j == 0) ? a * hs[0] : fma(a, hs[j], cs);
        if constexpr (j == N1 - 1) v = (k == 0) ? cs * ht[0] : fma(cs, ht[k], v);
    }
};

// Element groups staged in LDS, one field at a time.  A 256-thread block
// takes a work unit: G consecutive elements and a run of up to kUnitGrp of
// their points (contiguous in the element-grouped order); for each field it stages the G element blocks
// (padded by 16 bytes so lanes on different elements use different LDS
// banks) and every thread interpolates its points.
constexpr int kEvThreads = 256;
constexpr int kUnitGrp = 1024;  // points of one element group per work unit

template <int N1>
struct EvGroup {
    static constexpr int V = N1 * N1 * N1;
    static constexpr int stride = V + 2;
    static constexpr int G0 = (6 * 8192) / (stride * 8);
    static constexpr int G = G0 < 1 ? 1 : (G0 > 32 ? 32 : G0);
};

template <int N1>
__global__ __launch_bounds__(kEvThreads) void k_eval_grp(EvArgs a, FieldPtrs F,
                                                         const double *__restrict__ basis)
{
    using Gr = EvGroup<N1>;
    constexpr int V = Gr::V, G = Gr::G, S = Gr::stride;
    __shared__ double sF[G * S];
    const BasisPtr<double> B{as_const(basis)};
    const int ns = (a.E + G - 1) / G;
    const UnitList units(a.off, ns, G, a.E, kUnitGrp);
    for (long long unit = xcd_unit(blockIdx.x, gridDim.x); unit < units.end; unit += gridDim.x) {
        Unit U;
        if (!units.at(unit, U)) continue;  // uniform
        const int e0 = U.seg * G;
        const int ne = min(G, a.E - e0);
        const int pb = U.beg, pe = U.end;
        for (int f = 0; f < a.nf; ++f) {
            const double *src = F.f[f] + (long long)e0 * V;
            for (int q = threadIdx.x; q < ne * V; q += kEvThreads) {
                const int g = q / V;
                sF[g * S + (q - g * V)] = src[q];
            }
            __syncthreads();
            for (int u = pb + threadIdx.x; u < pe; u += kEvThreads) {
                const int p = a.order[u];
                const int g = a.el[p] - e0;
                FieldAcc<N1> acc;
                lagrange<N1>(B, a.rst[3 * (long long)p], acc.hr);
                lagrange<N1>(B, a.rst[3 * (long long)p + 1], acc.hs);
                lagrange<N1>(B, a.rst[3 * (long long)p + 2], acc.ht);
                double buf[kPrefetch + 1][N1];
                walk_rows<N1, 1, 0>((lptr<double>)(sF + g * S), buf, acc);
                a.out[f * a.ostride + p] = acc.v;
            }
            __syncthreads();
        }
    }
}

// Interpolation on the matrix cores (orders 1..7): one wavefront per work
// unit (up to kUnitEvalMfma points of one element), points in batches of 16.
// For field f the first contraction a_f(k, j; point) = sum_i F_f[k][j][i]
// h_i(r_point) is a dense product of the field's rows (n1^2 x n1) with the
// basis values of 16 points, one 16x16x4 matrix product per 16 rows and 4
// i-values; the fields' A fragments stay in registers for all points of the
// element.  Lane n + 16 g supplies h_i(r) for i = 4 kb + g of point n
// (evaluating only its own i and j, in its rotated node order), contracts its
// rows j = g + 4 w with h_j(s) and every plane k with h_k(t), and the 4 lanes
// of point n add their partial sums (same order in all 4: the total is
// bit-identical).  T is the arithmetic: binary64, or binary32 with binary32
// accumulation for mixed precision (binary32 basis and matrix products; the
// nodal values are rounded to binary32, the result widened to binary64).  NF
// is the launch's field count (at most 8), so one pass reads each point's r
// and evaluates its basis once for all fields, and no register holds the
// fragments of a field the launch does not have.
constexpr int kUnitEvalMfma = 256;  // points of one element per work unit
constexpr int kEvMfmaMaxN1 = 8;      // orders with the matrix-core kernel
// Smallest pass that takes the staged path: below it the grouping's launches
// cost more than the scattered stores they avoid.
constexpr int kEvStageMin = 1 << 18;
// Wavefronts per SIMD the binary64 interpolation kernel with up to 5 fields
// is held to: three (at most 168 registers; a few bytes of spills at order 7
// with 5 fields, 12 % faster than two wavefronts on the large box); the
// other instances take what their registers allow.
template <class T, int NF>
constexpr int kEvMfmaWaves = (sizeof(T) == sizeof(double) && NF <= 5) ? 3 : 1;

template <int N1, class T, int NF>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(kEvMfmaWaves<T, NF>)))
void k_eval_mfma(EvArgs a, FieldPtrs F,
                                                     const double *__restrict__ basis,
                                                     const float *__restrict__ basis32)
{
    using S = MShape<N1>;
    constexpr int V = N1 * N1 * N1;
    constexpr int MBF = (N1 + S::PPB - 1) / S::PPB;  // M blocks per field (planes k)
    const BasisPtr<double> B{as_const(basis)};
    const BasisPtr<float> B32{as_const(basis32)};
    LaneNodes<N1, T> Z;  // h_i(r), h_j(s) only for the lane's own i, j = g + 4 w
    lane_nodes<N1, T>(B, threadIdx.x >> 4, Z);
    const UnitList units(a.off, a.E, 1, a.E, kUnitEvalMfma);
    for (long long unit = xcd_unit(blockIdx.x, gridDim.x); unit < units.end; unit += gridDim.x) {
        Unit U;
        if (!units.at(unit, U)) continue;
        const int e = U.seg, beg = U.beg, end = U.end;
        const int lane = threadIdx.x, n = lane & 15, g = lane >> 4;
        // A fragment coordinates of this lane: row -> plane p, row jj; column i
        const int row = lane & 15, q = lane >> 4;
        const int gr = MF<T>::grp(row), vr = MF<T>::comp(row);
        const int pr = vr / S::EPP, jj = gr + 4 * (vr % S::EPP);
        T A[NF][MBF][S::KB];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const double *src = F.f[f] + (long long)e * V;
            double raw[MBF][S::KB];
#pragma unroll
            for (int mb = 0; mb < MBF; ++mb) {
                const int k = mb * S::PPB + pr;
#pragma unroll
                for (int kb = 0; kb < S::KB; ++kb) {
                    const int i = 4 * kb + q;
                    const bool ok = k < N1 && jj < N1 && i < N1;
                    if constexpr (sizeof(T) == sizeof(double)) {
                        raw[mb][kb] = ok ? src[N1 * (jj + N1 * k) + i] : 0.0;
                    } else {
                        // binary32: every load is issued unconditionally
                        // (entries past the element's nodes read its first
                        // value and are zeroed below), so that the loads are
                        // in flight together before their conversions wait
                        raw[mb][kb] = src[ok ? N1 * (jj + N1 * k) + i : 0];
                    }
                }
            }
#pragma unroll
            for (int mb = 0; mb < MBF; ++mb) {
                const int k = mb * S::PPB + pr;
#pragma unroll
                for (int kb = 0; kb < S::KB; ++kb) {
                    const bool ok = k < N1 && jj < N1 && 4 * kb + q < N1;
                    A[f][mb][kb] = ok ? (T)raw[mb][kb] : T(0);
                }
            }
        }
        // Software pipeline over the batches of 16 points: the point ids of
        // batch b + 2 and the r of batch b + 1 are in flight while batch b
        // computes.  The loop body has no branch: loads past the unit read
        // its first point again, and the slots past the unit store into the
        // sink, so the wait for the next batch's r counts only the memory
        // operations issued after it and never waits for this batch's stores.
        const auto at = [&](int u) { return u < end ? u : beg; };
        int p_next = a.order[at(beg + n)], j_next = a.slot[at(beg + n)];
        double r_next[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) r_next[d] = a.rst[3 * (long long)p_next + d];
        int p_after = a.order[at(beg + 16 + n)], j_after = a.slot[at(beg + 16 + n)];
        for (int b0 = beg; b0 < end; b0 += 16) {
            const bool act = b0 + n < end;
            const int p = p_next, j = j_next;
            const double r0 = r_next[0], r1 = r_next[1], r2 = r_next[2];
            p_next = p_after;
            j_next = j_after;
#pragma unroll
            for (int d = 0; d < 3; ++d) r_next[d] = a.rst[3 * (long long)p_next + d];
            p_after = a.order[at(b0 + 32 + n)];
            j_after = a.slot[at(b0 + 32 + n)];
            static_assert(S::KB == S::EPP, "r and s rows use the same lane indices");
            T hrl[S::KB], hsl[S::EPP], ht[N1];
            lagrange_lane<N1, T>(Z, (T)r0, hrl);
            lagrange_lane<N1, T>(Z, (T)r1, hsl);
            if constexpr (sizeof(T) == sizeof(double))
                lagrange<N1>(B, r2, ht);
            else
                lagrange<N1>(B32, (float)r2, ht);
            // the 4 lanes of a slot hold bit-identical totals and all store
            // them (to the staging list, or to the caller's output); the
            // slots past the unit store into the sink
            const long long fs = a.stage ? 1 : a.ostride;
            double *dst = !act     ? a.sink + ((unit * 16 + n) & (kEvSink - 1))
                          : a.stage ? a.stage + (long long)j * NF
                                    : a.out + p;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                T v = 0;
#pragma unroll
                for (int mb = 0; mb < MBF; ++mb) {
                    typename MF<T>::acc c = {0, 0, 0, 0};
#pragma unroll
                    for (int kb = 0; kb < S::KB; ++kb) c = MF<T>::mma(A[f][mb][kb], hrl[kb], c);
#pragma unroll
                    for (int pp = 0; pp < S::PPB; ++pp) {
                        const int k = mb * S::PPB + pp;
                        if (k < N1) {
                            T sa = 0;
#pragma unroll
                            for (int w = 0; w < S::EPP; ++w) sa = fma(c[pp * S::EPP + w], hsl[w], sa);
                            v = fma(sa, ht[k], v);
                        }
                    }
                }
                v = slot_sum(v);
                dst[act ? f * fs : 0] = (double)v;
            }
        }
    }
}

// Launches the order's interpolation kernel over the work units of n points.
static hipError_t launch_eval_kernel(int n1, int E, int n, const EvArgs &a, const FieldPtrs &F,
                                     const double *B, const float *B32, bool mixed, hipStream_t s)
{
#define FP_EVAL_MFMA(N1, T, NF) \
    k_eval_mfma<N1, T, NF><<<unit_grid(E, n, kUnitEvalMfma), kWave, 0, s>>>(a, F, B, B32)
#define FP_EVAL_NF(N1, T)                   \
    do {                                    \
        switch (a.nf) {                     \
            case 1: FP_EVAL_MFMA(N1, T, 1); break; \
            case 2: FP_EVAL_MFMA(N1, T, 2); break; \
            case 3: FP_EVAL_MFMA(N1, T, 3); break; \
            case 4: FP_EVAL_MFMA(N1, T, 4); break; \
            case 5: FP_EVAL_MFMA(N1, T, 5); break; \
            case 6: FP_EVAL_MFMA(N1, T, 6); break; \
            case 7: FP_EVAL_MFMA(N1, T, 7); break; \
            default: FP_EVAL_MFMA(N1, T, 8); break; \
        }                                   \
    } while (0)
#define FP_LAUNCH_MFMA(N1)             \
    do {                               \
        if (mixed)                     \
            FP_EVAL_NF(N1, float);     \
        else                           \
            FP_EVAL_NF(N1, double);    \
    } while (0)
    switch (n1) {
        case 2: FP_LAUNCH_MFMA(2); return hipGetLastError();
        case 3: FP_LAUNCH_MFMA(3); return hipGetLastError();
        case 4: FP_LAUNCH_MFMA(4); return hipGetLastError();
        case 5: FP_LAUNCH_MFMA(5); return hipGetLastError();
        case 6: FP_LAUNCH_MFMA(6); return hipGetLastError();
        case 7: FP_LAUNCH_MFMA(7); return hipGetLastError();
        case 8: FP_LAUNCH_MFMA(8); return hipGetLastError();
        default: break;
    }
#undef FP_LAUNCH_MFMA
#undef FP_EVAL_NF
#undef FP_EVAL_MFMA
#define FP_LAUNCH_GRP(N1)                                                                 \
    k_eval_grp<N1><<<unit_grid((E + EvGroup<N1>::G - 1) / EvGroup<N1>::G, n, kUnitGrp),   \
                     kEvThreads, 0, s>>>(a, F, B)
    switch (n1) {
        case 9: FP_LAUNCH_GRP(9); return hipGetLastError();
        case 10: FP_LAUNCH_GRP(10); return hipGetLastError();
        default: break;
    }
#undef FP_LAUNCH_GRP
#define FP_LAUNCH_EVAL(N1) k_eval<N1><<<unit_grid(E, n, kUnitEval), kWave, 0, s>>>(a, F, B)
    switch (n1) {
        case 2: FP_LAUNCH_EVAL(2); break;
        case 3: FP_LAUNCH_EVAL(3); break;
        case 4: FP_LAUNCH_EVAL(4); break;
        case 5: FP_LAUNCH_EVAL(5); break;
        case 6: FP_LAUNCH_EVAL(6); break;
        case 7: FP_LAUNCH_EVAL(7); break;
        case 8: FP_LAUNCH_EVAL(8); break;
        case 9: FP_LAUNCH_EVAL(9); break;
        case 10: FP_LAUNCH_EVAL(10); break;
        case 11: FP_LAUNCH_EVAL(11); break;
        case 12: FP_LAUNCH_EVAL(12); break;
        case 13: FP_LAUNCH_EVAL(13); break;
        case 14: FP_LAUNCH_EVAL(14); break;
        case 15: FP_LAUNCH_EVAL(15); break;
        case 16: FP_LAUNCH_EVAL(16); break;
        default: return hipErrorInvalidValue;
    }
#undef FP_LAUNCH_EVAL
    return hipGetLastError();
}

int run_eval(fp_handle *h, const Work &w, int npts, const int *code, const int *el,
             const double *rst, int nfields, const double *const *h_fields, double *out,
             hipStream_t s, bool timed)
{
    const size_t res_bytes = w.res ? (size_t)w.M * w.MC * 4 * sizeof(double) : 0;
    for (int start = 0; start < npts; start += w.M) {
        const int n = (npts - start < w.M) ? npts - start : w.M;
        hipEvent_t t0 = nullptr, t1 = nullptr, l0 = nullptr, l1 = nullptr;
        if (timed) {
            t0 = pool_event(h);
            t1 = pool_event(h);
            l0 = pool_event(h);
            l1 = pool_event(h);
            FP_HIP(hipEventRecord(t0, s));
        }
        // Staged path (matrix-core orders, passes of at least kEvStageMin
        // points): points grouped by element with the two-level counting
        // sort, values staged in the grouping's bucket order and moved to the
        // output by k_ev_unstage.  The grouping's
        // transient arrays and the staged values live in the pair-results
        // array of the workspace, dead once findpts has returned.  Without
        // that array (the allocation-free entry) or room in it: per-element
        // counters with atomic ranks, values written to the output directly.
        bool plan_ok = false;
        const GroupPlan gp = group_plan(n, h->E, &plan_ok);
        const int nf_max = nfields < kMaxEvalFields ? nfields : kMaxEvalFields;
        const bool staged = h->n1 <= kEvMfmaMaxN1 && n >= kEvStageMin && plan_ok && w.ev_slot &&
                            res_bytes >= group_transient_bytes(gp) &&
                            res_bytes >= (size_t)n * nf_max * sizeof(double);
        for (int f0 = 0; f0 < nfields; f0 += kMaxEvalFields) {
            const int nf = (nfields - f0 < kMaxEvalFields) ? nfields - f0 : kMaxEvalFields;
            EvArgs a{};
            a.code = code + start;
            a.el = el + start;
            a.rst = rst + 3 * (long long)start;
            a.npts = n;
            a.E = h->E;
            a.cnt = w.ev_cnt;
            a.off = w.ev_off;
            a.pos = w.ev_pos;
            a.order = w.ev_order;
            a.out = out + (long long)f0 * npts + start;
            a.ostride = npts;
            a.nf = nf;
            a.out_all = out + start;
            a.nf_all = nfields;
            a.sink = w.ev_sink;
            a.stage = staged ? w.res : nullptr;
            a.slot = staged ? w.ev_slot : w.ev_order;
            FieldPtrs F{};
            for (int f = 0; f < nf; ++f) F.f[f] = h_fields[f0 + f];
            const int pb = (n + 255) / 256;
            if (f0 == 0) {
                if (staged) {
                    GroupBufs gb;
                    gb.off = w.ev_off;
                    gb.order = w.ev_order;
                    gb.slot = w.ev_slot;
                    gb.posb = w.ev_pos;
                    group_carve(gp, (char *)w.res, gb);
                    FP_HIP(group_by_key(EvKey{a.code, a.el, h->E}, gp, gb, s));
                } else {
                    FP_HIP(fill_int(w.ev_cnt, 0, (long long)h->E + 1, s));
                    k_ev_count<<<pb, 256, 0, s>>>(a);
                    FP_HIP(hipGetLastError());
                    FP_HIP(scan_exclusive(w.ev_cnt, w.ev_off, h->E, w.scan_tmp, s));
                    k_ev_scatter<<<pb, 256, 0, s>>>(a);
                    FP_HIP(hipGetLastError());
                }
                if (timed) FP_HIP(hipEventRecord(l0, s));
            }
            FP_HIP(launch_eval_kernel(h->n1, h->E, n, a, F, h->d_basis, h->d_basis32,
                                      h->precision == FP_PREC_MIXED, s));
            if (staged) {
                launch_unstage(a, pb, s);
                FP_HIP(hipGetLastError());
            }
        }
        if (timed) {
            FP_HIP(hipEventRecord(l1, s));
            FP_HIP(hipEventRecord(t1, s));
            h->timed.push_back(TimedPair{1, l0, l1});
            h->timed.push_back(TimedPair{3, t0, t1});
        }
    }
    return FP_OK;
}

// ---------------------------------------------------------------------------
// Interpolation without any allocation: the grouping arrays (element
// counters and offsets, the scan's block sums, each point's rank and the
// element-ordered point list) live in one file-scope device array.  Each
// device holds its own copy at its own address, found once per device with
// hipGetSymbolAddress; the host never passes the array's name to a kernel.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per device
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kScratchDevices] = {};

// Address of the current device's scratch array (resolved on first use,
// with that device current).
int scratch_ptr(int dev, char **p)
{
    if (dev < 0 || dev >= kScratchDevices) {
        set_error("scratch: device ordinal out of range");
        return FP_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *q = nullptr;
        const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q) return hip_fail(e == hipSuccess ? hipErrorUnknown : e,
                                                   "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = (char *)q;
    }
    *p = g_scratch_ptr[dev];
    return FP_OK;
}

// Eval-only workspace carved from the scratch array: counters and offsets
// of E + 1 elements and the scan's block sums, then two arrays of M points
// per pass, M as large as the array allows.  Returns false when E leaves no
// room for a pass of kScratchMinPass points.
constexpr int kScratchMinPass = 1024;

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

static bool scratch_carve(char *base, int E, int npts, Work &w)
{
    const size_t e1 = (size_t)E + 1;
    const size_t fixed = 2 * round256(e1 * sizeof(int)) +
                         round256((size_t)scan_tmp_size((long long)E + 1) * sizeof(int)) +
                         round256(kEvSink * sizeof(double));
    if (fixed >= kScratchBytes) return false;
    const size_t per = (kScratchBytes - fixed) / 2 / 256 * 256 / sizeof(int);  // ints per array
    if (per < (size_t)kScratchMinPass) return false;
    const int M = (int)std::min<size_t>(per, (size_t)std::max(npts, 1));
    char *q = base;
    w = Work{};
    w.M = M;
    w.E = E;
    w.ev_cnt = (int *)q;
    q += round256(e1 * sizeof(int));
    w.ev_off = (int *)q;
    q += round256(e1 * sizeof(int));
    w.scan_tmp = (int *)q;
    q += round256((size_t)scan_tmp_size((long long)E + 1) * sizeof(int));
    w.ev_sink = (double *)q;
    q += round256(kEvSink * sizeof(double));
    w.ev_pos = (int *)q;
    q += per * sizeof(int);
    w.ev_order = (int *)q;
    return true;
}

}  // namespace fp

using namespace fp;

extern "C" int findpts_eval_noalloc(fp_handle *h, int npts, const int *code, const int *el,
                                    const double *rst, int nfields,
                                    const double *const *h_fields, double *out, void *stream)
{
    if (!h) {
        set_error("findpts_eval_noalloc: NULL handle");
        return FP_EINVAL;
    }
    if (npts < 0 || nfields < 1) {
        set_error("findpts_eval_noalloc: npts < 0 or nfields < 1");
        return FP_EINVAL;
    }
    if (npts == 0) return FP_OK;
    if (!code || !el || !rst || !h_fields || !out) {
        set_error("findpts_eval_noalloc: NULL argument");
        return FP_EINVAL;
    }
    for (int f = 0; f < nfields; ++f)
        if (!h_fields[f]) {
            set_error("findpts_eval_noalloc: NULL field pointer");
            return FP_EINVAL;
        }
    int dev = 0;
    FP_HIP(hipGetDevice(&dev));
    if (dev != h->device) FP_HIP(hipSetDevice(h->device));
    char *base = nullptr;
    const int rc = scratch_ptr(h->device, &base);
    if (rc != FP_OK) return rc;
    Work w;
    if (!scratch_carve(base, h->E, npts, w)) {
        set_error("findpts_eval_noalloc: the mesh has too many elements for the 32 MiB scratch "
                  "array (at most about 4 million)");
        return FP_ERANGE;
    }
    return run_eval(h, w, npts, code, el, rst, nfields, h_fields, out, (hipStream_t)stream,
                    false);
}

extern "C" int findpts_eval(fp_handle *h, int npts, const int *code, const int *el,
                            const double *rst, int nfields, const double *const *h_fields,
                            double *out, void *stream)
{
    if (!h) {
        set_error("findpts_eval: NULL handle");
        return FP_EINVAL;
    }
    if (npts < 0 || nfields < 1) {
        set_error("findpts_eval: npts < 0 or nfields < 1");
        return FP_EINVAL;
    }
    if (npts == 0) return FP_OK;
    if (!code || !el || !rst || !h_fields || !out) {
        set_error("findpts_eval: NULL argument");
        return FP_EINVAL;
    }
    for (int f = 0; f < nfields; ++f)
        if (!h_fields[f]) {
            set_error("findpts_eval: NULL field pointer");
            return FP_EINVAL;
        }
    int dev = 0;
    FP_HIP(hipGetDevice(&dev));
    if (dev != h->device) FP_HIP(hipSetDevice(h->device));
    return run_eval(h, h->work, npts, code, el, rst, nfields, h_fields, out, (hipStream_t)stream,
                    h->timing);
}
