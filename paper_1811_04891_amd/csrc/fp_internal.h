// Internal declarations of the gfx950 findpts library (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/findpts.h"

namespace fp {

constexpr int kMaxN1 = 16;       // N <= 15
constexpr int kMaxEvalFields = 8; // fields per interpolation launch
constexpr int kEvSink = 512;       // doubles in Work::ev_sink (a power of two)
constexpr int kStats = 6;          // device counters of a handle (findpts_stats)
constexpr int kTimedPhases = 5;    // timed phases (findpts_timing_read)
constexpr int kWave = 64;
constexpr int kXcds = 8;  // accelerator dies; workgroups are dealt to them in turn

// Block index remapped so that each accelerator die (XCD, own L2) runs one
// contiguous range of the G block indices: workgroup b is dispatched to die
// b mod kXcds, and becomes number b / kXcds of that die's range.  A bijection
// of [0, G); neighbouring work then shares one L2.
__device__ __forceinline__ int xcd_block(int b, int G)
{
    const int x = b % kXcds, i = b / kXcds, q = G / kXcds, r = G % kXcds;
    return x * q + (x < r ? x : r) + i;
}

// Unit walked first by block b of a grid of G blocks (blocks go to the dies
// in turn, b mod kXcds): each die takes runs of kXcdRun consecutive units,
// the runs of the dies interleaved, so that the units of a crowded element
// (consecutive indices) mostly share one die's L2 while the work stays spread
// over all dies.  A bijection of [0, G) (the last partial round of runs
// keeps b).
constexpr int kXcdRun = 8;
__device__ __forceinline__ long long xcd_unit(long long b, long long G)
{
    constexpr long long P = (long long)kXcds * kXcdRun;
    if (b >= (G / P) * P) return b;
    const long long i = b / kXcds, x = b % kXcds;
    return (i / kXcdRun) * P + x * kXcdRun + i % kXcdRun;
}

// GLL nodes z_i and barycentric weights wb_i = 1 / prod_{m != i} (z_i - z_m),
// passed to kernels by value (kernel arguments are read through the scalar
// cache).
struct Basis {
    double z[kMaxN1];
    double wb[kMaxN1];
};

struct Basis32 {
    float z[kMaxN1];
    float wb[kMaxN1];
};

// Hash grid parameters passed by value.
struct Grid {
    double lo[3];
    double hi[3];
    double inv[3];  // cells per unit length
    int nc[3];
};

struct TimedPair {
    int phase;
    hipEvent_t a, b;
};

// Workspace of one findpts / findpts_eval call on one stream: M points per
// pass, MC candidate slots per point (the longest hash-cell list), E + 1
// element counters.  Carved from one device block; a handle owns one, the
// serving layer carves one per admitted request from its arena.
struct Work {
    int M = 0, MC = 1, E = 0;
    int *ncand = nullptr;     // M
    int *cand_el = nullptr;   // M x MC
    int *cand_pos = nullptr;  // M x MC, rank of the pair within its element
    int *elem_cnt = nullptr;  // E + 1
    int *elem_off = nullptr;  // E + 1
    int *order = nullptr;     // M x MC pair slots grouped by element
    double *res = nullptr;    // M x MC x 4: r, s, t, d2
    double *res_dl = nullptr; // M x MC: delta at the candidate (if delta)
    int *res_in = nullptr;    // M x MC: inside flag
    int *redo = nullptr;      // M: second-pass flag per point
    int *gate = nullptr;      // 1: nonzero when the first pass flagged any point
    int *scan_tmp = nullptr;  // block sums of the device scans
    unsigned *cand_part = nullptr;  // ceil(M / 256): per-block candidate counts
    unsigned *iter_part = nullptr;  // unit_grid(E, M, kUnitMin): Newton iterations per block
    int *ev_cnt = nullptr;    // E + 1
    int *ev_off = nullptr;    // E + 1
    int *ev_pos = nullptr;    // M
    int *ev_order = nullptr;  // M
    int *ev_slot = nullptr;   // M: stage row of each list position (grouped path)
    double *ev_sink = nullptr;  // kEvSink: stores of interpolation slots past a unit
};

// Bytes of a workspace (256-byte aligned sub-arrays); carve() lays it out
// from `base` (which must be 256-byte aligned).
size_t work_bytes(int E, int MC, int M, bool delta);
void work_carve(Work &w, char *base, int E, int MC, int M, bool delta);

}  // namespace fp

struct fp_handle {
    int device = 0;
    int E = 0, N = 0, n1 = 0, V = 0;
    double tol = 0.0;
    int precision = 0;
    int max_points = 0;

    // mesh (handle-owned)
    double *geom = nullptr;    // E x 3 x V, element-blocked, r index fastest
    float *geom32 = nullptr;   // binary32 copy (mixed precision)
    double *esize = nullptr;   // E: h_e
    double *bbox = nullptr;    // E x 6
    double *erec = nullptr;    // E x 16 doubles (one 128-byte line per element): the
                               // axis-aligned box (6 doubles) then the oriented box
                               // (18 binary32 values), for the candidate tests
    float *obb = nullptr;      // E x 18 binary32: frame Q (9, row-major, rows = axes),
                               // centre (3), rotated lo (3), rotated hi (3)
    int *esess = nullptr;      // E or null
    double *delta = nullptr;   // E x V or null

    // hash grid
    fp::Grid grid{};
    long long ncell = 0, nnz = 0;
    int max_cell = 0;
    int *cell_off = nullptr;   // ncell + 1
    int *cell_cnt = nullptr;   // ncell + 1 (hash build)
    long long cell_cap = 0;    // allocated length of cell_off / cell_cnt
    long long nnz_cap = 0;     // allocated entries of cell_el / cell_box
    int *cell_el = nullptr;    // nnz
    float4 *cell_box = nullptr; // 2 nnz: binary32 outward box + element id per entry

    // workspace of the handle's own calls (max_points per pass)
    int MC = 1;                 // longest hash-cell list (>= 1)
    fp::Work work{};
    void *work_mem = nullptr;
    size_t work_bytes = 0;
    int *d_flag = nullptr;      // setup scratch: flags, longest cell list
    double *d_g = nullptr;      // setup scratch: global box
    double *d_binv = nullptr;   // Bernstein-to-nodal inverse (n1 x n1)
    int *scan_tmp = nullptr;    // setup's scans (cells)
    int scan_tmp_n = 0;

    // [pairs solved, Newton iterations, points located, axis-aligned box
    //  candidates (the hash + box candidate count of the method), pairs
    //  solved by first passes, their Newton iterations]
    unsigned long long *stats = nullptr;

    fp::Basis basis{};
    fp::Basis32 basis32{};
    double *d_basis = nullptr;   // device copy of basis (z, wb)
    double *d_dnode = nullptr;   // n1 x n1: h_b'(z_a) at row a, column b
    float *d_basis32 = nullptr;  // device copy of basis32
    size_t bytes = 0;

    bool timing = false;
    std::vector<fp::TimedPair> timed;
    std::vector<hipEvent_t> event_pool;
};

namespace fp {

void set_error(const std::string &msg);
int hip_fail(hipError_t e, const char *what);
// Device address of the interpolation scratch array of device dev (resolved
// once per device, with dev current); FP_OK or an error code.
int scratch_ptr(int dev, char **p);
hipEvent_t pool_event(fp_handle *h);

#define FP_HIP(call)                                         \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return fp::hip_fail(e_, #call); \
    } while (0)

// Work units of an element-grouped list.  Segment s (a run of gs consecutive
// elements, s < ns) owns list positions [b(s), b(s + 1)) with
// b(s) = off[min(s gs, ne)]; it is cut at the multiples of K and its piece in
// window j (positions [j K, (j + 1) K)) is unit s + j.  Along the list both s
// and j never decrease and at least one of them grows from one piece to the
// next, so the unit indices of the pieces are distinct and increasing, and
// the segment holding unit u is the last s with s + b(s) / K <= u, which lies
// in [u - T, u] for T = b(ns) / K.  A block takes units blockIdx.x,
// blockIdx.x + gridDim.x, ... below ns + T + 1: an element with many points
// is spread over many blocks, and a sparse list (T small) needs no search.
// Units of gaps (empty segments, cuts that fall on a segment's start) are
// empty.
struct Unit {
    int seg, beg, end;
};

struct UnitList {
    const int *off;
    int ns, gs, ne, K, T;
    long long end;  // one past the last unit index

    __host__ __device__ __forceinline__ UnitList(const int *off_, int ns_, int gs_, int ne_, int K_)
        : off(off_), ns(ns_), gs(gs_), ne(ne_), K(K_)
    {
        T = off[ne] / K;
        end = (long long)ns + T + 1;
    }
    __host__ __device__ __forceinline__ int b(long long s) const
    {
        return off[s * gs < ne ? s * gs : ne];
    }
    // Unit u of the list (false for a gap).  Called by every lane of a
    // wavefront with the same u (converged code, full wavefront): the 64
    // lanes probe 64 evenly spaced segments of the bracket at once, and the
    // prefix of probes with s + b(s) / K <= u (a prefix, since that sum grows
    // with s) narrows the bracket to one 64th per round, so a list of T
    // windows takes log64 T dependent loads instead of log2 T.
    __device__ __forceinline__ bool at(long long u, Unit &U) const
    {
        long long lo = u - T, hi = u;  // s + b(s) / K <= u holds at lo
        if (lo < 0) lo = 0;
        if (hi > ns - 1) hi = ns - 1;
        const long long lane = (long long)(threadIdx.x & (kWave - 1));
        while (lo < hi) {
            const long long span = hi - lo;
            const long long p = lo + ((lane + 1) * span + kWave - 1) / kWave;  // in (lo, hi]
            const long long cnt = __popcll(__ballot(p + b(p) / K <= u));
            const long long nlo = cnt == 0 ? lo : lo + (cnt * span + kWave - 1) / kWave;
            const long long nhi = cnt == kWave ? hi : lo + ((cnt + 1) * span + kWave - 1) / kWave - 1;
            lo = nlo;
            hi = nhi;
        }
        const int b0 = b(lo), b1 = b(lo + 1);
        const long long j = u - lo;
        if (b0 >= b1 || j * K >= b1) return false;
        U.seg = (int)lo;
        U.beg = (int)(j * K > b0 ? j * K : b0);
        U.end = (int)((j + 1) * K < b1 ? (j + 1) * K : b1);
        return true;
    }
};

// Blocks of a unit launch over ns segments for a list of about n entries:
// one per segment plus up to 2 n / K (at most kUnitSpare) for the pieces of
// crowded segments.  Units beyond the grid are taken by the grid-stride walk.
constexpr long long kUnitSpare = 4096;
inline int unit_grid(int ns, long long n, int K)
{
    long long extra = 2 * ((n + K - 1) / K);
    if (extra > kUnitSpare) extra = kUnitSpare;
    const long long g = (long long)ns + extra;
    return (int)(g < 1 ? 1 : (g > 0x7fffffffLL ? 0x7fffffffLL : g));
}

// Grid of a second-pass launch: usually nearly empty, so a bounded grid walks
// the units with its grid-stride loop instead of one block per element.
constexpr int kSecondPassGrid = 8192;

// Rank of each active lane's entry in its group's counter, cnt[e] += 1 per
// entry.  Lanes of a wavefront that share the group of the first pending
// lane take their ranks from one atomic add (up to four such groups); any
// other lane adds alone.  Call from converged code (every lane of the
// wavefront), act false for lanes without an entry.  The ranks of a group are
// distinct and fill [old count, new count).
__device__ __forceinline__ int wave_rank(int *cnt, int e, bool act)
{
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long pending = __ballot(act);
    int rank = 0;
    for (int it = 0; it < 4 && pending; ++it) {
        const int leader = __ffsll((long long)pending) - 1;
        const int e0 = __shfl(e, leader, kWave);
        const unsigned long long grp = __ballot(act && e == e0) & pending;
        const int m = __popcll(grp);
        if (m < 2) break;  // no sharing: the rest add alone
        int base = 0;
        if (lane == leader) base = atomicAdd(&cnt[e0], m);
        base = __shfl(base, leader, kWave);
        if ((grp >> lane) & 1ull) rank = base + __popcll(grp & below);
        pending &= ~grp;
    }
    if ((pending >> lane) & 1ull) rank = atomicAdd(&cnt[e], 1);
    return rank;
}
constexpr int kUnitMin = 64;  // smallest K of the locate kernels

// Exclusive scan of n ints: out[0..n], out[n] = total.  tmp needs
// scan_tmp_size(n) ints.  With gate non-null the kernels do nothing while
// *gate is zero (a pass with no work), as does the gated fill.
int scan_tmp_size(long long n);
hipError_t scan_exclusive(const int *in, int *out, int n, int *tmp,
                          hipStream_t s, const int *gate = nullptr);
hipError_t fill_int_gated(int *p, int value, long long n, const int *gate, hipStream_t s);

// GLL nodes and barycentric weights of order N; the inverse of the
// Bernstein-to-nodal matrix (n1 x n1, row-major), both computed on the host.
Basis make_basis(int N);
// Differentiation matrix at the nodes, D[a n1 + b] = h_b'(z_a), from the
// barycentric weights (off-diagonal (wb_b / wb_a) / (z_a - z_b), diagonal
// minus the row sum).
std::vector<double> node_derivatives(const Basis &b, int N);
std::vector<double> bernstein_to_nodal_inverse(int N, const double *z);

// Fill n ints with a value (a kernel, so that it may be graph-captured).
hipError_t fill_int(int *p, int value, long long n, hipStream_t s);

// findpts / findpts_eval on a given workspace and stream (the public calls
// pass the handle's own workspace; `timed` records the handle's events).
int run_findpts(fp_handle *h, const Work &w, int npts, const double *pts, const int *pt_session,
                int *code, int *el, double *rst, double *dist2, hipStream_t s, bool timed);
int run_eval(fp_handle *h, const Work &w, int npts, const int *code, const int *el,
             const double *rst, int nfields, const double *const *h_fields, double *out,
             hipStream_t s, bool timed);

}  // namespace fp
