// Grouping of n items by an integer key in [0, K), without device-scope
// atomics: a counting sort in two levels.  Items whose key is negative are
// left out.
//
//   k_grp_hist     per tile of kGrpTile items: item counts per bucket (a run
//                  of 2^shift consecutive keys), counted in LDS
//   scan           bucket-major exclusive scan of the tile counts: each
//                  (bucket, tile) pair gets its run in bucket order
//   k_grp_scatter  per tile: the items and keys into bucket order (ranks
//                  within the tile's run from LDS counters); each item's
//                  bucket-order index j is stored in item order
//   k_grp_chunks   each bucket cut into chunks of kGrpChunk items (so that a
//                  crowded bucket is spread over many blocks)
//   k_grp_lcount   per chunk: key counts and ranks from LDS counters
//   scan           counts in (bucket, key, chunk) order -> offsets
//   k_grp_lplace   per chunk: each item to its key's run
//   k_grp_off      key offsets
//
// Scattered stores stay within a tile's runs or a bucket's window of the
// list, which the caches hold, instead of one device-scope atomic and one
// store anywhere in the list per item.  Positions within a key's run follow
// the order of LDS atomics (not deterministic); every consumer here treats
// the items of a run independently.
#pragma once

#include <algorithm>

#include "fp_internal.h"

namespace fp {

constexpr int kGrpThreads = 256;
constexpr int kGrpItems = 32;  // items per thread and tile
constexpr int kGrpTile = kGrpThreads * kGrpItems;
constexpr int kGrpChunk = 4096;  // items per chunk of a bucket
constexpr int kGrpMaxBuckets = 1024;
constexpr int kGrpMaxShift = 12;  // keys per bucket: LDS tables of k_grp_lplace (2 x 16 KB)

struct GroupPlan {
    int n;      // items
    int K;      // keys: [0, K)
    int shift;  // bucket of key e: e >> shift
    int B;      // buckets
    int T;      // tiles
};

// Plan for n items and K keys: at most kGrpMaxBuckets buckets of at least 64
// keys; ok is false when a bucket's key counters would not fit in LDS (K
// above kGrpMaxBuckets << kGrpMaxShift).
inline GroupPlan group_plan(int n, int K, bool *ok)
{
    GroupPlan g{n, K, 6, 1, 1};
    while ((((long long)K + (1LL << g.shift) - 1) >> g.shift) > kGrpMaxBuckets) ++g.shift;
    const long long B = ((long long)K + (1LL << g.shift) - 1) >> g.shift;
    g.B = B < 1 ? 1 : (int)B;
    g.T = n < 1 ? 1 : (int)(((long long)n + kGrpTile - 1) / kGrpTile);
    // the scans take int counts
    const long long gc = ((long long)1 << g.shift) * (g.B + ((long long)n + kGrpChunk - 1) / kGrpChunk);
    *ok = g.shift <= kGrpMaxShift && gc < 0x7fffffffLL && (long long)g.B * g.T < 0x7fffffffLL;
    return g;
}

// Entries of the (bucket, key, chunk) count array: keys per bucket times a
// bound on the chunks.
inline long long grp_gcnt_size(const GroupPlan &g)
{
    return ((long long)1 << g.shift) * (g.B + ((long long)g.n + kGrpChunk - 1) / kGrpChunk);
}

// Device arrays of a grouping.  Results: off (K + 1: start of each key's
// run, off[K] = items kept), order (list position -> item), slot (list
// position -> bucket-order index), posb (item -> bucket-order index, -1 if
// left out).  Transient (carved by group_carve): items, keys and ranks in
// bucket order, tile counts and their scan, the chunk table, the chunk key
// counts and their scan, scan workspace.
struct GroupBufs {
    int *off = nullptr, *order = nullptr, *slot = nullptr, *posb = nullptr;
    int *items_b = nullptr, *keys_b = nullptr, *rank_b = nullptr;
    int *h = nullptr, *hoff = nullptr, *cstart = nullptr, *gcnt = nullptr, *goff = nullptr;
    int *scan_tmp = nullptr;
};

inline size_t grp_round(size_t b) { return (b + 255) / 256 * 256; }

// Transient arrays of a plan carved from base (256-byte aligned; null base:
// sizes only); returns their bytes.
inline size_t group_carve(const GroupPlan &g, char *base, GroupBufs &b)
{
    const size_t n = (size_t)(g.n < 1 ? 1 : g.n), bt = (size_t)g.B * g.T + 1;
    const size_t gc = (size_t)grp_gcnt_size(g) + 1;
    const size_t st = (size_t)scan_tmp_size((long long)std::max(bt, gc));
    const size_t sizes[9] = {n, n, n, bt, bt, (size_t)g.B + 1, gc, gc, st};
    int **dst[9] = {&b.items_b, &b.keys_b, &b.rank_b, &b.h, &b.hoff,
                    &b.cstart, &b.gcnt, &b.goff, &b.scan_tmp};
    size_t off = 0;
    for (int k = 0; k < 9; ++k) {
        if (base) *dst[k] = (int *)(base + off);
        off += grp_round(sizes[k] * sizeof(int));
    }
    return off;
}

inline size_t group_transient_bytes(const GroupPlan &g)
{
    GroupBufs b;
    return group_carve(g, nullptr, b);
}

template <class Key>
__global__ __launch_bounds__(kGrpThreads) void k_grp_hist(Key key, GroupPlan g, int *__restrict__ h)
{
    extern __shared__ int cnt[];  // g.B
    for (int b = threadIdx.x; b < g.B; b += kGrpThreads) cnt[b] = 0;
    __syncthreads();
    const int t = xcd_block(blockIdx.x, gridDim.x);  // neighbouring tiles on one die
    const long long base = (long long)t * kGrpTile;
#pragma unroll 4
    for (int k = 0; k < kGrpItems; ++k) {
        const long long i = base + (long long)k * kGrpThreads + threadIdx.x;
        const int e = i < g.n ? key((int)i) : -1;
        if (e >= 0) atomicAdd(&cnt[e >> g.shift], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < g.B; b += kGrpThreads) h[(long long)b * g.T + t] = cnt[b];
}

// Exclusive scan of cnt[0..m) in LDS by one block of kGrpThreads threads
// (each thread a contiguous run of entries); cnt holds the offsets
// afterwards.  Called by every thread of the block.
__device__ __forceinline__ void grp_block_scan(int *cnt, int m)
{
    __shared__ int part[kGrpThreads];
    const int per = (m + kGrpThreads - 1) / kGrpThreads;
    const int b = threadIdx.x * per;
    int s = 0;
    for (int i = 0; i < per; ++i)
        if (b + i < m) s += cnt[b + i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < kWave) {  // the 256 partial sums, 4 per lane of one wavefront
        int v[4], t = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            v[r] = part[4 * threadIdx.x + r];
            t += v[r];
        }
        int inc = t;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(inc, o, kWave);
            if ((int)threadIdx.x >= o) inc += y;
        }
        int ex = inc - t;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            part[4 * threadIdx.x + r] = ex;
            ex += v[r];
        }
    }
    __syncthreads();
    int off = part[threadIdx.x];
    for (int i = 0; i < per; ++i)
        if (b + i < m) {
            const int v = cnt[b + i];
            cnt[b + i] = off;
            off += v;
        }
    __syncthreads();
}

// Per tile: the tile's items are first ordered by bucket in LDS (local
// index, 16 bits), then written out in that order, so that consecutive
// lanes store consecutive entries of one run.
template <class Key>
__global__ __launch_bounds__(kGrpThreads) void k_grp_scatter(Key key, GroupPlan g,
                                                             const int *__restrict__ hoff,
                                                             int *__restrict__ items_b,
                                                             int *__restrict__ keys_b,
                                                             int *__restrict__ posb)
{
    static_assert(kGrpTile <= 65536, "local indices are 16-bit");
    extern __shared__ int lds[];
    int *start = lds;                                // g.B: tile-local start of each bucket
    int *gbase = lds + g.B;                          // g.B: bucket-order index minus local start
    unsigned short *sorted = (unsigned short *)(lds + 2 * g.B);  // kGrpTile local indices
    // neighbouring tiles on one die: their runs of a bucket are adjacent, so
    // that die's L2 gathers the partial lines
    const int t = xcd_block(blockIdx.x, gridDim.x);
    const long long base = (long long)t * kGrpTile;
    for (int b = threadIdx.x; b < g.B; b += kGrpThreads) start[b] = 0;
    __syncthreads();
    int bk[kGrpItems];
#pragma unroll
    for (int k = 0; k < kGrpItems; ++k) {
        const long long i = base + (long long)k * kGrpThreads + threadIdx.x;
        const int e = i < g.n ? key((int)i) : -1;
        bk[k] = e >= 0 ? e >> g.shift : -1;
        if (e >= 0) atomicAdd(&start[bk[k]], 1);
    }
    __syncthreads();
    grp_block_scan(start, g.B);
    for (int b = threadIdx.x; b < g.B; b += kGrpThreads)
        gbase[b] = hoff[(long long)b * g.T + t] - start[b];
    __syncthreads();
    // local positions: start[b] advances as the bucket's entries are taken;
    // each item's bucket-order index is stored in item order (coalesced)
#pragma unroll
    for (int k = 0; k < kGrpItems; ++k) {
        const int li = k * kGrpThreads + (int)threadIdx.x;
        const int lp = wave_rank(start, bk[k], bk[k] >= 0);  // converged: uniform loop
        if (bk[k] >= 0) sorted[lp] = (unsigned short)li;
        if (base + li < g.n) posb[base + li] = bk[k] >= 0 ? gbase[bk[k]] + lp : -1;
    }
    __syncthreads();
    // kept items of the tile: the last bucket's end
    const int kept = start[g.B - 1];
    for (int lp = threadIdx.x; lp < kept; lp += kGrpThreads) {
        const int i = (int)(base + sorted[lp]);
        const int e = key(i);  // the tile's keys again (cache-resident)
        const int j = gbase[e >> g.shift] + lp;
        items_b[j] = i;
        keys_b[j] = e;
    }
}

// Chunk table: bucket b's items are cut into ceil(size_b / kGrpChunk) chunks,
// cstart[b] = chunks of the buckets before b, cstart[B] = all chunks.  One
// block of kGrpMaxBuckets threads, one per bucket.
__global__ __launch_bounds__(kGrpMaxBuckets) void k_grp_chunks(GroupPlan g,
                                                              const int *__restrict__ hoff,
                                                              int *__restrict__ cstart)
{
    __shared__ int wsum[kGrpMaxBuckets / kWave];
    const int b = threadIdx.x, lane = b & (kWave - 1), w = b / kWave;
    int nc = 0;
    if (b < g.B) {
        const int size = hoff[(long long)(b + 1) * g.T] - hoff[(long long)b * g.T];
        nc = (size + kGrpChunk - 1) / kGrpChunk;
    }
    int inc = nc;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += y;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int before = 0;
    for (int k = 0; k < w; ++k) before += wsum[k];
    inc += before;
    if (b < g.B) cstart[b] = inc - nc;
    if (b == g.B - 1) cstart[g.B] = inc;
}

// Bucket of chunk c: the last b with cstart[b] <= c (empty buckets repeat
// the next bucket's start and are passed over).
__device__ __forceinline__ int grp_bucket_of(const int *cstart, int B, int c)
{
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cstart[mid] <= c)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Per chunk: key counts in LDS (ranks within the chunk from the same LDS
// atomics), written key-major within the bucket: gcnt[KB cstart[b] + k nc_b +
// ci] for local key k and chunk ci of bucket b.  One exclusive scan of gcnt
// then orders the list by bucket, key and chunk.
__global__ __launch_bounds__(kGrpThreads) void k_grp_lcount(GroupPlan g, const int *__restrict__ hoff,
                                                            const int *__restrict__ cstart,
                                                            const int *__restrict__ keys_b,
                                                            int *__restrict__ rank_b,
                                                            int *__restrict__ gcnt)
{
    extern __shared__ int cnt[];  // 1 << g.shift keys of the bucket
    const int c = xcd_block(blockIdx.x, gridDim.x);  // a bucket's chunks on one die
    if (c >= cstart[g.B]) return;
    const int b = grp_bucket_of(cstart, g.B, c), KB = 1 << g.shift;
    const int ci = c - cstart[b], nc = cstart[b + 1] - cstart[b];
    const int beg = hoff[(long long)b * g.T] + ci * kGrpChunk;
    const int end = min(beg + kGrpChunk, hoff[(long long)(b + 1) * g.T]);
    for (int k = threadIdx.x; k < KB; k += kGrpThreads) cnt[k] = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kGrpChunk / kGrpThreads; ++q) {
        const int j = beg + q * kGrpThreads + (int)threadIdx.x;
        const int k = j < end ? (keys_b[j] & (KB - 1)) : -1;
        const int r = wave_rank(cnt, k, j < end);  // converged: uniform loop
        if (j < end) rank_b[j] = r;
    }
    __syncthreads();
    int *dst = gcnt + (long long)KB * cstart[b] + ci;
    for (int k = threadIdx.x; k < KB; k += kGrpThreads) dst[(long long)k * nc] = cnt[k];
}

// Per chunk: each item to its key's run, at the chunk's offset for that key
// plus its rank in the chunk.  The chunk is first ordered by key in LDS
// (local index, 16 bits), so that consecutive lanes store consecutive
// entries of a run.
__global__ __launch_bounds__(kGrpThreads) void k_grp_lplace(GroupPlan g, const int *__restrict__ hoff,
                                                            const int *__restrict__ cstart,
                                                            const int *__restrict__ items_b,
                                                            const int *__restrict__ keys_b,
                                                            const int *__restrict__ rank_b,
                                                            const int *__restrict__ goff,
                                                            int *__restrict__ order,
                                                            int *__restrict__ slot)
{
    static_assert(kGrpChunk <= 65536, "local indices are 16-bit");
    extern __shared__ int lds[];
    const int KB = 1 << g.shift;
    int *start = lds;        // KB: chunk-local start of each key
    int *gofs = lds + KB;    // KB: list position minus chunk-local start
    unsigned short *sorted = (unsigned short *)(lds + 2 * KB);  // kGrpChunk
    const int c = xcd_block(blockIdx.x, gridDim.x);  // a bucket's window in one L2
    if (c >= cstart[g.B]) return;
    const int b = grp_bucket_of(cstart, g.B, c);
    const int ci = c - cstart[b], nc = cstart[b + 1] - cstart[b];
    const int beg = hoff[(long long)b * g.T] + ci * kGrpChunk;
    const int end = min(beg + kGrpChunk, hoff[(long long)(b + 1) * g.T]);
    for (int k = threadIdx.x; k < KB; k += kGrpThreads) start[k] = 0;
    __syncthreads();
    constexpr int U = kGrpChunk / kGrpThreads;
    int kk[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
        const int j = beg + q * kGrpThreads + (int)threadIdx.x;
        kk[q] = j < end ? (keys_b[j] & (KB - 1)) : -1;
        if (kk[q] >= 0) atomicAdd(&start[kk[q]], 1);
    }
    __syncthreads();
    grp_block_scan(start, KB);
    const int *src = goff + (long long)KB * cstart[b] + ci;
    for (int k = threadIdx.x; k < KB; k += kGrpThreads) gofs[k] = src[(long long)k * nc] - start[k];
#pragma unroll
    for (int q = 0; q < U; ++q) {
        const int j = beg + q * kGrpThreads + (int)threadIdx.x;
        if (kk[q] >= 0) sorted[start[kk[q]] + rank_b[j]] = (unsigned short)(j - beg);
    }
    __syncthreads();
    for (int lp = threadIdx.x; lp < end - beg; lp += kGrpThreads) {
        const int j = beg + sorted[lp];
        const int u = gofs[keys_b[j] & (KB - 1)] + lp;
        order[u] = items_b[j];
        slot[u] = j;
    }
}

// Key offsets: the first chunk's offset of each key; keys of an empty bucket
// start where the bucket starts.
__global__ __launch_bounds__(kGrpThreads) void k_grp_off(GroupPlan g, const int *__restrict__ hoff,
                                                         const int *__restrict__ cstart,
                                                         const int *__restrict__ goff,
                                                         int *__restrict__ off)
{
    const int e = blockIdx.x * kGrpThreads + threadIdx.x;
    if (e > g.K) return;
    if (e == g.K) {
        off[e] = hoff[(long long)g.B * g.T];
        return;
    }
    const int b = e >> g.shift, KB = 1 << g.shift;
    const int nc = cstart[b + 1] - cstart[b];
    off[e] = nc ? goff[(long long)KB * cstart[b] + (long long)(e & (KB - 1)) * nc]
                : hoff[(long long)b * g.T];
}

// Groups the n items of the plan by key on stream s.  b holds the result
// arrays (off and cnt: K + 1, order/slot/posb: n) and transient arrays carved
// by group_carve.
template <class Key>
hipError_t group_by_key(const Key &key, const GroupPlan &g, const GroupBufs &b, hipStream_t s)
{
    const size_t shb = (size_t)g.B * sizeof(int);
    k_grp_hist<Key><<<g.T, kGrpThreads, shb, s>>>(key, g, b.h);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_exclusive(b.h, b.hoff, g.B * g.T, b.scan_tmp, s);
    if (e != hipSuccess) return e;
    const size_t shs = 2 * shb + kGrpTile * sizeof(unsigned short);
    k_grp_scatter<Key><<<g.T, kGrpThreads, shs, s>>>(key, g, b.hoff, b.items_b, b.keys_b, b.posb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_grp_chunks<<<1, kGrpMaxBuckets, 0, s>>>(g, b.hoff, b.cstart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nch = g.B + (g.n + kGrpChunk - 1) / kGrpChunk;  // bound on the chunks
    const size_t shk = (size_t)sizeof(int) << g.shift;
    k_grp_lcount<<<nch, kGrpThreads, shk, s>>>(g, b.hoff, b.cstart, b.keys_b, b.rank_b, b.gcnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = scan_exclusive(b.gcnt, b.goff, (int)grp_gcnt_size(g), b.scan_tmp, s);
    if (e != hipSuccess) return e;
    const size_t shp = 2 * shk + kGrpChunk * sizeof(unsigned short);
    k_grp_lplace<<<nch, kGrpThreads, shp, s>>>(g, b.hoff, b.cstart, b.items_b, b.keys_b, b.rank_b,
                                             b.goff, b.order, b.slot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_grp_off<<<(g.K + kGrpThreads) / kGrpThreads, kGrpThreads, 0, s>>>(g, b.hoff, b.cstart,
                                                                        b.goff, b.off);
    return hipGetLastError();
}

}  // namespace fp
