// Device utilities: exclusive prefix sum, fill, copy, error state.
#include <cstdio>
#include <string>

#include "fp_internal.h"

namespace fp {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return FP_ENOMEM;
    return FP_EHIP;
}

// ---------------------------------------------------------------------------
// Exclusive scan, three launches: tile sums, scan of the tile sums in one
// block, tile-local scan plus the tile's offset.  A tile is 256 threads x 16
// items.  Wave-level inclusive scans use cross-lane shuffles (wave64).
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the thread's
// exclusive prefix and writes the block total.
__device__ __forceinline__ int block_excl_scan(int v, int *total)
{
    __shared__ int wsum[kScanThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        if (i < w) off += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(
    const int *__restrict__ in, int n, int *__restrict__ tsum, const int *__restrict__ gate)
{
    if (gate && !*gate) return;
    const long long base = (long long)blockIdx.x * kScanTile;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long long i = base + (long long)k * kScanThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    int tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(int *__restrict__ tsum,
                                                           int nt, const int *__restrict__ gate)
{
    if (gate && !*gate) return;
    // each thread scans a contiguous run of tile sums
    const int per = (nt + kScanThreads - 1) / kScanThreads;
    const int b = threadIdx.x * per;
    int s = 0;
    for (int i = 0; i < per; ++i)
        if (b + i < nt) s += tsum[b + i];
    int tot;
    int off = block_excl_scan(s, &tot);
    for (int i = 0; i < per; ++i)
        if (b + i < nt) {
            int v = tsum[b + i];
            tsum[b + i] = off;
            off += v;
        }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(
    const int *__restrict__ in, int n, const int *__restrict__ toff,
    int *__restrict__ out, int nt, const int *__restrict__ gate)
{
    if (gate && !*gate) return;
    const long long base = (long long)blockIdx.x * kScanTile;
    // each thread owns kScanItems consecutive items
    const long long my = base + (long long)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long long i = my + k;
        v[k] = (i < n) ? in[i] : 0;
        s += v[k];
    }
    int tot;
    int off = block_excl_scan(s, &tot) + toff[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long long i = my + k;
        if (i < n) out[i] = off;
        off += v[k];
    }
    if (blockIdx.x == nt - 1 && threadIdx.x == kScanThreads - 1) out[n] = off;
}

__global__ void k_zero_total(int *out, int n) { out[n] = 0; }

int scan_tmp_size(long long n) { return (int)((n + kScanTile - 1) / kScanTile) + 1; }

hipError_t scan_exclusive(const int *in, int *out, int n, int *tmp, hipStream_t s,
                          const int *gate)
{
    if (n <= 0) {
        k_zero_total<<<1, 1, 0, s>>>(out, 0);
        return hipGetLastError();
    }
    const int nt = (n + kScanTile - 1) / kScanTile;
    k_scan_tiles<<<nt, kScanThreads, 0, s>>>(in, n, tmp, gate);
    k_scan_top<<<1, kScanThreads, 0, s>>>(tmp, nt, gate);
    k_scan_down<<<nt, kScanThreads, 0, s>>>(in, n, tmp, out, nt, gate);
    return hipGetLastError();
}

__global__ void k_fill_int(int *__restrict__ p, int v, long long n, const int *__restrict__ gate)
{
    if (gate && !*gate) return;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

hipError_t fill_int(int *p, int value, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_fill_int<<<(int)blocks, 256, 0, s>>>(p, value, n, nullptr);
    return hipGetLastError();
}

hipError_t fill_int_gated(int *p, int value, long long n, const int *gate, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_fill_int<<<(int)blocks, 256, 0, s>>>(p, value, n, gate);
    return hipGetLastError();
}

// Plain streaming copy, 16 bytes per lane per iteration (grid-stride).
__global__ __launch_bounds__(256) void k_copy16(const uint4 *__restrict__ a,
                                               uint4 *__restrict__ b, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) b[i] = a[i];
}

}  // namespace fp

extern "C" const char *fp_last_error(void) { return fp::g_err.c_str(); }

extern "C" int fp_copy(const void *src, void *dst, size_t bytes, void *stream)
{
    if (!src || !dst || (bytes & 15) || (((uintptr_t)src | (uintptr_t)dst) & 15)) {
        fp::set_error("fp_copy: pointers must be 16-byte aligned and bytes a multiple of 16");
        return FP_EINVAL;
    }
    long long n = (long long)(bytes / 16);
    if (n == 0) return FP_OK;
    long long blocks = (n + 255) / 256;
    if (blocks > 256 * 32) blocks = 256 * 32;
    fp::k_copy16<<<(int)blocks, 256, 0, (hipStream_t)stream>>>(
        (const uint4 *)src, (uint4 *)dst, n);
    FP_HIP(hipGetLastError());
    return FP_OK;
}
