// contour_reorder.hip -- group the edge list by blocks of source ids.
//
// The asynchronous sweep may take the edges in any order (Section III-B-1),
// so a solve may work on a copy of the edge list that is grouped by the
// source block b = src >> shift (at most 1024 blocks).  Neighbouring edges of
// the copy then gather labels from a narrow id range, which the sweep stages
// in LDS.  The order of the edges inside a block is left free.
//
// One counting pass and one scatter pass:
//   count    a histogram of the blocks (per-workgroup LDS histograms, then
//            one global atomic add per block and workgroup);
//   scan     one workgroup turns it into the first slot of every block and
//            sets each block's cursor there;
//   scatter  a workgroup loads 16 Ki edges, ranks them by block in LDS
//            (LDS atomics), reserves each block's run of slots with one
//            global atomic add on the block's cursor, places the edges in
//            block order in LDS and writes them out with consecutive lanes
//            on consecutive slots, so each block's run (16 edges on average
//            for 1024 blocks) is stored as contiguous words.
// An id outside [0, n) goes to the last block unchanged; the sweep's own
// range check rejects it.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "contour_runtime.hpp"

namespace contour {

static constexpr int kMaxBuckets = 1024;
static constexpr int kThreads = 1024;                       // count, scan and scatter workgroups
static constexpr int kCountPer = 32;                        // edges per thread of the count pass
static constexpr int kScatterPer = 16;                      // edges per thread of the scatter pass
static constexpr int kScatterChunk = kThreads * kScatterPer;  // 16 Ki edges per scatter workgroup
// dynamic LDS of the scatter: the chunk in block order (src and dst)
static constexpr size_t kScatterLds = (size_t)kScatterChunk * 2 * sizeof(int);

__device__ __forceinline__ int block_of(int w, int shift, int K)
{
    const unsigned b = (unsigned)w >> shift;
    return b < (unsigned)K ? (int)b : K - 1;
}

__global__ __launch_bounds__(kThreads) void k_blk_count(const int* __restrict__ src, long long m, int shift, int K,
                                                        int* __restrict__ hist)
{
    __shared__ int h[kMaxBuckets];
    for (int i = threadIdx.x; i < K; i += kThreads) h[i] = 0;
    __syncthreads();
    const long long e0 = (long long)blockIdx.x * kThreads * kCountPer;
    int w[kCountPer];
#pragma unroll
    for (int k = 0; k < kCountPer; ++k)
        w[k] = ld_edge(src + std::min(e0 + (long long)k * kThreads + threadIdx.x, m - 1));
#pragma unroll
    for (int k = 0; k < kCountPer; ++k)
        if (e0 + (long long)k * kThreads + threadIdx.x < m) atomicAdd(&h[block_of(w[k], shift, K)], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < K; i += kThreads)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Inclusive scan of v over the workgroup's threads (kThreads of them);
// `tot` is LDS scratch of one int per wave.
__device__ __forceinline__ int block_inclusive_scan(int v, int* tot)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int x = __shfl_up(v, off, 64);
        if (lane >= off) v += x;
    }
    if (lane == 63) tot[wave] = v;
    __syncthreads();
    int add = 0;
    for (int k = 0; k < wave; ++k) add += tot[k];
    return v + add;
}

// One workgroup: first slot of every block, and the scatter's cursors.
__global__ __launch_bounds__(kThreads) void k_blk_scan(const int* __restrict__ hist, int K, int* __restrict__ cursor)
{
    __shared__ int tot[kThreads / 64];
    const int b = threadIdx.x;
    const int c = b < K ? hist[b] : 0;
    const int incl = block_inclusive_scan(c, tot);
    if (b < K) cursor[b] = incl - c;
}

__global__ __launch_bounds__(kThreads) void k_blk_scatter(const int* __restrict__ src, const int* __restrict__ dst,
                                                          long long m, int shift, int K, int* __restrict__ cursor,
                                                          int* __restrict__ osrc, int* __restrict__ odst)
{
    extern __shared__ __align__(16) int lds[];
    int* out_s = lds;
    int* out_d = lds + kScatterChunk;
    __shared__ int cnt[kMaxBuckets];    // edges of the chunk per block, then rank cursor
    __shared__ int lstart[kMaxBuckets]; // first position of each block in the chunk
    __shared__ int gbase[kMaxBuckets];  // first global slot of the chunk's run of each block
    __shared__ int tot[kThreads / 64];
    const int t = threadIdx.x;
    const long long e0 = (long long)blockIdx.x * kScatterChunk;
    const int len = (int)std::min<long long>(kScatterChunk, m - e0);
    for (int i = t; i < K; i += kThreads) cnt[i] = 0;
    int es[kScatterPer], ed[kScatterPer];
#pragma unroll
    for (int k = 0; k < kScatterPer; ++k) {
        const int i = std::min(k * kThreads + t, len - 1);
        es[k] = ld_edge(src + e0 + i);
        ed[k] = ld_edge(dst + e0 + i);
    }
    __syncthreads();
    int rank[kScatterPer];
#pragma unroll
    for (int k = 0; k < kScatterPer; ++k)
        rank[k] = k * kThreads + t < len ? atomicAdd(&cnt[block_of(es[k], shift, K)], 1) : 0;
    __syncthreads();
    // positions of the blocks inside the chunk, and their global runs
    const int c = t < K ? cnt[t] : 0;
    const int incl = block_inclusive_scan(c, tot);
    if (t < K) {
        lstart[t] = incl - c;
        gbase[t] = c ? atomicAdd(&cursor[t], c) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScatterPer; ++k) {
        if (k * kThreads + t < len) {
            const int pos = lstart[block_of(es[k], shift, K)] + rank[k];
            out_s[pos] = es[k];
            out_d[pos] = ed[k];
        }
    }
    __syncthreads();
    for (int i = t; i < len; i += kThreads) {
        const int w = out_s[i];
        const int b = block_of(w, shift, K);
        const int slot = gbase[b] + (i - lstart[b]);
        osrc[slot] = w;
        odst[slot] = out_d[i];
    }
}

// Zero the histogram (a kernel rather than a memset, so that the sequence
// can be captured in a graph).
__global__ void k_blk_zero(int* __restrict__ hist, int K)
{
    for (int i = threadIdx.x; i < K; i += blockDim.x) hist[i] = 0;
}

void reorder_geometry(const DeviceInfo& d, long long m, int n, Reorder* r)
{
    (void)d;
    // the scatter stages 128 KiB of edges in LDS (set on the current device)
    (void)hipFuncSetAttribute((const void*)k_blk_scatter, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kScatterLds);
    int shift = 0;
    while (((unsigned)(n - 1) >> shift) >= (unsigned)kMaxBuckets) ++shift;
    r->shift = shift;
    r->K = (int)(((unsigned)(n - 1) >> shift) + 1);
    r->m = m;
    // every array starts on a 16-byte boundary (the sweep reads edges with
    // 16-byte loads when it can)
    const long long mp = (m + 3) & ~3LL;
    r->elems = 2 * mp + 2 * kMaxBuckets;
}

void reorder_bind(Reorder* r, int* ws)
{
    const long long mp = (r->m + 3) & ~3LL;
    r->src2 = ws;
    r->dst2 = ws + mp;
    r->hist = ws + 2 * mp;
    r->cursor = r->hist + kMaxBuckets;
}

int enqueue_reorder(const Reorder& r, const int* src, const int* dst, hipStream_t stream)
{
    if (r.m <= 0) return CONTOUR_OK;
    const unsigned gc = (unsigned)((r.m + (long long)kThreads * kCountPer - 1) / ((long long)kThreads * kCountPer));
    const unsigned gs = (unsigned)((r.m + kScatterChunk - 1) / kScatterChunk);
    hipLaunchKernelGGL(k_blk_zero, dim3(1), dim3(kThreads), 0, stream, r.hist, r.K);
    hipLaunchKernelGGL(k_blk_count, dim3(gc), dim3(kThreads), 0, stream, src, r.m, r.shift, r.K, r.hist);
    hipLaunchKernelGGL(k_blk_scan, dim3(1), dim3(kThreads), 0, stream, (const int*)r.hist, r.K, r.cursor);
    hipLaunchKernelGGL(k_blk_scatter, dim3(gs), dim3(kThreads), kScatterLds, stream, src, dst, r.m, r.shift, r.K,
                       r.cursor, r.src2, r.dst2);
    CONTOUR_HIP(hipGetLastError());
    return CONTOUR_OK;
}

}  // namespace contour
