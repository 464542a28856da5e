// contour_reorder.hip -- group the edge list by blocks of source ids.
//
// The asynchronous sweep may take the edges in any order (Section III-B-1),
// so a solve may work on a copy of the edge list that is grouped by the
// source block b = src >> shift (at most 1024 blocks).  Neighbouring edges of
// the copy then gather labels from a narrow id range, which the sweep stages
// in LDS.
//
// The grouping is a stable least-significant-digit radix partition of b in
// 5-bit digits (two passes for 1024 blocks).  Each pass:
//   count    workgroup g counts the digits of its chunk of 2048 edges into
//            counts[d * G + g] (digit-major);
//   scan     an exclusive prefix sum of that matrix gives workgroup g the
//            first output slot of each digit;
//   scatter  workgroup g loads its chunk into LDS, ranks it by digit there
//            (stable: each thread owns eight consecutive edges and a column
//            of per-digit counters), places it in rank order in LDS, and
//            then writes it out with consecutive lanes on consecutive
//            ranks, so each digit's run (64 edges on average) is stored as
//            contiguous words rather than scattered ones.
// An id outside [0, n) goes to the last block unchanged; the sweep's own
// range check rejects it.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "contour_runtime.hpp"

namespace contour {

static constexpr int kMaxBuckets = 1024;
static constexpr int kDigitBits = 5;
static constexpr int kDigits = 1 << kDigitBits;
static constexpr int kRxThreads = 256;
static constexpr int kRxPer = 8;
static constexpr int kRxChunk = kRxThreads * kRxPer;  // 2048 edges per workgroup
static constexpr int kScanThreads = 1024;
static constexpr int kScanPerThread = 8;
static constexpr long long kScanSegment = (long long)kScanThreads * kScanPerThread;

// Chunk handled by workgroup `blk` of `G`.  Workgroups are dispatched to the
// eight XCDs round-robin; this mapping gives each XCD a contiguous range of
// chunks, so the pieces of a digit's output run written by neighbouring
// chunks are mostly written through the same L2 and merge into whole lines.
__device__ __forceinline__ long long chunk_of(unsigned blk, unsigned G)
{
    const unsigned per = (G + 7) / 8;
    const unsigned x = blk % 8, k = blk / 8;
    const unsigned full = G - (per - 1) * 8;  // XCDs that get `per` chunks (the rest get per - 1)
    const unsigned start = x < full ? x * per : full * per + (x - full) * (per - 1);
    return (long long)(start + k);
}

__device__ __forceinline__ int digit_of(int w, int shift, int K, int pass)
{
    const unsigned b0 = (unsigned)w >> shift;
    const unsigned b = b0 < (unsigned)K ? b0 : (unsigned)(K - 1);
    return (int)((b >> (kDigitBits * pass)) & (kDigits - 1));
}

__global__ __launch_bounds__(kRxThreads) void k_rx_count(const int* __restrict__ src, long long m, int shift,
                                                         int K, int pass, int* __restrict__ counts)
{
    __shared__ int h[kDigits];
    if (threadIdx.x < kDigits) h[threadIdx.x] = 0;
    __syncthreads();
    const long long c = chunk_of(blockIdx.x, gridDim.x);
    const long long e0 = c * kRxChunk;
    const int len = (int)std::min<long long>(kRxChunk, m - e0);
    int w[kRxPer];
#pragma unroll
    for (int k = 0; k < kRxPer; ++k) w[k] = ld_edge(src + e0 + min(k * kRxThreads + (int)threadIdx.x, len - 1));
#pragma unroll
    for (int k = 0; k < kRxPer; ++k)
        if (k * kRxThreads + (int)threadIdx.x < len) atomicAdd(&h[digit_of(w[k], shift, K, pass)], 1);
    __syncthreads();
    if (threadIdx.x < kDigits) counts[(long long)threadIdx.x * gridDim.x + c] = h[threadIdx.x];
}

// Exclusive scan, level 1: each block scans kScanSegment elements in place
// and writes its total to sums[block].
__global__ __launch_bounds__(kScanThreads) void k_scan_local(int* a, long long len, int* sums)
{
    __shared__ int tot[kScanThreads];
    const long long base = (long long)blockIdx.x * kScanSegment + (long long)threadIdx.x * kScanPerThread;
    int v[kScanPerThread];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        v[k] = base + k < len ? a[base + k] : 0;
        s += v[k];
    }
    tot[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int t = threadIdx.x >= (unsigned)off ? tot[threadIdx.x - off] : 0;
        __syncthreads();
        tot[threadIdx.x] += t;
        __syncthreads();
    }
    int run = threadIdx.x ? tot[threadIdx.x - 1] : 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        if (base + k < len) a[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = tot[kScanThreads - 1];
}

// Level 2: exclusive scan of the block totals (at most kScanSegment of them)
// by a single block.
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int* sums, int nblk)
{
    __shared__ int tot[kScanThreads];
    const long long base = (long long)threadIdx.x * kScanPerThread;
    int v[kScanPerThread];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        v[k] = base + k < nblk ? sums[base + k] : 0;
        s += v[k];
    }
    tot[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int t = threadIdx.x >= (unsigned)off ? tot[threadIdx.x - off] : 0;
        __syncthreads();
        tot[threadIdx.x] += t;
        __syncthreads();
    }
    int run = threadIdx.x ? tot[threadIdx.x - 1] : 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        if (base + k < nblk) sums[base + k] = run;
        run += v[k];
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int* a, long long len, const int* sums)
{
    const int add = sums[blockIdx.x];
    const long long base = (long long)blockIdx.x * kScanSegment;
    for (long long i = threadIdx.x; i < kScanSegment; i += kScanThreads)
        if (base + i < len) a[base + i] += add;
}

// Counter matrix of the scatter, cnt[d * threads + t], stored with one
// padding word after every 32 so that a thread walking 32 consecutive
// entries and its neighbours walking theirs hit different LDS banks.
__device__ __forceinline__ int padded(int i) { return i + (i >> 5); }
static constexpr int kRxCells = kDigits * kRxThreads;
static constexpr int kRxCellsPadded = kRxCells + kRxCells / 32;

__global__ __launch_bounds__(kRxThreads) void k_rx_scatter(const int* __restrict__ src, const int* __restrict__ dst,
                                                           long long m, int shift, int K, int pass,
                                                           const int* __restrict__ offsets, int* __restrict__ osrc,
                                                           int* __restrict__ odst)
{
    __shared__ int in_s[kRxChunk], in_d[kRxChunk];
    // the counters, later reused for the output slot of each sorted edge
    __shared__ int cnt[kRxCellsPadded];
    __shared__ int tot[kRxThreads];
    __shared__ int dstart[kDigits];
    __shared__ int gbase[kDigits];
    const int t = threadIdx.x;
    const long long c = chunk_of(blockIdx.x, gridDim.x);
    const long long e0 = c * kRxChunk;
    const int len = (int)std::min<long long>(kRxChunk, m - e0);
    {
        // every load of the chunk in flight at once (indices past the end
        // re-read the last edge and store it again in its own slot)
        int vs[kRxPer], vd[kRxPer];
#pragma unroll
        for (int k = 0; k < kRxPer; ++k) {
            const int i = min(k * kRxThreads + t, len - 1);
            vs[k] = ld_edge(src + e0 + i);
            vd[k] = ld_edge(dst + e0 + i);
        }
#pragma unroll
        for (int k = 0; k < kRxPer; ++k) {
            const int i = min(k * kRxThreads + t, len - 1);
            in_s[i] = vs[k];
            in_d[i] = vd[k];
        }
    }
    for (int i = t; i < kRxCellsPadded; i += kRxThreads) cnt[i] = 0;
    // output slots fit int32: reordering is only used for m < 2^31
    if (t < kDigits) gbase[t] = offsets[(long long)t * gridDim.x + c];
    __syncthreads();
    // thread t owns edges [t * kRxPer, (t + 1) * kRxPer) of the chunk
    int es[kRxPer], ed[kRxPer], dig[kRxPer], rank[kRxPer];
#pragma unroll
    for (int k = 0; k < kRxPer; ++k) {
        const int i = t * kRxPer + k;
        es[k] = in_s[min(i, len - 1)];
        ed[k] = in_d[min(i, len - 1)];
        dig[k] = i < len ? digit_of(es[k], shift, K, pass) : -1;
        if (dig[k] >= 0) cnt[padded(dig[k] * kRxThreads + t)] += 1;
    }
    __syncthreads();
    // exclusive scan of cnt in digit-major order: thread t scans entries
    // [t * 32, t * 32 + 32), then the thread totals are scanned
    int run = 0;
    for (int k = 0; k < kDigits; ++k) {
        const int j = padded(t * kDigits + k);
        const int x = cnt[j];
        cnt[j] = run;
        run += x;
    }
    tot[t] = run;
    __syncthreads();
    for (int off = 1; off < kRxThreads; off <<= 1) {
        const int x = t >= off ? tot[t - off] : 0;
        __syncthreads();
        tot[t] += x;
        __syncthreads();
    }
    const int add = t ? tot[t - 1] : 0;
    for (int k = 0; k < kDigits; ++k) cnt[padded(t * kDigits + k)] += add;
    __syncthreads();
    // cnt[d * threads + t] is now the chunk-local rank of thread t's first
    // digit-d edge (stable order), and digit d's run starts at rank
    // dstart[d]
    if (t < kDigits) dstart[t] = cnt[padded(t * kRxThreads)];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRxPer; ++k)
        rank[k] = dig[k] >= 0 ? cnt[padded(dig[k] * kRxThreads + t)]++ : 0;
    __syncthreads();
    // place the chunk in rank order in LDS, with each edge's output slot
    // (its digit's run start plus its offset in the run) in cnt
#pragma unroll
    for (int k = 0; k < kRxPer; ++k) {
        if (dig[k] >= 0) {
            in_s[rank[k]] = es[k];
            in_d[rank[k]] = ed[k];
            cnt[rank[k]] = gbase[dig[k]] + (rank[k] - dstart[dig[k]]);
        }
    }
    __syncthreads();
    // consecutive lanes write consecutive ranks: each digit's run is stored
    // as contiguous words
    for (int i = t; i < len; i += kRxThreads) {
        const int slot = cnt[i];
        osrc[slot] = in_s[i];
        odst[slot] = in_d[i];
    }
}

void reorder_geometry(const DeviceInfo& d, long long m, int n, Reorder* r)
{
    (void)d;
    int shift = 0;
    while (((unsigned)(n - 1) >> shift) >= (unsigned)kMaxBuckets) ++shift;
    r->shift = shift;
    r->K = (int)(((unsigned)(n - 1) >> shift) + 1);
    int passes = 0;
    while ((1 << (kDigitBits * passes)) < r->K) ++passes;
    r->passes = std::max(passes, 1);
    r->G = (int)((m + kRxChunk - 1) / kRxChunk);
    r->chunk = kRxChunk;
    const long long cells = (long long)kDigits * r->G;
    r->nblk = (int)((cells + kScanSegment - 1) / kScanSegment);
    r->m = m;
    // every array starts on a 16-byte boundary (the sweep reads edges with
    // 16-byte loads when it can)
    const long long mp = (m + 3) & ~3LL;
    r->elems = 4 * mp + cells + ((r->nblk + 3) & ~3);
}

void reorder_bind(Reorder* r, int* ws)
{
    const long long mp = (r->m + 3) & ~3LL;
    r->src2 = ws;
    r->dst2 = ws + mp;
    r->tmp_src = ws + 2 * mp;
    r->tmp_dst = ws + 3 * mp;
    r->counts = ws + 4 * mp;
    r->sums = r->counts + (long long)kDigits * r->G;
}

int enqueue_reorder(const Reorder& r, const int* src, const int* dst, hipStream_t stream)
{
    const long long cells = (long long)kDigits * r.G;
    // the last pass writes src2/dst2; earlier passes alternate through tmp
    const int* in_s = src;
    const int* in_d = dst;
    for (int pass = 0; pass < r.passes; ++pass) {
        int* out_s = ((r.passes - 1 - pass) & 1) ? r.tmp_src : r.src2;
        int* out_d = ((r.passes - 1 - pass) & 1) ? r.tmp_dst : r.dst2;
        hipLaunchKernelGGL(k_rx_count, dim3(r.G), dim3(kRxThreads), 0, stream, in_s, r.m, r.shift, r.K, pass, r.counts);
        hipLaunchKernelGGL(k_scan_local, dim3(r.nblk), dim3(kScanThreads), 0, stream, r.counts, cells, r.sums);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, stream, r.sums, r.nblk);
        hipLaunchKernelGGL(k_scan_add, dim3(r.nblk), dim3(kScanThreads), 0, stream, r.counts, cells,
                           (const int*)r.sums);
        hipLaunchKernelGGL(k_rx_scatter, dim3(r.G), dim3(kRxThreads), 0, stream, in_s, in_d, r.m, r.shift, r.K, pass,
                           (const int*)r.counts, out_s, out_d);
        in_s = out_s;
        in_d = out_d;
    }
    CONTOUR_HIP(hipGetLastError());
    return CONTOUR_OK;
}

}  // namespace contour
