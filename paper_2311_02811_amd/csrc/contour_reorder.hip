// contour_reorder.hip -- group the edge list by blocks of source ids.
//
// The asynchronous sweep may take the edges in any order (Section III-B-1),
// so a solve may work on a copy of the edge list that is grouped by
// src >> shift into at most 1024 buckets.  Neighbouring edges of the copy
// then gather labels from a narrow id range and share cache lines, instead
// of every gather touching its own line of the label array.
//
// A counting sort, three kernels and a scan:
//   count    workgroup g counts the bucket of every edge of its contiguous
//            chunk into LDS and writes the counts to column g of a
//            bucket-major matrix counts[b * G + g];
//   scan     exclusive prefix sum of the matrix in that (bucket-major) order
//            gives workgroup g the first slot of each of its buckets;
//   scatter  workgroup g walks its chunk again and writes each edge at its
//            bucket's next slot (an LDS cursor per bucket).
// An id outside [0, n) goes to the last bucket unchanged; the sweep's own
// range check then rejects it.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "contour_runtime.hpp"

namespace contour {

static constexpr int kMaxBuckets = 1024;
static constexpr int kScanThreads = 1024;
static constexpr int kScanPerThread = 8;
static constexpr long long kScanSegment = (long long)kScanThreads * kScanPerThread;

__device__ __forceinline__ int bucket_of(int w, int shift, int K)
{
    const unsigned b = (unsigned)w >> shift;
    return b < (unsigned)K ? (int)b : K - 1;
}

__global__ __launch_bounds__(256) void k_bucket_count(const int* __restrict__ src, long long m, long long chunk,
                                                      int shift, int K, int* __restrict__ counts)
{
    __shared__ int h[kMaxBuckets];
    for (int i = threadIdx.x; i < K; i += 256) h[i] = 0;
    __syncthreads();
    const long long e0 = (long long)blockIdx.x * chunk;
    const long long e1 = std::min(m, e0 + chunk);
    for (long long e = e0 + threadIdx.x; e < e1; e += 256) atomicAdd(&h[bucket_of(ld_edge(src + e), shift, K)], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < K; i += 256) counts[(long long)i * gridDim.x + blockIdx.x] = h[i];
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
    __shared__ int scratch_sums[kScanThreads];
    const long long base = (long long)threadIdx.x * kScanPerThread;
    int v[kScanPerThread];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        v[k] = base + k < nblk ? sums[base + k] : 0;
        s += v[k];
    }
    scratch_sums[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int t = threadIdx.x >= (unsigned)off ? scratch_sums[threadIdx.x - off] : 0;
        __syncthreads();
        scratch_sums[threadIdx.x] += t;
        __syncthreads();
    }
    int run = threadIdx.x ? scratch_sums[threadIdx.x - 1] : 0;
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

__global__ __launch_bounds__(256) void k_bucket_scatter(const int* __restrict__ src, const int* __restrict__ dst,
                                                        long long m, long long chunk, int shift, int K,
                                                        const int* __restrict__ offsets, int* __restrict__ src2,
                                                        int* __restrict__ dst2)
{
    __shared__ int cur[kMaxBuckets];
    for (int i = threadIdx.x; i < K; i += 256) cur[i] = offsets[(long long)i * gridDim.x + blockIdx.x];
    __syncthreads();
    const long long e0 = (long long)blockIdx.x * chunk;
    const long long e1 = std::min(m, e0 + chunk);
    for (long long e = e0 + threadIdx.x; e < e1; e += 256) {
        const int w = ld_edge(src + e);
        const int v = ld_edge(dst + e);
        const int pos = atomicAdd(&cur[bucket_of(w, shift, K)], 1);
        src2[pos] = w;
        dst2[pos] = v;
    }
}

void reorder_geometry(const DeviceInfo& d, long long m, int n, Reorder* r)
{
    int shift = 0;
    while (((unsigned)(n - 1) >> shift) >= (unsigned)kMaxBuckets) ++shift;
    r->shift = shift;
    r->K = (int)(((unsigned)(n - 1) >> shift) + 1);
    r->G = (int)std::max<long long>(1, std::min<long long>((m + 4095) / 4096, (long long)d.cus * 4));
    r->chunk = (m + r->G - 1) / r->G;
    const long long cells = (long long)r->K * r->G;
    r->nblk = (int)((cells + kScanSegment - 1) / kScanSegment);
    r->m = m;
    r->elems = 2 * m + cells + r->nblk;
}

void reorder_bind(Reorder* r, int* ws)
{
    r->src2 = ws;
    r->dst2 = ws + r->m;
    r->counts = ws + 2 * r->m;
    r->sums = r->counts + (long long)r->K * r->G;
}

int enqueue_reorder(const Reorder& r, const int* src, const int* dst, hipStream_t stream)
{
    const long long cells = (long long)r.K * r.G;
    hipLaunchKernelGGL(k_bucket_count, dim3(r.G), dim3(256), 0, stream, src, r.m, r.chunk, r.shift, r.K, r.counts);
    hipLaunchKernelGGL(k_scan_local, dim3(r.nblk), dim3(kScanThreads), 0, stream, r.counts, cells, r.sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, stream, r.sums, r.nblk);
    hipLaunchKernelGGL(k_scan_add, dim3(r.nblk), dim3(kScanThreads), 0, stream, r.counts, cells, (const int*)r.sums);
    hipLaunchKernelGGL(k_bucket_scatter, dim3(r.G), dim3(256), 0, stream, src, dst, r.m, r.chunk, r.shift, r.K,
                       (const int*)r.counts, r.src2, r.dst2);
    CONTOUR_HIP(hipGetLastError());
    return CONTOUR_OK;
}

}  // namespace contour
