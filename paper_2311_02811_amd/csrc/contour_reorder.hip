// contour_reorder.hip -- group the edge list by blocks of source ids.
//
// The asynchronous sweep may take the edges in any order (Section III-B-1),
// so a solve may work on a copy of the edge list that is grouped by the
// source block b = src >> shift (at most 1024 blocks).  Neighbouring edges of
// the copy then gather labels from a narrow id range, which the sweep stages
// in LDS.  The order of the edges inside a block is left free.
//
// The edge list is cut into chunks of 8 Ki edges; the grouped copy holds,
// for every block, the chunks' edges of that block in chunk order:
//   count    per chunk, a histogram of the blocks (LDS), written as one row
//            of the chunk x block count matrix;
//   offsets  per group of 128 chunks, the offset of every (chunk, block)
//            run inside the group's run of the block, written over the count
//            matrix, and the group's total per block;
//   scan     one workgroup: the first slot of every block, and from it the
//            first slot of every (chunk group, block) run;
//   scatter  a workgroup loads one chunk, ranks its edges by block in LDS
//            (LDS atomics), places them in block order in LDS and writes
//            them out with consecutive lanes on consecutive slots (8 edges
//            per block on average for 1024 blocks).  Each XCD takes one
//            eighth of the chunks in order, so the runs of neighbouring
//            chunks, which lie next to each other in the copy, are written
//            through one L2 at about the same time and leave it as whole
//            lines.  A workgroup holds 64 KiB of LDS, so two share a CU and
//            one's loads overlap the other's ranking and writes.
// Every slot is known before the scatter (no global atomics at all), and
// each block lists its edges chunk by chunk
// in input order, which on power-law graphs also saves sweeps (the edges of
// a block keep the input's locality).
//
// Second pass (optional): the grouped copy is grouped again, stably, by
// destination range dst >> dshift (at most 64 ranges), with the same count,
// offsets and scan kernels and a scatter that ranks a chunk's edges in
// element order (wave ballots over the key bits, then a scan over the
// chunk's waves).  The result lists the edges by destination range and,
// within a range, by source block: a task of consecutive edges then gathers
// its source labels from a window in LDS and its destination labels from one
// range that fits an XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "contour_runtime.hpp"

namespace contour {

static constexpr int kMaxBuckets = 1024;
static constexpr int kThreads = 1024;                       // count, scan and scatter workgroups
static constexpr int kScatterPer = 8;                       // edges per thread and chunk
static constexpr int kChunk = kThreads * kScatterPer;       // 8 Ki edges per chunk
static constexpr int kCountChunks = 2;                      // chunks per count workgroup
static constexpr int kGroupChunks = 128;                    // chunks per group of the offset scan
static constexpr int kOffThreads = 256;                     // offsets workgroup: 4 waves x 32 chunks x 64 blocks
static constexpr int kOffRows = kGroupChunks / (kOffThreads / 64);
static constexpr unsigned kXcds = 8;                        // accelerator complex dies of the MI355X
// dynamic LDS of the scatter: the chunk in block order (src and dst)
static constexpr size_t kScatterLds = (size_t)kChunk * 2 * sizeof(int);
static constexpr int kMaxRanges = 64;                       // destination ranges of the second pass
static constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ int block_of(int w, int shift, int K)
{
    const unsigned b = (unsigned)w >> shift;
    return b < (unsigned)K ? (int)b : K - 1;
}

// Chunks kCountChunks * blockIdx.x + j: row j of the count matrix (K blocks)
// each.
__global__ __launch_bounds__(kThreads) void k_blk_count(const int* __restrict__ src, long long m, int shift, int K,
                                                        int* __restrict__ cnt)
{
    __shared__ int h[kCountChunks][kMaxBuckets];
    for (int i = threadIdx.x; i < kCountChunks * kMaxBuckets; i += kThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const long long c0 = (long long)blockIdx.x * kCountChunks;
    int w[kCountChunks][kScatterPer];
#pragma unroll
    for (int j = 0; j < kCountChunks; ++j)
#pragma unroll
        for (int k = 0; k < kScatterPer; ++k)
            w[j][k] = ld_edge(src + std::min((c0 + j) * kChunk + (long long)k * kThreads + threadIdx.x, m - 1));
#pragma unroll
    for (int j = 0; j < kCountChunks; ++j)
#pragma unroll
        for (int k = 0; k < kScatterPer; ++k)
            if ((c0 + j) * kChunk + (long long)k * kThreads + threadIdx.x < m) atomicAdd(&h[j][block_of(w[j][k], shift, K)], 1);
    __syncthreads();
    const long long nch = (m + kChunk - 1) / kChunk;
    for (int b = threadIdx.x; b < K; b += kThreads)
#pragma unroll
        for (int j = 0; j < kCountChunks; ++j)
            if (c0 + j < nch) cnt[(c0 + j) * K + b] = h[j][b];
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

// One workgroup: the first slot of every block (exclusive scan of the
// column sums of `part`), then each row of `part` replaced by the first slot
// of its chunk group's run of each block.
__global__ __launch_bounds__(kThreads) void k_blk_scan(int* __restrict__ part, int groups, int K)
{
    __shared__ int tot[kThreads / 64];
    const int b = threadIdx.x;
    int c = 0;
    if (b < K) {
#pragma unroll 8
        for (int g = 0; g < groups; ++g) c += part[(long long)g * K + b];
    }
    int run = block_inclusive_scan(c, tot) - c;
    if (b < K)
#pragma unroll 8
        for (int g = 0; g < groups; ++g) {
            const long long i = (long long)g * K + b;
            const int v = part[i];
            part[i] = run;
            run += v;
        }
}

// Workgroup (x, y): blocks 64x .. 64x+63 of chunk group y.  Each wave takes
// kOffRows consecutive chunks of the group, one block per lane, and writes
// over each count the offset of that (chunk, block) run inside the group's
// run of the block; the group's total per block goes to `part`.
__global__ __launch_bounds__(kOffThreads) void k_blk_offsets(int* __restrict__ cnt, int* __restrict__ part,
                                                             long long nch, int K)
{
    __shared__ int wsum[kOffThreads / 64][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.x * 64 + lane;
    const long long r0 = (long long)blockIdx.y * kGroupChunks + (long long)wave * kOffRows;
    int v[kOffRows];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kOffRows; ++k) {
        v[k] = b < K && r0 + k < nch ? cnt[(r0 + k) * K + b] : 0;
        s += v[k];
    }
    wsum[wave][lane] = s;
    __syncthreads();
    if (b >= K) return;
    int run = 0;
    for (int k = 0; k < wave; ++k) run += wsum[k][lane];
    if (wave == 0) {
        int total = 0;
        for (int k = 0; k < kOffThreads / 64; ++k) total += wsum[k][lane];
        part[(long long)blockIdx.y * K + b] = total;
    }
#pragma unroll
    for (int k = 0; k < kOffRows; ++k) {
        if (r0 + k < nch) cnt[(r0 + k) * K + b] = run;
        run += v[k];
    }
}

__global__ __launch_bounds__(kThreads) void k_blk_scatter(const int* __restrict__ src, const int* __restrict__ dst,
                                                          long long m, int shift, int K, const int* __restrict__ off,
                                                          const int* __restrict__ part,
                                                          int* __restrict__ osrc, int* __restrict__ odst)
{
    extern __shared__ __align__(16) int lds[];
    int* out_s = lds;
    int* out_d = lds + kChunk;
    __shared__ int cnt[kMaxBuckets];    // edges of the chunk per block, then rank cursor
    __shared__ int lstart[kMaxBuckets]; // first position of each block in the chunk
    __shared__ int gbase[kMaxBuckets];  // first global slot of the chunk's run of each block
    __shared__ int tot[kThreads / 64];
    const int t = threadIdx.x;
    // Workgroups go to the XCDs in turn; XCD x takes the x-th eighth of the
    // chunks in order, so the runs that neighbouring chunks write next to
    // each other meet in one L2 and leave it as whole lines.
    const unsigned per = gridDim.x / kXcds, rem = gridDim.x % kXcds;
    const unsigned x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
    const long long chunk = (long long)x * per + std::min(x, rem) + j;
    const long long e0 = chunk * kChunk;
    const int len = (int)std::min<long long>(kChunk, m - e0);
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
        gbase[t] = c ? part[(chunk / kGroupChunks) * K + t] + off[chunk * K + t] : 0;
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

// Second pass: chunk `chunk` (XCD-ordered as in k_blk_scatter) of the
// grouped copy, placed stably by destination range.  Element i = k * kThreads
// + t of the chunk is edge k of thread t; an edge's rank among the chunk's
// edges of its range counts the earlier elements of that range: those of
// earlier (k, wave) slots (a scan of per-slot counts) plus those of earlier
// lanes of its own wave and slot (wave ballots over the key bits).
__global__ __launch_bounds__(kThreads) void k_rng_scatter(const int* __restrict__ src, const int* __restrict__ dst,
                                                          long long m, int shift, int R, const int* __restrict__ off,
                                                          const int* __restrict__ part, int* __restrict__ osrc,
                                                          int* __restrict__ odst)
{
    extern __shared__ __align__(16) int lds[];
    int* out_s = lds;
    int* out_d = lds + kChunk;
    // per (k, wave) slot and range: count, then first rank within the chunk
    // (both below 2^16), R columns: with R <= 32 the workgroup needs under
    // 80 KiB of LDS, so two share a CU
    unsigned short* hist = reinterpret_cast<unsigned short*>(lds + 2 * kChunk);
    __shared__ int segsum[kWaves][kMaxRanges];
    __shared__ int total[kMaxRanges], lstart[kMaxRanges], gbase[kMaxRanges];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const unsigned per = gridDim.x / kXcds, rem = gridDim.x % kXcds;
    const unsigned x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
    const long long chunk = (long long)x * per + std::min(x, rem) + j;
    const long long e0 = chunk * kChunk;
    const int len = (int)std::min<long long>(kChunk, m - e0);
    for (int i = t; i < kScatterPer * kWaves * R; i += kThreads) hist[i] = 0;
    int es[kScatterPer], ed[kScatterPer];
#pragma unroll
    for (int k = 0; k < kScatterPer; ++k) {
        const int i = std::min(k * kThreads + t, len - 1);
        es[k] = ld_edge(src + e0 + i);
        ed[k] = ld_edge(dst + e0 + i);
    }
    __syncthreads();
    const unsigned long long below = lane ? (~0ULL >> (64 - lane)) : 0ULL;
    int key[kScatterPer], rank[kScatterPer];
#pragma unroll
    for (int k = 0; k < kScatterPer; ++k) {
        const bool valid = k * kThreads + t < len;
        key[k] = valid ? block_of(ed[k], shift, R) : 0;
        unsigned long long peers = __builtin_amdgcn_ballot_w64(valid);
        for (int b = 0; (1 << b) < R; ++b) {
            const bool bit = (key[k] >> b) & 1;
            const unsigned long long bal = __builtin_amdgcn_ballot_w64(bit);
            peers &= bit ? bal : ~bal;
        }
        rank[k] = __popcll(peers & below);
        if (valid && rank[k] == 0) hist[(k * kWaves + wave) * R + key[k]] = (unsigned short)__popcll(peers);
    }
    __syncthreads();
    // exclusive scan of each range's counts over the 128 slots in element
    // order, cut into 16 segments of 8 slots: thread (seg, r) sums its
    // segment's slots, wave 0 scans the segment sums, then each thread writes
    // its slots' first ranks
    constexpr int kSegSlots = kScatterPer;
    const int r = t & 63, seg = t >> 6;
    int sum = 0;
    if (r < R)
        for (int s = 0; s < kSegSlots; ++s) sum += hist[(seg * kSegSlots + s) * R + r];
    segsum[seg][r] = sum;
    __syncthreads();
    if (t < kMaxRanges) {
        int run = 0;
        for (int s = 0; s < kWaves; ++s) {
            const int v = segsum[s][t];
            segsum[s][t] = run;
            run += v;
        }
        total[t] = run;
    }
    __syncthreads();
    if (r < R) {
        int run = segsum[seg][r];
        for (int s = 0; s < kSegSlots; ++s) {
            const int i = (seg * kSegSlots + s) * R + r;
            const int v = hist[i];
            hist[i] = (unsigned short)run;
            run += v;
        }
    }
    if (t < kMaxRanges) {
        // first position of each range in the chunk (wave 0: inclusive scan)
        const int c = t < R ? total[t] : 0;
        int v = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(v, o, 64);
            if (lane >= o) v += y;
        }
        lstart[t] = v - c;
        gbase[t] = (t < R && c) ? part[(chunk / kGroupChunks) * R + t] + off[chunk * R + t] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScatterPer; ++k) {
        if (k * kThreads + t < len) {
            const int pos = lstart[key[k]] + hist[(k * kWaves + wave) * R + key[k]] + rank[k];
            out_s[pos] = es[k];
            out_d[pos] = ed[k];
        }
    }
    __syncthreads();
    for (int i = t; i < len; i += kThreads) {
        const int v = out_d[i];
        const int b = block_of(v, shift, R);
        const int slot = gbase[b] + (i - lstart[b]);
        osrc[slot] = out_s[i];
        odst[slot] = v;
    }
}

// dynamic LDS of the second-pass scatter: the chunk in range order and the
// per-slot counts of R ranges
static size_t rng_scatter_lds(int R)
{
    return kScatterLds + (size_t)kScatterPer * kWaves * R * sizeof(unsigned short);
}

void reorder_geometry(const DeviceInfo& d, long long m, int n, Reorder* r, int dshift)
{
    (void)d;
    // the scatters stage 64 KiB of edges in LDS (set on the current device)
    (void)hipFuncSetAttribute((const void*)k_blk_scatter, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kScatterLds);
    int shift = 0;
    while (((unsigned)(n - 1) >> shift) >= (unsigned)kMaxBuckets) ++shift;
    r->shift = shift;
    r->K = (int)(((unsigned)(n - 1) >> shift) + 1);
    r->dshift = 0;
    r->R = 0;
    if (dshift > 0) {
        while (((unsigned)(n - 1) >> dshift) >= (unsigned)kMaxRanges) ++dshift;
        const int R = (int)(((unsigned)(n - 1) >> dshift) + 1);
        if (R > 1) {
            r->dshift = dshift;
            r->R = R;
            (void)hipFuncSetAttribute((const void*)k_rng_scatter, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)rng_scatter_lds(R));
        }
    }
    r->m = m;
    // every array starts on a 16-byte boundary (the sweep reads edges with
    // 16-byte loads when it can)
    const long long mp = (m + 3) & ~3LL;
    r->chunks = (m + kChunk - 1) / kChunk;
    r->groups = (r->chunks + kGroupChunks - 1) / kGroupChunks;
    r->elems = (r->R ? 4 : 2) * mp + reorder_table_elems(*r);
}

long long reorder_table_elems(const Reorder& r) { return (r.chunks + r.groups) * (r.K + r.R); }

void reorder_bind_tables(Reorder* r, int* tables)
{
    r->cnt = tables;
    r->part = tables + r->chunks * r->K;
    r->cnt2 = r->part + r->groups * r->K;
    r->part2 = r->cnt2 + r->chunks * r->R;
}

void reorder_bind(Reorder* r, int* ws)
{
    const long long mp = (r->m + 3) & ~3LL;
    r->src2 = ws;
    r->dst2 = ws + mp;
    if (r->R) {
        r->src1 = ws + 2 * mp;
        r->dst1 = ws + 3 * mp;
    }
    reorder_bind_tables(r, ws + (r->R ? 4 : 2) * mp);
}

// count, offsets and scan of one pass: keys from `key_src` (>> shift, K keys)
static void enqueue_counts(const Reorder& r, const int* key_src, int shift, int K, int* cnt, int* part,
                           hipStream_t stream)
{
    const unsigned gc = (unsigned)((r.chunks + kCountChunks - 1) / kCountChunks);
    hipLaunchKernelGGL(k_blk_count, dim3(gc), dim3(kThreads), 0, stream, key_src, r.m, shift, K, cnt);
    hipLaunchKernelGGL(k_blk_offsets, dim3((unsigned)((K + 63) / 64), (unsigned)r.groups), dim3(kOffThreads), 0,
                       stream, cnt, part, r.chunks, K);
    hipLaunchKernelGGL(k_blk_scan, dim3(1), dim3(kThreads), 0, stream, part, (int)r.groups, K);
}

int enqueue_reorder(const Reorder& r, const int* src, const int* dst, hipStream_t stream)
{
    if (r.m <= 0) return CONTOUR_OK;
    int* s1 = r.R ? r.src1 : r.src2;
    int* d1 = r.R ? r.dst1 : r.dst2;
    enqueue_counts(r, src, r.shift, r.K, r.cnt, r.part, stream);
    hipLaunchKernelGGL(k_blk_scatter, dim3((unsigned)r.chunks), dim3(kThreads), kScatterLds, stream, src, dst, r.m,
                       r.shift, r.K, (const int*)r.cnt, (const int*)r.part, s1, d1);
    if (r.R) {
        enqueue_counts(r, d1, r.dshift, r.R, r.cnt2, r.part2, stream);
        hipLaunchKernelGGL(k_rng_scatter, dim3((unsigned)r.chunks), dim3(kThreads), rng_scatter_lds(r.R), stream,
                           (const int*)s1, (const int*)d1, r.m, r.dshift, r.R, (const int*)r.cnt2,
                           (const int*)r.part2, r.src2, r.dst2);
    }
    CONTOUR_HIP(hipGetLastError());
    return CONTOUR_OK;
}

}  // namespace contour
