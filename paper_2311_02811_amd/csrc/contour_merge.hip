// contour_merge.hip -- elementwise minimum of two label arrays.
//
// Under an edge split of one graph over several devices, each device sweeps
// its share of the edges against a full copy of the labels, and the copies
// are combined by an elementwise minimum.  In the pointer-graph view of the
// labels (Section II-A) every label names a vertex of the same component at
// or below its own id; the minimum of two such states keeps that, and never
// raises a label, so rounds of local sweeps and merges reach the same unique
// fixed point.  This file holds that combine step for one peer copy: an
// HBM-bound pass (8 bytes read and at most 4 written per label) that also
// counts the labels it lowered, so that a round that changed nothing ends the
// rounds.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "contour_runtime.hpp"

namespace contour {

static constexpr int kMergeThreads = 256;
static constexpr int kMergeUnroll = 4;  // vectors of each array in flight per thread

__global__ __launch_bounds__(64) void k_merge_zero(int* lowered)
{
    if (threadIdx.x == 0) *lowered = 0;
}

// labels[i] = min(labels[i], peer[i]); VEC: both arrays 16-byte aligned, four
// labels per load, kMergeUnroll loads of each array issued before any is
// used (indices past the end clamped to the last vector, whose result is then
// dropped), and a vector written back only where one of its labels dropped.
// One atomic per workgroup adds the count of lowered labels.
template <bool VEC>
__global__ __launch_bounds__(kMergeThreads) void k_merge_min(const int* __restrict__ peer, int* __restrict__ L,
                                                             unsigned n, int* __restrict__ lowered)
{
    __shared__ int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    int c = 0;
    const unsigned stride = gridDim.x * blockDim.x;
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned done = 0;
    if (VEC) {
        const unsigned q = n >> 2;
        const int4* p4 = reinterpret_cast<const int4*>(peer);
        int4* l4 = reinterpret_cast<int4*>(L);
        for (unsigned i0 = t; i0 < q; i0 += stride * kMergeUnroll) {
            int4 a[kMergeUnroll], b[kMergeUnroll];
#pragma unroll
            for (int u = 0; u < kMergeUnroll; ++u) {
                const unsigned i = min(i0 + u * stride, q - 1);
                a[u] = p4[i];
                b[u] = l4[i];
            }
#pragma unroll
            for (int u = 0; u < kMergeUnroll; ++u) {
                const unsigned i = i0 + u * stride;
                if (i >= q) break;
                const bool x = a[u].x < b[u].x, y = a[u].y < b[u].y, z = a[u].z < b[u].z, w = a[u].w < b[u].w;
                c += (int)x + (int)y + (int)z + (int)w;
                if (x || y || z || w) {
                    int4 r;
                    r.x = min(a[u].x, b[u].x);
                    r.y = min(a[u].y, b[u].y);
                    r.z = min(a[u].z, b[u].z);
                    r.w = min(a[u].w, b[u].w);
                    l4[i] = r;
                }
            }
        }
        done = q << 2;
    }
    for (unsigned i = done + t; i < n; i += stride) {
        const int a = peer[i];
        if (a < L[i]) {
            L[i] = a;
            ++c;
        }
    }
    if (c) atomicAdd(&s_cnt, c);
    __syncthreads();
    if (threadIdx.x == 0 && lowered && s_cnt) atomicAdd(lowered, s_cnt);
}

}  // namespace contour

extern "C" {

int contour_merge_min(const int32_t* peer, int32_t* labels_inout, int32_t n, int32_t* lowered,
                      contour_stream_t stream)
{
    if (n < 0) return CONTOUR_EINVAL;
    if (n > 0 && (!peer || !labels_inout)) return CONTOUR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (lowered) {
        hipLaunchKernelGGL(contour::k_merge_zero, dim3(1), dim3(64), 0, s, lowered);
        CONTOUR_HIP(hipGetLastError());
    }
    if (n == 0) return CONTOUR_OK;
    contour::DeviceInfo d;
    int rc = contour::device_info(&d);
    if (rc) return rc;
    const bool vec = ((reinterpret_cast<uintptr_t>(peer) | reinterpret_cast<uintptr_t>(labels_inout)) & 15) == 0;
    const long long per_block = (long long)contour::kMergeThreads * (vec ? 4 * contour::kMergeUnroll : 1);
    // enough workgroups to cover the array once, at most eight per CU
    const unsigned grid = (unsigned)std::max<long long>(
        1, std::min<long long>(((long long)n + per_block - 1) / per_block, (long long)d.cus * 8));
    if (vec)
        hipLaunchKernelGGL(contour::k_merge_min<true>, dim3(grid), dim3(contour::kMergeThreads), 0, s, peer,
                           labels_inout, (unsigned)n, lowered);
    else
        hipLaunchKernelGGL(contour::k_merge_min<false>, dim3(grid), dim3(contour::kMergeThreads), 0, s, peer,
                           labels_inout, (unsigned)n, lowered);
    CONTOUR_HIP(hipGetLastError());
    return CONTOUR_OK;
}

}  // extern "C"
