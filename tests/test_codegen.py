"""Code-generation checks of the HIP kernels (CPU only: hipcc cross-compiles).

Every kernel that loops around a workgroup barrier must keep all lanes of a
wave together at that barrier.  A loop that masks some lanes out while others
go round again (which the compiler may produce when a loop's control looks
lane-dependent) deadlocks the workgroup; the persistent kernels read their
loop control from shared memory through readfirstlane to prevent it.
"""
import os
import shutil
import subprocess

import pytest

from tests.asm_loops import check_file

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_02811_amd", "csrc")


@pytest.mark.parametrize("src", ["contour_single.hip", "contour_batch.hip", "contour_reorder.hip"])
def test_no_divergent_loop_around_a_barrier(src, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    from paper_2311_02811_amd._build import HIPCC_FLAGS
    out = tmp_path / (src + ".s")
    cmd = [hipcc, *[f for f in HIPCC_FLAGS if f != "-Wall"], "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, "--cuda-device-only", "-S", "-o", str(out), os.path.join(CSRC, src)]
    subprocess.run(cmd, check=True, capture_output=True)
    bad = check_file(str(out))
    assert not bad, bad
    # no kernel may spill vector registers to scratch memory
    import re
    spills = []
    for blk in out.read_text().split("  - ."):
        name = re.search(r"\.name:\s+(\S+)", blk)
        spill = re.search(r"\.vgpr_spill_count:\s+(\d+)", blk)
        if name and spill and int(spill.group(1)) > 0:
            spills.append((name.group(1), int(spill.group(1))))
    assert not spills, spills


def test_checker_flags_a_divergent_barrier_loop(tmp_path):
    # a task loop whose control is read from LDS without readfirstlane and
    # whose thread-0 sections (task pick with a spin wait, task completion)
    # sit at both ends of the body: this compiles to a lane-split loop around
    # the barrier, the pattern the persistent kernels must avoid
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "bad.hip"
    src.write_text(r'''
#include <hip/hip_runtime.h>
struct C { unsigned long long next, done; int last, state; };
__global__ void bad(C* c, int* L, const int* src, long long tasks, long long m) {
    __shared__ long long s_t; __shared__ int s_go;
    for (;;) {
        if (threadIdx.x == 0) {
            int go = 0; long long t = 0;
            if (__hip_atomic_load(&c->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                t = (long long)__hip_atomic_fetch_add(&c->next, 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                long long sweep = t / tasks;
                if (sweep > 0) {
                    while (__hip_atomic_load(&c->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned long long)(sweep * tasks)) {
                        if (__hip_atomic_load(&c->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
                if (sweep > 0 && c->last <= sweep - 1) { int e = 0; __hip_atomic_compare_exchange_strong(&c->state, &e, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
                else go = 1;
            }
            s_go = go; s_t = t;
        }
        __syncthreads();
        if (!s_go) break;
        long long t = s_t; long long sweep = t / tasks; long long chunk = t - sweep * tasks;
        long long e = chunk * blockDim.x + threadIdx.x;
        bool pred = false;
        if (e < m) { int w = src[e]; int a = L[w]; int b = L[a]; if (b < a) { L[w] = b; pred = true; } }
        int any = __syncthreads_or(pred);
        if (threadIdx.x == 0) {
            if (any) __hip_atomic_fetch_max(&c->last, (int)sweep + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&c->done, 1ULL, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}
''')
    out = tmp_path / "bad.s"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O3", "--cuda-device-only", "-S", "-o", str(out),
                    str(src)], check=True, capture_output=True)
    assert check_file(str(out)), "the checker missed a lane-split loop"
