/*
 * contour_omp.c -- the paper's own multicore CPU design of Contour, as a
 * timed CPU baseline.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite and the benchmark's CPU
 * baseline leg load this library; nothing on the product path calls, links
 * or loads it, and it shares no code, header or constant with the HIP
 * library.
 *
 * What it runs is Algorithm 1 with the three implementation choices of
 * Section III-B, on all host threads (OpenMP):
 *   asynchronous update (III-B-1)  one label array updated in place; an edge
 *                                  reads whatever the other threads stored;
 *   early convergence (III-B-2)    an edge flags a change when its chains
 *                                  read, before its own stores, show a value
 *                                  above z; a sweep that flags nothing ends
 *                                  the loop;
 *   no atomics (III-B-3)           the conditional assignment of Definition 1
 *                                  is a plain load, a compare and a plain
 *                                  store, so concurrent stores may overwrite
 *                                  each other (lost updates).  The loads and
 *                                  stores go through relaxed atomic builtins
 *                                  only so that the race is defined in C11;
 *                                  on x86 they are ordinary moves, with no
 *                                  read-modify-write.
 * The operator is MM^h (Definition 3): for edge <w, v> the chains
 * x_0 = w, x_{i+1} = L[x_i] (and the same from v) are read to level h or to
 * a root; z = min(x_h(w), x_h(v)); every chain vertex x_i, i < h, whose value
 * read there exceeds z is assigned z.  h = 0 follows each chain to its root
 * and includes the root among the targets (the paper's order-m operator with
 * m larger than any chain).
 */
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static inline int32_t ld(const int32_t* L, int32_t x) { return __atomic_load_n(L + x, __ATOMIC_RELAXED); }
static inline void st(int32_t* L, int32_t x, int32_t z) { __atomic_store_n(L + x, z, __ATOMIC_RELAXED); }

#define MAX_CHAIN 64

/* One chain from x: tgt[0..k) are the targets, val[i] the value read at
 * tgt[i]; returns k and the chain's last value (its level-h label, or the
 * root).  Chains longer than MAX_CHAIN levels (order 0 only) are cut there:
 * cutting a chain only makes z larger, which is still a valid label, so the
 * result stays exact and the loop still converges (a cut chain reads a value
 * above z or reaches a root in a later sweep). */
static int chain(const int32_t* L, int32_t x, int h, int32_t* tgt, int32_t* val, int32_t* top)
{
    int k = 0;
    int32_t cur = x;
    for (;;) {
        int32_t nxt = ld(L, cur);
        tgt[k] = cur;
        val[k] = nxt;
        ++k;
        if (nxt == cur || (h > 0 && k == h) || k == MAX_CHAIN) {
            *top = nxt;
            return k;
        }
        cur = nxt;
    }
}

/* Contour on (src, dst) with MM^h (h >= 1, or 0 for chase to the root).
 * labels[n] receives the result; *sweeps the number of sweeps including the
 * final one that flagged nothing; *threads the OpenMP threads used.
 * Returns 0, or -1 for a bad size or an id outside [0, n). */
int contour_omp_cc(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t h, int32_t* labels,
                   int32_t* sweeps, int32_t* threads)
{
    if (m < 0 || n < 0 || h < 0) return -1;
    for (int64_t e = 0; e < m; ++e)
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -1;
    int nt = 1;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        nt = omp_get_num_threads();
#endif
    }
    *threads = nt;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) labels[i] = i;
    int32_t s = 0;
    for (;;) {
        int changed = 0;
        ++s;
#pragma omp parallel for schedule(dynamic, 65536) reduction(| : changed)
        for (int64_t e = 0; e < m; ++e) {
            int32_t tw[MAX_CHAIN], vw[MAX_CHAIN], tv[MAX_CHAIN], vv[MAX_CHAIN], zw, zv;
            const int kw = chain(labels, src[e], h, tw, vw, &zw);
            const int kv = chain(labels, dst[e], h, tv, vv, &zv);
            const int32_t z = zw < zv ? zw : zv;
            int act = 0;
            for (int i = 0; i < kw; ++i) act |= vw[i] > z;
            for (int i = 0; i < kv; ++i) act |= vv[i] > z;
            if (!act) continue;
            changed = 1;
            for (int i = 0; i < kw; ++i)
                if (vw[i] > z) st(labels, tw[i], z);
            for (int i = 0; i < kv; ++i)
                if (vv[i] > z) st(labels, tv[i], z);
        }
        if (!changed || m == 0) break;
    }
    *sweeps = m == 0 ? 0 : s;
    return 0;
}
