/*
 * graphgen.c -- seeded synthetic graph generators.
 *
 * This module only makes inputs.  It holds none of the connectivity
 * arithmetic: no labels, no union-find, no minimum mapping.  Both the HIP
 * path and the CPU oracle are fed from here, and neither side's code is
 * shared with the other through this file.
 *
 * Randomness is counter based, so every output is a pure function of
 * (seed, stream, index) and does not depend on the number of threads:
 *   draw(seed, stream, i) = splitmix64_mix(key(seed, stream) + (i+1) * GAMMA)
 * where splitmix64_mix is the output function of SplitMix64 (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) and
 * GAMMA is its golden-ratio increment.  Bounded integers use Lemire's
 * multiply-shift ("Fast random integer generation in an interval", 2019,
 * without the rejection step), normals use Box-Muller.
 *
 * Graph families (all ids are int32, edges are SoA src[]/dst[]):
 *   gg_er          Erdos-Renyi G(n, m): uniform ordered pairs, self-loops and
 *                  duplicate undirected pairs rejected, drawn order and
 *                  orientation kept, exactly m edges.
 *   gg_grid_holes  rows x cols 4-neighbour lattice in row-major ids; a seeded
 *                  partial Fisher-Yates keeps exactly `keep` lattice edges in
 *                  uniformly random order (the rest are the holes); optional
 *                  seeded permutation of the vertex ids.
 *   gg_rmat        R-MAT / Kronecker: every edge descends `scale` levels of
 *                  the 2x2 quadrant probabilities (a, b, c, d); vertex ids
 *                  are then permuted by a seeded Fisher-Yates permutation.
 *                  Self-loops and duplicates are kept.
 *   gg_batch_*     a batch of independent graphs with log-normal sizes, a
 *                  uniform average degree and a 50/50 ER / grid-with-holes mix.
 *   gg_poisson_trace  Poisson arrival times and request kinds for a serving
 *                  trace.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GG_GAMMA 0x9e3779b97f4a7c15ULL

/* stream ids: one per independent use of the generator */
enum {
    GG_S_ER = 1, GG_S_GRID = 2, GG_S_RMAT = 3, GG_S_PERM = 4,
    GG_S_BATCH_SIZE = 5, GG_S_BATCH_GRAPH = 6, GG_S_TRACE = 7, GG_S_SHUFFLE = 8
};

uint64_t gg_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t gg_key(uint64_t seed, uint64_t stream)
{
    return gg_mix64(gg_mix64(seed + GG_GAMMA) ^ (stream * 0xd1b54a32d192ed03ULL));
}

static inline uint64_t gg_draw_k(uint64_t key, uint64_t i)
{
    return gg_mix64(key + (i + 1) * GG_GAMMA);
}

uint64_t gg_draw(uint64_t seed, uint64_t stream, uint64_t i)
{
    return gg_draw_k(gg_key(seed, stream), i);
}

/* uniform integer in [0, range) by multiply-shift */
static inline uint64_t gg_bounded(uint64_t r, uint64_t range)
{
    return (uint64_t)(((unsigned __int128)r * (unsigned __int128)range) >> 64);
}

/* uniform double in [0, 1) from the top 53 bits */
static inline double gg_unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* ---------------------------------------------------------------- ER -- */

typedef struct { uint64_t* slot; uint64_t mask; } gg_set;

static int gg_set_init(gg_set* s, int64_t expect)
{
    uint64_t cap = 16;
    while (cap < (uint64_t)expect * 2 + 16) cap <<= 1;
    s->slot = (uint64_t*)calloc(cap, sizeof(uint64_t));
    s->mask = cap - 1;
    return s->slot ? 0 : -1;
}

/* returns 1 when inserted, 0 when already present; keys are stored +1 */
static int gg_set_insert(gg_set* s, uint64_t key)
{
    uint64_t k = key + 1, h = gg_mix64(key) & s->mask;
    for (;;) {
        uint64_t cur = s->slot[h];
        if (cur == 0) { s->slot[h] = k; return 1; }
        if (cur == k) return 0;
        h = (h + 1) & s->mask;
    }
}

/* Exactly m distinct undirected edges with u != v drawn uniformly.  Returns m,
 * or -1 when m exceeds n(n-1)/2 or memory runs out. */
static int64_t gg_er_key(int32_t n, int64_t m, uint64_t key, int32_t* src, int32_t* dst)
{
    if (n < 0 || m < 0) return -1;
    if (m == 0) return 0;
    if ((double)m > 0.5 * (double)n * (double)(n - 1)) return -1;
    gg_set s;
    if (gg_set_init(&s, m)) return -1;
    int64_t got = 0;
    for (uint64_t i = 0; got < m; ++i) {
        uint64_t u = gg_bounded(gg_draw_k(key, 2 * i), (uint64_t)n);
        uint64_t v = gg_bounded(gg_draw_k(key, 2 * i + 1), (uint64_t)n);
        if (u == v) continue;
        uint64_t lo = u < v ? u : v, hi = u < v ? v : u;
        if (!gg_set_insert(&s, (lo << 32) | hi)) continue;
        src[got] = (int32_t)u;
        dst[got] = (int32_t)v;
        ++got;
    }
    free(s.slot);
    return got;
}

int64_t gg_er(int32_t n, int64_t m, uint64_t seed, int32_t* src, int32_t* dst)
{
    return gg_er_key(n, m, gg_key(seed, GG_S_ER), src, dst);
}

/* ------------------------------------------------------- permutations -- */

/* perm[0..n) = seeded Fisher-Yates permutation of 0..n-1 */
int gg_permutation(int32_t n, uint64_t seed, uint64_t stream, int32_t* perm)
{
    if (n < 0) return -1;
    uint64_t key = gg_key(seed, stream);
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    for (int64_t i = (int64_t)n - 1; i > 0; --i) {
        int64_t j = (int64_t)gg_bounded(gg_draw_k(key, (uint64_t)i), (uint64_t)i + 1);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    return 0;
}

/* ------------------------------------------------------- grid lattice -- */

/* Lattice edges of the first nv vertices (row-major) of a rows x cols grid;
 * with nv = rows*cols this is the full lattice.  Edge e < H is horizontal,
 * otherwise vertical.  Returns the count, or fills (u, v) for index e. */
static int64_t gg_lattice_count(int64_t rows, int64_t cols, int64_t nv)
{
    /* horizontal: (r, c)-(r, c+1) with r*cols + c + 1 < nv */
    int64_t h = 0, v = 0;
    int64_t full_rows = nv / cols, rem = nv % cols;
    h = full_rows * (cols - 1) + (rem > 0 ? rem - 1 : 0);
    /* vertical: (r, c)-(r+1, c) with (r+1)*cols + c < nv */
    v = nv > cols ? nv - cols : 0;
    (void)rows;
    return h + v;
}

static void gg_lattice_edge(int64_t cols, int64_t nv, int64_t e, int64_t* u, int64_t* w)
{
    int64_t full_rows = nv / cols, rem = nv % cols;
    int64_t h = full_rows * (cols - 1) + (rem > 0 ? rem - 1 : 0);
    if (e < h) {
        int64_t r = e / (cols - 1), c = e % (cols - 1);
        *u = r * cols + c;
        *w = *u + 1;
    } else {
        int64_t x = e - h;        /* vertical edges in row-major order of the upper end */
        *u = x;
        *w = x + cols;
    }
}

/* Keep exactly `keep` of the lattice edges of the first nv vertices of a
 * rows x cols grid, chosen and ordered by a partial Fisher-Yates shuffle, so
 * the kept edges come out in uniformly random order.  Orientation (min, max)
 * of the final ids.  perm may be NULL (row-major ids).  Returns keep or -1. */
static int64_t gg_grid_key(int64_t rows, int64_t cols, int64_t nv, int64_t keep, uint64_t key,
                           const int32_t* perm, int32_t* src, int32_t* dst)
{
    if (rows <= 0 || cols <= 0 || nv < 0 || nv > rows * cols) return -1;
    int64_t total = gg_lattice_count(rows, cols, nv);
    if (keep < 0 || keep > total) return -1;
    if (keep == 0) return 0;
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)total);
    if (!idx) return -1;
    for (int64_t i = 0; i < total; ++i) idx[i] = i;
    for (int64_t i = 0; i < keep; ++i) {
        int64_t j = i + (int64_t)gg_bounded(gg_draw_k(key, (uint64_t)i), (uint64_t)(total - i));
        int64_t t = idx[i]; idx[i] = idx[j]; idx[j] = t;
        int64_t u, w;
        gg_lattice_edge(cols, nv, idx[i], &u, &w);
        int32_t a = perm ? perm[u] : (int32_t)u, b = perm ? perm[w] : (int32_t)w;
        src[i] = a < b ? a : b;
        dst[i] = a < b ? b : a;
    }
    free(idx);
    return keep;
}

int64_t gg_lattice_edges(int64_t rows, int64_t cols, int64_t nv)
{
    if (rows <= 0 || cols <= 0 || nv < 0 || nv > rows * cols) return -1;
    return gg_lattice_count(rows, cols, nv);
}

int64_t gg_grid_holes(int32_t rows, int32_t cols, int64_t keep, uint64_t seed, int permute_ids,
                      int32_t* src, int32_t* dst)
{
    int64_t nv = (int64_t)rows * cols;
    if (nv > 0x7fffffffLL) return -1;
    int32_t* perm = NULL;
    if (permute_ids) {
        perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)nv);
        if (!perm) return -1;
        gg_permutation((int32_t)nv, seed, GG_S_PERM, perm);
    }
    int64_t r = gg_grid_key(rows, cols, nv, keep, gg_key(seed, GG_S_GRID), perm, src, dst);
    free(perm);
    return r;
}

/* -------------------------------------------------------------- R-MAT -- */

int64_t gg_rmat(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed,
                int permute_ids, int32_t* src, int32_t* dst)
{
    if (scale < 1 || scale > 30 || m < 0) return -1;
    int32_t n = (int32_t)(1u << scale);
    int32_t* perm = NULL;
    if (permute_ids) {
        perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        if (!perm) return -1;
        gg_permutation(n, seed, GG_S_PERM, perm);
    }
    const uint64_t key = gg_key(seed, GG_S_RMAT);
    const double ab = a + b, abc = a + b + c;
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        uint32_t u = 0, v = 0;
        uint64_t base = (uint64_t)e * (uint64_t)scale;
        for (int32_t l = 0; l < scale; ++l) {
            double p = gg_unit(gg_draw_k(key, base + (uint64_t)l));
            uint32_t bu = p >= ab, bv = (p >= a && p < ab) || p >= abc;
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        src[e] = perm ? perm[u] : (int32_t)u;
        dst[e] = perm ? perm[v] : (int32_t)v;
    }
    free(perm);
    return m;
}

/* -------------------------------------------------------------- batch -- */

/* Per-graph parameters of a batch: n_g = clamp(round(exp(ln(median) +
 * sigma * N(0,1))), n_lo, n_hi); average degree d_g ~ U[d_lo, d_hi];
 * kind_g = 0 (ER) or 1 (grid with holes) with probability 1/2 each.
 * ER: m_g = round(n_g d_g / 2).  Grid: rows = floor(sqrt(n_g)),
 * cols = ceil(n_g / rows), the first n_g row-major vertices, keeping
 * round(min(0.9, d_g / 4) * lattice edges).  Returns 0. */
int gg_batch_sizes(int32_t G, uint64_t seed, double median, double sigma, int32_t n_lo,
                   int32_t n_hi, double d_lo, double d_hi, int32_t* n_out, int64_t* m_out,
                   int32_t* kind_out)
{
    const uint64_t key = gg_key(seed, GG_S_BATCH_SIZE);
    for (int32_t g = 0; g < G; ++g) {
        uint64_t base = (uint64_t)g * 4;
        double u1 = ((double)(gg_draw_k(key, base) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
        double u2 = gg_unit(gg_draw_k(key, base + 1));
        double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        double nf = floor(exp(log(median) + sigma * z) + 0.5);
        if (nf < n_lo) nf = n_lo;
        if (nf > n_hi) nf = n_hi;
        int64_t n = (int64_t)nf;
        double d = d_lo + (d_hi - d_lo) * gg_unit(gg_draw_k(key, base + 2));
        int32_t kind = (int32_t)(gg_draw_k(key, base + 3) >> 63);
        int64_t m;
        if (kind == 0) {
            m = (int64_t)floor((double)n * d * 0.5 + 0.5);
            int64_t cap = n * (n - 1) / 2;
            if (m > cap) m = cap;
        } else {
            int64_t rows = (int64_t)floor(sqrt((double)n));
            if (rows < 1) rows = 1;
            while ((rows + 1) * (rows + 1) <= n) ++rows;
            while (rows * rows > n) --rows;
            int64_t cols = (n + rows - 1) / rows;
            int64_t tot = gg_lattice_count(rows, cols, n);
            double f = d / 4.0 < 0.9 ? d / 4.0 : 0.9;
            m = (int64_t)floor(f * (double)tot + 0.5);
        }
        n_out[g] = (int32_t)n;
        m_out[g] = m;
        kind_out[g] = kind;
    }
    return 0;
}

/* Fill every graph's edges (local ids) at edge_off[g] .. edge_off[g+1].
 * Graphs are independent, so the fill runs in parallel over graphs. */
int gg_batch_fill(int32_t G, uint64_t seed, const int32_t* n_g, const int64_t* m_g,
                  const int32_t* kind_g, const int64_t* edge_off, int32_t* src, int32_t* dst)
{
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int32_t g = 0; g < G; ++g) {
        uint64_t key = gg_key(gg_mix64(seed ^ ((uint64_t)g * GG_GAMMA)), GG_S_BATCH_GRAPH);
        int64_t n = n_g[g], m = m_g[g];
        int32_t* s = src + edge_off[g];
        int32_t* d = dst + edge_off[g];
        int64_t r;
        if (kind_g[g] == 0) {
            r = gg_er_key((int32_t)n, m, key, s, d);
        } else {
            int64_t rows = (int64_t)floor(sqrt((double)n));
            if (rows < 1) rows = 1;
            while ((rows + 1) * (rows + 1) <= n) ++rows;
            while (rows * rows > n) --rows;
            int64_t cols = (n + rows - 1) / rows;
            r = gg_grid_key(rows, cols, n, m, key, NULL, s, d);
        }
        if (r != m) bad |= 1;
    }
    return bad ? -1 : 0;
}

/* -------------------------------------------------------------- trace -- */

/* Open-loop Poisson arrivals at `rate` per second: t[i] in seconds from 0;
 * big[i] = 1 with probability p_big; pick[i] uniform in [0, pool_small) or
 * [0, pool_big) according to big[i]. */
int gg_poisson_trace(int64_t count, double rate, double p_big, int64_t pool_small,
                     int64_t pool_big, uint64_t seed, double* t, int32_t* big, int64_t* pick)
{
    if (count < 0 || rate <= 0) return -1;
    const uint64_t key = gg_key(seed, GG_S_TRACE);
    double now = 0.0;
    for (int64_t i = 0; i < count; ++i) {
        uint64_t base = (uint64_t)i * 3;
        double u = ((double)(gg_draw_k(key, base) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
        now += -log(u) / rate;
        t[i] = now;
        int32_t b = gg_unit(gg_draw_k(key, base + 1)) < p_big && pool_big > 0;
        big[i] = b;
        uint64_t range = (uint64_t)(b ? pool_big : pool_small);
        pick[i] = range ? (int64_t)gg_bounded(gg_draw_k(key, base + 2), range) : 0;
    }
    return 0;
}

/* ------------------------------------------------------ edge shuffles -- */

/* In-place seeded Fisher-Yates shuffle of the edge order (src/dst together). */
int gg_shuffle_edges(int64_t m, uint64_t seed, int32_t* src, int32_t* dst)
{
    const uint64_t key = gg_key(seed, GG_S_SHUFFLE);
    for (int64_t i = m - 1; i > 0; --i) {
        int64_t j = (int64_t)gg_bounded(gg_draw_k(key, (uint64_t)i), (uint64_t)i + 1);
        int32_t t = src[i]; src[i] = src[j]; src[j] = t;
        t = dst[i]; dst[i] = dst[j]; dst[j] = t;
    }
    return 0;
}

int gg_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
