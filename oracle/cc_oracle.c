/*
 * cc_oracle.c -- CPU oracle for connected-component labels.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file's library: only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header or constant
 * with the HIP library.
 *
 * What it computes is the plain definition of the result of the Contour
 * algorithm (Sections II-A and II-D of the paper): vertex ids are 0..n-1, and
 * once the label array has converged to one star per component, each
 * component's root is its minimum vertex, so
 *
 *     labels[v] = min { u : u is connected to v },   v counted as connected
 *                                                   to itself.
 *
 * Two independent routes to that definition are given:
 *   oracle_uf_labels   sequential union-find, path halving, the larger root
 *                      linked under the smaller so every root stays the
 *                      minimum of its set; labels[v] = find(v).
 *   oracle_bfs_labels  breadth-first search started from s = 0, 1, ..., n-1
 *                      in increasing order; the first unvisited s of each
 *                      component is its minimum, and BFS labels the whole
 *                      component with s.
 *
 * Both reject an edge whose id is outside [0, n) by returning -1 before
 * touching labels.
 */
#include <stdint.h>
#include <stdlib.h>

static int32_t uf_find(int32_t* parent, int32_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];   /* path halving */
        x = parent[x];
    }
    return x;
}

static int ids_in_range(const int32_t* src, const int32_t* dst, int64_t m, int32_t n)
{
    for (int64_t e = 0; e < m; ++e)
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return 0;
    return 1;
}

/* labels[0..n) = minimum vertex id of each vertex's component.  Returns 0, or
 * -1 when n < 0, m < 0 or an id is out of range (labels untouched). */
int oracle_uf_labels(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                     int32_t* labels)
{
    if (n < 0 || m < 0) return -1;
    if (!ids_in_range(src, dst, m, n)) return -1;
    for (int32_t i = 0; i < n; ++i) labels[i] = i;      /* labels doubles as parent[] */
    for (int64_t e = 0; e < m; ++e) {
        int32_t ru = uf_find(labels, src[e]);
        int32_t rv = uf_find(labels, dst[e]);
        if (ru == rv) continue;
        if (ru < rv) labels[rv] = ru;                  /* larger root under smaller */
        else labels[ru] = rv;
    }
    for (int32_t i = 0; i < n; ++i) labels[i] = uf_find(labels, i);
    return 0;
}

/* Same result by breadth-first search over an adjacency list. */
int oracle_bfs_labels(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                      int32_t* labels)
{
    if (n < 0 || m < 0) return -1;
    if (!ids_in_range(src, dst, m, n)) return -1;
    int64_t* start = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!start || !adj || !queue || !fill) {
        free(start); free(adj); free(queue); free(fill);
        return -2;
    }
    for (int64_t e = 0; e < m; ++e) {
        start[src[e] + 1]++;
        start[dst[e] + 1]++;
    }
    for (int32_t i = 0; i < n; ++i) start[i + 1] += start[i];
    for (int32_t i = 0; i <= n; ++i) fill[i] = start[i];
    for (int64_t e = 0; e < m; ++e) {
        adj[fill[src[e]]++] = dst[e];
        adj[fill[dst[e]]++] = src[e];
    }
    for (int32_t i = 0; i < n; ++i) labels[i] = -1;
    for (int32_t s = 0; s < n; ++s) {
        if (labels[s] != -1) continue;
        int64_t head = 0, tail = 0;
        labels[s] = s;
        queue[tail++] = s;
        while (head < tail) {
            int32_t x = queue[head++];
            for (int64_t k = start[x]; k < start[x + 1]; ++k) {
                int32_t y = adj[k];
                if (labels[y] == -1) {
                    labels[y] = s;
                    queue[tail++] = y;
                }
            }
        }
    }
    free(start); free(adj); free(queue); free(fill);
    return 0;
}

/* Batched form: graph g has local ids 0..n_g-1 with n_g = vertex_off[g+1] -
 * vertex_off[g], and edges edge_off[g]..edge_off[g+1].  Each graph's labels
 * are its own local minimum ids, written at labels + vertex_off[g].  Returns
 * 0, or -1 - g for the first graph g that is rejected. */
int oracle_uf_batch(int32_t G, const int64_t* edge_off, const int64_t* vertex_off,
                    const int32_t* src, const int32_t* dst, int32_t* labels)
{
    for (int32_t g = 0; g < G; ++g) {
        int64_t e0 = edge_off[g], e1 = edge_off[g + 1];
        int64_t v0 = vertex_off[g], v1 = vertex_off[g + 1];
        if (e1 < e0 || v1 < v0 || v1 - v0 > 0x7fffffffLL) return -1 - g;
        if (oracle_uf_labels(src + e0, dst + e0, e1 - e0, (int32_t)(v1 - v0), labels + v0))
            return -1 - g;
    }
    return 0;
}

/* Eccentricity of s by BFS (hop count to the farthest reachable vertex), and
 * the farthest vertex in *far.  Used for a double-sweep lower bound on a
 * component's diameter when logging the paper's iteration bound. */
int64_t oracle_bfs_ecc(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t s,
                       int32_t* far)
{
    if (n <= 0 || s < 0 || s >= n || !ids_in_range(src, dst, m, n)) return -1;
    int64_t* start = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!start || !adj || !dist || !queue || !fill) {
        free(start); free(adj); free(dist); free(queue); free(fill);
        return -2;
    }
    for (int64_t e = 0; e < m; ++e) { start[src[e] + 1]++; start[dst[e] + 1]++; }
    for (int32_t i = 0; i < n; ++i) start[i + 1] += start[i];
    for (int32_t i = 0; i <= n; ++i) fill[i] = start[i];
    for (int64_t e = 0; e < m; ++e) { adj[fill[src[e]]++] = dst[e]; adj[fill[dst[e]]++] = src[e]; }
    for (int32_t i = 0; i < n; ++i) dist[i] = -1;
    int64_t head = 0, tail = 0, ecc = 0;
    int32_t last = s;
    dist[s] = 0;
    queue[tail++] = s;
    while (head < tail) {
        int32_t x = queue[head++];
        if (dist[x] > ecc) { ecc = dist[x]; last = x; }
        for (int64_t k = start[x]; k < start[x + 1]; ++k) {
            int32_t y = adj[k];
            if (dist[y] == -1) { dist[y] = dist[x] + 1; queue[tail++] = y; }
        }
    }
    if (far) *far = last;
    free(start); free(adj); free(dist); free(queue); free(fill);
    return ecc;
}
