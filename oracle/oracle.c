/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow, obviously correct single-threaded C for what the GPU traversal
 * library computes. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may call it; the library never does. It shares no code,
 * header or table with the GPU library (the only common input is the seeded
 * graph generator, which carries none of the method's arithmetic).
 *
 * Graphs are CSR: row_ptr[n+1], col[m] (int32). Floating point is fp64.
 *
 * Definitions followed (the paper names the five algorithms it evaluates in
 * its Evaluation section, "Algorithms" paragraph, but defines none beyond the
 * BFS program of its Algorithm Language section):
 *   BFS    FIFO queue; depth of the source 0, first discovery sets depth+1;
 *          -1 when unreachable. (The paper's BFS program records a parent;
 *          the depth is the unique part of that result.)
 *   SSSP   Dijkstra with a binary heap and lazy deletion, int64 sums;
 *          INT32_MAX when unreachable. Delta-stepping (Evaluation section and
 *          the priority-queue schedule of the Scheduling Language section)
 *          reaches exactly these distances for every delta.
 *   CC     union-find; label = smallest vertex id in the component.
 *   PR     power iteration from 1/n, exactly `iters` steps, damping d; the
 *          mass of zero-degree vertices is spread uniformly (variant 0) or
 *          dropped (variant 1).
 *   BC     Brandes: BFS path counts sigma (uint64, checked), dependencies
 *          delta[v] = sum over neighbours w one level deeper of
 *          sigma[v]/sigma[w] * (1 + delta[w]), in neighbour order; delta[s]=0.
 *   Directed graphs (rows are out-edges): BFS, SSSP and BC above follow
 *          out-edges as written. PR on a directed graph is its own function:
 *          every vertex passes rank/out-degree along each out-edge, and the
 *          vertices without out-edges are the dangling ones.
 *   EB     EdgeBlocking preprocessing (the Algorithm for preprocessing the
 *          input graph, GPU-Specific Optimizations section): count edges per
 *          destination segment floor(dst/N), exclusive prefix sum, stable
 *          scatter.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- CSR sanity: sorted, unique, in range, no self-loops, symmetric ------ */
/* returns 0 if fine, else a code naming the first violated property */
int oracle_check_csr(int64_t n, const int32_t *rp, const int32_t *col) {
    if (n < 0 || rp[0] != 0) return 1;
    for (int64_t v = 0; v < n; v++) {
        if (rp[v + 1] < rp[v]) return 2;
        for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
            if (col[e] < 0 || col[e] >= n) return 3;
            if (col[e] == v) return 4;
            if (e > rp[v] && col[e] <= col[e - 1]) return 5;
        }
    }
    /* symmetry: every (v,u) has (u,v), by binary search in u's row */
    for (int64_t v = 0; v < n; v++) {
        for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
            int64_t u = col[e], lo = rp[u], hi = rp[u + 1];
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (col[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (lo >= rp[u + 1] || col[lo] != v) return 6;
        }
    }
    return 0;
}

/* ---- CSR sanity for a directed graph: sorted, unique, in range, no
   self-loops (no symmetry). Same codes as oracle_check_csr. ---------------- */
int oracle_check_digraph(int64_t n, const int32_t *rp, const int32_t *col) {
    if (n < 0 || rp[0] != 0) return 1;
    for (int64_t v = 0; v < n; v++) {
        if (rp[v + 1] < rp[v]) return 2;
        for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
            if (col[e] < 0 || col[e] >= n) return 3;
            if (col[e] == v) return 4;
            if (e > rp[v] && col[e] <= col[e - 1]) return 5;
        }
    }
    return 0;
}

/* ---- BFS ------------------------------------------------------------------ */
int oracle_bfs(int64_t n, const int32_t *rp, const int32_t *col, int32_t src, int32_t *depth) {
    if (src < 0 || src >= n) return 1;
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t v = 0; v < n; v++) depth[v] = -1;
    int64_t head = 0, tail = 0;
    depth[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
            int32_t v = col[e];
            if (depth[v] == -1) {
                depth[v] = depth[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return 0;
}

/* ---- Dijkstra ------------------------------------------------------------- */
typedef struct { int64_t key; int32_t v; } heap_item;

static void heap_push(heap_item *h, int64_t *size, heap_item x) {
    int64_t i = (*size)++;
    h[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].key <= h[i].key) break;
        heap_item t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static heap_item heap_pop(heap_item *h, int64_t *size) {
    heap_item top = h[0];
    h[0] = h[--(*size)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < *size && h[l].key < h[s].key) s = l;
        if (r < *size && h[r].key < h[s].key) s = r;
        if (s == i) break;
        heap_item t = h[s]; h[s] = h[i]; h[i] = t;
        i = s;
    }
    return top;
}

/* returns 0, 1 for a bad source, 2 if a distance exceeds INT32_MAX-1 */
int oracle_sssp(int64_t n, const int32_t *rp, const int32_t *col, const uint32_t *w,
                int32_t src, int32_t *dist) {
    if (src < 0 || src >= n) return 1;
    int64_t m = rp[n];
    int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    heap_item *h = (heap_item *)malloc(sizeof(heap_item) * (size_t)(m + 1));
    int64_t hs = 0;
    const int64_t INF = INT64_MAX;
    for (int64_t v = 0; v < n; v++) d[v] = INF;
    d[src] = 0;
    heap_item s0 = {0, src};
    heap_push(h, &hs, s0);
    while (hs > 0) {
        heap_item it = heap_pop(h, &hs);
        if (it.key != d[it.v]) continue; /* stale entry */
        int32_t u = it.v;
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
            int64_t nd = d[u] + (int64_t)w[e];
            int32_t v = col[e];
            if (nd < d[v]) {
                d[v] = nd;
                heap_item x = {nd, v};
                heap_push(h, &hs, x);
            }
        }
    }
    int rc = 0;
    for (int64_t v = 0; v < n; v++) {
        if (d[v] == INF) dist[v] = INT32_MAX;
        else if (d[v] > (int64_t)INT32_MAX - 1) { dist[v] = INT32_MAX; rc = 2; }
        else dist[v] = (int32_t)d[v];
    }
    free(d); free(h);
    return rc;
}

/* ---- connected components --------------------------------------------------- */
static int32_t find_root(int32_t *p, int32_t x) {
    while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; } /* path halving */
    return x;
}

void oracle_cc(int64_t n, const int32_t *rp, const int32_t *col, int32_t *label) {
    int32_t *p = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t v = 0; v < n; v++) p[v] = (int32_t)v;
    for (int64_t u = 0; u < n; u++) {
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
            int32_t a = find_root(p, (int32_t)u), b = find_root(p, col[e]);
            if (a == b) continue;
            if (a < b) p[b] = a; else p[a] = b; /* smaller id becomes the root */
        }
    }
    for (int64_t v = 0; v < n; v++) label[v] = find_root(p, (int32_t)v);
    free(p);
}

/* ---- PageRank ------------------------------------------------------------- */
void oracle_pagerank(int64_t n, const int32_t *rp, const int32_t *col, double damping,
                     int iters, int variant, double *rank) {
    double *next = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t v = 0; v < n; v++) rank[v] = 1.0 / (double)n;
    for (int t = 0; t < iters; t++) {
        double dangling = 0.0;
        if (variant == 0)
            for (int64_t u = 0; u < n; u++)
                if (rp[u + 1] == rp[u]) dangling += rank[u];
        for (int64_t v = 0; v < n; v++) {
            double s = 0.0;
            for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
                int32_t u = col[e]; /* symmetric graph: in-neighbours = out-neighbours */
                s += rank[u] / (double)(rp[u + 1] - rp[u]);
            }
            next[v] = (1.0 - damping) / (double)n + damping * (s + dangling / (double)n);
        }
        memcpy(rank, next, sizeof(double) * (size_t)n);
    }
    free(next);
}

/* ---- PageRank on a directed graph ----------------------------------------------
   next[v] = (1-d)/n + d * (sum over edges u -> v of rank[u]/outdeg(u) + D/n),
   D = the rank held by vertices with no out-edge (variant 0) or 0 (variant 1). */
void oracle_pagerank_directed(int64_t n, const int32_t *rp, const int32_t *col, double damping,
                              int iters, int variant, double *rank) {
    double *in_sum = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t v = 0; v < n; v++) rank[v] = 1.0 / (double)n;
    for (int t = 0; t < iters; t++) {
        double dangling = 0.0;
        for (int64_t v = 0; v < n; v++) in_sum[v] = 0.0;
        for (int64_t u = 0; u < n; u++) {
            int64_t outdeg = rp[u + 1] - rp[u];
            if (outdeg == 0) {
                if (variant == 0) dangling += rank[u];
                continue;
            }
            for (int64_t e = rp[u]; e < rp[u + 1]; e++) in_sum[col[e]] += rank[u] / (double)outdeg;
        }
        for (int64_t v = 0; v < n; v++)
            rank[v] = (1.0 - damping) / (double)n + damping * (in_sum[v] + dangling / (double)n);
    }
    free(in_sum);
}

/* ---- betweenness (single source) -------------------------------------------- */
/* returns 0, 1 for a bad source, 2 if a path count overflows uint64 */
int oracle_bc(int64_t n, const int32_t *rp, const int32_t *col, int32_t src,
              uint64_t *sigma, double *delta) {
    if (src < 0 || src >= n) return 1;
    int32_t *depth = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int rc = 0;
    for (int64_t v = 0; v < n; v++) { depth[v] = -1; sigma[v] = 0; delta[v] = 0.0; }
    int64_t head = 0, tail = 0;
    depth[src] = 0;
    sigma[src] = 1;
    order[tail++] = src;
    while (head < tail) {
        int32_t u = order[head++];
        for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
            int32_t v = col[e];
            if (depth[v] == -1) { depth[v] = depth[u] + 1; order[tail++] = v; }
            if (depth[v] == depth[u] + 1) {
                uint64_t s = sigma[v] + sigma[u];
                if (s < sigma[v]) rc = 2;
                sigma[v] = s;
            }
        }
    }
    /* reverse BFS order: deeper vertices first, so delta[w] is final when read */
    for (int64_t i = tail - 1; i >= 0; i--) {
        int32_t v = order[i];
        double acc = 0.0;
        for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
            int32_t w = col[e];
            if (depth[w] == depth[v] + 1)
                acc += ((double)sigma[v] / (double)sigma[w]) * (1.0 + delta[w]);
        }
        delta[v] = (v == src) ? 0.0 : acc;
    }
    free(depth); free(order);
    return rc;
}

/* ---- EdgeBlocking preprocessing ------------------------------------------------ */
/* seg_start has ceil(n/N)+1 entries: segment s is [seg_start[s], seg_start[s+1]) */
int64_t oracle_edgeblock(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int64_t N,
                         int32_t *out_src, int32_t *out_dst, int64_t *seg_start) {
    int64_t S = (n + N - 1) / N;
    int64_t *count = (int64_t *)calloc((size_t)S + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; e++) count[dst[e] / N]++;
    /* exclusive prefix sum */
    int64_t run = 0;
    for (int64_t s = 0; s <= S; s++) { int64_t c = count[s]; seg_start[s] = run; run += c; }
    int64_t *cursor = (int64_t *)malloc(sizeof(int64_t) * ((size_t)S + 1));
    memcpy(cursor, seg_start, sizeof(int64_t) * ((size_t)S + 1));
    for (int64_t e = 0; e < m; e++) {
        int64_t s = dst[e] / N;
        int64_t i = cursor[s]++;
        out_src[i] = src[e];
        out_dst[i] = dst[e];
    }
    free(count); free(cursor);
    return S;
}
