/*
 * Seeded synthetic graph inputs: R-MAT edge lists, road-like weighted grids,
 * symmetric CSR construction and per-edge weights.
 *
 * This file holds input preparation only. It contains none of the traversal
 * method's arithmetic and is shared, unchanged, by the test oracle and by the
 * GPU library's tests and benchmark.
 *
 * Random numbers: output number `ctr` of a SplitMix64 stream (Steele, Lea and
 * Flood, OOPSLA 2014) whose state starts at mix64(seed):
 *     rng(seed, ctr) = mix64(mix64(seed) + (ctr + 1) * 0x9E3779B97F4A7C15)
 * so every draw is addressable by a counter and generation is order-free.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t gen_rng(uint64_t seed, uint64_t ctr) {
    return mix64(mix64(seed) + (ctr + 1) * GOLDEN);
}

/* uniform double in [0,1) from the top 53 bits */
static inline double u53(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* index in [0, bound) from a 64-bit draw (multiply-high, Lemire) */
static inline uint64_t bounded(uint64_t x, uint64_t bound) {
    return (uint64_t)(((unsigned __int128)x * bound) >> 64);
}

/* Seeded Fisher-Yates permutation of 0..n-1. */
void gen_permutation(int64_t n, uint64_t seed, int32_t *perm) {
    for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t j = (int64_t)bounded(gen_rng(seed, (uint64_t)i), (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

/*
 * R-MAT edge list: m = ef * 2^scale edges. Edge i descends `scale` levels,
 * most significant bit first; draw u = rng(seed, i*64 + level):
 * u < a -> (0,0), < a+b -> (0,1), < a+b+c -> (1,0), else (1,1).
 * Vertex ids are then relabelled by a Fisher-Yates permutation with seed+1.
 * Edges are independent draws, so the range is split over threads.
 */
typedef struct {
    int scale; int64_t lo, hi; double a, ab, abc; uint64_t s0;
    int32_t *src, *dst;
} rmat_job;

static void *rmat_worker(void *arg) {
    rmat_job *j = (rmat_job *)arg;
    for (int64_t i = j->lo; i < j->hi; i++) {
        uint32_t u = 0, v = 0;
        for (int l = 0; l < j->scale; l++) {
            uint64_t ctr = (uint64_t)i * 64u + (uint64_t)l;
            double r = u53(mix64(j->s0 + (ctr + 1) * GOLDEN));
            uint32_t bu, bv;
            if (r < j->a) { bu = 0; bv = 0; }
            else if (r < j->ab) { bu = 0; bv = 1; }
            else if (r < j->abc) { bu = 1; bv = 0; }
            else { bu = 1; bv = 1; }
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        j->src[i] = (int32_t)u;
        j->dst[i] = (int32_t)v;
    }
    return 0;
}

static int nthreads(void) {
    long t = sysconf(_SC_NPROCESSORS_ONLN);
    if (t < 1) t = 1;
    if (t > 16) t = 16;
    return (int)t;
}

void gen_rmat_edges(int scale, int64_t m, double a, double b, double c, uint64_t seed,
                    int32_t *src, int32_t *dst) {
    int T = nthreads();
    pthread_t th[16];
    rmat_job jobs[16];
    for (int t = 0; t < T; t++) {
        rmat_job jb = {scale, m * t / T, m * (t + 1) / T, a, a + b, a + b + c, mix64(seed), src, dst};
        jobs[t] = jb;
        pthread_create(&th[t], 0, rmat_worker, &jobs[t]);
    }
    for (int t = 0; t < T; t++) pthread_join(th[t], 0);
    int64_t n = (int64_t)1 << scale;
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    gen_permutation(n, seed + 1, perm);
    for (int64_t i = 0; i < m; i++) { src[i] = perm[src[i]]; dst[i] = perm[dst[i]]; }
    free(perm);
}

/*
 * Symmetric CSR from an edge list: drop self-loops, add every reverse edge,
 * sort each row ascending and remove duplicates. row_ptr has n+1 entries;
 * col must hold 2*m_in entries. Returns the number of directed entries.
 * Two stable counting sorts (by column, then by row) give (row, col) order.
 */
int64_t gen_build_csr(int64_t n, int64_t m_in, const int32_t *src, const int32_t *dst,
                      int32_t *row_ptr, int32_t *col) {
    int64_t m2 = 0;
    int32_t *eu = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m_in + 1));
    int32_t *ev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m_in + 1));
    for (int64_t i = 0; i < m_in; i++) {
        if (src[i] == dst[i]) continue;
        eu[m2] = src[i]; ev[m2] = dst[i]; m2++;
        eu[m2] = dst[i]; ev[m2] = src[i]; m2++;
    }
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *tu = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m2 + 1));
    int32_t *tv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m2 + 1));
    /* pass 1: stable by column */
    for (int64_t i = 0; i < m2; i++) cnt[ev[i] + 1]++;
    for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    for (int64_t i = 0; i < m2; i++) { int64_t p = cnt[ev[i]]++; tu[p] = eu[i]; tv[p] = ev[i]; }
    /* pass 2: stable by row */
    memset(cnt, 0, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < m2; i++) cnt[tu[i] + 1]++;
    for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    for (int64_t i = 0; i < m2; i++) { int64_t p = cnt[tu[i]]++; eu[p] = tu[i]; ev[p] = tv[i]; }
    free(tu); free(tv); free(cnt);
    /* dedup into CSR */
    int64_t out = 0;
    int64_t i = 0;
    for (int64_t r = 0; r < n; r++) {
        row_ptr[r] = (int32_t)out;
        int32_t last = -1;
        while (i < m2 && eu[i] == r) {
            if (ev[i] != last) { col[out++] = ev[i]; last = ev[i]; }
            i++;
        }
    }
    row_ptr[n] = (int32_t)out;
    free(eu); free(ev);
    return out;
}

/* Symmetric weight per undirected edge: 1 + rng(seed, min*2^32+max) mod (wmax). */
void gen_edge_weights(int64_t n, const int32_t *row_ptr, const int32_t *col, uint64_t seed,
                      uint32_t wmax, uint32_t *w) {
    for (int64_t u = 0; u < n; u++) {
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
            uint64_t a = (uint64_t)u, b = (uint64_t)(uint32_t)col[e];
            uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
            w[e] = 1u + (uint32_t)(gen_rng(seed, (lo << 32) | hi) % wmax);
        }
    }
}

/* ---- road-like grid ---------------------------------------------------- */

static int32_t uf_find(int32_t *p, int32_t x) {
    while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
    return x;
}

/*
 * W x H 4-neighbour grid, id = r*W + c. Undirected edge k of the full set
 * (horizontal edges first, row-major, then vertical edges, row-major) joins
 * the two cells it names. A seeded shuffle of all edges feeds Kruskal's
 * spanning-tree construction (unit cost, so the tree is a uniform random
 * order's tree); exactly `ndrop` of the non-tree edges, chosen uniformly by a
 * second seeded shuffle, are removed. Each kept undirected edge gets weight
 * 1 + rng(seed+2, k) mod wmax. Output is symmetric CSR with sorted rows;
 * col/w must hold 2*U entries. Returns the number of directed entries.
 */
int64_t gen_grid(int32_t W, int32_t H, uint64_t seed, int64_t ndrop, uint32_t wmax,
                 int32_t *row_ptr, int32_t *col, uint32_t *w) {
    int64_t n = (int64_t)W * H;
    int64_t nh = (int64_t)(W - 1) * H, nv = (int64_t)W * (H - 1);
    int64_t U = nh + nv;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(U > 0 ? U : 1));
    gen_permutation(U, seed, order);
    int32_t *par = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; i++) par[i] = (int32_t)i;
    uint8_t *keep = (uint8_t *)calloc((size_t)(U > 0 ? U : 1), 1);
    int32_t *nontree = (int32_t *)malloc(sizeof(int32_t) * (size_t)(U > 0 ? U : 1));
    int64_t nnt = 0;
    for (int64_t t = 0; t < U; t++) {
        int64_t k = order[t];
        int64_t a, b;
        if (k < nh) { int64_t r = k / (W - 1), c = k % (W - 1); a = r * W + c; b = a + 1; }
        else { int64_t kk = k - nh; int64_t r = kk / W, c = kk % W; a = r * W + c; b = a + W; }
        int32_t ra = uf_find(par, (int32_t)a), rb = uf_find(par, (int32_t)b);
        keep[k] = 1;
        if (ra != rb) { if (ra < rb) par[rb] = ra; else par[ra] = rb; }
        else nontree[nnt++] = (int32_t)k;
    }
    if (ndrop > nnt) ndrop = nnt;
    /* partial Fisher-Yates over the non-tree list, seed+1: first ndrop dropped */
    for (int64_t i = 0; i < ndrop; i++) {
        int64_t j = i + (int64_t)bounded(gen_rng(seed + 1, (uint64_t)i), (uint64_t)(nnt - i));
        int32_t t = nontree[i]; nontree[i] = nontree[j]; nontree[j] = t;
        keep[nontree[i]] = 0;
    }
    free(nontree); free(par); free(order);
    /* degree count then fill; neighbours of (r,c) in ascending id order:
       up (id-W), left (id-1), right (id+1), down (id+W) */
    for (int64_t i = 0; i <= n; i++) row_ptr[i] = 0;
    int64_t m = 0;
    for (int64_t r = 0; r < H; r++) {
        for (int64_t c = 0; c < W; c++) {
            int64_t id = r * W + c;
            row_ptr[id] = (int32_t)m;
            int64_t ks[4]; int64_t nb[4]; int q = 0;
            if (r > 0) { ks[q] = nh + (r - 1) * W + c; nb[q] = id - W; q++; }
            if (c > 0) { ks[q] = r * (W - 1) + (c - 1); nb[q] = id - 1; q++; }
            if (c < W - 1) { ks[q] = r * (W - 1) + c; nb[q] = id + 1; q++; }
            if (r < H - 1) { ks[q] = nh + r * W + c; nb[q] = id + W; q++; }
            for (int j = 0; j < q; j++) {
                if (!keep[ks[j]]) continue;
                col[m] = (int32_t)nb[j];
                w[m] = 1u + (uint32_t)(gen_rng(seed + 2, (uint64_t)ks[j]) % wmax);
                m++;
            }
        }
    }
    row_ptr[n] = (int32_t)m;
    free(keep);
    return m;
}
