/*
 * oracle.c -- plain CPU reference for the single-linkage dendrogram of a
 * minimum spanning tree.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header, table or helper with the GPU
 * library; the only thing the two sides have in common is the meaning of the
 * inputs and outputs.
 *
 * What it computes (paper, Section 2.3.2, bottom-up construction): visit the
 * MST edges from lightest to heaviest; each edge merges the two clusters that
 * contain its endpoints, and becomes the parent of the two nodes that
 * currently stand for those clusters (a vertex if the cluster is still a
 * single vertex, otherwise the edge that last merged it).  A union-find
 * structure (Tarjan) tracks cluster membership.
 *
 * Readings of the paper fixed here:
 *   - Order.  Section 3.1.1 asks for a consistent order on equal weights so
 *     that the dendrogram is unique.  We use the lexicographic order of
 *     (w, edge id), ascending: among equal weights the lower input id is the
 *     lighter edge.  Weights are compared by IEEE value, so -0.0 and +0.0
 *     tie and fall to the id; +-inf are ordinary values; NaN is rejected.
 *   - Numbering.  Every output names INPUT edge ids.  The root edge has
 *     parent -1; for a one-vertex tree vertex_parent[0] = -1.
 *   - Vertex parent.  The first edge in this order that touches a vertex
 *     (its lightest incident edge).  This is the paper's Eq. (vertexparent),
 *     whose "largest index" is the lightest edge because the paper indexes
 *     edges by descending weight.
 *   - Non-tree input (a repeated component while merging) is an error.
 *
 * Status codes (numeric values are part of the documented interface):
 *   0 ok, 1 invalid argument, 2 not a tree, 3 NaN weight, 6 vertex id out of
 *   range.  Checks run in the order: arguments, vertex ids, NaN, tree.
 */
#define _POSIX_C_SOURCE 200809L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>
#include <time.h>

enum {
    ORC_OK = 0,
    ORC_INVALID_ARG = 1,
    ORC_NOT_A_TREE = 2,
    ORC_NAN_WEIGHT = 3,
    ORC_BAD_VERTEX = 6,
};

typedef struct {
    float w;
    int32_t id;
} orc_edge_key;

/* Strict total order on (w, id): the order the whole method is defined on. */
static int orc_cmp(const void* pa, const void* pb)
{
    const orc_edge_key* a = (const orc_edge_key*)pa;
    const orc_edge_key* b = (const orc_edge_key*)pb;
    if (a->w < b->w) return -1;
    if (b->w < a->w) return 1;
    if (a->id < b->id) return -1;
    if (a->id > b->id) return 1;
    return 0;
}

/* Union-find with path halving.  parent[x] == x marks a root. */
static int32_t orc_find(int32_t* parent, int32_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

/*
 * Sorting by (w, id) on T host threads: the keys are cut into T runs, each run
 * is sorted by qsort with the comparator above on its own thread, and sorted
 * runs are merged pairwise, each merge of a round on its own thread, until
 * one run is left.  Every edge id is distinct, so the order is total and the
 * result does not depend on T.  (A comparison sort; it shares nothing with the
 * GPU's radix passes.)
 */
typedef struct {
    orc_edge_key* src;
    orc_edge_key* dst;
    int64_t lo, mid, hi;   /* sort: [lo, hi); merge: [lo, mid) with [mid, hi) */
} orc_job;

static void* orc_sort_run(void* p)
{
    orc_job* j = (orc_job*)p;
    qsort(j->src + j->lo, (size_t)(j->hi - j->lo), sizeof(orc_edge_key), orc_cmp);
    return NULL;
}

static void* orc_merge_runs(void* p)
{
    orc_job* j = (orc_job*)p;
    int64_t a = j->lo, b = j->mid, o = j->lo;
    while (a < j->mid && b < j->hi) {
        /* take the right run's key only when it is strictly lighter */
        if (orc_cmp(&j->src[b], &j->src[a]) < 0) j->dst[o++] = j->src[b++];
        else j->dst[o++] = j->src[a++];
    }
    while (a < j->mid) j->dst[o++] = j->src[a++];
    while (b < j->hi) j->dst[o++] = j->src[b++];
    return NULL;
}

/* Runs fn over jobs[0..k) on k threads (the calling thread takes the last). */
static int orc_run_jobs(void* (*fn)(void*), orc_job* jobs, int k)
{
    pthread_t tid[256];
    int started = 0, rc = 0;
    for (int i = 0; i + 1 < k; ++i) {
        if (pthread_create(&tid[i], NULL, fn, &jobs[i]) != 0) { rc = -1; break; }
        ++started;
    }
    for (int i = started; i < k; ++i) fn(&jobs[i]);   /* what did not get a thread runs here */
    for (int i = 0; i < started; ++i) pthread_join(tid[i], NULL);
    return rc;
}

/* keys[0..m) sorted in place by (w, id) on `threads` threads. */
static int orc_sort_keys(orc_edge_key* keys, int64_t m, int threads)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if ((int64_t)threads > m / 4096 + 1) threads = (int)(m / 4096 + 1);   /* tiny inputs: one run */
    if (threads == 1) {
        qsort(keys, (size_t)m, sizeof(orc_edge_key), orc_cmp);
        return ORC_OK;
    }
    orc_edge_key* tmp = (orc_edge_key*)malloc((size_t)m * sizeof(orc_edge_key));
    if (!tmp) return ORC_INVALID_ARG;
    int64_t bound[257];
    for (int t = 0; t <= threads; ++t) bound[t] = m * t / threads;
    orc_job jobs[256];
    for (int t = 0; t < threads; ++t) {
        jobs[t].src = keys;
        jobs[t].dst = NULL;
        jobs[t].lo = bound[t];
        jobs[t].mid = bound[t];
        jobs[t].hi = bound[t + 1];
    }
    orc_run_jobs(orc_sort_run, jobs, threads);
    orc_edge_key* src = keys;
    orc_edge_key* dst = tmp;
    for (int width = 1; width < threads; width *= 2) {
        int k = 0;
        for (int t = 0; t < threads; t += 2 * width) {
            const int tm = t + width < threads ? t + width : threads;
            const int th = t + 2 * width < threads ? t + 2 * width : threads;
            jobs[k].src = src;
            jobs[k].dst = dst;
            jobs[k].lo = bound[t];
            jobs[k].mid = bound[tm];
            jobs[k].hi = bound[th];
            ++k;
        }
        orc_run_jobs(orc_merge_runs, jobs, k);
        orc_edge_key* x = src;
        src = dst;
        dst = x;
    }
    if (src != keys) memcpy(keys, src, (size_t)m * sizeof(orc_edge_key));
    free(tmp);
    return ORC_OK;
}

/*
 * Sort edge ids 0..m-1 by (w, id) ascending into order[], on `threads` host
 * threads.  Returns a status.  Exposed on its own so tests can check the
 * ordering step by itself.
 */
int oracle_edge_order_mt(int64_t m, const float* w, int32_t* order, int threads)
{
    if (m < 0 || (m > 0 && (!w || !order))) return ORC_INVALID_ARG;
    orc_edge_key* keys = (orc_edge_key*)malloc((size_t)(m > 0 ? m : 1) * sizeof(orc_edge_key));
    if (!keys) return ORC_INVALID_ARG;
    for (int64_t i = 0; i < m; ++i) {
        if (isnan(w[i])) { free(keys); return ORC_NAN_WEIGHT; }
        keys[i].w = w[i];
        keys[i].id = (int32_t)i;
    }
    const int st = orc_sort_keys(keys, m, threads);
    if (st == ORC_OK)
        for (int64_t i = 0; i < m; ++i) order[i] = keys[i].id;
    free(keys);
    return st;
}

int oracle_edge_order(int64_t m, const float* w, int32_t* order)
{
    return oracle_edge_order_mt(m, w, order, 1);
}

static double orc_now(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/*
 * Dendrogram of one tree with n vertices and n-1 edges; edge i joins u[i] and
 * v[i] with weight w[i].  Writes edge_parent[n-1] and vertex_parent[n] (input
 * edge ids, -1 for "no parent").  All pointers are host pointers owned by the
 * caller.  The sort runs on `threads` host threads; the union-find sweep is
 * sequential.  When given, *sort_seconds and *sweep_seconds receive the wall
 * time of the two phases.
 */
int oracle_dendrogram_mt(int64_t n, const int32_t* u, const int32_t* v, const float* w,
                         int32_t* edge_parent, int32_t* vertex_parent, int threads,
                         double* sort_seconds, double* sweep_seconds)
{
    if (n < 1 || n > INT32_MAX) return ORC_INVALID_ARG;
    const int64_t m = n - 1;
    if (!vertex_parent) return ORC_INVALID_ARG;
    if (m > 0 && (!u || !v || !w || !edge_parent)) return ORC_INVALID_ARG;

    for (int64_t i = 0; i < m; ++i)
        if (u[i] < 0 || u[i] >= n || v[i] < 0 || v[i] >= n) return ORC_BAD_VERTEX;

    int32_t* order = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t* parent = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* size = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* top = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!order || !parent || !size || !top) {
        free(order); free(parent); free(size); free(top);
        return ORC_INVALID_ARG;
    }

    const double t0 = orc_now();
    int status = oracle_edge_order_mt(m, w, order, threads);
    const double t1 = orc_now();
    if (sort_seconds) *sort_seconds = t1 - t0;
    if (status != ORC_OK) goto done;

    for (int64_t x = 0; x < n; ++x) {
        parent[x] = (int32_t)x;
        size[x] = 1;
        top[x] = -1;          /* -1: the cluster is still the single vertex x */
        vertex_parent[x] = -1;
    }
    for (int64_t i = 0; i < m; ++i) edge_parent[i] = -1;

    for (int64_t k = 0; k < m; ++k) {
        const int32_t e = order[k];
        const int32_t a = orc_find(parent, u[e]);
        const int32_t b = orc_find(parent, v[e]);
        if (a == b) { status = ORC_NOT_A_TREE; goto done; }
        /* e becomes the parent of the node standing for each merged cluster. */
        const int32_t ends[2] = {a, b};
        for (int s = 0; s < 2; ++s) {
            const int32_t x = ends[s];
            if (top[x] < 0) vertex_parent[x] = e;   /* singleton: x is the vertex */
            else edge_parent[top[x]] = e;
        }
        /* union by size; the merged cluster is now represented by edge e */
        int32_t r = a, c = b;
        if (size[r] < size[c]) { r = b; c = a; }
        parent[c] = r;
        size[r] += size[c];
        top[r] = e;
    }
    /* The heaviest edge is the root and keeps edge_parent == -1. */
    if (sweep_seconds) *sweep_seconds = orc_now() - t1;

done:
    free(order); free(parent); free(size); free(top);
    return status;
}

int oracle_dendrogram(int64_t n, const int32_t* u, const int32_t* v, const float* w,
                      int32_t* edge_parent, int32_t* vertex_parent)
{
    return oracle_dendrogram_mt(n, u, v, w, edge_parent, vertex_parent, 1, NULL, NULL);
}

/*
 * Batched form: B independent trees.  Tree b owns global vertices
 * [voff[b], voff[b+1]) and global edges [voff[b]-b, voff[b+1]-b-1).  u, v and
 * both outputs use TREE-LOCAL indices.  Each tree is built by
 * oracle_dendrogram on its own slice; the first failing tree's status is
 * returned (its index in *bad_tree when bad_tree is not NULL).
 */
int oracle_dendrogram_batched(int32_t B, const int64_t* voff, const int32_t* u, const int32_t* v,
                              const float* w, int32_t* edge_parent, int32_t* vertex_parent,
                              int32_t* bad_tree)
{
    if (B < 1 || !voff) return ORC_INVALID_ARG;
    if (voff[0] != 0) return ORC_INVALID_ARG;
    for (int32_t b = 0; b < B; ++b)
        if (voff[b + 1] - voff[b] < 1) return ORC_INVALID_ARG;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t v0 = voff[b], nb = voff[b + 1] - voff[b];
        const int64_t e0 = v0 - b;
        int st = oracle_dendrogram(nb, u ? u + e0 : NULL, v ? v + e0 : NULL, w ? w + e0 : NULL,
                                   edge_parent ? edge_parent + e0 : NULL, vertex_parent + v0);
        if (st != ORC_OK) {
            if (bad_tree) *bad_tree = b;
            return st;
        }
    }
    return ORC_OK;
}

/*
 * Height of a dendrogram: the largest number of edge nodes on the path from a
 * vertex up to the root.  The paper's imbalance measure (Section 6, Table 2)
 * divides it by log2 n: near 1 for a balanced dendrogram, about n / log2 n
 * for a single chain.  Depths are filled iteratively: climb from an edge to
 * the first edge of known depth (or past the root), then walk the same path
 * again writing depths.  Returns -1 for malformed parents (an id out of
 * range, or a cycle).
 */
int64_t oracle_dendrogram_height(int64_t n, const int32_t* edge_parent, const int32_t* vertex_parent)
{
    if (n < 1 || !vertex_parent) return -1;
    if (n == 1) return 0;
    if (!edge_parent) return -1;
    const int64_t m = n - 1;
    int64_t* depth = (int64_t*)calloc((size_t)m, sizeof(int64_t));   /* 0 = not known yet */
    if (!depth) return -1;
    int64_t height = -1;
    for (int64_t e = 0; e < m; ++e) {
        if (depth[e]) continue;
        int64_t k = 0, base = 0, x = e;
        for (;;) {
            if (x < 0 || x >= m || k > m) goto bad;
            if (depth[x]) {
                base = depth[x];
                break;
            }
            ++k;
            if (edge_parent[x] == -1) {
                base = 0;
                break;
            }
            x = edge_parent[x];
        }
        x = e;
        for (int64_t d = base + k; d > base; --d) {
            depth[x] = d;
            x = edge_parent[x];
        }
    }
    for (int64_t v = 0; v < n; ++v) {
        const int32_t p = vertex_parent[v];
        if (p < 0 || p >= m) goto bad;
        if (depth[p] > height) height = depth[p];
    }
    free(depth);
    return height;
bad:
    free(depth);
    return -1;
}
