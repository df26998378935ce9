/*
 * pandora.h -- C ABI of libpandora.so: single-linkage dendrograms of minimum
 * spanning trees on an MI355X (gfx950), by recursive tree contraction.
 *
 * Method: Algorithm 1 of the paper ("Dendrogram Computation using Tree
 * Contraction", Section 3): sort the MST edges by weight (Section 3.1.1),
 * contract all non-alpha edges level by level (Section 3.2, Eq. alphaedge),
 * then expand: map every edge to a leaf chain of some level or to the root
 * chain (Section 3.3.2), sort the chains and stitch them (Section 3.3.3).
 *
 * Problem statement (Algorithm 1's input; Section 3.1.2 defines the output):
 * a tree with n vertices and n-1 edges, edge i joining u[i] and v[i] with
 * fp32 weight w[i].  Edges are totally ordered by (w, i) ascending: equal
 * weights fall to the lower edge id, and -0.0 ties with +0.0.  The
 * dendrogram is the parent function P over vertices and edges:
 *   edge_parent[i]   = id of the edge that merges edge i's cluster next
 *                      (-1 for the heaviest edge, the root);
 *   vertex_parent[x] = id of the lightest edge incident to x (Eq.
 *                      vertexparent; -1 when x has no edge, i.e. n == 1).
 * All ids are INPUT edge ids.
 *
 * Memory: every array pointer is a DEVICE pointer on the current HIP device,
 * owned by the caller; the library never frees caller memory.  Scratch space
 * is cached per (device, stream) and grows on demand (see
 * pandora_workspace_bytes / pandora_release_workspaces).
 *
 * Execution: work is enqueued on `hip_stream` (NULL = the default stream).
 * The plain calls (pandora_dendrogram, pandora_dendrogram_batched) return
 * when the dendrogram is complete: contraction reads one small counter block
 * back per large level, so the host waits for the stream, and every status,
 * input errors included, comes back from the call.  This blocking form is
 * the fastest for large trees (exact grids per level).  The stream-ordered
 * form that never waits and defers input errors to pandora_stream_status is
 * pandora_dendrogram_async / pandora_dendrogram_batched_async.  Calls on
 * different streams may run concurrently from different host threads; calls
 * on the same stream are serialized.
 *
 * Errors: the return value is a pandora_status_t.  Argument errors are
 * detected before any work is enqueued.  Input errors (ids out of range, NaN
 * weights, cycles/disconnected input) are detected on the device; the
 * outputs are then unspecified but every kernel still stays within its
 * buffers.  When several input errors are present the first of
 * BAD_VERTEX, NAN_WEIGHT, NOT_A_TREE is reported.
 */
#ifndef PANDORA_H
#define PANDORA_H

#include <stddef.h>
#include <stdint.h>

/* Only the functions below are exported from libpandora.so. */
#define PANDORA_API __attribute__((visibility("default")))

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PANDORA_OK = 0,
    PANDORA_ERR_INVALID_ARG = 1,   /* bad size, null pointer, bad offsets */
    PANDORA_ERR_NOT_A_TREE = 2,    /* cycle / disconnected graph / self loop */
    PANDORA_ERR_NAN_WEIGHT = 3,    /* some w[i] is NaN */
    PANDORA_ERR_OUT_OF_MEMORY = 4, /* scratch allocation failed */
    PANDORA_ERR_HIP = 5,           /* HIP runtime error or internal check */
    PANDORA_ERR_BAD_VERTEX = 6     /* some u[i]/v[i] outside [0, n) of its tree */
} pandora_status_t;

/*
 * Dendrogram of one tree.
 *   n              number of vertices, 1 <= n <= 2^31 - 1 (edges: n-1); the
 *                  vertices of all contraction levels share one int32 id
 *                  space (about 2n ids), so a tree may have at most
 *                  1,073,741,7xx vertices (pandora_workspace_bytes returns 0
 *                  beyond; the call returns INVALID_ARG)
 *   u, v           int32[n-1] edge endpoints in [0, n)      (device)
 *   w              float[n-1] edge weights, no NaN          (device)
 *   edge_parent    int32[n-1] output                        (device)
 *   vertex_parent  int32[n]   output                        (device)
 *   hip_stream     hipStream_t to enqueue on, or NULL
 * For n == 1 the edge arrays may be NULL.
 */
PANDORA_API int pandora_dendrogram(int64_t n, const int32_t* u, const int32_t* v, const float* w,
                       int32_t* edge_parent, int32_t* vertex_parent, void* hip_stream);

/*
 * Dendrograms of B independent trees in one pass (a forest).  Tree b owns
 * vertices [voff[b], voff[b+1]) and edges [voff[b]-b, voff[b+1]-b-1) of the
 * concatenated arrays; voff is a HOST int64[B+1] array with voff[0] = 0 and
 * voff[b+1] > voff[b].  u, v and both outputs use TREE-LOCAL ids: u/v of tree
 * b are in [0, voff[b+1]-voff[b]), and edge ids in the outputs count from
 * the tree's first edge.  Each tree's result is identical to what
 * pandora_dendrogram returns for it alone.
 */
PANDORA_API int pandora_dendrogram_batched(int32_t B, const int64_t* voff, const int32_t* u, const int32_t* v,
                               const float* w, int32_t* edge_parent, int32_t* vertex_parent,
                               void* hip_stream);

/*
 * Stream-ordered variants of the two calls above (same arguments, same
 * results).  They enqueue the whole computation on hip_stream and return
 * without waiting for the device: the contraction levels run without host
 * round trips.
 *   - Argument errors come back at once.
 *   - Input errors (NOT_A_TREE, NAN_WEIGHT, BAD_VERTEX) are recorded on the
 *     device and returned later by pandora_stream_status; the outputs of a
 *     failed call are unspecified.
 *   - u, v, w and the outputs must stay valid until the stream has passed
 *     the call.  voff (host memory) is read before the call returns.
 *   - Calls on one stream run in stream order and share its scratch.  A call
 *     that needs more scratch than the stream holds waits for the stream once
 *     while the scratch grows.
 *   - No statistics (pandora_last_stats) or profiler events are kept.
 */
PANDORA_API int pandora_dendrogram_async(int64_t n, const int32_t* u, const int32_t* v, const float* w,
                                         int32_t* edge_parent, int32_t* vertex_parent, void* hip_stream);
PANDORA_API int pandora_dendrogram_batched_async(int32_t B, const int64_t* voff, const int32_t* u,
                                                 const int32_t* v, const float* w, int32_t* edge_parent,
                                                 int32_t* vertex_parent, void* hip_stream);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results, errors and blocking behaviour as pandora_dendrogram,
 * but the call makes no hipMalloc, hipFree or pinned host allocation: all of
 * its scratch lives in one fixed device array of
 * PANDORA_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs
 * on until the process ends.
 *   - Trees with pandora_workspace_bytes(n, 1) > PANDORA_NOALLOC_SCRATCH_BYTES
 *     (more than PANDORA_NOALLOC_MAX_VERTICES vertices) return
 *     PANDORA_ERR_OUT_OF_MEMORY before any work is enqueued.
 *   - Every call on one GPU uses the same array, which keeps the last call's
 *     contents (each call clears what it needs cleared).  Overlapping calls
 *     would race on it, so the library holds a per-GPU lock from the start of
 *     a call until its stream has finished it: calls from several threads run
 *     one after the other.
 *   - No profiler events are recorded; pandora_last_stats is kept.
 */
#define PANDORA_NOALLOC_SCRATCH_BYTES (64u << 20)
#define PANDORA_NOALLOC_MAX_VERTICES 798594   /* largest n that fits, any tuning */
PANDORA_API int pandora_dendrogram_noalloc(int64_t n, const int32_t* u, const int32_t* v, const float* w,
                                           int32_t* edge_parent, int32_t* vertex_parent, void* hip_stream);

/*
 * Waits for hip_stream, then returns the deferred status of the
 * stream-ordered calls made on it since the last read, and clears it.
 * PANDORA_OK if none failed.  If several failed, their errors are merged and
 * the most specific status is returned (BAD_VERTEX, then NAN_WEIGHT, then
 * NOT_A_TREE).  PANDORA_ERR_HIP if the stream itself failed.
 */
PANDORA_API int pandora_stream_status(void* hip_stream);

/*
 * Caller-owned scratch for the calls made on hip_stream (current device).
 *   dev_ptr  256-byte aligned device memory of `bytes` bytes, or NULL to go
 *            back to scratch the library allocates.
 * Calls on that stream that need more than `bytes` (see
 * pandora_workspace_bytes) return PANDORA_ERR_OUT_OF_MEMORY.  The library
 * never frees the caller's buffer.  This waits for the stream first, since
 * earlier calls may still use the previous buffer.
 * pandora_release_workspaces drops the setting.  A small status word and
 * pinned host staging stay library-owned.  Returns INVALID_ARG for a
 * misaligned pointer or zero bytes.
 */
PANDORA_API int pandora_set_workspace(void* hip_stream, void* dev_ptr, size_t bytes);

/* Device scratch bytes a call with n_total_vertices over B trees needs under
 * any tuning (admission control, preallocation, pandora_set_workspace).  0 on
 * invalid sizes and for forests with no edges. */
PANDORA_API size_t pandora_workspace_bytes(int64_t n_total_vertices, int32_t B);

/*
 * HDBSCAN* flat clusters of one tree (paper, Section "HDBSCAN* Performance":
 * the optional step after the dendrogram; cluster and selection rules of
 * HDBSCAN*, Campello et al. 2015).  Builds the dendrogram (edge_parent,
 * vertex_parent exactly as pandora_dendrogram) and then:
 *   lambda(e) = 1 / w(e) in fp64 (w = +inf gives 0); every w must be > 0.
 *   Walking down from the root, an edge node whose two children both hold
 *   >= min_cluster_size vertices splits its cluster into two new clusters
 *   born at its lambda; a smaller child's vertices leave the cluster there;
 *   with no large child the cluster ends.  Stability of a cluster = sum over
 *   its vertices of (lambda at which the vertex leaves) - (birth lambda).
 *   Excess of mass: a cluster whose stability is >= the summed values of its
 *   two children is selected (ties go to the parent); the root is never
 *   selected; the chosen clusters are the selected ones with no selected
 *   ancestor.
 * Outputs (device memory, caller-owned):
 *   labels[n]     chosen cluster of each vertex, numbered 0..k-1 in order of
 *                 each cluster's smallest vertex id; -1 = noise
 *   stability     NULL, or room for n / min_cluster_size doubles: the
 *                 stability of cluster i at index i: the correctly rounded
 *                 sum of its fp64 terms (exact accumulation, rounded once),
 *                 so the same on every run
 *   num_clusters  host pointer receiving k (may be NULL)
 * min_cluster_size >= 2.  Synchronous: returns after the stream has
 * finished the call.  Errors: INVALID_ARG (also for a weight <= 0 or NaN),
 * the dendrogram's errors (NOT_A_TREE, BAD_VERTEX, NAN_WEIGHT),
 * OUT_OF_MEMORY, HIP.  Uses the stream's workspace (see
 * pandora_flat_clusters_workspace_bytes for a caller-owned one).
 */
PANDORA_API int pandora_flat_clusters(int64_t n, const int32_t* u, const int32_t* v, const float* w,
                                      int32_t min_cluster_size, int32_t* edge_parent, int32_t* vertex_parent,
                                      int32_t* labels, double* stability, int64_t* num_clusters,
                                      void* hip_stream);
/*
 * Mutual-reachability minimum spanning tree of a point cloud: the tree that
 * HDBSCAN* builds before the dendrogram (paper, Section "HDBSCAN*
 * Performance"; definitions of Campello et al. 2015).
 *   points   device, n x dim fp32, row-major; 1 <= dim <= 4; finite
 *   min_pts  1..min(32, n): the core distance of a point is the distance to
 *            its (min_pts - 1)-th nearest other point (0 for min_pts = 1)
 *   mutual reachability = max(core(i), core(j), |x_i - x_j|), evaluated on
 *   squared distances in fp64 (coordinates summed in order, each operation
 *   rounded on its own); edges are ordered by (squared mutual reachability,
 *   min(i, j), max(i, j)), which makes the tree unique.
 * Outputs (device, caller-owned, n-1 entries each): the tree's edges in that
 * order, u[k] < v[k], with weights w64 = sqrt(squared mutual reachability)
 * (correctly rounded; may be NULL) and w32 = its fp32 rounding, ready for
 * pandora_dendrogram / pandora_flat_clusters (edge k = k-th in the order).
 * Boruvka rounds (at most about log2 n); from 2,048 points on, the searches
 * run on a uniform grid (exact: the grid changes speed only), below that as
 * full sweeps.  n <= 2^24.  Synchronous.  Errors: INVALID_ARG (also for a
 * non-finite coordinate), OUT_OF_MEMORY, HIP.
 */
PANDORA_API int pandora_emst(int64_t n, int32_t dim, const float* points, int32_t min_pts, int32_t* u, int32_t* v,
                             double* w64, float* w32, void* hip_stream);

/* Device scratch bytes pandora_flat_clusters needs for n vertices under any
 * tuning; 0 for n < 2 or sizes the dendrogram rejects. */
PANDORA_API size_t pandora_flat_clusters_workspace_bytes(int64_t n);

/* Per-stage statistics of the last successful call on this thread:
 * out[0] = levels, out[1] = sum of edges over all levels, out[2] = pointer
 * jumping launches, out[3] = levels done in the LDS tail, out[4] = edges at
 * the level the LDS tail started from, out[5] = 1 if the call ran without
 * host round trips, out[6] = 1 if some levels ran in the persistent level
 * kernel.  Returns the number filled (<= cap), or
 * -PANDORA_ERR_INVALID_ARG for a NULL out or a negative cap. */
PANDORA_API int pandora_last_stats(int64_t* out, int cap);

/* Process-wide tuning knobs (defaults in brackets), read at the start of
 * every call.  They change speed only, never results.
 *   sync_free_max_edges  calls with at most this many edges run their level
 *                        loop without host round trips: grids sized by the
 *                        level bounds, empty levels return at once [0]
 *   jump_steps           pointer-jumping steps per thread per launch [16]
 *   chain_digit_bits     radix digit width of the chain sort: 8, 9, or 0 for
 *                        automatic (9 where that saves a pass, else 8) [0]
 *   sort_tile_cfg        radix tile: 0..3 = 1024, 2048, 4096, 8192 keys per
 *                        workgroup [3]
 *   persist_max_edges    levels with at most this many edges run in one
 *                        persistent launch (workgroups on a quarter of the
 *                        compute units, grid barriers between the steps of a
 *                        level) instead of one launch per step; 0 turns it
 *                        off [0: on gfx950 the per-step launches are faster]
 * pandora_set_tuning returns INVALID_ARG for out-of-range values.
 * pandora_set_thread_tuning overrides them for calls made by the calling
 * thread only (NULL removes the override), so concurrent callers can tune
 * per call size without affecting each other. */
typedef struct {
    int32_t sync_free_max_edges;
    int32_t jump_steps;
    int32_t chain_digit_bits;
    int32_t sort_tile_cfg;
    int32_t persist_max_edges;
} pandora_tuning_t;
PANDORA_API int pandora_set_tuning(const pandora_tuning_t* t);
PANDORA_API int pandora_get_tuning(pandora_tuning_t* t);
PANDORA_API int pandora_set_thread_tuning(const pandora_tuning_t* t);

/* Per-kernel profiler (tracing).  pandora_profile_enable(mask) clears the
 * counters and, for every kernel kind k with bit k set in mask, brackets each
 * launch with a pair of HIP events on the call's stream; mask 0 turns it
 * off.  pandora_profile_read fills, per kind, the summed event time in ms,
 * the summed algorithmic bytes (the minimum traffic of each launch) and the
 * launch count; it returns the number of kinds (<= cap).  Kind names come
 * from pandora_profile_name.  Counters are process-wide. */
PANDORA_API int pandora_profile_enable(uint32_t kind_mask);
PANDORA_API int pandora_profile_read(double* ms, double* bytes, int64_t* launches, int cap);
PANDORA_API const char* pandora_profile_name(int kind);

/* Captured calls (HIP graphs).  pandora_graph_create captures the whole
 * method for fixed arguments -- the same pointers and sizes as
 * pandora_dendrogram -- into a HIP graph with its own scratch memory (the
 * level loop runs in its sync-free form, so nothing waits for the device
 * inside the graph).  pandora_graph_launch replays it on hip_stream, waits
 * for it and returns the call's status; the arrays must hold the inputs
 * when it is launched.  Replays of one graph must not overlap.  The batched
 * form takes the same arguments as pandora_dendrogram_batched (voff is
 * copied at creation).  pandora_graph_destroy frees the graph and its
 * memory. */
typedef struct pandora_graph pandora_graph_t;
PANDORA_API int pandora_graph_create(int64_t n, const int32_t* u, const int32_t* v, const float* w,
                         int32_t* edge_parent, int32_t* vertex_parent, pandora_graph_t** out);
PANDORA_API int pandora_graph_create_batched(int32_t B, const int64_t* voff, const int32_t* u, const int32_t* v,
                                 const float* w, int32_t* edge_parent, int32_t* vertex_parent,
                                 pandora_graph_t** out);
PANDORA_API int pandora_graph_launch(pandora_graph_t* g, void* hip_stream);
PANDORA_API void pandora_graph_destroy(pandora_graph_t* g);

/* Free every cached scratch allocation (waits for the owning streams). */
PANDORA_API void pandora_release_workspaces(void);

/* Human-readable name of a status code (static string). */
PANDORA_API const char* pandora_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* PANDORA_H */
