// Kernel argument blocks and host-side launchers (internal interface between
// the orchestration code and the .hip kernel files).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace pandora {

// ---- radix sort (stable LSD, 8-bit digits, one-sweep chained scan) ----------
constexpr int kMaxRadixBits = 9;                      // digits of 8 or 9 bits
constexpr int kMaxRadix = 1 << kMaxRadixBits;

// Radix tile configurations (threads x keys per thread), chosen at run time:
// small inputs want small tiles (more workgroups), large ones long digit
// runs per tile (contiguous scatters).  9-bit digits need 512 threads (one
// per digit), so they use 512 threads at the same tile size.
constexpr int kNumSortCfg = 4;
constexpr int kDefaultSortCfg = 3;
__host__ __device__ constexpr int sort_cfg_tile(int cfg) {
    return cfg == 0 ? 1024 : cfg == 1 ? 2048 : cfg == 2 ? 4096 : 8192;
}
__host__ __device__ constexpr int sort_cfg_block(int cfg, int bits) {
    return bits == 9 ? 512 : (cfg == 3 ? 512 : 256);
}

enum SortSrc { SRC_WEIGHT = 0, SRC_KEYS = 1 };
enum SortDst { DST_KEYS = 0, DST_RANK = 1 };

struct SortPassArgs {
    int64_t n;
    int cfg;                   // tile configuration (sort_cfg_tile / sort_cfg_block)
    int bits;                  // digit width of this pass: 8 or 9
    int shift;                 // bit offset of this pass's digit
    int pass;                  // row of Control::hist / sort_tiles
    const float* w;            // SRC_WEIGHT: keys from weights, values = index
    const uint32_t* keys_in;   // SRC_KEYS
    const int32_t* vals_in;    // SRC_KEYS
    uint32_t* keys_out;        // DST_KEYS
    int32_t* vals_out;         // DST_KEYS values; DST_RANK: perm (rank -> edge id)
    int32_t* rank;             // DST_RANK: rank[edge id] (inverse of perm)
    uint64_t* lb;              // look-back words of this pass, [tiles][1 << bits]
    uint64_t* lb_zero;         // look-back words of the next pass, cleared here
    int64_t lb_zero_words;
    Control* ctrl;
};

struct SortHistArgs {
    int64_t n;
    int bits;                  // digit width: 8 or 9
    int hist_row;              // first Control::hist row written
    int passes;                // digits histogrammed (<= 4)
    const float* w;            // SRC_WEIGHT
    const uint32_t* keys;      // SRC_KEYS
    uint64_t* fill64;          // optional: fill64[0..fill_n) = all ones
    int64_t fill_n;
    uint32_t* zero32;          // optional: zero32[0..zero_n) = 0
    int64_t zero_n;
    uint64_t* lb_zero;         // look-back words of the first pass, cleared here
    int64_t lb_zero_words;
    Control* ctrl;
};

hipError_t launch_sort_hist(int src, const SortHistArgs& a, hipStream_t s);
hipError_t launch_sort_pass(int src, int dst, const SortPassArgs& a, hipStream_t s);

__host__ __device__ inline int64_t sort_tiles(int64_t n, int cfg) {
    return (n + sort_cfg_tile(cfg) - 1) / sort_cfg_tile(cfg);
}

// ---- contraction levels -------------------------------------------------------
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;   // 2048 edges per workgroup

__host__ __device__ inline int64_t scan_tiles(int64_t m) { return (m + kScanTile - 1) / kScanTile; }
// The classification scans tiles of two compaction tiles each (it records
// the alpha prefix at the start of both halves).
constexpr int kClsItems = 2 * kScanItems;
constexpr int kClsTile = kScanBlock * kClsItems;     // 4096 edges per workgroup
__host__ __device__ inline int64_t cls_tiles(int64_t m) { return (m + kClsTile - 1) / kClsTile; }

// One edge of a level: its endpoints (level-local ids) in an 8-byte record,
// and its global rank in a parallel array.  The pointer-chasing steps gather
// only records, so a smaller record means more of them per cached line.  At
// level 0 the rank array is the rank of every input edge, and an edge's
// input id is its position.
struct EdgeRec {
    int32_t u, v, r;
};

// Per flat vertex: rank of its lightest edge at its level (kInf if none) and
// the flat id of its supervertex one level up (-1 if none); one 8-byte record,
// so a step of the expansion walk touches one cache line.
struct alignas(8) VInfo {
    int32_t minInc, label;
};

constexpr uint64_t kNoEdge = ~0ull;          // min64 of a vertex without edges
constexpr int32_t kLabelFlag = INT32_MIN;    // ptr word holding a final label
constexpr int32_t kOtherEnd = 1 << 30;       // ... held by the larger endpoint of a leaf edge
                                             // (labels of a level are below 2^30)

// Level kernels read their sizes from Control::lv[level] on the device, so a
// level can be launched before the host knows how large it is; grids are
// sized by the capacities below and surplus threads return at once.  A level
// that fits the LDS tail (or is empty) is left to k_tail: all its kernels
// return immediately.
struct LevelArgs {
    int level;
    int32_t cap_m;             // edge capacity of this level's buffers (grid size)
    int32_t cap_n;             // vertex capacity of this level
    const int32_t* in_u;       // level 0: caller's endpoints (tree-local ids)
    const int32_t* in_v;
    const int32_t* rank;       // level 0: rank of each input edge
    Forest forest;
    i32x2* E;                  // this level's edge records (level 0: written by k_min_incident)
    const int32_t* Er;         // ... and their ranks (level 0: `rank`)
    uint64_t* min64;           // per vertex: (rank << 32) | position of its lightest edge
    VInfo* vinfo_all;          // flat per-vertex table of all levels (level 0 as min0, lab0)
    int32_t* min0;             // level 0: lightest incident rank of each vertex
    int32_t* lab0;             // level 0: flat id of each vertex's supervertex
                               // (both in level 0's part of vinfo_all)
    int32_t* ptr;              // contraction pointers / final labels (kLabelFlag set)
    uint16_t* own;             // per edge: byte 0 = owned by u, byte 1 = owned by v
    uint8_t* alpha;            // per-edge alpha flag
    uint64_t* scan_lb;         // look-back words, one per scan tile
    int32_t* tile_alpha_excl;  // alpha prefix at the start of each scan tile
    i32x2* out;                // next level's edge records
    int32_t* out_r;            // ... and their ranks
    int32_t cap_next_e;
    int32_t cap_next_v;
    int32_t* svflat;           // per rank: flat id of the supervertex the edge is contracted into
                               // (kLabelFlag set on a leaf edge: its chain is that supervertex)
    int32_t* vertex_parent;    // level 0 output (tree-local edge ids)
    Control* ctrl;
    int jump_steps;
    int round;
    int spread;                // k_min_incident visits edge blocks in a strided order (below)
    uint32_t compact_guard;    // k_compact returns at once if Control::not_converged has one of these bits
};

// A forest of many small trees: the workgroups that run at once would all
// work near the start of the same few trees, whose first vertices collect
// most of the early edges' minima updates (at every level: each level keeps
// the trees' edges and vertices together).  With `spread` set, the
// workgroups take the edge blocks in an order strided by kSpreadGroups, so
// that concurrent workgroups work in about kSpreadGroups places of the edge
// list.
constexpr int kSpreadGroups = 1024;
constexpr int64_t kSpreadMaxMeanEdges = 1 << 16;   // spread when M <= B * this

__host__ __device__ inline bool tail_level(int64_t m, int64_t n, int tail_e, int tail_v) {
    return m == 0 || (m <= tail_e && n <= tail_v);
}

hipError_t launch_min_incident(bool level0, const LevelArgs& a, hipStream_t s);

// Levels [first_level, last_level) in one persistent launch (stops at the
// first level small enough for the LDS tail).  a holds the pointers shared by
// all levels; the per-level fields are filled from the capacities.
struct PersistArgs {
    LevelArgs a;
    i32x2* E0;
    i32x2* EA;
    i32x2* EB;
    int32_t* EA_r;
    int32_t* EB_r;
    int32_t first_level, last_level;
    int32_t jump_rounds;     // pointer-jumping rounds; the last is bounded only by the level size
    int32_t capE[kMaxLevels + 1];
    int32_t capV[kMaxLevels + 1];
};
hipError_t launch_levels(const PersistArgs& p, int grid, hipStream_t s);
hipError_t launch_own(bool level0, const LevelArgs& a, hipStream_t s);
hipError_t launch_classify(const LevelArgs& a, hipStream_t s);
hipError_t launch_jump(const LevelArgs& a, hipStream_t s);
hipError_t launch_compact(const LevelArgs& a, hipStream_t s);

// All remaining levels inside one workgroup's LDS.
constexpr int kTailThreads = 1024;
constexpr int kTailE = 4096;
constexpr int kTailV = 8192;

struct TailArgs {
    const i32x2* EA;           // level edges of odd levels
    const i32x2* EB;           // level edges of even levels >= 2
    const int32_t* EA_r;       // their ranks
    const int32_t* EB_r;
    const int32_t* in_u;       // level-0 entry: caller's endpoints and ranks
    const int32_t* in_v;
    const int32_t* rank;
    int64_t flat_cap;
    VInfo* vinfo_all;
    int32_t* svflat;
    const int32_t* perm;
    int32_t* vertex_parent;
    Forest forest;
    Control* ctrl;
};

hipError_t launch_tail(const TailArgs& a, hipStream_t s);

// ---- expansion ----------------------------------------------------------------
struct WalkArgs {
    int64_t m;
    int64_t n0;                // vertices of level 0 = flat offset of level 1
    int64_t flat_cap;
    const int32_t* svflat;
    const VInfo* vinfo_all;
    uint32_t* ckey;            // out: chain key per rank
    int bits[4];               // digit width of each chain-sort pass, least significant first
    int hist_row;
    int passes;
    uint64_t* lb_zero;
    int64_t lb_zero_words;
    Control* ctrl;
};

struct StitchArgs {
    int64_t m;
    int64_t n0;
    int64_t flat_cap;
    const uint32_t* skey;      // chain keys sorted
    const int32_t* sid;        // edge ids in chain order
    const VInfo* vinfo_all;
    const int32_t* perm;
    int32_t* edge_parent;
    Forest forest;
};

hipError_t launch_walk_hist(const WalkArgs& a, hipStream_t s);
hipError_t launch_stitch(const StitchArgs& a, hipStream_t s);

// ---- HDBSCAN* flat clusters from the dendrogram ------------------------------------
// Per-edge arrays are indexed by edge id (a born cluster is named by the edge
// where it is born, the root cluster by m); the cluster tree then works on
// dense indices 0..K-1 of the born clusters (K for the root).
constexpr int kFcBlock = 1024;   // threads of a scan workgroup (4 elements each)
constexpr int kAccChunks = 13;   // 64-bit words of one cluster's exact stability accumulator
struct FlatArgs {
    int64_t n, m;
    int32_t mcs;               // minimum cluster size (>= 2)
    const uint32_t* skey;      // chain keys, sorted (as left by the expansion)
    const int32_t* sid;        // edge ids in chain order
    const int32_t* ep;         // dendrogram: parent edge of every edge (-1 at the root)
    const int32_t* vp;         // dendrogram: parent edge of every vertex
    const float* w;
    // per edge, [m]
    int32_t* ext;              // vertices and run sizes hanging at each edge
    int32_t* size;             // vertices below each edge node
    uint32_t* bigcnt;          // children with >= mcs vertices
    int32_t* bigmax;           // the largest such child
    int32_t* T;                // cluster of each edge node (birth edge id, or m)
    int32_t* cpar;             // parent cluster (edge id or m) of each born cluster
    double* stab;              // stability of each born cluster (written once its sum is exact)
    unsigned long long* acc;   // [K_max * kAccChunks] exact fixed-point stability sums (dense clusters)
    int32_t* cidx;             // dense index of each born cluster
    // per cluster, dense
    int64_t K;                 // born clusters: an upper bound before they are counted, then the count
    int32_t* clist;            // [K] birth edge of each cluster
    int32_t* cparD;            // [K] parent cluster, -1 = the root
    uint64_t* heavy;           // [K] (size << 32 | index) of the child with more vertices
    int32_t* up[2];            // [K] heavy paths: head (pointer jumping, double-buffered)
    int32_t* dist[2];          // [K] depth below the head
    int32_t* plen;             // [K] path length (at heads)
    int32_t* poff;             // [K] first layout position of each path (at heads)
    int32_t* posof;            // [K] layout position of each cluster
    int32_t* lay;              // [K] cluster at each layout position
    double* s_lay;             // [K] stabilities in layout order
    double* b_lay;             // [K] value of each cluster's light child, in layout order
    int32_t* pending;          // [K] light children not yet valued (at heads; -1 = done)
    int32_t* ready;            // [K] round in which the path became ready (at heads)
    uint8_t* sel;              // [K+1] selected by excess of mass
    int32_t* jp[2];            // [K+1] top-down pointer jumping: jump target
    int32_t* tp[2];            // [K+1] topmost selected cluster so far
    int32_t* minv;             // [K] smallest vertex of each chosen cluster
    int32_t* cnum;             // [K] label of each chosen cluster
    int32_t* labels;           // [n] output
    double* stab_out;          // [k] output stabilities in label order (may be null)
    int64_t* count;            // [2] born clusters, chosen clusters
    uint32_t* counters;        // [4] births, error bits, paths evaluated, path heads
    uint64_t* lb[2];           // scan look-back words, alternating between consecutive scans
    int64_t lb_words;          // words per look-back buffer (tiles of the longest scan)
    uint32_t* scan_ctr;        // [2] scan tile counters, alternating likewise
    int* scan_seq;             // host: scans launched so far
};

hipError_t launch_fc_bounds(const uint32_t* skey, int64_t m, const int64_t* keys, int64_t* pos, int count,
                            hipStream_t s);
hipError_t launch_fc_prepare(const FlatArgs& a, hipStream_t s);
hipError_t launch_fc_sizes(const FlatArgs& a, int64_t lo, int64_t hi, hipStream_t s);  // also large children
hipError_t launch_fc_clusters(const FlatArgs& a, int64_t lo, int64_t hi, hipStream_t s);
hipError_t launch_fc_stab(const FlatArgs& a, hipStream_t s);        // also numbers the born clusters
hipError_t launch_fc_tree(FlatArgs& a, int rounds, hipStream_t s);  // heavy paths; swaps a.up/a.dist
hipError_t launch_fc_eval(const FlatArgs& a, int round, hipStream_t s);
hipError_t launch_fc_label(const FlatArgs& a, int rounds, hipStream_t s);

// ---- mutual-reachability MST of a point cloud (HDBSCAN*'s first step) ---------------
constexpr int kEmstMaxDim = 4;
constexpr int kEmstMaxMinPts = 32;
constexpr int kEmstPairSlots = 32;   // slots of the examined-pair count (spread against contention)
// Per-point arrays are indexed by slot: the input index for small clouds,
// the position in cell order on the grid (sorted[] maps a slot to its input
// index, which the total order and the output use; slotof[] maps back).
struct EmstArgs {
    int64_t n;
    int dim, min_pts;
    const float* pts;          // [n * dim], row-major, input order
    double* core2;             // [n] squared core distances
    int32_t* comp;             // [n] component (its root point)
    int32_t* comp2;            // [n] next round's components
    double* best_w;            // [n] least outgoing mrd2 of each point
    int32_t* best_j;           // [n] its other endpoint's slot (-1: none)
    int32_t* active;           // [n] slots that search again this round
    uint64_t* cmin_w;          // [n] per component root: least mrd2 (bits)
    uint64_t* cmin_e;          // [n] per component root: least (lo << 32 | hi) input indices at that weight
    int32_t* parent[2];        // [n] hooking and pointer jumping
    const int32_t* roots;      // [nroots] this round's component roots (null: every point)
    int64_t nroots;
    int32_t* roots_next;       // [n] the next round's roots, appended by the relabelling
    uint64_t* ew;              // [n-1] tree edges as recorded: mrd2 bits, endpoints
    int32_t* ea;
    int32_t* eb;
    int32_t* u;                // [n-1] outputs, in (mrd2, u, v) order, u < v
    int32_t* v;
    double* w64;               // may be null
    float* w32;
    uint32_t* counters;        // [8] edges, components, error bits, pointer-jumping changes / active
                               // points, grid leftovers
    // uniform grid (large clouds): points sorted by cell; searches widen ring
    // by ring and stop once no farther cell can hold a better point
    int use_grid;
    double gmin[kEmstMaxDim];  // grid origin
    double h, inv_h;           // cell edge and its inverse
    double gslack;             // distance by which rounding may misplace a point across a cell boundary
    int32_t* fallback;         // [n] points the grid search left to a full sweep
    int32_t gdim[kEmstMaxDim]; // cells per dimension (1 for unused dimensions)
    int64_t gstride[kEmstMaxDim];
    int64_t ncells;
    // profiling only: the grid searches add the point pairs they examine
    // into pairs[block % kEmstPairSlots]
    int count_pairs;
    uint64_t* pairs;
    uint32_t* bbox;            // [2 * kEmstMaxDim] order-preserving bits of each min and of each max, complemented
    int32_t* cellof;           // [n] cell of each point
    int32_t* cstart;           // [ncells + 1] first sorted position of each cell
    int32_t* cfill;            // [ncells] points per cell, then a fill counter
    int32_t* sorted;           // [n] input index at each sorted position (slot)
    int32_t* slotof;           // [n] slot of each input index
    float* spts;               // [n * kEmstMaxDim] input coordinates in sorted order (16-byte slots)
    uint8_t* partial;          // [n] the point's search stopped early: search again next round
    uint64_t* scan_agg;        // cell-count scan: per-block sums
};
hipError_t launch_em_core(const EmstArgs& a, const int32_t* list, int64_t count, hipStream_t s);
hipError_t launch_em_active(const EmstArgs& a, hipStream_t s);   // counts into counters[3]
hipError_t launch_em_search(const EmstArgs& a, const int32_t* list, int64_t count, hipStream_t s);
hipError_t launch_em_merge_edges(const EmstArgs& a, hipStream_t s);
hipError_t launch_em_jump(const EmstArgs& a, int src, hipStream_t s);
hipError_t launch_em_relabel(const EmstArgs& a, int src, hipStream_t s);
hipError_t launch_em_sort_key(const EmstArgs& a, int word, const int32_t* order, uint32_t* keys, int32_t* order_out,
                              hipStream_t s);
hipError_t launch_em_out(const EmstArgs& a, const int32_t* order, hipStream_t s);
hipError_t launch_em_bbox(const EmstArgs& a, hipStream_t s);
hipError_t launch_em_grid(const EmstArgs& a, hipStream_t s);         // cells, counts, scan, scatter
hipError_t launch_em_core_grid(const EmstArgs& a, hipStream_t s);      // leftovers listed in fallback
hipError_t launch_em_search_grid(const EmstArgs& a, int64_t active, hipStream_t s);

// ---- misc -----------------------------------------------------------------------
// Clears the control block; voff1, if given, receives the offsets {0, n} of a
// single tree.
hipError_t launch_zero_control(Control* c, int32_t m, int32_t n, int64_t* voff1, hipStream_t s);
hipError_t launch_finalize(const Control* c, int32_t B, uint32_t* sticky, hipStream_t s);
// Fills the forest index (te: (m+63)/64 + 1 entries, tv: (n+63)/64 + 1).
hipError_t launch_forest_index(const Forest& f, int64_t m, int64_t n, int32_t* te, int32_t* tv, hipStream_t s);
hipError_t launch_clear_words(uint32_t* p, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t value, hipStream_t s);

}  // namespace pandora
