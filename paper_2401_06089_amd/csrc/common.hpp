// Shared device helpers for the dendrogram kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pandora {

constexpr int kWave = 64;
constexpr int32_t kInf = 0x7fffffff;   // "no incident edge" rank

// Deferred error bits, OR-ed into Control::err by the kernels.
enum : uint32_t {
    kErrNaN = 1u << 0,        // a weight is NaN
    kErrBadVertex = 1u << 1,  // a vertex id outside its tree
    kErrNotTree = 1u << 2,    // cycle / disconnected input
    kErrOverflow = 1u << 3,   // a level outgrew the tree bound (=> not a tree)
    kErrSpin = 1u << 4,       // a look-back wait hit its spin limit
    kErrWalk = 1u << 5,       // the expansion walk left the level tables
};

// Sizes of one contraction level, written on the device by the level before
// it: m edges, n vertices, flat offset of its vertex table.
struct LevelInfo {
    int32_t m, n;
    int64_t off;
};
constexpr int kMaxLevels = 40;   // > ceil(log2(2^31)) + 2

// Device-resident control block; zeroed at the start of every call.
struct Control {
    uint32_t err;
    uint32_t not_converged;   // pointer jumping left a vertex short of its root
    uint32_t isolated;        // isolated vertices seen (= finished components)
    uint32_t alpha_tiles;     // dynamic tile counter of the alpha/leaf scan
    int32_t m_next;           // alpha edges at the current level  (= m_{j+1})
    int32_t n_next;           // leaf edges at the current level   (= n_{j+1})
    int32_t tail_levels;      // levels finished inside the LDS tail kernel
    int32_t tail_vertices;    // vertices of the last level (all isolated)
    uint32_t grid_bar;        // arrivals at the persistent level kernel's grid barriers
    uint32_t sort_tiles[8];   // dynamic tile counters, one per radix pass
    LevelInfo lv[kMaxLevels]; // level sizes (lv[0] set at the start of a call)
    // Per-pass digit histograms (8- or 9-bit digits).  Thousands of
    // workgroups add into these words at once; their placement in cache lines
    // measurably changes the histogram kernels' speed, so it is pinned.
    alignas(256) uint32_t hist[8][512];
};

// A forest of B trees: tree b owns vertices [voff[b], voff[b+1]) and edges
// [voff[b]-b, voff[b+1]-b-1).  A single tree is B = 1, voff = {0, n}.
struct Forest {
    const int64_t* voff;   // device copy, B+1 entries
    int32_t B;
    // Index (B > 1): the tree of every 64th edge and vertex, plus a last
    // entry B-1, so that a lookup is two loads and a search between them.
    const int32_t* tree_at_edge64;
    const int32_t* tree_at_vertex64;

    __device__ __forceinline__ int32_t tree_of_edge(int64_t e) const {
        if (B == 1) return 0;
        int32_t lo = 0, hi = B - 1;          // largest b with voff[b]-b <= e
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (voff[mid] - mid <= e) lo = mid; else hi = mid - 1;
        }
        return lo;
    }
    __device__ __forceinline__ int32_t tree_of_vertex(int64_t x) const {
        if (B == 1) return 0;
        int32_t lo = 0, hi = B - 1;          // largest b with voff[b] <= x
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (voff[mid] <= x) lo = mid; else hi = mid - 1;
        }
        return lo;
    }
    __device__ __forceinline__ int64_t edge_base(int32_t b) const { return voff[b] - b; }
    // The same searches when the answer is known to lie in [lo, hi] (then
    // usually lo == hi and no step is taken).
    __device__ __forceinline__ int32_t tree_of_edge_in(int64_t e, int32_t lo, int32_t hi) const {
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (voff[mid] - mid <= e) lo = mid; else hi = mid - 1;
        }
        return lo;
    }
    __device__ __forceinline__ int32_t tree_of_vertex_in(int64_t x, int32_t lo, int32_t hi) const {
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (voff[mid] <= x) lo = mid; else hi = mid - 1;
        }
        return lo;
    }
    // Through the index: the trees of 64*floor(e/64) and of the next multiple
    // of 64 bound the tree of e (both searches are monotone in their id).
    __device__ __forceinline__ int32_t tree_of_edge_fast(int64_t e) const {
        if (B == 1) return 0;
        const int64_t k = e >> 6;
        return tree_of_edge_in(e, tree_at_edge64[k], tree_at_edge64[k + 1]);
    }
    __device__ __forceinline__ int32_t tree_of_vertex_fast(int64_t x) const {
        if (B == 1) return 0;
        const int64_t k = x >> 6;
        return tree_of_vertex_in(x, tree_at_vertex64[k], tree_at_vertex64[k + 1]);
    }
};

// Nontemporal loads and stores for streams that a kernel touches exactly
// once, so that they do not displace the randomly accessed vertex tables from
// the caches.  On MI355X this measured faster for streaming loads and
// sequential stores, and slower for random or run-scattered stores, which
// therefore keep the default policy.
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ T load_stream(const T* p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void store_stream(T* p, T v) { __builtin_nontemporal_store(v, p); }

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

// Agent-scope relaxed atomics for cross-workgroup look-back words.  The word
// itself carries all the information, so no fences are needed.
__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void raise_err(Control* c, uint32_t bits) { atomicOr(&c->err, bits); }

// Inclusive wave64 prefix sum.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, kWave);
        if (l >= d) x += y;
    }
    return x;
}

// Monotone u32 key of an fp32 weight: -0.0 is folded onto +0.0 so that the
// two tie (and fall to the edge id); negatives flip all bits, non-negatives
// flip the sign bit.  NaN is reported by the caller.
__device__ __forceinline__ uint32_t weight_key(float w) {
    uint32_t b = __float_as_uint(w);
    if (b == 0x80000000u) b = 0u;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ bool is_nan_bits(float w) {
    return (__float_as_uint(w) & 0x7fffffffu) > 0x7f800000u;
}

}  // namespace pandora
