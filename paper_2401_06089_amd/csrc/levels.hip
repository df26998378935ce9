// Recursive tree contraction (paper, Section 3.2) on gfx950.
//
// Ranks: r is an edge's position in the global ascending (weight, id) order,
// so the paper's descending index is m-1-r and its maxIncident is our
// lightest incident edge.  Level 0 is processed in the caller's edge order
// (its vertex accesses then follow whatever locality the input has); deeper
// levels in compaction order.  Every comparison uses ranks, never positions.
//
// One level, m_j edges and n_j vertices:
//   k_min_incident  min64[x] = min over incident edges of (rank << 32 | pos):
//                   the lightest incident edge (Eq. vertexparent) and where
//                   its record lives.  At level 0 it also builds the 8-byte
//                   (u, v) edge records from the caller's arrays (ranks stay in
//                   their own array), translating the tree-local ids of a
//                   forest and validating them.
//   k_own           per vertex: one gather of its lightest edge's record gives
//                   the hook ptr[x] = other endpoint, the rank table entry and
//                   (level 0) the vertex's dendrogram parent; the vertex marks
//                   itself as an owner of that edge.
//   k_classify      per edge: owned by neither endpoint = alpha (Eq.
//                   alphaedge); by both = leaf edge.  Ranks fall strictly along
//                   hooks except across a leaf edge, so every supervertex is one
//                   pointer tree whose root is its leaf edge's smaller endpoint.
//                   A decoupled look-back scan of leaf flags (alpha count
//                   alongside) numbers the next level's vertices; both
//                   endpoints of each leaf edge receive its label in their ptr
//                   words with the flag bit set.
//   k_jump          pointer jumping in place (bounded steps per launch; the
//                   host relaunches until every vertex has its label); each
//                   vertex writes its flat label and records its lightest
//                   edge's supervertex for the expansion.
//   k_compact       stable compaction of alpha edges, endpoints relabelled.
//
// Vertices of all levels share one flat id space: level j occupies
// [off_j, off_j + n_j).  Isolated vertices (finished components of a forest)
// are not carried to the next level.
//
// Sizes come from Control::lv on the device (the previous level's k_classify
// writes them), clamped to the buffers' capacities, so the same kernels serve
// a host loop that reads the sizes back and a fixed launch sequence with no
// host round trip at all.
//
// k_tail runs every remaining level inside one workgroup's LDS once a level
// is small, replacing ~5 launches per level.
#include "kernels.hpp"

namespace pandora {

namespace {

constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint64_t kFlagMask = 3ull << 62;
constexpr uint64_t kCountMask = ~kFlagMask;
constexpr uint64_t kLow31 = (1ull << 31) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;

struct LevelView {
    int32_t m, n;
    int64_t off, off_next;
    bool skip;   // empty, or small enough for the LDS tail
};

__device__ __forceinline__ LevelView level_view(const LevelArgs& a) {
    const LevelInfo L = a.ctrl->lv[a.level];
    LevelView v;
    v.m = L.m < a.cap_m ? L.m : a.cap_m;
    v.n = L.n < a.cap_n ? L.n : a.cap_n;
    v.off = L.off;
    v.off_next = L.off + v.n;
    v.skip = tail_level(v.m, v.n, kTailE, kTailV);
    return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)x, d, kWave);
        const uint32_t hi = __shfl_xor((uint32_t)(x >> 32), d, kWave);
        x += ((uint64_t)hi << 32) | lo;
    }
    return x;
}

// Decoupled look-back by a whole wave: lane l reads the word of tile p-l, so
// one hop covers 64 earlier tiles.  Words are consumed newest first up to the
// nearest inclusive one, or up to the first tile that has not published yet
// (then the wave waits there).  Every lane returns the same exclusive sum.
__device__ uint64_t wave_lookback(const uint64_t* lb, int64_t tile, Control* ctrl) {
    const int lane = lane_id();
    int64_t p = tile - 1;
    uint64_t excl = 0;
    uint32_t spins = 0;
    while (true) {
        const int64_t q = p - lane;
        const uint64_t wv = q >= 0 ? ld_relaxed(lb + q) : kFlagInc;
        const uint64_t flag = wv & kFlagMask;
        const uint64_t notready = ballot(flag == 0);
        const int nr = notready ? __ffsll((long long)notready) - 1 : kWave;
        const uint64_t usable = nr == kWave ? ~0ull : ((1ull << nr) - 1ull);
        const uint64_t inc = ballot(flag == kFlagInc) & usable;
        if (inc) {
            const int f = __ffsll((long long)inc) - 1;
            return excl + wave_sum64(lane <= f ? (wv & kCountMask) : 0ull);
        }
        if (nr == 0) {
            if (++spins > kSpinLimit) {
                if (lane == 0) raise_err(ctrl, kErrSpin);
                return excl;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        spins = 0;
        excl += wave_sum64(lane < nr ? (wv & kCountMask) : 0ull);
        p -= nr;
    }
}

// After an input error every level kernel returns at once: the call's outputs
// are unspecified then, and nothing may index with the damaged tables.
// Workgroup b of G goes to group b % K; group x takes a contiguous run of the
// block ids (a permutation of [0, G)).
template <int K>
__device__ __forceinline__ int64_t spread_block(uint32_t b, uint32_t G) {
    const uint32_t q = G / K, r = G % K, x = b % K;
    return (int64_t)x * q + (x < r ? x : r) + b / K;
}

template <bool L0>
__global__ __launch_bounds__(256) void k_min_incident(LevelArgs a) {
    const LevelView L = level_view(a);
    if (L.skip || a.ctrl->err) return;
    const int64_t blk = a.spread ? spread_block<kSpreadGroups>(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t i = blk * 256 + threadIdx.x;
    if (i < scan_tiles(L.m)) a.scan_lb[i] = 0;
    if (i == 0) {
        a.ctrl->alpha_tiles = 0;
        a.ctrl->not_converged = 0;
    }
    if (i >= L.m) return;
    EdgeRec e;
    if (L0) {
        int64_t x = load_stream(a.in_u + i);
        int64_t y = load_stream(a.in_v + i);
        e.r = load_stream(a.rank + i);
        // a single tree owns every vertex; a forest's tree comes from the index
        int64_t v0 = 0, nb = L.n;
        if (a.forest.B > 1) {
            const int32_t b = a.forest.tree_of_edge_fast(i);
            v0 = a.forest.voff[b];
            nb = a.forest.voff[b + 1] - v0;
        }
        if (x < 0 || x >= nb || y < 0 || y >= nb) {
            raise_err(a.ctrl, kErrBadVertex);
            x = (x < 0 || x >= nb) ? 0 : x;
            y = (y < 0 || y >= nb) ? 0 : y;
        }
        e.u = (int32_t)(v0 + x);
        e.v = (int32_t)(v0 + y);
        store_stream(a.E + i, i32x2{e.u, e.v});
    } else {
        const i32x2 uv = load_stream(a.E + i);
        e = EdgeRec{uv.x, uv.y, load_stream(a.Er + i)};
    }
    const uint64_t key = ((uint64_t)(uint32_t)e.r << 32) | (uint64_t)(uint32_t)i;
    // Read first: values only decrease, so a stale read can only cause a
    // redundant atomic, never a missed one.  Both reads go out together.
    uint64_t mu = a.min64[e.u], mv = a.min64[e.v];
    asm volatile("" : "+v"(mu), "+v"(mv));
    if (mu > key) atomicMin((unsigned long long*)&a.min64[e.u], (unsigned long long)key);
    if (mv > key) atomicMin((unsigned long long*)&a.min64[e.v], (unsigned long long)key);
}

// ---- per-item and per-tile bodies ---------------------------------------------
// Shared by the per-level kernels below and by the persistent kernel k_levels.

// One vertex x (x >= L.n is a no-op; called by whole waves).
template <bool L0>
__device__ __forceinline__ void own_item(const LevelArgs& a, const LevelView& L, int64_t x) {
    VInfo* vinfo = a.vinfo_all + L.off;
    const bool live = x < L.n;
    const uint64_t mm = live ? load_stream(a.min64 + x) : 0;
    const bool isolated = live && mm == kNoEdge;
    const uint64_t b = ballot(isolated);
    if (b != 0 && lane_id() == __ffsll((long long)b) - 1) atomicAdd(&a.ctrl->isolated, (uint32_t)popc64(b));
    if (!live) return;
    if (isolated) {
        if (L0) a.min0[x] = kInf;
        else vinfo[x].minInc = kInf;
        if (L0) a.vertex_parent[x] = -1;
        return;
    }
    const uint32_t pos = (uint32_t)mm;
    if (pos >= (uint32_t)L.m) {
        raise_err(a.ctrl, kErrOverflow);
        return;
    }
    const i32x2 e = a.E[pos];
    const int side = (e.x == (int32_t)x) ? 0 : 1;
    a.ptr[x] = side ? e.x : e.y;
    reinterpret_cast<uint8_t*>(a.own)[2 * (int64_t)pos + side] = 1;
    if (L0) a.min0[x] = (int32_t)(mm >> 32);
    else vinfo[x].minInc = (int32_t)(mm >> 32);
    if (L0) {
        int32_t vp = (int32_t)pos;   // level 0: the edge's input id is its position
        if (a.forest.B > 1) vp = (int32_t)(vp - a.forest.edge_base(a.forest.tree_of_vertex_fast(x)));
        store_stream(a.vertex_parent + x, vp);
    }
}

// One claimed tile of the alpha/leaf classification (whole workgroup): the
// edges of two consecutive compaction tiles.
template <bool L0>
__device__ __forceinline__ void classify_tile(const LevelArgs& a, const LevelView& L, int64_t tile) {
    constexpr int W = kScanBlock / kWave;
    static_assert(kClsItems * W == kWave, "one (item, wave) count per lane of the prefix wave");
    __shared__ uint32_t s_cnt[kClsItems][W];   // alpha count << 16 | leaf count, then their prefix
    __shared__ uint64_t s_excl;
    const int tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
    const int64_t base = tile * kClsTile;
    const uint64_t lt = lanemask_lt();

    uint32_t lmask = 0;
    uint32_t lpre[kClsItems];
    int32_t root[kClsItems], other[kClsItems];
    bool selfloop = false;
    // All of the thread's loads go out before any is used (past the end the
    // last edge is read instead).
    uint32_t ov[kClsItems];
    i32x2 ev[kClsItems];
#pragma unroll
    for (int k = 0; k < kClsItems; ++k) {
        int64_t idx = base + k * kScanBlock + tid;
        idx = idx < L.m ? idx : L.m - 1;
        ov[k] = a.own[idx];
        ev[k] = load_stream(a.E + idx);
    }
#pragma unroll
    for (int k = 0; k < kClsItems; ++k) {
        const int64_t idx = base + k * kScanBlock + tid;
        bool al = false, lf = false;
        root[k] = 0;
        other[k] = 0;
        if (idx < L.m) {
            const uint32_t o = ov[k];
            a.own[idx] = 0;
            const EdgeRec e{ev[k].x, ev[k].y, 0};
            selfloop |= e.u == e.v;
            al = o == 0;
            lf = o == 0x0101;
            root[k] = e.u < e.v ? e.u : e.v;
            other[k] = e.u < e.v ? e.v : e.u;
            store_stream(a.alpha + idx, (uint8_t)(al ? 1 : 0));
        }
        const uint64_t ba = ballot(al);
        const uint64_t bl = ballot(lf);
        lpre[k] = (uint32_t)popc64(bl & lt);
        lmask |= (lf ? 1u : 0u) << k;
        if (lane == 0) s_cnt[k][wave] = ((uint32_t)popc64(ba) << 16) | (uint32_t)popc64(bl);
    }
    if (ballot(selfloop) != 0 && lane == 0) raise_err(a.ctrl, kErrNotTree);
    __syncthreads();
    if (wave == 0) {
        // Prefix of the (item, wave) counts in edge order, one per lane (both
        // counts are at most 4096, so they add as one word).
        const int k = lane / W, w = lane % W;
        const uint32_t c = s_cnt[k][w];
        const uint32_t inc = wave_incl_scan(c);
        s_cnt[k][w] = inc - c;
        const uint32_t all = __shfl(inc, kWave - 1, kWave);
        const uint32_t half = __shfl(inc - c, kScanItems * W, kWave);   // before the second half
        const uint64_t agg = ((uint64_t)(all >> 16) << 31) | (uint64_t)(all & 0xffffu);
        if (lane == 0) st_relaxed(a.scan_lb + tile, (tile == 0 ? kFlagInc : kFlagAgg) | agg);
        const uint64_t excl = tile > 0 ? wave_lookback(a.scan_lb, tile, a.ctrl) : 0;
        if (lane == 0) {
            if (tile > 0) st_relaxed(a.scan_lb + tile, kFlagInc | (excl + agg));
            s_excl = excl;
            const int32_t ea = (int32_t)(excl >> 31);
            a.tile_alpha_excl[2 * tile] = ea;
            if (2 * tile + 1 < scan_tiles(L.m)) a.tile_alpha_excl[2 * tile + 1] = ea + (int32_t)(half >> 16);
            if (tile == cls_tiles(L.m) - 1) {
                const uint64_t tot = excl + agg;
                int32_t mn = (int32_t)(tot >> 31), nn = (int32_t)(tot & kLow31);
                a.ctrl->m_next = mn;
                a.ctrl->n_next = nn;
                // Section 4.2 bounds the next level; a larger one is not a tree.
                if (mn > a.cap_next_e || nn > a.cap_next_v || mn >= L.m) {
                    raise_err(a.ctrl, kErrOverflow);
                    mn = 0;
                    nn = 0;
                }
                if (a.level + 1 < kMaxLevels) {
                    LevelInfo nx;
                    nx.m = mn;
                    nx.n = nn;
                    nx.off = L.off_next;
                    a.ctrl->lv[a.level + 1] = nx;
                }
            }
        }
    }
    __syncthreads();
    // Both endpoints of a leaf edge receive the label of their supervertex
    // (the larger one marked as such), so pointer jumping stops at either.
    const int64_t leaf_base = (int64_t)(s_excl & kLow31);
#pragma unroll
    for (int k = 0; k < kClsItems; ++k) {
        if (lmask & (1u << k)) {
            const int64_t pos = leaf_base + (s_cnt[k][wave] & 0xffffu) + lpre[k];
            const int32_t word = kLabelFlag | (int32_t)pos;
            a.ptr[root[k]] = word;
            a.ptr[other[k]] = word | kOtherEnd;
        }
    }
}

// One vertex x < L.n, one pointer-jumping round of at most `steps` steps.
// Level 0 keeps its minima and labels in two plain arrays (no expansion walk
// reads them, and the compaction's label gathers then find twice as many
// labels per cached line); deeper levels in the flat records.
template <bool L0>
__device__ __forceinline__ void jump_item(const LevelArgs& a, const LevelView& L, int64_t x, int round,
                                          int steps) {
    VInfo* vinfo = a.vinfo_all + L.off;
    auto set_label = [&](int32_t lab) {
        if (L0) a.lab0[x] = lab;
        else vinfo[x].label = lab;
    };
    // After the first round a labelled pointer means the vertex was finished
    // in an earlier round (label and supervertex record already written); an
    // isolated vertex returns below either way.
    if (round > 0 && (a.ptr[x] & kLabelFlag)) return;
    if (round == 0) {
        int32_t nn = a.ctrl->lv[a.level + 1].n;
        if (nn > a.cap_next_v) nn = a.cap_next_v;
        if (x < nn) store_stream(a.min64 + x, kNoEdge);     // the next level starts clean
    }
    // both loads go out together (the pointer is not needed for an isolated
    // vertex, which is rare, but waiting for the minimum first would put a
    // second memory round trip in front of every chase)
    const int32_t r = L0 ? load_stream(a.min0 + x) : load_stream(&vinfo[x].minInc);
    int32_t q = a.ptr[x];
    asm volatile("" : "+v"(q));   // keeps the load here, ahead of the branch below
    if (r == kInf) {
        if (round == 0) set_label(-1);
        return;
    }
    int32_t lab;
    // In the first round only the two endpoints of a leaf edge start with a
    // label (the classification wrote it), and their lightest edge is that
    // leaf edge.  It is lighter than every alpha edge of its supervertex, so
    // its chain is that supervertex itself: the smaller endpoint writes its
    // expansion record with the flag bit set (the walk then skips it), the
    // larger one writes nothing.
    const bool leaf_end = round == 0 && (q & kLabelFlag);
    const bool leaf_root = leaf_end && !(q & kOtherEnd);
    if (q & kLabelFlag) {
        lab = q & ~(kLabelFlag | kOtherEnd);
    } else {
        int32_t t = a.ptr[q];
        for (int s = 0; !(t & kLabelFlag) && s < steps; ++s) {
            q = t;
            t = a.ptr[q];
        }
        if (!(t & kLabelFlag)) {
            a.ptr[x] = q;                        // progress for the next round
            atomicOr(&a.ctrl->not_converged, 1u << (round & 31));
            return;
        }
        lab = t & ~(kLabelFlag | kOtherEnd);
        a.ptr[x] = t;                            // x now holds its label directly
    }
    const int32_t flat = (int32_t)(L.off_next + lab);
    set_label(flat);
    if (leaf_root) a.svflat[r] = flat | kLabelFlag;
    else if (!leaf_end) a.svflat[r] = flat;      // the lightest edge of x falls into this supervertex
}

// Sizes of the level after a (written by its classification), clamped.
struct NextSizes {
    int32_t m, n;
};
__device__ __forceinline__ NextSizes next_sizes(const LevelArgs& a) {
    const bool has_next = a.level + 1 < kMaxLevels;
    int32_t n_next = has_next ? a.ctrl->lv[a.level + 1].n : 0;
    int32_t m_next = has_next ? a.ctrl->lv[a.level + 1].m : 0;
    n_next = n_next < a.cap_next_v ? n_next : a.cap_next_v;
    m_next = m_next < a.cap_next_e ? m_next : a.cap_next_e;
    return {m_next, n_next};
}

// Before the compaction: the next level's scan starts clean (this level's scan
// is finished) and the scan counters restart.  g is a global thread index.
__device__ __forceinline__ void compact_prepare(const LevelArgs& a, const NextSizes& nx, int64_t g) {
    if (g < scan_tiles(nx.m)) a.scan_lb[g] = 0;
    if (g == 0) {
        a.ctrl->alpha_tiles = 0;
        a.ctrl->not_converged = 0;
    }
}

// One tile of the stable alpha compaction (whole workgroup).  With BID each
// written edge also bids for the next level's minima (the persistent kernel
// saves a grid barrier that way; with one launch per step a separate
// k_min_incident is faster, measured).
template <bool L0, bool BID>
__device__ __forceinline__ void compact_tile(const LevelArgs& a, const LevelView& L, const NextSizes& nx,
                                             int64_t tile) {
    constexpr int W = kScanBlock / kWave;
    __shared__ uint32_t s_ca[kScanItems][W];
    const int tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
    const VInfo* vinfo = a.vinfo_all + L.off;
    const int64_t base = tile * kScanTile;
    const uint64_t lt = lanemask_lt();
    // All of the thread's loads go out before any is used: the alpha flags,
    // and the records and ranks (their lines come in whole anyway, for the
    // alpha edges among them).  Past the end the last edge is read instead.
    uint32_t alv[kScanItems];
    i32x2 uv[kScanItems];
    int32_t rk[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t idx = base + k * kScanBlock + tid;
        idx = idx < L.m ? idx : L.m - 1;
        alv[k] = load_stream(a.alpha + idx);
        uv[k] = load_stream(a.E + idx);
        rk[k] = load_stream(a.Er + idx);
    }
    uint32_t amask = 0;
    uint32_t apre[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t idx = base + k * kScanBlock + tid;
        const bool al = idx < L.m && alv[k] != 0;
        const uint64_t ba = ballot(al);
        apre[k] = (uint32_t)popc64(ba & lt);
        amask |= (al ? 1u : 0u) << k;
        if (lane == 0) s_ca[k][wave] = (uint32_t)popc64(ba);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t sa = 0;
        for (int k = 0; k < kScanItems; ++k)
            for (int w = 0; w < W; ++w) {
                const uint32_t c = s_ca[k][w];
                s_ca[k][w] = sa;
                sa += c;
            }
    }
    __syncthreads();
    const int64_t abase = a.tile_alpha_excl[tile];
    // the endpoints' labels, all requested before any is used
    int32_t lx[kScanItems], ly[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        lx[k] = 0;
        ly[k] = 0;
        if (amask & (1u << k)) {
            lx[k] = L0 ? a.lab0[uv[k].x] : vinfo[uv[k].x].label;
            ly[k] = L0 ? a.lab0[uv[k].y] : vinfo[uv[k].y].label;
        }
    }
    bool selfloop = false, overflow = false;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (!(amask & (1u << k))) continue;
        const int64_t pos = abase + s_ca[k][wave] + apre[k];
        selfloop |= lx[k] == ly[k];
        const int64_t ux = (int64_t)lx[k] - L.off_next, vx = (int64_t)ly[k] - L.off_next;
        if (pos < nx.m && ux >= 0 && ux < nx.n && vx >= 0 && vx < nx.n) {
            store_stream(a.out + pos, i32x2{(int32_t)ux, (int32_t)vx});
            store_stream(a.out_r + pos, rk[k]);
            if (BID) {
                // the next level's lightest incident edges (its min64 words
                // were reset by this level's pointer jumping)
                const uint64_t key = ((uint64_t)(uint32_t)rk[k] << 32) | (uint64_t)pos;
                if (a.min64[ux] > key) atomicMin((unsigned long long*)&a.min64[ux], (unsigned long long)key);
                if (a.min64[vx] > key) atomicMin((unsigned long long*)&a.min64[vx], (unsigned long long)key);
            }
        } else {
            overflow = true;
        }
    }
    if (ballot(selfloop) != 0 && lane == 0) raise_err(a.ctrl, kErrNotTree);
    if (ballot(overflow) != 0 && lane == 0) raise_err(a.ctrl, kErrOverflow);
    __syncthreads();   // s_ca is reused by the workgroup's next tile
}

// ---- one kernel per step and level ----------------------------------------------

template <bool L0>
__global__ __launch_bounds__(256) void k_own(LevelArgs a) {
    const LevelView L = level_view(a);
    if (L.skip || a.ctrl->err) return;
    own_item<L0>(a, L, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// Level 0 and the deeper levels get separate instantiations of the remaining
// kernels too, so that per-kernel profiles separate the two (their sizes
// differ by the contraction factor).
template <bool L0>
__global__ __launch_bounds__(kScanBlock) void k_classify(LevelArgs a) {
    __shared__ uint32_t s_tile;
    const LevelView L = level_view(a);
    // The error check comes before a tile is claimed: a claimed tile is always
    // finished, so no claimed tile ever waits on a tile that nobody claimed.
    if (L.skip || a.ctrl->err) return;
    if (threadIdx.x == 0) s_tile = atomicAdd(&a.ctrl->alpha_tiles, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    if (tile >= cls_tiles(L.m)) return;        // surplus workgroup of a capacity-sized grid
    classify_tile<L0>(a, L, tile);
}

template <bool L0>
__global__ __launch_bounds__(256) void k_jump(LevelArgs a) {
    const LevelView L = level_view(a);
    if (L.skip) return;
    // a later round runs only if the previous one left some vertex unresolved
    if (a.round > 0 && !(a.ctrl->not_converged & (1u << ((a.round - 1) & 31)))) return;
    if (a.ctrl->err) return;                     // invalid input: outputs are unspecified
    const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (x >= L.n) return;
    jump_item<L0>(a, L, x, a.round, a.jump_steps);
}

template <bool L0>
__global__ __launch_bounds__(kScanBlock) void k_compact(LevelArgs a) {
    const LevelView L = level_view(a);
    if (L.skip || a.ctrl->err) return;
    // Launched before the host knows whether pointer jumping has finished:
    // then every workgroup returns here (nothing below has run yet).
    if (a.ctrl->not_converged & a.compact_guard) return;
    const NextSizes nx = next_sizes(a);
    // the grid has at least as many threads as the next level has scan tiles
    compact_prepare(a, nx, (int64_t)blockIdx.x * kScanBlock + threadIdx.x);
    const int64_t tile = blockIdx.x;
    if (tile >= scan_tiles(L.m)) return;
    compact_tile<L0, false>(a, L, nx, tile);
}

// ---- persistent kernel: all mid-size levels in one launch -------------------------
//
// A fixed grid of workgroups walks through the levels; grid barriers separate
// the steps.  Every decision that shapes the loop (a level's size, whether pointer
// jumping converged) is read after a barrier from words written before it, so
// all workgroups take the same path.  Barrier waits are bounded and stop once
// an input error is flagged (then every step returns at once and the outputs
// are unspecified anyway).

__device__ __forceinline__ void grid_barrier(Control* c, uint32_t& target) {
    __syncthreads();
    if (threadIdx.x == 0) {
        target += gridDim.x;
        __threadfence();
        atomicAdd(&c->grid_bar, 1u);
        uint32_t spins = 0;
        while (__hip_atomic_load(&c->grid_bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (++spins > kSpinLimit) {
                raise_err(c, kErrSpin);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
    }
    __syncthreads();
}

__device__ __forceinline__ bool err_set(Control* c) {
    return __hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

template <bool L0>
__device__ void persistent_level(const LevelArgs& a, const LevelView& L, int jump_rounds, uint32_t& bar,
                                 uint32_t* s_tile) {
    Control* c = a.ctrl;
    const int tid = threadIdx.x;
    const int64_t gsize = (int64_t)gridDim.x * kScanBlock;
    const int64_t gtid = (int64_t)blockIdx.x * kScanBlock + tid;

    // 1. ownership: whole waves step through the vertices together
    if (!err_set(c))
        for (int64_t xb = gtid - lane_id(); xb < L.n; xb += gsize) own_item<L0>(a, L, xb + lane_id());
    grid_barrier(c, bar);

    // 2. alpha / leaf classification and the label scan over claimed tiles
    while (true) {
        __syncthreads();
        if (tid == 0) *s_tile = err_set(c) ? 0xffffffffu : atomicAdd(&c->alpha_tiles, 1u);
        __syncthreads();
        const uint32_t t = *s_tile;
        if (t >= (uint32_t)cls_tiles(L.m)) break;
        classify_tile<L0>(a, L, t);
    }
    grid_barrier(c, bar);

    // 3. pointer jumping: bounded rounds, then one bounded only by the level size
    for (int round = 0;; ++round) {
        const bool last = round + 1 >= jump_rounds;
        const int steps = last ? (L.n > 16 ? L.n : 16) : a.jump_steps;
        // the bit of the next round is not read or written during this one
        if (gtid == 0) atomicAnd(&c->not_converged, ~(1u << ((round + 1) & 31)));
        if (!err_set(c))
            for (int64_t x = gtid; x < L.n; x += gsize) jump_item<L0>(a, L, x, round, steps);
        grid_barrier(c, bar);
        const uint32_t nc = __hip_atomic_load(&c->not_converged, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!(nc & (1u << (round & 31)))) break;
        if (last) {
            if (gtid == 0) raise_err(c, kErrNotTree);   // only a cycle keeps a vertex from its root
            break;
        }
    }

    // 4. compaction into the next level (which also bids for its minima); the
    // tiles hold workgroup barriers, so the whole workgroup takes one decision
    const NextSizes nx = next_sizes(a);
    __syncthreads();
    if (tid == 0) *s_tile = err_set(c) ? 1u : 0u;
    __syncthreads();
    if (*s_tile == 0) {
        for (int64_t g = gtid; g < scan_tiles(nx.m) || g == 0; g += gsize) compact_prepare(a, nx, g);
        for (int64_t t = blockIdx.x; t < scan_tiles(L.m); t += gridDim.x) compact_tile<L0, true>(a, L, nx, t);
    }
    grid_barrier(c, bar);
}

__global__ __launch_bounds__(kScanBlock) void k_levels(PersistArgs p) {
    __shared__ uint32_t s_tile;
    uint32_t bar = 0;
    for (int j = p.first_level; j < p.last_level; ++j) {
        LevelArgs a = p.a;
        a.level = j;
        a.cap_m = p.capE[j];
        a.cap_n = p.capV[j];
        a.cap_next_e = p.capE[j + 1];
        a.cap_next_v = p.capV[j + 1];
        a.E = j == 0 ? p.E0 : (j % 2 == 1 ? p.EA : p.EB);
        a.Er = j == 0 ? p.a.rank : (j % 2 == 1 ? p.EA_r : p.EB_r);
        a.out = j % 2 == 0 ? p.EA : p.EB;
        a.out_r = j % 2 == 0 ? p.EA_r : p.EB_r;
        const LevelView L = level_view(a);   // written before the last barrier: the same everywhere
        if (L.skip) break;
        if (j == 0) persistent_level<true>(a, L, p.jump_rounds, bar, &s_tile);
        else persistent_level<false>(a, L, p.jump_rounds, bar, &s_tile);
    }
}

// ---- the LDS tail: all remaining levels in one workgroup ----------------------

template <int BLOCK>
__device__ __forceinline__ uint32_t tail_excl_scan(uint32_t x, uint32_t* s_wsum, uint32_t* total) {
    constexpr int W = BLOCK / kWave;
    const int wave = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(x);
    if (lane_id() == kWave - 1) s_wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t s = s_wsum[w];
        if (w < wave) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

constexpr int kTailPer = kTailE / kTailThreads;   // edges per thread (blocked)

__global__ __launch_bounds__(kTailThreads) void k_tail(TailArgs a) {
    __shared__ int32_t s_u[kTailE], s_v[kTailE], s_r[kTailE];
    __shared__ int32_t s_min[kTailV], s_ptr[kTailV], s_lab[kTailV];
    __shared__ uint32_t s_wsum[kTailThreads / kWave];
    __shared__ uint32_t s_flag;
    const int tid = threadIdx.x;

    if (a.ctrl->err) return;
    // Entry: the first level that is empty or fits in LDS.
    int entry = 0;
    while (entry + 1 < kMaxLevels && !tail_level(a.ctrl->lv[entry].m, a.ctrl->lv[entry].n, kTailE, kTailV))
        ++entry;
    const LevelInfo E0 = a.ctrl->lv[entry];
    const bool level0 = entry == 0;
    const i32x2* ent = (entry % 2 == 1) ? a.EA : a.EB;
    const int32_t* ent_r = (entry % 2 == 1) ? a.EA_r : a.EB_r;
    int32_t m = E0.m, n = E0.n;
    int64_t off = E0.off;
    if (!tail_level(m, n, kTailE, kTailV) || off + (m > 0 ? n : 0) > a.flat_cap) {
        if (tid == 0) raise_err(a.ctrl, kErrOverflow);
        return;
    }
    bool first = true;
    int levels = 0;
    uint32_t err = 0;
    for (int i = tid; i < m; i += kTailThreads) {
        if (level0) {
            const int32_t b = a.forest.tree_of_edge(i);
            const int64_t v0 = a.forest.voff[b];
            const int64_t nb = a.forest.voff[b + 1] - v0;
            int64_t x = a.in_u[i], y = a.in_v[i];
            if (x < 0 || x >= nb || y < 0 || y >= nb) {
                err |= kErrBadVertex;
                x = (x < 0 || x >= nb) ? 0 : x;
                y = (y < 0 || y >= nb) ? 0 : y;
            }
            s_u[i] = (int32_t)(v0 + x);
            s_v[i] = (int32_t)(v0 + y);
            s_r[i] = a.rank[i];
        } else {
            const i32x2 e = ent[i];
            s_u[i] = e.x;
            s_v[i] = e.y;
            s_r[i] = ent_r[i];
        }
    }
    __syncthreads();

    while (m > 0) {
        const int64_t off_next = off + n;
        // lightest incident rank
        for (int x = tid; x < n; x += kTailThreads) s_min[x] = kInf;
        __syncthreads();
        for (int i = tid; i < m; i += kTailThreads) {
            atomicMin(&s_min[s_u[i]], s_r[i]);
            atomicMin(&s_min[s_v[i]], s_r[i]);
        }
        __syncthreads();
        // alpha test, hooks, leaf/alpha counts (thread t owns edges [4t, 4t+4))
        uint32_t amask = 0, lmask = 0, ca = 0, cl = 0;
#pragma unroll
        for (int q = 0; q < kTailPer; ++q) {
            const int i = tid * kTailPer + q;
            if (i >= m) break;
            const int32_t r = s_r[i], x = s_u[i], y = s_v[i];
            if (x == y) err |= kErrNotTree;
            const bool ax = s_min[x] == r, ay = s_min[y] == r;
            if (ax && ay) {
                const int32_t lo = x < y ? x : y, hi = x < y ? y : x;
                s_ptr[lo] = lo;
                s_ptr[hi] = lo;
                lmask |= 1u << q;
                ++cl;
            } else if (ax) {
                s_ptr[x] = y;
            } else if (ay) {
                s_ptr[y] = x;
            } else {
                amask |= 1u << q;
                ++ca;
            }
        }
        uint32_t tot;
        const uint32_t ex = tail_excl_scan<kTailThreads>(ca | (cl << 16), s_wsum, &tot);
        const uint32_t A = tot & 0xffffu, L = tot >> 16;
        uint32_t ea = ex & 0xffffu, el = ex >> 16;
        for (int q = 0; q < kTailPer; ++q) {
            if (lmask & (1u << q)) {
                const int i = tid * kTailPer + q;
                const int32_t lo = s_u[i] < s_v[i] ? s_u[i] : s_v[i];
                s_lab[lo] = (int32_t)(off_next + el);
                ++el;
            }
        }
        __syncthreads();
        // pointer jumping to the leaf-edge roots
        int it = 0;
        for (;; ++it) {
            __syncthreads();
            if (tid == 0) s_flag = 0;
            __syncthreads();
            bool changed = false;
            for (int x = tid; x < n; x += kTailThreads) {
                if (s_min[x] == kInf) continue;
                const int32_t p = s_ptr[x], pp = s_ptr[p];
                if (p != pp) {
                    s_ptr[x] = pp;
                    changed = true;
                }
            }
            if (changed) s_flag = 1;
            __syncthreads();
            if (s_flag == 0 || it >= 64) break;
        }
        if (it >= 64) err |= kErrNotTree;
        // labels and the level tables
        uint32_t iso = 0;
        for (int x = tid; x < n; x += kTailThreads) {
            const int32_t mi = s_min[x];
            int32_t lab = -1;
            if (mi == kInf) ++iso;
            else lab = s_lab[s_ptr[x]];
            VInfo vi;
            vi.minInc = mi;
            vi.label = lab;
            a.vinfo_all[off + x] = vi;
            if (first && level0) {
                int32_t vp = -1;
                if (mi != kInf) {
                    vp = a.perm[mi];
                    if (a.forest.B > 1) vp = (int32_t)(vp - a.forest.edge_base(a.forest.tree_of_vertex(x)));
                }
                a.vertex_parent[x] = vp;
            }
        }
        if (iso) atomicAdd(&a.ctrl->isolated, iso);
        __syncthreads();
        for (int x = tid; x < n; x += kTailThreads)
            if (s_min[x] != kInf) s_lab[x] = s_lab[s_ptr[x]];
        __syncthreads();
        // compaction: read everything first, then write (positions only move down)
        int32_t nu[kTailPer], nv[kTailPer], nr[kTailPer];
        for (int q = 0; q < kTailPer; ++q) {
            const int i = tid * kTailPer + q;
            if (i >= m) break;
            const int32_t lx = s_lab[s_u[i]];
            if (amask & (1u << q)) {
                const int32_t ly = s_lab[s_v[i]];
                if (lx == ly) err |= kErrNotTree;
                nu[q] = (int32_t)(lx - off_next);
                nv[q] = (int32_t)(ly - off_next);
                nr[q] = s_r[i];
            } else {
                a.svflat[s_r[i]] = lx;
            }
        }
        __syncthreads();
        for (int q = 0; q < kTailPer; ++q) {
            if (amask & (1u << q)) {
                s_u[ea] = nu[q];
                s_v[ea] = nv[q];
                s_r[ea] = nr[q];
                ++ea;
            }
        }
        __syncthreads();
        off = off_next;
        n = (int32_t)L;
        m = (int32_t)A;
        first = false;
        ++levels;
        if (tid == 0 && entry + levels < kMaxLevels) {   // the level table covers the tail levels too
            LevelInfo li;
            li.m = m;
            li.n = n;
            li.off = off;
            a.ctrl->lv[entry + levels] = li;
        }
        if (off + n > a.flat_cap) {
            err |= kErrOverflow;
            break;
        }
    }
    // last level: no edges left, every vertex is its component's root chain
    if (!(err & kErrOverflow) && off + n <= a.flat_cap) {
        for (int x = tid; x < n; x += kTailThreads) {
            VInfo vi;
            vi.minInc = kInf;
            vi.label = -1;
            a.vinfo_all[off + x] = vi;
            if (first && level0) a.vertex_parent[x] = -1;
        }
    }
    if (err) raise_err(a.ctrl, err);
    if (tid == 0) {
        atomicAdd(&a.ctrl->isolated, (uint32_t)n);
        a.ctrl->tail_levels = levels;
        a.ctrl->tail_vertices = n;
    }
}

inline unsigned blocks_for(int64_t n, int per) {
    const int64_t b = (n + per - 1) / per;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_min_incident(bool level0, const LevelArgs& a, hipStream_t s) {
    const int64_t work = a.cap_m > scan_tiles(a.cap_m) ? a.cap_m : scan_tiles(a.cap_m);
    if (level0) k_min_incident<true><<<blocks_for(work, 256), 256, 0, s>>>(a);
    else k_min_incident<false><<<blocks_for(work, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_own(bool level0, const LevelArgs& a, hipStream_t s) {
    if (level0) k_own<true><<<blocks_for(a.cap_n, 256), 256, 0, s>>>(a);
    else k_own<false><<<blocks_for(a.cap_n, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_classify(const LevelArgs& a, hipStream_t s) {
    if (a.level == 0) k_classify<true><<<blocks_for(cls_tiles(a.cap_m), 1), kScanBlock, 0, s>>>(a);
    else k_classify<false><<<blocks_for(cls_tiles(a.cap_m), 1), kScanBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_jump(const LevelArgs& a, hipStream_t s) {
    if (a.level == 0) k_jump<true><<<blocks_for(a.cap_n, 256), 256, 0, s>>>(a);
    else k_jump<false><<<blocks_for(a.cap_n, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_compact(const LevelArgs& a, hipStream_t s) {
    if (a.level == 0) k_compact<true><<<blocks_for(scan_tiles(a.cap_m), 1), kScanBlock, 0, s>>>(a);
    else k_compact<false><<<blocks_for(scan_tiles(a.cap_m), 1), kScanBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_levels(const PersistArgs& p, int grid, hipStream_t s) {
    k_levels<<<grid, kScanBlock, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_tail(const TailArgs& a, hipStream_t s) {
    k_tail<<<1, kTailThreads, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace pandora
