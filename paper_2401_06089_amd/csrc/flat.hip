// HDBSCAN* flat clusters from the dendrogram on gfx950: the optional step
// after the dendrogram that the paper names in its HDBSCAN* section, with the
// cluster definition and the excess-of-mass selection of HDBSCAN* (Campello
// et al. 2015, the paper's reference for it).
//
// The expansion leaves every dendrogram chain sorted and contiguous: runs of
// equal chain keys, lightest edge first, in ascending key order.  An edge's
// parent is the next edge of its run; the heaviest edge of a run hangs below
// the run's head edge, which lies in a run whose key belongs to a later
// contraction level.  So with the runs grouped by level:
//   sizes     size(e_k) = size(e_{k-1}) + ext(e_k), a segmented prefix sum
//             along each run, where ext(e) = vertices hanging at e plus the
//             sizes of the runs headed by e (added by earlier levels).
//             Levels run in ascending order.
//   clusters  T(e) = e if e is born (it and its sibling both hold >= mcs
//             vertices), else T(parent): the last birth along the run from its
//             heavy end, seeded by T(head).  Levels run in descending order.
// Both are ordered scans (an associative, non-commutative combine) over one
// level's positions, in one pass: tiles are claimed in order and find their
// prefix by a decoupled look-back in which a wave combines 64 earlier tiles.
// The size scan also counts, at each parent, the children with >= mcs
// vertices.
//
// Stabilities are sums of fp64 count * lambda terms (lambda = 1 / w), each
// accumulated exactly in fixed point and rounded once, so they are the
// correctly rounded sums whatever order the atomics land in; the selection
// compares them in fp64.
//
// Excess of mass runs on the cluster tree (each cluster splits into exactly
// two or ends), whose depth reaches tens of thousands on skewed trees.  It is
// cut into heavy paths (each cluster continues into its child with more
// vertices), so that any cluster has O(log n) light ancestors.  Every path is
// laid out contiguously, bottom first, and evaluated by one wave in order:
//   v = max(s_i, v_below + v_light_child_i)
// exactly the oracle's operations, so values and decisions are the same.
// A path runs once the values of all its light children are in, so there are
// at most about log2 n rounds.  The chosen clusters (selected, no selected
// ancestor) come from pointer jumping; labels are numbered by the smallest
// vertex of each cluster.
#include <utility>

#include "kernels.hpp"

namespace pandora {

namespace {

constexpr int kFcItems = 4;
constexpr int kFcTile = kFcBlock * kFcItems;
constexpr int kFcWaves = kFcBlock / kWave;
constexpr uint64_t kSegStart = 1ull << 61;         // inside the 62 state bits of a look-back word
constexpr uint64_t kLbAgg = 1ull << 62;            // look-back word: aggregate of its tile only
constexpr uint64_t kLbInc = 2ull << 62;            // look-back word: inclusive of all tiles before
constexpr uint64_t kLbState = (1ull << 62) - 1;
constexpr uint32_t kLbSpinLimit = 1u << 22;

struct OpSegSum {   // (run-start flag, sum): a start discards everything before it
    __device__ static uint64_t identity() { return 0; }
    __device__ static uint64_t combine(uint64_t a, uint64_t b) {
        return (b & kSegStart) ? b : ((a & kSegStart) | ((a & ~kSegStart) + b));
    }
};
struct OpLastSet {  // value + 1, 0 = unset: the last set value wins
    __device__ static uint64_t identity() { return 0; }
    __device__ static uint64_t combine(uint64_t a, uint64_t b) { return b ? b : a; }
};
struct OpSum {
    __device__ static uint64_t identity() { return 0; }
    __device__ static uint64_t combine(uint64_t a, uint64_t b) { return a + b; }
};

// Exclusive scan of one value per thread in thread order (whole workgroup);
// *total receives the combination of all of them.
template <class Op>
__device__ uint64_t block_scan(uint64_t x, uint64_t* s_w, uint64_t* total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    uint64_t inc = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t y = __shfl_up(inc, d, kWave);
        if (lane >= d) inc = Op::combine(y, inc);
    }
    uint64_t lex = __shfl_up(inc, 1, kWave);
    if (lane == 0) lex = Op::identity();
    if (lane == kWave - 1) s_w[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = Op::identity();
        for (int w = 0; w < kFcWaves; ++w) {
            const uint64_t t = s_w[w];
            s_w[w] = run;
            run = Op::combine(run, t);
        }
        s_w[kFcWaves] = run;
    }
    __syncthreads();
    const uint64_t res = Op::combine(s_w[wave], lex);
    *total = s_w[kFcWaves];
    __syncthreads();   // s_w is reused by the next scan
    return res;
}

// ---- the three scans ------------------------------------------------------------

// Sizes over one level's positions [lo, lo + cnt).
// Each final size is also counted at the edge node's parent when it reaches
// mcs (the parent's large children), so no separate pass is needed.
struct SizeScan {
    const uint32_t* skey;
    const int32_t* sid;
    int32_t* ext;
    int32_t* size;
    const int32_t* ep;
    uint32_t* bigcnt;
    int32_t* bigmax;
    int32_t mcs;
    int64_t lo, cnt, m;
    __device__ uint64_t load(int64_t k) const {
        const int64_t i = lo + k;
        const bool start = k == 0 || skey[i] != skey[i - 1];
        const int32_t e = sid[i];
        const uint32_t x = (e >= 0 && e < m) ? (uint32_t)ext[e] : 0u;
        return (start ? kSegStart : 0ull) | (uint64_t)x;
    }
    __device__ void store(int64_t k, uint64_t incl, uint64_t) const {
        const int64_t i = lo + k;
        const int32_t e = sid[i];
        if (e < 0 || e >= m) return;
        const int32_t sz = (int32_t)(incl & ~kSegStart);
        size[e] = sz;
        int32_t parent;
        if (k == cnt - 1 || skey[i + 1] != skey[i]) {   // heaviest edge of its run: hangs at the head
            parent = ep[e];
            if (parent >= 0 && parent < m) atomicAdd(&ext[parent], sz);
        } else {
            parent = sid[i + 1];
        }
        if (sz >= mcs && parent >= 0 && parent < m) {
            atomicAdd(&bigcnt[parent], 1u);
            atomicMax(&bigmax[parent], sz);
        }
    }
};

// Clusters over one level's positions, heaviest first: position hi-1-k.
struct ClusterScan {
    const uint32_t* skey;
    const int32_t* sid;
    const int32_t* size;
    const int32_t* ep;
    const uint32_t* bigcnt;
    int32_t* T;
    int32_t mcs, root;
    int64_t hi, cnt, m;
    __device__ uint64_t load(int64_t k) const {
        const int64_t i = hi - 1 - k;
        const int32_t e = sid[i];
        if (e < 0 || e >= m) return 0;
        const int32_t p = ep[e];
        const bool parent_ok = p >= 0 && p < m;
        if (parent_ok && size[e] >= mcs && bigcnt[p] == 2u) return (uint64_t)e + 1;   // born here
        if (k == 0 || skey[i + 1] != skey[i]) {                                        // heavy end of a run
            const int32_t t = parent_ok ? T[p] : root;
            return (uint64_t)(uint32_t)t + 1;
        }
        return 0;
    }
    __device__ void store(int64_t k, uint64_t incl, uint64_t) const {
        const int32_t e = sid[hi - 1 - k];
        if (e >= 0 && e < m) T[e] = incl ? (int32_t)(incl - 1) : root;
    }
};

// Dense numbering of the born clusters (edges with T(e) = e), in edge order.
struct BirthScan {
    const int32_t* T;
    int32_t* clist;
    int32_t* cidx;
    int64_t* count;
    int64_t cnt;
    __device__ uint64_t load(int64_t k) const { return T[k] == (int32_t)k ? 1ull : 0ull; }
    __device__ void store(int64_t k, uint64_t incl, uint64_t v) const {
        if (v) {
            clist[incl - 1] = (int32_t)k;
            cidx[k] = (int32_t)(incl - 1);
        }
        if (k == cnt - 1) *count = (int64_t)incl;
    }
};

// Offsets of the heavy paths in the layout (one entry per path head).
struct PathScan {
    const int32_t* up;
    const int32_t* plen;
    int32_t* poff;
    int64_t cnt;
    __device__ uint64_t load(int64_t i) const { return up[i] == (int32_t)i ? (uint64_t)plen[i] : 0ull; }
    __device__ void store(int64_t i, uint64_t incl, uint64_t v) const {
        if (up[i] == (int32_t)i) poff[i] = (int32_t)(incl - v);
    }
};

// Label numbering over the vertices: the first vertex of each chosen cluster.
struct NumberScan {
    const int32_t* labels;     // chosen cluster (dense index) or -1
    const int32_t* minv;
    const int32_t* clist;
    int32_t* cnum;
    const double* stab;
    double* stab_out;          // may be null
    int64_t* count;
    int64_t cnt;
    __device__ uint64_t load(int64_t k) const {
        const int32_t c = labels[k];
        return (c >= 0 && minv[c] == (int32_t)k) ? 1ull : 0ull;
    }
    __device__ void store(int64_t k, uint64_t incl, uint64_t v) const {
        if (v) {
            const int32_t c = labels[k];
            cnum[c] = (int32_t)(incl - 1);
            if (stab_out) stab_out[incl - 1] = stab[clist[c]];
        }
        if (k == cnt - 1) *count = (int64_t)incl;
    }
};

struct ScanState {
    uint64_t* lb;              // this scan's look-back words (cleared by the scan before)
    uint64_t* lb_next;         // the next scan's, cleared here
    int64_t words;
    uint32_t* ctr;             // this scan's tile counter
    uint32_t* ctr_next;
    uint32_t* err;
};

// Ordered combination of the lanes' values, lane L-1 (the oldest tile) first;
// lanes >= L contribute nothing.  Lane 0 returns the result.
template <class Op>
__device__ uint64_t wave_combine_desc(uint64_t v, int L) {
    const int lane = lane_id();
    uint64_t x = lane < L ? v : Op::identity();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t y = __shfl_down(x, d, kWave);
        x = Op::combine(lane + d < kWave ? y : Op::identity(), x);
    }
    return x;
}

// Decoupled look-back by wave 0: lane l reads the word of tile p-l; words are
// consumed newest first up to the nearest inclusive one (or the first tile
// that has not published: the wave waits there).  Lane 0 gets the exclusive
// prefix of the tile.
template <class Op>
__device__ uint64_t scan_lookback(const uint64_t* lb, int64_t tile, uint32_t* err) {
    const int lane = lane_id();
    int64_t p = tile - 1;
    uint64_t excl = Op::identity();
    uint32_t spins = 0;
    while (true) {
        const int64_t q = p - lane;
        const uint64_t w = q >= 0 ? ld_relaxed(lb + q) : (kLbInc | Op::identity());
        const uint64_t flag = w & ~kLbState;
        const uint64_t notready = ballot(flag == 0);
        const int nr = notready ? __ffsll((long long)notready) - 1 : kWave;
        const uint64_t inc = ballot(flag == kLbInc) & (nr == kWave ? ~0ull : ((1ull << nr) - 1ull));
        if (inc) {
            const int f = __ffsll((long long)inc) - 1;
            return Op::combine(wave_combine_desc<Op>(w & kLbState, f + 1), excl);
        }
        if (nr == 0) {
            if (++spins > kLbSpinLimit) {
                if (lane == 0) atomicOr(err, 32u);
                return excl;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        spins = 0;
        excl = Op::combine(wave_combine_desc<Op>(w & kLbState, nr), excl);
        p -= nr;
    }
}

// One pass over the range: tiles are claimed in order, each loads its
// elements once, publishes its aggregate, looks back for its prefix and
// finishes.  It also clears the other look-back buffer and tile counter for
// the scan after it.
template <class Op, class P>
__global__ __launch_bounds__(kFcBlock) void k_scan(P p, ScanState st) {
    __shared__ uint64_t s_w[kFcWaves + 1];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_excl;
    {
        const int64_t stride = (int64_t)gridDim.x * kFcBlock;
        for (int64_t i = (int64_t)blockIdx.x * kFcBlock + threadIdx.x; i < st.words; i += stride) st.lb_next[i] = 0;
        if (blockIdx.x == 0 && threadIdx.x == 0) *st.ctr_next = 0;
    }
    if (threadIdx.x == 0) s_tile = atomicAdd(st.ctr, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t base = tile * kFcTile + (int64_t)threadIdx.x * kFcItems;
    uint64_t v[kFcItems];
    uint64_t acc = Op::identity();
#pragma unroll
    for (int j = 0; j < kFcItems; ++j) {
        v[j] = base + j < p.cnt ? p.load(base + j) : Op::identity();
        acc = Op::combine(acc, v[j]);
    }
    uint64_t total;
    const uint64_t ex = block_scan<Op>(acc, s_w, &total);
    if (threadIdx.x < kWave) {
        if (threadIdx.x == 0) st_relaxed(st.lb + tile, (tile == 0 ? kLbInc : kLbAgg) | total);
        const uint64_t excl = tile > 0 ? scan_lookback<Op>(st.lb, tile, st.err) : Op::identity();
        if (threadIdx.x == 0) {
            if (tile > 0) st_relaxed(st.lb + tile, kLbInc | Op::combine(excl, total));
            s_excl = excl;
        }
    }
    __syncthreads();
    uint64_t run = Op::combine(s_excl, ex);
#pragma unroll
    for (int j = 0; j < kFcItems; ++j) {
        if (base + j >= p.cnt) break;
        run = Op::combine(run, v[j]);
        p.store(base + j, run, v[j]);
    }
}

template <class Op, class P>
hipError_t run_scan(const P& p, const FlatArgs& a, hipStream_t s) {
    if (p.cnt < 1) return hipSuccess;
    const int64_t tiles = (p.cnt + kFcTile - 1) / kFcTile;
    // the look-back buffers alternate between consecutive scans
    const int cur = a.scan_seq[0] & 1;
    ScanState st{a.lb[cur], a.lb[cur ^ 1], a.lb_words, a.scan_ctr + cur, a.scan_ctr + (cur ^ 1), &a.counters[1]};
    ++a.scan_seq[0];
    k_scan<Op, P><<<(unsigned)tiles, kFcBlock, 0, s>>>(p, st);
    return hipGetLastError();
}

// ---- per-element passes ----------------------------------------------------------

inline unsigned grid_for(int64_t n, int per = 256, int64_t cap = 1 << 16) {
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

__global__ void k_fc_clear(FlatArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.m; i += stride) {
        a.ext[i] = 0;
        a.bigcnt[i] = 0;
        a.bigmax[i] = 0;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.lb_words; i += stride) a.lb[0][i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 4) a.counters[threadIdx.x] = 0;   // births, errors, paths done, heads
    if (blockIdx.x == 0 && threadIdx.x < 2) {
        a.count[threadIdx.x] = 0;
        a.scan_ctr[threadIdx.x] = 0;
    }
}

// Vertices count at their parent edge; every weight must be > 0.
__global__ void k_fc_prepare(FlatArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        const int32_t p = a.vp[i];
        if (p >= 0 && p < a.m) atomicAdd(&a.ext[p], 1);
        else bad = true;
        if (i < a.m && !(a.w[i] > 0.0f)) bad = true;    // also NaN
    }
    if (ballot(bad) != 0 && lane_id() == 0) atomicOr(&a.counters[1], 1u);
}

// Exact stabilities.  Every term is an fp64 value t = d * lambda (or the birth
// term -size * lambda_birth) with lambda = 1/w for an fp32 weight w > 0, so
// |t| lies in [2^-180, 2^180] and is an integer multiple of 2^-180.  Each
// cluster therefore sums its terms exactly in a fixed-point accumulator of
// kAccChunks signed 64-bit words, word k holding a multiple of
// 2^(32k + kAccBase): a term adds its 53-bit significand, shifted into place,
// as three 32-bit pieces.  At most n - 1 < 2^31 pieces below 2^32 meet in a
// word, so no word overflows, and integer sums do not depend on their order.
// A sum of fewer than 2^31 terms is below 2^211 in magnitude, so the 13 words
// (bits 2^-192 .. 2^224) hold it, and the carry out of the top word is its
// sign.
// The finished sum is rounded once to the nearest double (ties to even): the
// correctly rounded sum of the terms, whatever the order of the additions.
constexpr int kAccBase = -192;

struct TermPieces {
    int k;                  // first accumulator word
    int64_t p0, p1, p2;     // signed pieces for words k, k+1, k+2
};

__device__ __forceinline__ TermPieces term_pieces(double t) {
    TermPieces r{0, 0, 0, 0};
    const uint64_t bits = (uint64_t)__double_as_longlong(t);
    const int bexp = (int)((bits >> 52) & 0x7ff);
    if (bexp == 0) return r;                        // zero (the range above has no subnormal terms)
    const uint64_t mant = (bits & ((1ull << 52) - 1)) | (1ull << 52);
    const int shift = (bexp - 1075) - kAccBase;     // t = mant * 2^(bexp - 1075)
    const int k = shift >> 5, o = shift & 31;
    const uint64_t lo = mant << o;                  // bits [0, 64) of mant * 2^o
    const uint64_t hi = o ? (mant >> (64 - o)) : 0; // bits [64, 85)
    r.k = k;
    r.p0 = (int64_t)(lo & 0xffffffffull);
    r.p1 = (int64_t)(lo >> 32);
    r.p2 = (int64_t)hi;
    if (bits >> 63) {
        r.p0 = -r.p0;
        r.p1 = -r.p1;
        r.p2 = -r.p2;
    }
    return r;
}

// Adds the pieces of t into accumulator acc (kAccChunks words; pieces beyond
// the last word cannot occur for terms in range).
__device__ __forceinline__ void acc_add_term(unsigned long long* acc, double t) {
    const TermPieces q = term_pieces(t);
    if (q.p0) atomicAdd(acc + q.k, (unsigned long long)q.p0);
    if (q.p1) atomicAdd(acc + q.k + 1, (unsigned long long)q.p1);
    if (q.p2 && q.k + 2 < kAccChunks) atomicAdd(acc + q.k + 2, (unsigned long long)q.p2);
}

// Sums the terms of the lanes with act into cluster accumulators.  Lanes that
// share the first active lane's cluster (edges of one large cluster, usually)
// add their pieces word by word across the wave first (exact integer sums)
// and send one atomic per word.  Every lane of the wave must call it.
__device__ void wave_acc_into(unsigned long long* acc, int32_t ci, double t, bool act) {
    const uint64_t m = ballot(act);
    if (!m) return;
    const int leader = __ffsll((long long)m) - 1;
    const int32_t c0 = __shfl(ci, leader, kWave);
    const bool same = act && ci == c0;
    const TermPieces q = same ? term_pieces(t) : TermPieces{0, 0, 0, 0};
    // the lanes' first words span a range [kmin, kmax]; combine word by word
    int kmin = same ? q.k : kAccChunks, kmax = same ? q.k + 2 : -1;
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        kmin = min(kmin, __shfl_xor(kmin, d, kWave));
        kmax = max(kmax, __shfl_xor(kmax, d, kWave));
    }
    if (kmax >= kAccChunks) kmax = kAccChunks - 1;
    for (int w = kmin; w <= kmax; ++w) {
        int64_t x = (w == q.k ? q.p0 : 0) + (w == q.k + 1 ? q.p1 : 0) + (w == q.k + 2 ? q.p2 : 0);
        if (!same) x = 0;
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
        if (lane_id() == leader && x != 0) atomicAdd(acc + (int64_t)c0 * kAccChunks + w, (unsigned long long)x);
    }
    if (act && !same) acc_add_term(acc + (int64_t)ci * kAccChunks, t);
}

// Departure terms count * lambda per edge node of a cluster region, the birth
// term -size * lambda_birth, and each born cluster's parent cluster.  Born
// clusters are already numbered (cidx), and their accumulators cleared.
__global__ void k_fc_stab(FlatArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t root = (int32_t)a.m;
    const int lane = lane_id();
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); e0 < a.m; e0 += stride) {
        const int64_t e = e0 + lane;
        int32_t ci = -1;
        double term = 0.0;
        bool born = false;
        const int32_t sz = e < a.m ? a.size[e] : 0;
        if (e < a.m && sz >= a.mcs) {
            const int32_t ce = a.T[e];
            if (ce < 0 || ce > root) {
                atomicOr(&a.counters[1], 2u);
            } else {
                const int32_t d = a.bigcnt[e] == 1u ? sz - a.bigmax[e] : sz;
                if (ce != root) {
                    ci = a.cidx[ce];
                    term = (double)d * (1.0 / (double)a.w[e]);
                    if (ci < 0 || ci >= a.K) {               // not a numbered cluster
                        atomicOr(&a.counters[1], 2u);
                        ci = -1;
                    }
                }
                if (ce == (int32_t)e && ci >= 0) {
                    const int32_t p = a.ep[e];                // a born edge always has a parent
                    if (p < 0 || p >= a.m) {
                        atomicOr(&a.counters[1], 2u);
                    } else {
                        const double lamb = 1.0 / (double)a.w[p];
                        acc_add_term(a.acc + (int64_t)ci * kAccChunks, -((double)sz * lamb));
                        a.cpar[e] = a.T[p];
                        born = true;
                    }
                }
            }
        }
        wave_acc_into(a.acc, ci, term, ci >= 0);
        const uint64_t b = ballot(born);
        if (b != 0 && lane == __ffsll((long long)b) - 1) atomicAdd(&a.counters[0], (uint32_t)popc64(b));
    }
}

__global__ void k_fc_acc_clear(FlatArgs a) {
    const int64_t K = *a.count < a.K ? *a.count : a.K;   // born clusters, counted by the birth scan
    const int64_t words = K * kAccChunks;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) a.acc[i] = 0;
}

// The exact sum of cluster i, rounded to the nearest double (ties to even),
// into stab[birth edge].
__global__ void k_fc_acc_round(FlatArgs a) {
    const int64_t K = *a.count < a.K ? *a.count : a.K;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += stride) {
        const unsigned long long* w = a.acc + i * kAccChunks;
        // carries: limbs of 32 bits, two's complement, with the sign in the top carry
        uint32_t limb[kAccChunks];
        int64_t carry = 0;
        for (int k = 0; k < kAccChunks; ++k) {
            const int64_t x = (int64_t)w[k] + carry;
            limb[k] = (uint32_t)x;
            carry = x >> 32;                          // arithmetic shift: floor division
        }
        const bool neg = carry < 0;
        if (neg) {                                   // magnitude of the negative sum
            uint64_t c = 1;
            for (int k = 0; k < kAccChunks; ++k) {
                const uint64_t x = (uint64_t)(uint32_t)~limb[k] + c;
                limb[k] = (uint32_t)x;
                c = x >> 32;
            }
        }
        int top = kAccChunks - 1;
        while (top >= 0 && limb[top] == 0) --top;
        double val = 0.0;
        if (top >= 0) {
            const int hb = 32 * top + (31 - __clz((int)limb[top]));   // highest set bit of the magnitude
            // the 53 bits from hb down, then the rounding bit and the sticky rest
            auto bit = [&](int b) -> uint32_t { return b < 0 ? 0u : (limb[b >> 5] >> (b & 31)) & 1u; };
            uint64_t mant = 0;
            for (int b = hb; b > hb - 53; --b) mant = (mant << 1) | bit(b);
            const int rb = hb - 53;
            const uint32_t round = bit(rb);
            bool sticky = false;                          // any bit below the rounding bit
            if (rb > 0) {
                const int lw = rb >> 5, lb = rb & 31;
                sticky = lb != 0 && (limb[lw] & ((1u << lb) - 1u)) != 0;
                for (int k = 0; k < lw && !sticky; ++k) sticky = limb[k] != 0;
            }
            int e2 = hb - 52 + kAccBase;                 // value = mant * 2^e2
            if (round && (sticky || (mant & 1))) {
                ++mant;
                if (mant >> 53) {
                    mant >>= 1;
                    ++e2;
                }
            }
            val = ldexp((double)mant, e2);
        }
        a.stab[a.clist[i]] = neg ? -val : val;
    }
}

// ---- the cluster tree, on dense cluster indices 0..K-1 -------------------------------

__global__ void k_fc_dense_clear(FlatArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= a.K; i += stride) {
        if (i < a.K) {
            a.heavy[i] = 0;
            a.plen[i] = 0;
            a.minv[i] = INT32_MAX;
        }
        a.sel[i] = 0;
    }
}

// Parent cluster (dense; -1 = the root) and the child with more vertices.
__global__ void k_fc_tree(FlatArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.K; i += stride) {
        const int32_t c = a.clist[i];
        const int32_t p = a.cpar[c];
        int32_t pd = -1;
        if (p >= 0 && p < a.m && a.T[p] == p) pd = a.cidx[p];
        else if (p != (int32_t)a.m) atomicOr(&a.counters[1], 8u);
        a.cparD[i] = pd;
        if (pd >= 0) atomicMax((unsigned long long*)&a.heavy[pd],
                               (unsigned long long)(((uint64_t)(uint32_t)a.size[c] << 32) | (uint32_t)i));
    }
}

// Heavy-path heads by pointer jumping: up = path head, dist = depth below it.
__global__ void k_fc_hp_init(FlatArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.K; i += stride) {
        const int32_t pd = a.cparD[i];
        const bool heavy = pd >= 0 && (uint32_t)a.heavy[pd] == (uint32_t)i;
        a.up[0][i] = heavy ? pd : (int32_t)i;
        a.dist[0][i] = heavy ? 1 : 0;
    }
}

__global__ void k_fc_hp_jump(FlatArgs a, int src) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t* uin = a.up[src];
    const int32_t* din = a.dist[src];
    int32_t* uout = a.up[src ^ 1];
    int32_t* dout = a.dist[src ^ 1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.K; i += stride) {
        const int32_t j = uin[i];
        if (j == (int32_t)i || j < 0 || j >= a.K) {
            uout[i] = j;
            dout[i] = din[i];
        } else {
            uout[i] = uin[j];
            dout[i] = din[i] + din[j];
        }
    }
}

__global__ void k_fc_hp_len(FlatArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.K; i += stride) {
        const int32_t h = a.up[0][i];
        if (h < 0 || h >= a.K || a.up[0][h] != h) {
            atomicOr(&a.counters[1], 16u);
            continue;
        }
        if (a.heavy[i] == 0) a.plen[h] = a.dist[0][i] + 1;   // the bottom: a leaf, one per path
        if (h == (int32_t)i) atomicAdd(&a.counters[3], 1u);
    }
}

// Layout: each path contiguous, bottom (a leaf cluster) first.
__global__ void k_fc_hp_place(FlatArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.K; i += stride) {
        const int32_t h = a.up[0][i];
        if (h < 0 || h >= a.K) continue;                  // reported by k_fc_hp_len
        const int64_t pos = (int64_t)a.poff[h] + a.plen[h] - 1 - a.dist[0][i];
        if (pos < 0 || pos >= a.K) {
            atomicOr(&a.counters[1], 16u);
            continue;
        }
        a.lay[pos] = (int32_t)i;
        a.posof[i] = (int32_t)pos;
        a.s_lay[pos] = a.stab[a.clist[i]];
        if (h == (int32_t)i) {
            a.pending[h] = a.plen[h] - 1;                 // one light child per cluster above the bottom
            a.ready[h] = a.plen[h] == 1 ? -1 : INT32_MAX;
        }
    }
}

// One round: every path whose light children were all valued in earlier
// rounds is evaluated bottom up by one wave: the lanes load 64 consecutive
// positions, and every lane runs the same sequential recurrence on them,
// reading each position's operands from its lane (readlane); the lane that
// owns a position keeps its decision.  The head's value goes to the parent's
// light-child slot in the parent's path.
__device__ __forceinline__ double readlane_f64(double x, int k) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), k);
    return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(256) void k_fc_hp_eval(FlatArgs a, int round) {
    const int64_t h = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    const int lane = lane_id();
    if (h >= a.K) return;                                 // whole waves
    // every lane takes lane 0's reads, so the wave branches as one
    const int32_t up = __builtin_amdgcn_readfirstlane(a.up[0][h]);
    const int32_t pend = __builtin_amdgcn_readfirstlane(a.pending[h]);
    const int32_t rdy = __builtin_amdgcn_readfirstlane(a.ready[h]);
    if (up != (int32_t)h || pend != 0 || rdy >= round) return;
    const int64_t base = __builtin_amdgcn_readfirstlane(a.poff[h]);
    const int32_t len = __builtin_amdgcn_readfirstlane(a.plen[h]);
    if (base < 0 || len < 1 || base + len > a.K) {
        if (lane == 0) {
            atomicOr(&a.counters[1], 16u);
            a.pending[h] = -1;
        }
        return;
    }
    double v = 0.0;
    double ns = 0.0, nb = 0.0;
    if (lane < len) {
        ns = a.s_lay[base + lane];
        nb = a.b_lay[base + lane];
    }
    for (int32_t c0 = 0; c0 < len; c0 += kWave) {
        const double ms = ns, mb = nb;
        const int64_t idx = (int64_t)c0 + lane;
        if (idx + kWave < len) {                          // the next chunk loads during this one
            ns = a.s_lay[base + idx + kWave];
            nb = a.b_lay[base + idx + kWave];
        }
        const int cnt = len - c0 < kWave ? len - c0 : kWave;
        bool mine = false;
        int k0 = 0;
        if (c0 == 0) {                                    // the bottom is a leaf cluster
            v = readlane_f64(ms, 0);
            mine = lane == 0;
            k0 = 1;
        }
        if (cnt == kWave && k0 == 0) {                    // a full chunk: constant lane indices
#pragma unroll
            for (int k = 0; k < kWave; ++k) {
                const double cs = v + readlane_f64(mb, k);
                const double sk = readlane_f64(ms, k);
                const bool take = sk >= cs;
                v = take ? sk : cs;
                mine = lane == k ? take : mine;
            }
        } else {
            for (int k = k0; k < cnt; ++k) {
                const double cs = v + readlane_f64(mb, k);
                const double sk = readlane_f64(ms, k);
                const bool take = sk >= cs;
                v = take ? sk : cs;
                mine = lane == k ? take : mine;
            }
        }
        if (idx < len) a.sel[a.lay[base + idx]] = mine ? 1 : 0;
    }
    if (lane == 0) {
        a.pending[h] = -1;                                // done
        const int32_t P = a.cparD[h];
        if (P >= 0) {
            a.b_lay[a.posof[P]] = v;
            const int32_t H = a.up[0][P];
            if (atomicSub(&a.pending[H], 1) == 1) a.ready[H] = round;
        }
        atomicAdd(&a.counters[2], 1u);
    }
}

// Pointer jumping over the cluster tree (index K = the root): tp = the
// topmost selected cluster on the path up to (not including) the root, or -1.
__global__ void k_fc_top_init(FlatArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t root = (int32_t)a.K;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= a.K; c += stride) {
        if (c == root) {
            a.jp[0][c] = root;
            a.tp[0][c] = -1;
        } else {
            const int32_t pd = a.cparD[c];
            a.jp[0][c] = pd >= 0 ? pd : root;
            a.tp[0][c] = a.sel[c] ? (int32_t)c : -1;
        }
    }
}

__global__ void k_fc_top_round(FlatArgs a, int src) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t root = (int32_t)a.K;
    const int32_t* jin = a.jp[src];
    const int32_t* tin = a.tp[src];
    int32_t* jout = a.jp[src ^ 1];
    int32_t* tout = a.tp[src ^ 1];
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= a.K; c += stride) {
        const int32_t j = jin[c];
        if (j == root || j < 0 || j > root) {
            jout[c] = root;
            tout[c] = tin[c];
        } else {
            const int32_t tj = tin[j];
            tout[c] = tj >= 0 ? tj : tin[c];
            jout[c] = jin[j];
        }
    }
}

// Cluster of every vertex (its parent edge's cluster), its chosen cluster,
// and the first vertex of each chosen cluster.
// Few large clusters would make every vertex hit the same few minv words:
// within a wave (consecutive vertices) only the first lane of each label
// competes, since it holds that label's smallest vertex there.
__global__ void k_fc_label(FlatArgs a, int src) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t* tp = a.tp[src];
    const int lane = lane_id();
    for (int64_t x0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); x0 < a.n; x0 += stride) {
        const int64_t x = x0 + lane;
        int32_t lab = -1;
        if (x < a.n) {
            const int32_t p = a.vp[x];
            if (p >= 0 && p < a.m) {
                const int32_t c = a.T[p];
                if (c >= 0 && c < a.m) lab = tp[a.cidx[c]];  // c is a born cluster or the root (m)
            }
            a.labels[x] = lab;
        }
        const bool mine = lab >= 0 && lab < a.K;
        uint64_t open = ballot(mine);
        while (open) {
            const int leader = __ffsll((long long)open) - 1;
            const int32_t l = __shfl(lab, leader, kWave);
            const uint64_t same = ballot(mine && lab == l);
            // a load first: with a few huge clusters most atomics would change nothing
            if (lane == leader && (int32_t)x < __hip_atomic_load(&a.minv[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                atomicMin(&a.minv[l], (int32_t)x);
            open &= ~same;
        }
    }
}

__global__ void k_fc_relabel(FlatArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < a.n; x += stride) {
        const int32_t c = a.labels[x];
        a.labels[x] = c >= 0 ? a.cnum[c] : -1;
    }
}

// Position of the first key >= bound[j] in the sorted chain keys, per level.
__global__ void k_fc_bounds(const uint32_t* skey, int64_t m, const int64_t* keys, int64_t* pos, int count) {
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= count) return;
    const int64_t key = keys[j];
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)skey[mid] < key) lo = mid + 1; else hi = mid;
    }
    pos[j] = lo;
}

}  // namespace

hipError_t launch_fc_bounds(const uint32_t* skey, int64_t m, const int64_t* keys, int64_t* pos, int count,
                            hipStream_t s) {
    k_fc_bounds<<<1, 64, 0, s>>>(skey, m, keys, pos, count);
    return hipGetLastError();
}

hipError_t launch_fc_prepare(const FlatArgs& a, hipStream_t s) {
    k_fc_clear<<<grid_for(a.m), 256, 0, s>>>(a);
    k_fc_prepare<<<grid_for(a.n), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_fc_sizes(const FlatArgs& a, int64_t lo, int64_t hi, hipStream_t s) {
    SizeScan p{a.skey, a.sid, a.ext, a.size, a.ep, a.bigcnt, a.bigmax, a.mcs, lo, hi - lo, a.m};
    return run_scan<OpSegSum>(p, a, s);
}

hipError_t launch_fc_clusters(const FlatArgs& a, int64_t lo, int64_t hi, hipStream_t s) {
    ClusterScan p{a.skey, a.sid, a.size, a.ep, a.bigcnt, a.T, a.mcs, (int32_t)a.m, hi, hi - lo, a.m};
    return run_scan<OpLastSet>(p, a, s);
}

hipError_t launch_fc_stab(const FlatArgs& a, hipStream_t s) {
    // number the born clusters first: each owns one exact accumulator
    BirthScan p{a.T, a.clist, a.cidx, a.count, a.m};
    hipError_t e = run_scan<OpSum>(p, a, s);
    if (e != hipSuccess) return e;
    k_fc_acc_clear<<<grid_for(a.K * kAccChunks), 256, 0, s>>>(a);
    k_fc_stab<<<grid_for(a.m), 256, 0, s>>>(a);
    k_fc_acc_round<<<grid_for(a.K), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_fc_tree(FlatArgs& a, int rounds, hipStream_t s) {
    k_fc_dense_clear<<<grid_for(a.K + 1), 256, 0, s>>>(a);
    k_fc_tree<<<grid_for(a.K), 256, 0, s>>>(a);
    k_fc_hp_init<<<grid_for(a.K), 256, 0, s>>>(a);
    int src = 0;
    for (int r = 0; r < rounds; ++r) {
        k_fc_hp_jump<<<grid_for(a.K), 256, 0, s>>>(a, src);
        src ^= 1;
    }
    if (src == 1) {   // the final heads and depths are read from index 0 from here on
        std::swap(a.up[0], a.up[1]);
        std::swap(a.dist[0], a.dist[1]);
    }
    k_fc_hp_len<<<grid_for(a.K), 256, 0, s>>>(a);
    PathScan p{a.up[0], a.plen, a.poff, a.K};
    hipError_t e = run_scan<OpSum>(p, a, s);
    if (e != hipSuccess) return e;
    k_fc_hp_place<<<grid_for(a.K), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_fc_eval(const FlatArgs& a, int round, hipStream_t s) {
    k_fc_hp_eval<<<(unsigned)((a.K + 3) / 4), 256, 0, s>>>(a, round);
    return hipGetLastError();
}

hipError_t launch_fc_label(const FlatArgs& a, int rounds, hipStream_t s) {
    k_fc_top_init<<<grid_for(a.K + 1), 256, 0, s>>>(a);
    int src = 0;
    for (int r = 0; r < rounds; ++r) {
        k_fc_top_round<<<grid_for(a.K + 1), 256, 0, s>>>(a, src);
        src ^= 1;
    }
    k_fc_label<<<grid_for(a.n), 256, 0, s>>>(a, src);
    NumberScan p{a.labels, a.minv, a.clist, a.cnum, a.stab, a.stab_out, a.count + 1, a.n};
    hipError_t e = run_scan<OpSum>(p, a, s);
    if (e != hipSuccess) return e;
    k_fc_relabel<<<grid_for(a.n), 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace pandora
