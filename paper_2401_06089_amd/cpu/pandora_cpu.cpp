// Multithreaded CPU version of the dendrogram path (OpenMP), for hosts
// without a GPU and for comparing the method's CPU and GPU forms: the paper
// reports its multithreaded CPU implementation beside the GPU one (Section 6).
//
// It follows the same steps as the GPU library, shaped for a few dozen cores:
//   1. a stable parallel LSD radix sort of (weight key, edge id): ranks
//      (Section 3.1.1);
//   2. per level (Section 3.2): lightest incident edge of every vertex by
//      atomic minimum of (rank << 32 | position); ownership marks; alpha
//      edges (owned by neither endpoint, Eq. alphaedge) and leaf edges (owned
//      by both); supervertex labels by a scan of leaf edges; pointer jumping
//      to the labelled roots; stable compaction of the alpha edges;
//   3. expansion (Section 3.3): each edge walks up the levels to its chain,
//      a stable radix sort groups the chains in rank order, and each edge's
//      parent is the next one of its chain (Algorithm 1).
// The result is identical to the union-find definition (bottom-up
// construction, Section 2.3.2) for the total order (weight, edge id).
// Separate from the GPU library: nothing here is called by it, and it
// shares no code with it.
#include <omp.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <vector>

namespace {

constexpr int32_t kInf = INT32_MAX;          // no incident edge
constexpr int32_t kLabel = INT32_MIN;        // pointer word that holds a final label
constexpr uint64_t kNone = ~0ull;            // minimum of a vertex without edges

enum Status { kOk = 0, kInvalid = 1, kNotTree = 2, kNaN = 3, kBadVertex = 6 };

struct Edge {
    int32_t u, v, r, id;
};

// Monotone image of an fp32 weight; -0.0 folds onto +0.0 so that the two tie.
uint32_t weight_key(float w) {
    uint32_t b;
    std::memcpy(&b, &w, 4);
    if (b == 0x80000000u) b = 0;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

int64_t chunk_lo(int64_t n, int t, int T) { return n * t / T; }

// Stable LSD radix sort of (key, val) by the low `bits` bits of key, 8 bits
// per pass; each thread keeps its contiguous chunk in order in every pass.
void radix_sort(std::vector<uint32_t>& key, std::vector<int32_t>& val, int bits, int T) {
    const int64_t n = (int64_t)key.size();
    std::vector<uint32_t> k2(n);
    std::vector<int32_t> v2(n);
    std::vector<int64_t> cnt((size_t)T * 256);
    for (int shift = 0; shift < bits; shift += 8) {
        std::fill(cnt.begin(), cnt.end(), 0);
#pragma omp parallel num_threads(T)
        {
            const int t = omp_get_thread_num();
            int64_t* c = &cnt[(size_t)t * 256];
            for (int64_t i = chunk_lo(n, t, T); i < chunk_lo(n, t + 1, T); ++i) ++c[(key[i] >> shift) & 255u];
        }
        int64_t run = 0;   // digit-major, thread-minor offsets keep the sort stable
        for (int d = 0; d < 256; ++d)
            for (int t = 0; t < T; ++t) {
                const int64_t c = cnt[(size_t)t * 256 + d];
                cnt[(size_t)t * 256 + d] = run;
                run += c;
            }
#pragma omp parallel num_threads(T)
        {
            const int t = omp_get_thread_num();
            int64_t* o = &cnt[(size_t)t * 256];
            for (int64_t i = chunk_lo(n, t, T); i < chunk_lo(n, t + 1, T); ++i) {
                const int64_t p = o[(key[i] >> shift) & 255u]++;
                k2[p] = key[i];
                v2[p] = val[i];
            }
        }
        key.swap(k2);
        val.swap(v2);
    }
}

void atomic_min(std::atomic<uint64_t>& a, uint64_t v) {
    uint64_t cur = a.load(std::memory_order_relaxed);
    while (v < cur && !a.compare_exchange_weak(cur, v, std::memory_order_relaxed)) {
    }
}

// Exclusive scan of per-thread counts (small arrays).
int64_t exclusive_scan(std::vector<int64_t>& c) {
    int64_t run = 0;
    for (auto& x : c) {
        const int64_t y = x;
        x = run;
        run += y;
    }
    return run;
}

int run(int64_t n, const int32_t* u, const int32_t* v, const float* w, int32_t* edge_parent,
        int32_t* vertex_parent, int T) {
    const int64_t m = n - 1;
    // ---- validation -----------------------------------------------------------------
    int bad_vertex = 0, nan_seen = 0;
#pragma omp parallel for num_threads(T) reduction(| : bad_vertex, nan_seen)
    for (int64_t i = 0; i < m; ++i) {
        bad_vertex |= (u[i] < 0 || u[i] >= n || v[i] < 0 || v[i] >= n) ? 1 : 0;
        nan_seen |= std::isnan(w[i]) ? 1 : 0;
    }
    if (bad_vertex) return kBadVertex;
    if (nan_seen) return kNaN;

    // ---- 1. ranks: stable radix sort of (weight key, id) ------------------------------
    std::vector<uint32_t> key(m);
    std::vector<int32_t> perm(m);
#pragma omp parallel for num_threads(T)
    for (int64_t i = 0; i < m; ++i) {
        key[i] = weight_key(w[i]);
        perm[i] = (int32_t)i;
    }
    radix_sort(key, perm, 32, T);
    std::vector<int32_t> rank(m);
#pragma omp parallel for num_threads(T)
    for (int64_t r = 0; r < m; ++r) rank[perm[r]] = (int32_t)r;

    // ---- 2. contraction levels ---------------------------------------------------------
    // Flat vertex ids: level j occupies [off_j, off_j + n_j); at most 2n in all.
    std::vector<int32_t> minInc, label;
    minInc.reserve(2 * n);
    label.reserve(2 * n);
    std::vector<int32_t> svflat(m, -1);
    std::vector<Edge> E(m), E2;
#pragma omp parallel for num_threads(T)
    for (int64_t i = 0; i < m; ++i) E[i] = {u[i], v[i], rank[i], (int32_t)i};
    std::unique_ptr<std::atomic<uint64_t>[]> mn(new std::atomic<uint64_t>[n]);
    std::unique_ptr<std::atomic<int32_t>[]> ptr(new std::atomic<int32_t>[n]);
    std::vector<uint8_t> own(2 * m), alpha(m);
    int64_t mj = m, nj = n, off = 0, isolated = 0;
    for (int level = 0;; ++level) {
        if (level > 64) return kNotTree;
        const int64_t off_next = off + nj;
        minInc.resize(off_next);
        label.resize(off_next);
#pragma omp parallel for num_threads(T)
        for (int64_t x = 0; x < nj; ++x) mn[x].store(kNone, std::memory_order_relaxed);
        int selfloop = 0;
#pragma omp parallel for num_threads(T) reduction(| : selfloop)
        for (int64_t i = 0; i < mj; ++i) {
            const Edge e = E[i];
            selfloop |= e.u == e.v;
            const uint64_t k = ((uint64_t)(uint32_t)e.r << 32) | (uint64_t)i;
            atomic_min(mn[e.u], k);
            atomic_min(mn[e.v], k);
            own[2 * i] = own[2 * i + 1] = 0;
        }
        if (selfloop) return kNotTree;
        // ownership: the hook of every vertex and the mark on its lightest edge
        int64_t iso = 0;
#pragma omp parallel for num_threads(T) reduction(+ : iso)
        for (int64_t x = 0; x < nj; ++x) {
            const uint64_t k = mn[x].load(std::memory_order_relaxed);
            if (k == kNone) {
                ++iso;
                minInc[off + x] = kInf;
                label[off + x] = -1;
                if (level == 0) vertex_parent[x] = -1;
                continue;
            }
            const int64_t pos = (int64_t)(k & 0xffffffffu);
            const Edge e = E[pos];
            const int side = e.u == (int32_t)x ? 0 : 1;
            ptr[x].store(side ? e.u : e.v, std::memory_order_relaxed);
            own[2 * pos + side] = 1;
            minInc[off + x] = (int32_t)(k >> 32);
            if (level == 0) vertex_parent[x] = e.id;
        }
        isolated += iso;
        if (mj == 0) break;

        // alpha and leaf edges; leaf edges number the next level's vertices
        std::vector<int64_t> cl(T, 0), ca(T, 0);
#pragma omp parallel num_threads(T)
        {
            const int t = omp_get_thread_num();
            int64_t l = 0, a = 0;
            for (int64_t i = chunk_lo(mj, t, T); i < chunk_lo(mj, t + 1, T); ++i) {
                const bool both = own[2 * i] && own[2 * i + 1];
                const bool none = !own[2 * i] && !own[2 * i + 1];
                alpha[i] = none;
                l += both;
                a += none;
            }
            cl[t] = l;
            ca[t] = a;
        }
        const int64_t n_next = exclusive_scan(cl);
        const int64_t m_next = exclusive_scan(ca);
        // Section 4.2: at most half the edges survive a level
        if (2 * m_next > mj) return kNotTree;
#pragma omp parallel num_threads(T)
        {
            const int t = omp_get_thread_num();
            int64_t l = cl[t];
            for (int64_t i = chunk_lo(mj, t, T); i < chunk_lo(mj, t + 1, T); ++i)
                if (own[2 * i] && own[2 * i + 1]) {
                    const Edge e = E[i];
                    ptr[std::min(e.u, e.v)].store(kLabel | (int32_t)l++, std::memory_order_relaxed);
                }
        }
        // pointer jumping with path compression, a bounded number of steps per
        // round; every round at least doubles the resolved prefix of each path
        for (int round = 0;; ++round) {
            if (round > 64) return kNotTree;
            int open = 0;
#pragma omp parallel for num_threads(T) reduction(| : open) schedule(dynamic, 4096)
            for (int64_t x = 0; x < nj; ++x) {
                if (minInc[off + x] == kInf) continue;
                int32_t q = ptr[x].load(std::memory_order_relaxed);
                if (q & kLabel) continue;
                int32_t t = ptr[q].load(std::memory_order_relaxed);
                for (int s = 0; !(t & kLabel) && s < 32; ++s) {
                    q = t;
                    t = ptr[q].load(std::memory_order_relaxed);
                }
                if (t & kLabel) {
                    ptr[x].store(t, std::memory_order_relaxed);
                } else {
                    ptr[x].store(q, std::memory_order_relaxed);
                    open = 1;
                }
            }
            if (!open) break;
        }
#pragma omp parallel for num_threads(T)
        for (int64_t x = 0; x < nj; ++x) {
            if (minInc[off + x] == kInf) continue;
            const int32_t flat = (int32_t)(off_next + (ptr[x].load(std::memory_order_relaxed) & ~kLabel));
            label[off + x] = flat;
            svflat[minInc[off + x]] = flat;   // x's lightest edge falls into this supervertex
        }
        // stable compaction of the alpha edges, endpoints relabelled
        E2.resize(m_next);
        int bad = 0;
#pragma omp parallel num_threads(T) reduction(| : bad)
        {
            const int t = omp_get_thread_num();
            int64_t a = ca[t];
            for (int64_t i = chunk_lo(mj, t, T); i < chunk_lo(mj, t + 1, T); ++i)
                if (alpha[i]) {
                    const Edge e = E[i];
                    const int32_t lx = label[off + e.u], ly = label[off + e.v];
                    bad |= lx == ly;
                    E2[a++] = {(int32_t)(lx - off_next), (int32_t)(ly - off_next), e.r, 0};
                }
        }
        if (bad) return kNotTree;
        E.swap(E2);
        off = off_next;
        nj = n_next;
        mj = m_next;
    }
    if (isolated != 1) return kNotTree;   // one tree ends as one isolated vertex

    // ---- 3. expansion ------------------------------------------------------------------
    const int64_t flat_total = (int64_t)minInc.size();
    std::vector<uint32_t> ckey(m);
    std::vector<int32_t> crank(m);
    int walk_bad = 0;
#pragma omp parallel for num_threads(T) reduction(| : walk_bad)
    for (int64_t r = 0; r < m; ++r) {
        int32_t x = svflat[r];
        int steps = 0;
        while (x >= 0 && x < flat_total && r >= minInc[x] && steps++ < 64) x = label[x];
        walk_bad |= (x < n || x >= flat_total) ? 1 : 0;
        ckey[r] = (uint32_t)(x - n);
        crank[r] = (int32_t)r;
    }
    if (walk_bad) return kNotTree;
    int bits = 8;
    while (bits < 32 && ((uint64_t)(flat_total - n) >> bits) != 0) bits += 8;
    radix_sort(ckey, crank, bits, T);
#pragma omp parallel for num_threads(T)
    for (int64_t i = 0; i < m; ++i) {
        const int32_t r = crank[i];
        int32_t p;
        if (i + 1 < m && ckey[i + 1] == ckey[i]) {
            p = perm[crank[i + 1]];
        } else {
            const int32_t head = minInc[(int64_t)ckey[i] + n];
            p = head == kInf ? -1 : perm[head];
        }
        edge_parent[perm[r]] = p;
    }
    return kOk;
}

}  // namespace

extern "C" {

// Dendrogram of one tree on the CPU with `threads` OpenMP threads (0: the
// OpenMP default).  Arguments and outputs as pandora_dendrogram, in host
// memory; returns the same status codes.
__attribute__((visibility("default"))) int pandora_cpu_dendrogram(int64_t n, const int32_t* u, const int32_t* v,
                                                                  const float* w, int32_t* edge_parent,
                                                                  int32_t* vertex_parent, int threads) {
    if (n < 1 || n > INT32_MAX || !vertex_parent) return kInvalid;
    if (n > 1 && (!u || !v || !w || !edge_parent)) return kInvalid;
    if (n == 1) {
        vertex_parent[0] = -1;
        return kOk;
    }
    const int T = threads > 0 ? threads : omp_get_max_threads();
    return run(n, u, v, w, edge_parent, vertex_parent, T);
}

}  // extern "C"
