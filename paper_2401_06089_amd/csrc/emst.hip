// Mutual-reachability minimum spanning tree of a low-dimensional point cloud
// on gfx950: HDBSCAN*'s first step, which the paper's HDBSCAN* section runs
// before the dendrogram (with ArborX there).  Definitions of HDBSCAN*
// (Campello et al. 2015):
//   d2(i, j)  squared distance, summed over coordinates in order, every
//             operation rounded to fp64 on its own (no fused multiply-add)
//   core2(i)  the (min_pts - 1)-th smallest d2(i, j), j != i (0 for min_pts 1)
//   mrd2      max(core2(i), core2(j), d2(i, j))
// Edges are totally ordered by (mrd2, min(i, j), max(i, j)), so the tree is
// unique.  Since sqrt is monotone and correctly rounded, ordering by mrd2
// orders the weights sqrt(mrd2).
//
// Borůvka rounds: every point finds its least edge to another component.
// Small clouds sweep all points in LDS tiles (dense fp64 vector work, no
// matrix-core shape); clouds of 2,048+ points search a uniform grid ring by
// ring, stop at exact distance bounds, and leave isolated points to a full
// sweep.  A search also stops once no farther point can beat an edge its
// component already has; the point then keeps the distance bound it reached
// as a lower bound on its least edge, and later rounds skip it while its
// component has a lighter edge.  On the grid every per-point array is kept
// in cell order (a point's slot), so that the passes over all points read
// and write them in order and a search's neighbours sit next to it.  A point
// whose previous least edge still leaves its component keeps it.
// Components take the least edge of their points (two atomic minima: weight
// bits, then endpoints), hook along it (a mutual pair keeps the smaller
// root), and pointer jumping relabels.  Each round at least halves the
// components.  The tree's edges are then sorted by the total order (the
// library's stable LSD radix passes, one 32-bit key word at a time) and
// handed out with fp64 and fp32 weights.
#include "kernels.hpp"

namespace pandora {

namespace {

constexpr int kEmBlock = 256;
constexpr int kEmMaxK = kEmstMaxMinPts - 1;       // core-distance rank held in registers (at most)
constexpr int kGridRingCap = 4;                    // rings searched in the grid before a full sweep

__device__ __forceinline__ double d2_of(const double* a, const double* b, int dim) {
#pragma clang fp contract(off)   // every product and sum rounded on its own, as defined
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kEmstMaxDim; ++k) {
        if (k < dim) {
            const double t = a[k] - b[k];
            acc = acc + t * t;
        }
    }
    return acc;
}

// The same with the second point as stored on the grid: its fp32 input
// coordinates, four to a 16-byte slot, widened here (exactly).
__device__ __forceinline__ double d2_of(const double* a, const float* b4, int dim) {
    const float4 q = *reinterpret_cast<const float4*>(b4);
    const double b[kEmstMaxDim] = {(double)q.x, (double)q.y, (double)q.z, (double)q.w};
    return d2_of(a, b, dim);
}

__device__ __forceinline__ bool key_less(double w, int32_t lo, int32_t hi, double bw, int32_t blo, int32_t bhi) {
    return w < bw || (w == bw && (lo < blo || (lo == blo && hi < bhi)));
}

// Input index of the point in slot p, and the slot of input index id (slots
// are sorted positions on the grid, input indices otherwise).
__device__ __forceinline__ int32_t id_of(const EmstArgs& a, int64_t p) {
    return a.use_grid ? a.sorted[p] : (int32_t)p;
}
__device__ __forceinline__ int64_t slot_of(const EmstArgs& a, int32_t id) {
    return a.use_grid ? (int64_t)a.slotof[id] : (int64_t)id;
}

// Coordinate k of the point in slot p, widened to fp64.
__device__ __forceinline__ double coord(const EmstArgs& a, int64_t p, int k) {
    return a.use_grid ? (double)a.spts[p * kEmstMaxDim + k] : (double)a.pts[p * a.dim + k];
}

// Atomic minimum of val into base[key] for the lanes with act.  Lanes that
// share the first active lane's key (neighbouring points usually share a
// component) send one combined minimum.  Every lane of the wave must call it.
__device__ void wave_min_into(uint64_t* base, int32_t key, uint64_t val, bool act) {
    const uint64_t m = ballot(act);
    if (!m) return;
    const int leader = __ffsll((long long)m) - 1;
    const int32_t k0 = __shfl(key, leader, kWave);
    const bool same = act && key == k0;
    uint64_t v = same ? val : ~0ull;
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const uint64_t o = __shfl_xor(v, d, kWave);
        v = o < v ? o : v;
    }
    // a load first: late in the merging many waves share a few large
    // components, and most of their atomics would change nothing
    if (lane_id() == leader && v < __hip_atomic_load(&base[k0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMin((unsigned long long*)&base[k0], (unsigned long long)v);
    if (act && !same && val < __hip_atomic_load(&base[key], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMin((unsigned long long*)&base[key], (unsigned long long)val);
}

// Adds every lane's count into one slot per block, one atomic per wave.
// Every lane of the wave must call it.
__device__ void wave_count(uint64_t* slots, uint32_t v) {
    uint64_t t = v;
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) t += __shfl_xor(t, d, kWave);
    if (lane_id() == 0 && t != 0)
        atomicAdd((unsigned long long*)&slots[blockIdx.x % kEmstPairSlots], (unsigned long long)t);
}

// A list append for a whole block of kThreads, with one atomic per block
// (an atomic from every wave of a pass over all points serialises on the
// counter): returns each wanting thread's slot, consecutive in thread order.
// Every thread of the block must call it.
template <int kThreads>
__device__ uint32_t block_append(uint32_t* ctr, bool want) {
    constexpr int kWaves = kThreads / kWave;
    __shared__ uint32_t s_cnt[kWaves];
    __shared__ uint32_t s_base;
    const uint64_t m = ballot(want);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) s_cnt[w] = (uint32_t)popc64(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int k = 0; k < kWaves; ++k) {
            const uint32_t t = s_cnt[k];
            s_cnt[k] = run;
            run += t;
        }
        s_base = run ? atomicAdd(ctr, run) : 0u;
    }
    __syncthreads();
    const uint32_t slot = s_base + s_cnt[w] + (uint32_t)popc64(m & lanemask_lt());
    __syncthreads();
    return slot;
}

constexpr int kEmPass = 1024;    // block of the passes over all points that append or count

// Core distances: each thread keeps the K smallest d2 of its point in
// registers (sorted, fully unrolled so that nothing spills).
// With a list, only the listed slots (the grid search's leftovers), and
// nothing but their core distance is written.
template <int KMAX>
__global__ __launch_bounds__(kEmBlock) void k_em_core(EmstArgs a, const int32_t* list, int64_t count) {
    __shared__ double s_p[kEmBlock][kEmstMaxDim];
    const int64_t slot = (int64_t)blockIdx.x * kEmBlock + threadIdx.x;
    const int64_t i = list ? (slot < count ? list[slot] : a.n) : slot;
    const int K = a.min_pts - 1;
    double me[kEmstMaxDim];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kEmstMaxDim; ++k) {
        me[k] = 0.0;
        if (i < a.n && k < a.dim) {
            me[k] = coord(a, i, k);
            bad |= !isfinite(me[k]);
        }
    }
    double top[KMAX];
#pragma unroll
    for (int t = 0; t < KMAX; ++t) top[t] = INFINITY;
    double thr = INFINITY;                                // top[K-1], kept in a register
    for (int64_t j0 = 0; j0 < a.n; j0 += kEmBlock) {
        __syncthreads();
        const int64_t jl = j0 + threadIdx.x;
#pragma unroll
        for (int k = 0; k < kEmstMaxDim; ++k)
            s_p[threadIdx.x][k] = (jl < a.n && k < a.dim) ? coord(a, jl, k) : 0.0;
        __syncthreads();
        if (i >= a.n || K == 0) continue;
        const int cnt = a.n - j0 < kEmBlock ? (int)(a.n - j0) : kEmBlock;
        for (int jj = 0; jj < cnt; ++jj) {
            if (j0 + jj == i) continue;
            const double d = d2_of(me, s_p[jj], a.dim);
            if (d >= thr) continue;
            // insert d into the sorted list and drop the largest (constant
            // indices only, so the list stays in registers)
#pragma unroll
            for (int t = KMAX - 1; t >= 1; --t) top[t] = fmin(top[t], fmax(top[t - 1], d));
            top[0] = fmin(top[0], d);
#pragma unroll
            for (int t = 0; t < KMAX; ++t)
                if (t == K - 1) thr = top[t];
        }
    }
    if (i < a.n) {
        double c = 0.0;
#pragma unroll
        for (int t = 0; t < KMAX; ++t)
            if (t == K - 1) c = top[t];
        a.core2[i] = c;
        if (!list) {
            a.comp[i] = (int32_t)i;
            a.best_j[i] = -1;
            a.cmin_w[i] = ~0ull;
            a.cmin_e[i] = ~0ull;
        }
    }
    if (ballot(bad) != 0 && lane_id() == 0) atomicOr(&a.counters[2], 1u);
}

// A point's least edge to another component stays its least edge while its
// other end is still outside the point's (grown) component: the candidates
// only lose points.  Such points report it at once; the others are listed
// for a new search (in slot order: on the grid, neighbouring threads then
// search neighbouring cells and share lines in the caches).
__global__ __launch_bounds__(kEmPass) void k_em_active(EmstArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool keep = false;
    int32_t mc = 0;
    uint64_t w = 0;
    if (i < a.n) {
        const int32_t j = a.best_j[i];
        mc = a.comp[i];
        keep = j >= 0 && a.comp[j] != mc && !(a.use_grid && a.partial[i]);
        if (keep) w = (uint64_t)__double_as_longlong(a.best_w[i]);
    }
    const bool search = i < a.n && !keep;
    const uint32_t k = block_append<kEmPass>(&a.counters[3], search);
    if (search) a.active[k] = (int32_t)i;
    wave_min_into(a.cmin_w, mc, w, keep);
}

// Every listed point's least edge to another component.
__global__ __launch_bounds__(kEmBlock) void k_em_best(EmstArgs a, const int32_t* list, int64_t count) {
    __shared__ double s_p[kEmBlock][kEmstMaxDim];
    __shared__ double s_c[kEmBlock];
    __shared__ int32_t s_comp[kEmBlock];
    __shared__ int32_t s_id[kEmBlock];
    const int64_t slot = (int64_t)blockIdx.x * kEmBlock + threadIdx.x;
    const int64_t i = slot < count ? list[slot] : a.n;
    double me[kEmstMaxDim];
#pragma unroll
    for (int k = 0; k < kEmstMaxDim; ++k) me[k] = (i < a.n && k < a.dim) ? coord(a, i, k) : 0.0;
    const double ci = i < a.n ? a.core2[i] : 0.0;
    const int32_t mc = i < a.n ? a.comp[i] : -1;
    const int32_t io = i < a.n ? id_of(a, i) : 0;
    double bw = INFINITY;
    int32_t blo = INT32_MAX, bhi = INT32_MAX, bj = -1;
    for (int64_t j0 = 0; j0 < a.n; j0 += kEmBlock) {
        __syncthreads();
        const int64_t jl = j0 + threadIdx.x;
#pragma unroll
        for (int k = 0; k < kEmstMaxDim; ++k)
            s_p[threadIdx.x][k] = (jl < a.n && k < a.dim) ? coord(a, jl, k) : 0.0;
        s_c[threadIdx.x] = jl < a.n ? a.core2[jl] : 0.0;
        s_comp[threadIdx.x] = jl < a.n ? a.comp[jl] : mc;
        s_id[threadIdx.x] = jl < a.n ? id_of(a, jl) : 0;
        __syncthreads();
        if (i >= a.n) continue;
        const int cnt = a.n - j0 < kEmBlock ? (int)(a.n - j0) : kEmBlock;
        for (int jj = 0; jj < cnt; ++jj) {
            if (s_comp[jj] == mc) continue;
            const double d = d2_of(me, s_p[jj], a.dim);
            const double w = fmax(fmax(ci, s_c[jj]), d);
            const int32_t j = s_id[jj];
            const int32_t lo = j < io ? j : io, hi = j < io ? io : j;
            if (key_less(w, lo, hi, bw, blo, bhi)) {
                bw = w;
                blo = lo;
                bhi = hi;
                bj = (int32_t)(j0 + jj);
            }
        }
    }
    if (i < a.n) {
        a.best_w[i] = bw;
        a.best_j[i] = bj;
    }
    wave_min_into(a.cmin_w, mc, (uint64_t)__double_as_longlong(bw), i < a.n && bj >= 0);
}

// The t-th component root of this round (every point in the first round);
// a.n past the end.
__device__ __forceinline__ int64_t root_at(const EmstArgs& a, int64_t t) {
    if (!a.roots) return t < a.n ? t : a.n;
    return t < a.nroots ? (int64_t)a.roots[t] : a.n;
}

// Among the points whose edge has the component's least weight, the least endpoints.
__global__ void k_em_cmin(EmstArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int32_t j = a.best_j[i];
    if (j < 0) return;
    const int32_t c = a.comp[i];
    if ((uint64_t)__double_as_longlong(a.best_w[i]) != a.cmin_w[c]) return;
    const int32_t io = id_of(a, i), jo = id_of(a, j);
    const uint64_t lo = (uint64_t)(uint32_t)(jo < io ? jo : io), hi = (uint64_t)(uint32_t)(jo < io ? io : jo);
    atomicMin((unsigned long long*)&a.cmin_e[c], (unsigned long long)((lo << 32) | hi));
}

// Each component hooks to the one across its least edge; of a mutual pair
// the smaller root stays a root and records the edge once.
__global__ __launch_bounds__(kEmPass) void k_em_hook(EmstArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = root_at(a, t);
    bool record = false;
    int32_t lo = 0, hi = 0;
    if (c < a.n && a.comp[c] == (int32_t)c) {
        const uint64_t e = a.cmin_e[c];
        if (e == ~0ull) {                                 // no edge out: the last component
            a.parent[0][c] = (int32_t)c;
        } else {
            lo = (int32_t)(e >> 32);
            hi = (int32_t)(e & 0xffffffffu);
            if (lo < 0 || hi >= a.n || lo >= hi) {
                atomicOr(&a.counters[2], 2u);
                a.parent[0][c] = (int32_t)c;
            } else {
                const int32_t clo = a.comp[slot_of(a, lo)], chi = a.comp[slot_of(a, hi)];
                const int32_t other = clo == (int32_t)c ? chi : clo;
                const bool mutual = a.cmin_e[other] == e;
                const bool stays = mutual && (int32_t)c < other;
                a.parent[0][c] = stays ? (int32_t)c : other;
                record = !mutual || stays;
            }
        }
    }
    const uint32_t k = block_append<kEmPass>(&a.counters[0], record);
    if (record) {
        if (k < (uint32_t)(a.n - 1)) {
            a.ew[k] = a.cmin_w[c];
            a.ea[k] = lo;
            a.eb[k] = hi;
        } else {
            atomicOr(&a.counters[2], 4u);
        }
    }
}

__global__ void k_em_jump(EmstArgs a, int src) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = root_at(a, t);
    bool changed = false;
    if (c < a.n && a.comp[c] == (int32_t)c) {
        const int32_t p = a.parent[src][c];
        const int32_t pp = (p >= 0 && p < a.n) ? a.parent[src][p] : p;
        a.parent[src ^ 1][c] = pp;
        changed = pp != p;
    }
    if (__syncthreads_or(changed) && threadIdx.x == 0 &&
        __hip_atomic_load(&a.counters[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        atomicOr(&a.counters[3], 1u);
}

// New component of every point; the per-component minima start over.
__global__ __launch_bounds__(kEmPass) void k_em_relabel(EmstArgs a, int src) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool root = false;
    if (i < a.n) {
        const int32_t r = a.parent[src][a.comp[i]];
        a.comp2[i] = r;
        a.cmin_w[i] = ~0ull;
        a.cmin_e[i] = ~0ull;
        root = r == (int32_t)i;
    }
    const uint32_t k = block_append<kEmPass>(&a.counters[1], root);
    if (root) a.roots_next[k] = (int32_t)i;
}

__global__ void k_em_copy_comp(EmstArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.n) a.comp[i] = a.comp2[i];
}

// Keys of the radix sort of the tree's edges, one 32-bit word per sort,
// from the least significant word of the total order's key: 0 = the larger
// endpoint, 1 = the smaller, 2 and 3 = the low and high halves of the mrd2
// bits (non-negative doubles order like their bits).  keys[i] = that word of
// edge order[i]; with order == nullptr the order is the identity, which is
// then written to order_out.
__global__ void k_em_sort_key(EmstArgs a, int word, const int32_t* order, uint32_t* keys, int32_t* order_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n - 1) return;
    int32_t e = (int32_t)i;
    if (order) e = order[i];
    else order_out[i] = e;
    uint32_t k;
    if (word == 0) k = (uint32_t)a.eb[e];
    else if (word == 1) k = (uint32_t)a.ea[e];
    else if (word == 2) k = (uint32_t)a.ew[e];
    else k = (uint32_t)(a.ew[e] >> 32);
    keys[i] = k;
}

// Correctly rounded square root.  The device square root is within one unit
// in the last place; the result is then fixed by comparing x with the square
// of the midpoint between adjacent candidates, in exact 128-bit integers:
// with a = A * 2^e, the midpoint to the next double up is (2A + 1) * 2^(e-1).
// (x is never that square exactly: (2A + 1)^2 is odd and has more than 53
// significant bits.)  Inputs are zero, +inf or normal (squared distances of
// fp32 points are at least 2^-298).
__device__ __forceinline__ void split_normal(double v, uint64_t& M, int& e) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    M = (b & ((1ull << 52) - 1)) | (1ull << 52);
    e = (int)((b >> 52) & 0x7ff) - 1075;              // v = M * 2^e
}

__device__ bool above_mid_square(double x, double a) {   // x > (a + ulp(a)/2)^2
    uint64_t A, X;
    int ea, ex;
    split_normal(a, A, ea);
    split_normal(x, X, ex);
    const unsigned __int128 m = (unsigned __int128)(2 * A + 1);
    const unsigned __int128 mm = m * m;                   // < 2^108
    const int g = ex - (2 * ea - 2);                      // x = X * 2^g in units of 2^(2ea-2)
    if (g < 0) return false;                              // x < 2^(53 + 2ea - 2) <= mm * 2^(2ea-2)
    if (g > 74) return true;                              // X * 2^g >= 2^(52 + 75) > mm
    return ((unsigned __int128)X << g) > mm;
}

__device__ double sqrt_rn(double x) {
    if (!(x > 0.0) || isinf(x)) return __dsqrt_rn(x);
    double y = __dsqrt_rn(x);
    for (int it = 0; it < 2; ++it) {
        const uint64_t b = (uint64_t)__double_as_longlong(y);
        if (above_mid_square(x, y)) {
            y = __longlong_as_double((long long)(b + 1));
        } else {
            const double dn = __longlong_as_double((long long)(b - 1));
            if (dn > 0.0 && !above_mid_square(x, dn)) y = dn;
            else break;
        }
    }
    return y;
}

// The k-th edge of the sorted tree is edge order[k] of the recorded list.
__global__ void k_em_out(EmstArgs a, const int32_t* order) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n - 1) return;
    const int32_t e = order[k];
    const double w2 = __longlong_as_double((long long)a.ew[e]);
    const double w = sqrt_rn(w2);
    a.u[k] = a.ea[e];
    a.v[k] = a.eb[e];
    if (a.w64) a.w64[k] = w;
    a.w32[k] = __double2float_rn(w);
}

// ---- uniform grid ------------------------------------------------------------------

__device__ __forceinline__ uint32_t order_bits(float f) {      // monotone in f
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__global__ void k_em_bbox(EmstArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t lo[kEmstMaxDim], hi[kEmstMaxDim];
#pragma unroll
    for (int k = 0; k < kEmstMaxDim; ++k) {
        lo[k] = 0xffffffffu;
        hi[k] = 0u;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
#pragma unroll
        for (int k = 0; k < kEmstMaxDim; ++k) {
            if (k < a.dim) {
                const uint32_t b = order_bits(a.pts[i * a.dim + k]);
                lo[k] = lo[k] < b ? lo[k] : b;
                hi[k] = hi[k] > b ? hi[k] : b;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kEmstMaxDim; ++k) {
        if (k < a.dim) {
            atomicMin(&a.bbox[2 * k], lo[k]);
            atomicMin(&a.bbox[2 * k + 1], ~hi[k]);         // the maximum, complemented
        }
    }
}

// Cell coordinate of x along dimension k (clamped: the floor of a rounded
// quotient may land one cell off, which the search bounds allow for).
__device__ __forceinline__ int32_t cell_coord(const EmstArgs& a, double x, int k) {
    const double q = floor((x - a.gmin[k]) * a.inv_h);
    const double c = q < 0.0 ? 0.0 : (q > (double)(a.gdim[k] - 1) ? (double)(a.gdim[k] - 1) : q);
    return (int32_t)c;
}

__global__ void k_em_cells(EmstArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    int64_t cell = 0;
    for (int k = 0; k < a.dim; ++k) cell += (int64_t)cell_coord(a, (double)a.pts[i * a.dim + k], k) * a.gstride[k];
    a.cellof[i] = (int32_t)cell;
    atomicAdd(&a.cfill[cell], 1);
}

// Exclusive scan of the cell counts into cstart (block sums, one block over
// the sums, then the block offsets); cfill is cleared for the scatter.
constexpr int kScanB = 1024, kScanI = 4;
__device__ uint64_t em_block_excl(uint64_t x, uint64_t* s_w, uint64_t* total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    uint64_t inc = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t y = __shfl_up(inc, d, kWave);
        if (lane >= d) inc += y;
    }
    if (lane == kWave - 1) s_w[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = 0;
        for (int w = 0; w < kScanB / kWave; ++w) {
            const uint64_t t = s_w[w];
            s_w[w] = run;
            run += t;
        }
        s_w[kScanB / kWave] = run;
    }
    __syncthreads();
    const uint64_t res = s_w[wave] + inc - x;
    *total = s_w[kScanB / kWave];
    __syncthreads();
    return res;
}

__global__ __launch_bounds__(kScanB) void k_em_scan1(EmstArgs a) {
    __shared__ uint64_t s_w[kScanB / kWave + 1];
    const int64_t base = ((int64_t)blockIdx.x * kScanB + threadIdx.x) * kScanI;
    uint64_t v = 0;
    for (int j = 0; j < kScanI; ++j)
        if (base + j < a.ncells) v += (uint64_t)a.cfill[base + j];
    uint64_t total;
    (void)em_block_excl(v, s_w, &total);
    if (threadIdx.x == 0) a.scan_agg[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanB) void k_em_scan2(EmstArgs a, int64_t blocks) {
    __shared__ uint64_t s_w[kScanB / kWave + 1];
    uint64_t run = 0;
    for (int64_t c0 = 0; c0 < blocks; c0 += kScanB) {
        const int64_t t = c0 + threadIdx.x;
        const uint64_t x = t < blocks ? a.scan_agg[t] : 0;
        uint64_t total;
        const uint64_t ex = em_block_excl(x, s_w, &total);
        if (t < blocks) a.scan_agg[t] = run + ex;
        run += total;
    }
    if (threadIdx.x == 0) a.cstart[a.ncells] = (int32_t)a.n;
}

__global__ __launch_bounds__(kScanB) void k_em_scan3(EmstArgs a) {
    __shared__ uint64_t s_w[kScanB / kWave + 1];
    const int64_t base = ((int64_t)blockIdx.x * kScanB + threadIdx.x) * kScanI;
    int32_t c[kScanI];
    uint64_t v = 0;
    for (int j = 0; j < kScanI; ++j) {
        c[j] = base + j < a.ncells ? a.cfill[base + j] : 0;
        v += (uint64_t)c[j];
    }
    uint64_t total;
    uint64_t run = a.scan_agg[blockIdx.x] + em_block_excl(v, s_w, &total);
    for (int j = 0; j < kScanI; ++j) {
        if (base + j >= a.ncells) break;
        a.cstart[base + j] = (int32_t)run;
        a.cfill[base + j] = 0;
        run += (uint64_t)c[j];
    }
}

// Points in cell order (the order inside a cell does not matter: every
// search takes the least key under the total order).
__global__ void k_em_scatter(EmstArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int32_t cell = a.cellof[i];
    const int64_t pos = (int64_t)a.cstart[cell] + atomicAdd(&a.cfill[cell], 1);
    a.sorted[pos] = (int32_t)i;
    a.slotof[i] = (int32_t)pos;
#pragma unroll
    for (int k = 0; k < kEmstMaxDim; ++k) a.spts[pos * kEmstMaxDim + k] = k < a.dim ? a.pts[i * a.dim + k] : 0.0f;
}

// Visits the points of Chebyshev ring r around cell coordinates c (only
// cells inside the grid) of the point at me; ring 1 includes the point's own
// cell.  Cells are row-major with the first coordinate fastest, so the
// ring's cells along a row of the first coordinate are one contiguous range
// of sorted positions: f(first, last, b2) gets such a range (a whole row, or
// one of a row's two end cells when the row passes through the ring's
// inside) and a lower bound b2 on the squared distance from me to any point
// placed in it: the distance to the range's box, less twice the placement
// slack per coordinate, squared and shrunk against its own rounding.
__device__ __forceinline__ double gap2(const EmstArgs& a, int k, double x, int32_t c0, int32_t c1) {
    const double lo = a.gmin[k] + (double)c0 * a.h, hi = a.gmin[k] + (double)(c1 + 1) * a.h;
    const double gap = fmax(lo - x, x - hi) - 2.0 * a.gslack;
    return gap > 0.0 ? gap * gap : 0.0;
}

template <class F>
__device__ __forceinline__ void for_ring(const EmstArgs& a, const int32_t* c, const double* me, int r, F&& f) {
    // offsets of coordinates 1.. in [-r, r], counted like an odometer
    // (constant indices only, so that nothing leaves the registers)
    int d[kEmstMaxDim];
#pragma unroll
    for (int k = 0; k < kEmstMaxDim; ++k) d[k] = (k >= 1 && k < a.dim) ? -r : 0;
    const int32_t gx = a.gdim[0];
    for (;;) {
        int64_t row = 0;
        bool inside = true, shell = false;
        double b2 = 0.0;
#pragma unroll
        for (int k = 1; k < kEmstMaxDim; ++k) {
            if (k < a.dim) {
                shell |= (d[k] == r || d[k] == -r);
                const int32_t ck = c[k] + d[k];
                inside &= ck >= 0 && ck < a.gdim[k];
                row += (int64_t)ck * a.gstride[k];
                b2 += gap2(a, k, me[k], ck, ck);
            }
        }
        if (inside) {
            if (shell || r == 1) {                            // the whole row
                const int32_t x0 = c[0] - r > 0 ? c[0] - r : 0;
                const int32_t x1 = c[0] + r < gx - 1 ? c[0] + r : gx - 1;
                f(a.cstart[row + x0], a.cstart[row + x1 + 1], (b2 + gap2(a, 0, me[0], x0, x1)) * (1.0 - 1e-12));
            } else {                                          // the row's two end cells
                const int32_t xl = c[0] - r, xr = c[0] + r;
                if (xl >= 0) f(a.cstart[row + xl], a.cstart[row + xl + 1], (b2 + gap2(a, 0, me[0], xl, xl)) * (1.0 - 1e-12));
                if (xr < gx) f(a.cstart[row + xr], a.cstart[row + xr + 1], (b2 + gap2(a, 0, me[0], xr, xr)) * (1.0 - 1e-12));
            }
        }
        bool carry = true;
#pragma unroll
        for (int k = 1; k < kEmstMaxDim; ++k) {
            if (carry && k < a.dim) {
                if (d[k] < r) {
                    ++d[k];
                    carry = false;
                } else {
                    d[k] = -r;
                }
            }
        }
        if (carry) break;
    }
}

// A point of a cell R rings away is at least R - 1 cell edges away, less
// the few rounding units by which a rounded floor can misplace a point at a
// cell boundary (gslack, from the coordinate magnitudes); the square is
// shrunk once more against its own rounding.
__device__ __forceinline__ double ring_bound2(const EmstArgs& a, int r) {
    if (r < 1) return 0.0;
    const double lb = (double)(r - 1) * a.h - a.gslack;
    return lb > 0.0 ? lb * lb * (1.0 - 1e-12) : 0.0;
}

__device__ __forceinline__ int max_ring(const EmstArgs& a) {
    int m = 0;
    for (int k = 0; k < a.dim; ++k) m = a.gdim[k] > m ? a.gdim[k] : m;
    return m;
}

// Core distances by widening rings: stop once the K-th smallest is no more
// than the bound for everything farther out.
// Returns the pairs examined.
template <int KMAX>
__device__ __forceinline__ uint32_t core_grid_point(const EmstArgs& a, int64_t i) {
    const int K = a.min_pts - 1;
    double me[kEmstMaxDim];
    int32_t c[kEmstMaxDim];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kEmstMaxDim; ++k) {
        me[k] = 0.0;
        c[k] = 0;
        if (k < a.dim) {
            me[k] = (double)a.spts[i * kEmstMaxDim + k];
            bad |= !isfinite(me[k]);
            c[k] = cell_coord(a, me[k], k);
        }
    }
    if (bad) atomicOr(&a.counters[2], 1u);
    double top[KMAX];
#pragma unroll
    for (int t = 0; t < KMAX; ++t) top[t] = INFINITY;
    double thr = INFINITY;
    uint32_t pairs = 0;
    bool done = K == 0;
    if (K > 0) {
        const int rmax = max_ring(a);
        const int rcap = rmax < kGridRingCap ? rmax : kGridRingCap;
        for (int r = 1; r <= rcap; ++r) {
            for_ring(a, c, me, r, [&](int32_t p0, int32_t p1, double b2) {
                if (b2 >= thr) return;                    // nothing in the cell can enter the list
                for (int32_t p = p0; p < p1; ++p) {
                    if (p == i) continue;
                    const double d = d2_of(me, a.spts + (int64_t)p * kEmstMaxDim, a.dim);
                    ++pairs;
                    if (d >= thr) continue;
#pragma unroll
                    for (int t = KMAX - 1; t >= 1; --t) top[t] = fmin(top[t], fmax(top[t - 1], d));
                    top[0] = fmin(top[0], d);
#pragma unroll
                    for (int t = 0; t < KMAX; ++t)
                        if (t == K - 1) thr = top[t];
                }
            });
            if (thr <= ring_bound2(a, r + 1) || r == rmax) {
                done = true;
                break;
            }
        }
    }
    if (!done) {                                          // far from its neighbours: full sweep later
        const uint32_t k = atomicAdd(&a.counters[4], 1u);
        a.fallback[k] = (int32_t)i;
    }
    double core = 0.0;
#pragma unroll
    for (int t = 0; t < KMAX; ++t)
        if (t == K - 1) core = top[t];
    a.core2[i] = core;
    a.comp[i] = (int32_t)i;
    a.best_j[i] = -1;
    a.partial[i] = 0;
    a.cmin_w[i] = ~0ull;
    a.cmin_e[i] = ~0ull;
    return pairs;
}

template <int KMAX>
__global__ __launch_bounds__(kEmBlock) void k_em_core_grid(EmstArgs a) {
    const int64_t q = (int64_t)blockIdx.x * kEmBlock + threadIdx.x;   // sorted position: cell order
    const uint32_t pairs = q < a.n ? core_grid_point<KMAX>(a, q) : 0u;
    if (a.count_pairs) wave_count(a.pairs, pairs);
}

// Least edge to another component by widening rings.  The search ends when
// nothing farther out can beat the best so far (complete), or when nothing
// farther out can beat the least edge some point of the same component has
// already reported (then this point cannot hold the component's least edge;
// it searches again next round).
__global__ __launch_bounds__(kEmBlock) void k_em_best_grid(EmstArgs a, int64_t count) {
    const int64_t slot = (int64_t)blockIdx.x * kEmBlock + threadIdx.x;
    const bool live = slot < count;
    const int32_t i = live ? a.active[slot] : 0;
    const int32_t mc = a.comp[i];
    double bw = INFINITY;
    int32_t blo = INT32_MAX, bhi = INT32_MAX, bj = -1;
    bool partial = false, done = !live, unchanged = false;
    double lower = 0.0;                                   // after an early stop: least edge >= lower
    uint32_t pairs = 0;
    // An earlier early stop left a lower bound on this point's least edge,
    // which still holds (the candidates only lose points as components
    // grow): if its component already has a lighter edge, nothing to do.
    if (live && a.partial[i]) {
        const double L = a.best_w[i];
        const uint64_t cb = __hip_atomic_load(&a.cmin_w[mc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cb != ~0ull && L > __longlong_as_double((long long)cb)) unchanged = partial = done = true;
    }
    const int32_t io = done ? 0 : a.sorted[i];
    double me[kEmstMaxDim];
    int32_t c[kEmstMaxDim];
#pragma unroll
    for (int k = 0; k < kEmstMaxDim; ++k) {
        me[k] = (k < a.dim && !done) ? (double)a.spts[(int64_t)i * kEmstMaxDim + k] : 0.0;
        c[k] = k < a.dim ? cell_coord(a, me[k], k) : 0;
    }
    const double ci = done ? 0.0 : a.core2[i];
    const int rmax = max_ring(a);
    const int rcap = rmax < kGridRingCap ? rmax : kGridRingCap;
    for (int r = 1; !done && r <= rcap; ++r) {
        for_ring(a, c, me, r, [&](int32_t p0, int32_t p1, double b2) {
            if (b2 > bw) return;                              // nothing in the cell can beat bw
            for (int32_t p = p0; p < p1; ++p) {
                if (a.comp[p] == mc) continue;
                const double d = d2_of(me, a.spts + (int64_t)p * kEmstMaxDim, a.dim);
                ++pairs;
                const double w = fmax(fmax(ci, a.core2[p]), d);
                if (w > bw) continue;
                const int32_t j = a.sorted[p];
                const int32_t lo = j < io ? j : io, hi = j < io ? io : j;
                if (key_less(w, lo, hi, bw, blo, bhi)) {
                    bw = w;
                    blo = lo;
                    bhi = hi;
                    bj = p;
                }
            }
        });
        const double lb2 = ring_bound2(a, r + 1);
        if (bw < lb2 || r == rmax) {                          // complete
            done = true;
            break;
        }
        const uint64_t cb = __hip_atomic_load(&a.cmin_w[mc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cb != ~0ull && lb2 > __longlong_as_double((long long)cb)) {
            partial = true;                                   // stopped early: bw >= lb2 > cb
            lower = lb2;
            done = true;
            break;
        }
    }
    if (live && !done) {                                  // far from other components: full sweep
        a.partial[i] = 0;
        const uint32_t k = atomicAdd(&a.counters[4], 1u);
        a.fallback[k] = i;
    }
    if (live && done && !unchanged) {
        a.best_w[i] = partial ? lower : bw;               // a partial point holds its lower bound
        a.best_j[i] = partial ? -1 : bj;
        a.partial[i] = partial ? 1 : 0;
    }
    wave_min_into(a.cmin_w, mc, (uint64_t)__double_as_longlong(bw), live && done && !partial && bj >= 0);
    if (a.count_pairs) wave_count(a.pairs, pairs);
}

inline unsigned em_blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// The list of the K smallest squared distances lives in registers: its
// capacity is the next of 1, 3, 7, 15, 31 at or above K = min_pts - 1.
template <template <int> class Launch, class... Args>
void with_core_capacity(int K, Args&&... args) {
    if (K <= 1) Launch<1>::run(args...);
    else if (K <= 3) Launch<3>::run(args...);
    else if (K <= 7) Launch<7>::run(args...);
    else if (K <= 15) Launch<15>::run(args...);
    else Launch<kEmMaxK>::run(args...);
}
template <int KMAX>
struct CoreSweep {
    static void run(const EmstArgs& a, const int32_t* list, int64_t count, int64_t m, hipStream_t s) {
        k_em_core<KMAX><<<em_blocks(m, kEmBlock), kEmBlock, 0, s>>>(a, list, count);
    }
};
template <int KMAX>
struct CoreGrid {
    static void run(const EmstArgs& a, hipStream_t s) {
        k_em_core_grid<KMAX><<<em_blocks(a.n, kEmBlock), kEmBlock, 0, s>>>(a);
    }
};

hipError_t launch_em_core(const EmstArgs& a, const int32_t* list, int64_t count, hipStream_t s) {
    const int64_t m = list ? count : a.n;
    if (m > 0) with_core_capacity<CoreSweep>(a.min_pts - 1, a, list, count, m, s);
    return hipGetLastError();
}

hipError_t launch_em_active(const EmstArgs& a, hipStream_t s) {
    k_em_active<<<em_blocks(a.n, kEmPass), kEmPass, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_em_search(const EmstArgs& a, const int32_t* list, int64_t count, hipStream_t s) {
    if (count > 0) k_em_best<<<em_blocks(count, kEmBlock), kEmBlock, 0, s>>>(a, list, count);
    return hipGetLastError();
}

hipError_t launch_em_merge_edges(const EmstArgs& a, hipStream_t s) {
    k_em_cmin<<<em_blocks(a.n, 256), 256, 0, s>>>(a);
    k_em_hook<<<em_blocks(a.roots ? a.nroots : a.n, kEmPass), kEmPass, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_em_bbox(const EmstArgs& a, hipStream_t s) {
    k_em_bbox<<<em_blocks(a.n, 256) < 1024 ? em_blocks(a.n, 256) : 1024, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_em_grid(const EmstArgs& a, hipStream_t s) {
    k_em_cells<<<em_blocks(a.n, 256), 256, 0, s>>>(a);
    const int64_t blocks = (a.ncells + kScanB * kScanI - 1) / (kScanB * kScanI);
    k_em_scan1<<<(unsigned)blocks, kScanB, 0, s>>>(a);
    k_em_scan2<<<1, kScanB, 0, s>>>(a, blocks);
    k_em_scan3<<<(unsigned)blocks, kScanB, 0, s>>>(a);
    k_em_scatter<<<em_blocks(a.n, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_em_core_grid(const EmstArgs& a, hipStream_t s) {
    with_core_capacity<CoreGrid>(a.min_pts - 1, a, s);
    return hipGetLastError();
}

hipError_t launch_em_search_grid(const EmstArgs& a, int64_t active, hipStream_t s) {
    if (active > 0) k_em_best_grid<<<em_blocks(active, kEmBlock), kEmBlock, 0, s>>>(a, active);
    return hipGetLastError();
}

hipError_t launch_em_jump(const EmstArgs& a, int src, hipStream_t s) {
    k_em_jump<<<em_blocks(a.roots ? a.nroots : a.n, 256), 256, 0, s>>>(a, src);
    return hipGetLastError();
}

hipError_t launch_em_relabel(const EmstArgs& a, int src, hipStream_t s) {
    k_em_relabel<<<em_blocks(a.n, kEmPass), kEmPass, 0, s>>>(a, src);
    k_em_copy_comp<<<em_blocks(a.n, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_em_sort_key(const EmstArgs& a, int word, const int32_t* order, uint32_t* keys, int32_t* order_out,
                              hipStream_t s) {
    if (a.n > 1) k_em_sort_key<<<em_blocks(a.n - 1, 256), 256, 0, s>>>(a, word, order, keys, order_out);
    return hipGetLastError();
}

hipError_t launch_em_out(const EmstArgs& a, const int32_t* order, hipStream_t s) {
    if (a.n > 1) k_em_out<<<em_blocks(a.n - 1, 256), 256, 0, s>>>(a, order);
    return hipGetLastError();
}

}  // namespace pandora
