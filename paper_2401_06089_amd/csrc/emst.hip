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
// Borůvka rounds: every point finds its least edge to another component by a
// brute-force sweep over LDS tiles of all points (dense fp64 vector work,
// no matrix core shape); a point whose previous least edge still leaves its
// component keeps it.  Components take the least edge of their points
// (two atomic minima: weight bits, then endpoints), hook along it (a
// mutual pair keeps the smaller root), and pointer jumping relabels.  Each
// round at least halves the components.  The tree's edges are then sorted
// by the total order (bitonic network) and handed out with fp64 and fp32
// weights.
#include "kernels.hpp"

namespace pandora {

namespace {

constexpr int kEmBlock = 256;
constexpr int kEmMaxK = kEmstMaxMinPts - 1;       // core-distance rank held in registers

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

__device__ __forceinline__ bool key_less(double w, int32_t lo, int32_t hi, double bw, int32_t blo, int32_t bhi) {
    return w < bw || (w == bw && (lo < blo || (lo == blo && hi < bhi)));
}

// Core distances: each thread keeps the K smallest d2 of its point in
// registers (sorted, fully unrolled so that nothing spills).
__global__ __launch_bounds__(kEmBlock) void k_em_core(EmstArgs a) {
    __shared__ double s_p[kEmBlock][kEmstMaxDim];
    const int64_t i = (int64_t)blockIdx.x * kEmBlock + threadIdx.x;
    const int K = a.min_pts - 1;
    double me[kEmstMaxDim];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kEmstMaxDim; ++k) {
        me[k] = 0.0;
        if (i < a.n && k < a.dim) {
            const float f = a.pts[i * a.dim + k];
            bad |= !isfinite(f);
            me[k] = (double)f;
        }
    }
    double top[kEmMaxK];
#pragma unroll
    for (int t = 0; t < kEmMaxK; ++t) top[t] = INFINITY;
    double thr = INFINITY;                                // top[K-1], kept in a register
    for (int64_t j0 = 0; j0 < a.n; j0 += kEmBlock) {
        __syncthreads();
        const int64_t jl = j0 + threadIdx.x;
#pragma unroll
        for (int k = 0; k < kEmstMaxDim; ++k)
            s_p[threadIdx.x][k] = (jl < a.n && k < a.dim) ? (double)a.pts[jl * a.dim + k] : 0.0;
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
            for (int t = kEmMaxK - 1; t >= 1; --t) top[t] = fmin(top[t], fmax(top[t - 1], d));
            top[0] = fmin(top[0], d);
#pragma unroll
            for (int t = 0; t < kEmMaxK; ++t)
                if (t == K - 1) thr = top[t];
        }
    }
    if (i < a.n) {
        double c = 0.0;
#pragma unroll
        for (int t = 0; t < kEmMaxK; ++t)
            if (t == K - 1) c = top[t];
        a.core2[i] = c;
        a.comp[i] = (int32_t)i;
        a.best_j[i] = -1;
        a.cmin_w[i] = ~0ull;
        a.cmin_e[i] = ~0ull;
    }
    if (ballot(bad) != 0 && lane_id() == 0) atomicOr(&a.counters[2], 1u);
}

// A point's least edge to another component stays its least edge while its
// other end is still outside the point's (grown) component: the candidates
// only lose points.  Such points report it at once; the others are listed
// for a new search.
__global__ void k_em_active(EmstArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int32_t j = a.best_j[i];
    const int32_t mc = a.comp[i];
    if (j >= 0 && a.comp[j] != mc) {
        atomicMin((unsigned long long*)&a.cmin_w[mc], (unsigned long long)__double_as_longlong(a.best_w[i]));
    } else {
        const uint32_t k = atomicAdd(&a.counters[3], 1u);
        a.active[k] = (int32_t)i;
    }
}

// Every listed point's least edge to another component.
__global__ __launch_bounds__(kEmBlock) void k_em_best(EmstArgs a, int64_t count) {
    __shared__ double s_p[kEmBlock][kEmstMaxDim];
    __shared__ double s_c[kEmBlock];
    __shared__ int32_t s_comp[kEmBlock];
    const int64_t slot = (int64_t)blockIdx.x * kEmBlock + threadIdx.x;
    const int64_t i = slot < count ? a.active[slot] : a.n;
    double me[kEmstMaxDim];
#pragma unroll
    for (int k = 0; k < kEmstMaxDim; ++k) me[k] = (i < a.n && k < a.dim) ? (double)a.pts[i * a.dim + k] : 0.0;
    const double ci = i < a.n ? a.core2[i] : 0.0;
    const int32_t mc = i < a.n ? a.comp[i] : -1;
    double bw = INFINITY;
    int32_t blo = INT32_MAX, bhi = INT32_MAX, bj = -1;
    for (int64_t j0 = 0; j0 < a.n; j0 += kEmBlock) {
        __syncthreads();
        const int64_t jl = j0 + threadIdx.x;
#pragma unroll
        for (int k = 0; k < kEmstMaxDim; ++k)
            s_p[threadIdx.x][k] = (jl < a.n && k < a.dim) ? (double)a.pts[jl * a.dim + k] : 0.0;
        s_c[threadIdx.x] = jl < a.n ? a.core2[jl] : 0.0;
        s_comp[threadIdx.x] = jl < a.n ? a.comp[jl] : mc;
        __syncthreads();
        if (i >= a.n) continue;
        const int cnt = a.n - j0 < kEmBlock ? (int)(a.n - j0) : kEmBlock;
        for (int jj = 0; jj < cnt; ++jj) {
            if (s_comp[jj] == mc) continue;
            const double d = d2_of(me, s_p[jj], a.dim);
            const double w = fmax(fmax(ci, s_c[jj]), d);
            const int32_t j = (int32_t)(j0 + jj);
            const int32_t lo = j < (int32_t)i ? j : (int32_t)i, hi = j < (int32_t)i ? (int32_t)i : j;
            if (key_less(w, lo, hi, bw, blo, bhi)) {
                bw = w;
                blo = lo;
                bhi = hi;
                bj = j;
            }
        }
    }
    if (i < a.n) {
        a.best_w[i] = bw;
        a.best_j[i] = bj;
        if (bj >= 0) atomicMin((unsigned long long*)&a.cmin_w[mc], (unsigned long long)__double_as_longlong(bw));
    }
}

// Among the points whose edge has the component's least weight, the least endpoints.
__global__ void k_em_cmin(EmstArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int32_t j = a.best_j[i];
    if (j < 0) return;
    const int32_t c = a.comp[i];
    if ((uint64_t)__double_as_longlong(a.best_w[i]) != a.cmin_w[c]) return;
    const uint64_t lo = (uint64_t)(uint32_t)(j < i ? j : (int32_t)i), hi = (uint64_t)(uint32_t)(j < i ? (int32_t)i : j);
    atomicMin((unsigned long long*)&a.cmin_e[c], (unsigned long long)((lo << 32) | hi));
}

// Each component hooks to the one across its least edge; of a mutual pair
// the smaller root stays a root and records the edge once.
__global__ void k_em_hook(EmstArgs a) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n || a.comp[c] != (int32_t)c) return;
    const uint64_t e = a.cmin_e[c];
    if (e == ~0ull) {                                     // no edge out: the last component
        a.parent[0][c] = (int32_t)c;
        return;
    }
    const int32_t lo = (int32_t)(e >> 32), hi = (int32_t)(e & 0xffffffffu);
    if (lo < 0 || hi >= a.n || lo >= hi) {
        atomicOr(&a.counters[2], 2u);
        a.parent[0][c] = (int32_t)c;
        return;
    }
    const int32_t clo = a.comp[lo], chi = a.comp[hi];
    const int32_t other = clo == (int32_t)c ? chi : clo;
    const bool mutual = a.cmin_e[other] == e;
    const bool stays = mutual && (int32_t)c < other;
    a.parent[0][c] = stays ? (int32_t)c : other;
    if (!mutual || stays) {
        const uint32_t k = atomicAdd(&a.counters[0], 1u);
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
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n || a.comp[c] != (int32_t)c) return;
    const int32_t p = a.parent[src][c];
    const int32_t pp = (p >= 0 && p < a.n) ? a.parent[src][p] : p;
    a.parent[src ^ 1][c] = pp;
    if (pp != p) atomicOr(&a.counters[3], 1u);
}

// New component of every point; the per-component minima start over.
__global__ void k_em_relabel(EmstArgs a, int src) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int32_t r = a.parent[src][a.comp[i]];
    a.comp2[i] = r;
    a.cmin_w[i] = ~0ull;
    a.cmin_e[i] = ~0ull;
    if (r == (int32_t)i) atomicAdd(&a.counters[1], 1u);
}

__global__ void k_em_copy_comp(EmstArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.n) a.comp[i] = a.comp2[i];
}

// One compare-exchange step of a bitonic sorting network over the padded
// edge list (keys: weight bits, then the two endpoints).
__global__ void k_em_bitonic(EmstArgs a, int64_t len, int64_t k, int64_t j) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    const int64_t l = i ^ j;
    if (l <= i) return;
    const bool up = (i & k) == 0;
    const uint64_t wi = a.ew[i], wl = a.ew[l];
    const int32_t ai = a.ea[i], al = a.ea[l], bi = a.eb[i], bl = a.eb[l];
    const bool gt = wi > wl || (wi == wl && (ai > al || (ai == al && bi > bl)));
    if (gt == up) {
        a.ew[i] = wl;
        a.ew[l] = wi;
        a.ea[i] = al;
        a.ea[l] = ai;
        a.eb[i] = bl;
        a.eb[l] = bi;
    }
}

__global__ void k_em_pad(EmstArgs a, int64_t from, int64_t len) {
    const int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    a.ew[i] = ~0ull;
    a.ea[i] = INT32_MAX;
    a.eb[i] = INT32_MAX;
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

__global__ void k_em_out(EmstArgs a) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n - 1) return;
    const double w2 = __longlong_as_double((long long)a.ew[k]);
    const double w = sqrt_rn(w2);
    a.u[k] = a.ea[k];
    a.v[k] = a.eb[k];
    if (a.w64) a.w64[k] = w;
    a.w32[k] = __double2float_rn(w);
}

inline unsigned em_blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_em_core(const EmstArgs& a, hipStream_t s) {
    k_em_core<<<em_blocks(a.n, kEmBlock), kEmBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_em_active(const EmstArgs& a, hipStream_t s) {
    k_em_active<<<em_blocks(a.n, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_em_round(const EmstArgs& a, int64_t active, hipStream_t s) {
    if (active > 0) k_em_best<<<em_blocks(active, kEmBlock), kEmBlock, 0, s>>>(a, active);
    k_em_cmin<<<em_blocks(a.n, 256), 256, 0, s>>>(a);
    k_em_hook<<<em_blocks(a.n, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_em_jump(const EmstArgs& a, int src, hipStream_t s) {
    k_em_jump<<<em_blocks(a.n, 256), 256, 0, s>>>(a, src);
    return hipGetLastError();
}

hipError_t launch_em_relabel(const EmstArgs& a, int src, hipStream_t s) {
    k_em_relabel<<<em_blocks(a.n, 256), 256, 0, s>>>(a, src);
    k_em_copy_comp<<<em_blocks(a.n, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_em_sort_out(const EmstArgs& a, int64_t len, hipStream_t s) {
    const int64_t m = a.n - 1;
    if (len > m) k_em_pad<<<em_blocks(len - m, 256), 256, 0, s>>>(a, m, len);
    for (int64_t k = 2; k <= len; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1) k_em_bitonic<<<em_blocks(len, 256), 256, 0, s>>>(a, len, k, j);
    k_em_out<<<em_blocks(m, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace pandora
