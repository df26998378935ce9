// Dendrogram expansion (paper, Sections 3.3.2 and 3.3.3) on gfx950.
//
// Chain assignment.  An edge e of rank r that was contracted at level l into
// the supervertex S of level l+1 is tested against S's lightest incident
// edge p = minInc_{l+1}(S): if r < p, e belongs to the leaf chain of S at that
// level, whose head hangs below p.  Otherwise S is itself contracted at level
// l+1 and the test repeats one level up with S's own supervertex.  A vertex
// with no incident edge (the last level, or a finished component of a forest)
// has p = +inf and ends the walk: that is the component's root chain.  With
// the flat vertex numbering the walk is a pointer chase
//   x <- svflat[r];  while (r >= vinfo[x].minInc) x <- vinfo[x].label;
// and the final x identifies the chain (k_walk_hist, which also histograms
// the chain keys for the sort that follows).  A leaf edge is lighter than
// every alpha edge of its supervertex, so it always stays there: the level
// kernels flag its record and the walk takes it as it is.
//
// Chain construction.  A stable sort of ranks by chain key lists every chain
// lightest first.  Each edge's parent is the next, heavier edge of its chain;
// the heaviest edge of a chain hangs below the chain's head edge p, or is the
// dendrogram root when p = +inf (k_stitch).  Outputs use input edge ids.
#include "kernels.hpp"

namespace pandora {

namespace {

constexpr int kWalkLimit = 64;
constexpr int kWalkBlock = 1024;   // threads of a walk workgroup

__global__ __launch_bounds__(kWalkBlock) void k_walk_hist(WalkArgs a) {
    __shared__ uint32_t s_h[4][kMaxRadix];
    for (int i = threadIdx.x; i < 4 * kMaxRadix; i += blockDim.x) (&s_h[0][0])[i] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    for (int64_t r = t0; r < a.m; r += stride) {
        const int32_t sv = a.svflat[r];
        int64_t x = sv & ~kLabelFlag;
        // a flagged record is a leaf edge, whose chain is its supervertex
        for (int it = 0;; ++it) {
            if (x < a.n0 || x >= a.flat_cap || it >= kWalkLimit) {
                bad = true;
                x = a.n0;
                break;
            }
            if (sv & kLabelFlag) break;
            // one 8-byte load: both fields arrive together (separate loads
            // would fetch the label only after the comparison, a second
            // dependent trip per step)
            const i32x2 vi = *reinterpret_cast<const i32x2*>(a.vinfo_all + x);
            if (r < (int64_t)vi.x) break;
            x = vi.y;
        }
        const uint32_t key = (uint32_t)(x - a.n0);
        a.ckey[r] = key;
        for (int p = 0, shift = 0; p < a.passes; shift += a.bits[p], ++p)
            atomicAdd(&s_h[p][(key >> shift) & ((1u << a.bits[p]) - 1u)], 1u);
    }
    for (int64_t i = t0; i < a.lb_zero_words; i += stride) a.lb_zero[i] = 0;
    if (ballot(bad) != 0 && lane_id() == 0) raise_err(a.ctrl, kErrWalk);
    __syncthreads();
    for (int i = threadIdx.x; i < a.passes * kMaxRadix; i += blockDim.x) {
        const uint32_t c = s_h[i / kMaxRadix][i % kMaxRadix];
        if (c) atomicAdd(&a.ctrl->hist[a.hist_row + i / kMaxRadix][i % kMaxRadix], c);
    }
}

__global__ __launch_bounds__(256) void k_stitch(StitchArgs a) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.m) return;
    // The four sequential loads go out together: waiting for each before the
    // next (as the branches below would otherwise order them) costs a memory
    // round trip apiece.
    const bool has_next = i + 1 < a.m;
    uint32_t c = a.skey[i];
    int32_t id = a.sid[i];
    uint32_t c_next = has_next ? a.skey[i + 1] : 0u;
    int32_t id_next = has_next ? a.sid[i + 1] : -1;
    asm volatile("" : "+v"(c), "+v"(id), "+v"(c_next), "+v"(id_next));
    if (id < 0 || id >= a.m || (int64_t)c >= a.flat_cap - a.n0) return;   // only after a reported error
    int32_t parent;
    if (has_next && c_next == c) {
        parent = id_next;
    } else {
        const int32_t p = a.vinfo_all[a.n0 + (int64_t)c].minInc;
        parent = (p < 0 || p >= a.m) ? -1 : a.perm[p];
    }
    if (parent >= 0 && a.forest.B > 1)
        parent = (int32_t)(parent - a.forest.edge_base(a.forest.tree_of_edge_fast(id)));
    a.edge_parent[id] = parent;
}

__global__ void k_zero_control(Control* c, int32_t m, int32_t n, int64_t* voff1) {
    uint32_t* p = reinterpret_cast<uint32_t*>(c);
    const int words = (int)(sizeof(Control) / sizeof(uint32_t));
    for (int i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        c->lv[0].m = m;
        c->lv[0].n = n;
        c->lv[0].off = 0;
        if (voff1) {            // a single tree: its offsets need no copy from the host
            voff1[0] = 0;
            voff1[1] = n;
        }
    }
}

// End of a stream-ordered call: its input errors (and a component count other
// than the number of trees) are OR-ed into the stream's sticky status word.
__global__ void k_finalize(const Control* c, int32_t B, uint32_t* sticky) {
    if (threadIdx.x != 0) return;
    uint32_t e = c->err;
    if (e == 0 && (int64_t)c->isolated != B) e = kErrNotTree;
    if (e) atomicOr(sticky, e);
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = value;
}

// The forest index: the tree of every 64th edge and vertex, closed by B-1.
__global__ void k_forest_index(Forest f, int64_t m, int64_t n, int32_t* te, int32_t* tv) {
    const int64_t ke = (m + 63) >> 6, kv = (n + 63) >> 6;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= ke + kv + 1; k += stride) {
        if (k < ke) te[k] = f.tree_of_edge(k << 6);
        else if (k == ke) te[k] = f.B - 1;
        else if (k - ke - 1 < kv) tv[k - ke - 1] = f.tree_of_vertex((k - ke - 1) << 6);
        else tv[kv] = f.B - 1;
    }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = value;
}

}  // namespace

hipError_t launch_walk_hist(const WalkArgs& a, hipStream_t s) {
    // Fewer, larger workgroups: each adds its chain-key histogram to the
    // global one with atomics (512 x 1024 threads still fill the GPU).
    int64_t blocks = (a.m + kWalkBlock * 8 - 1) / (kWalkBlock * 8);
    if (blocks < 1) blocks = 1;
    if (blocks > 512) blocks = 512;
    k_walk_hist<<<(unsigned)blocks, kWalkBlock, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_stitch(const StitchArgs& a, hipStream_t s) {
    if (a.m < 1) return hipSuccess;
    k_stitch<<<(unsigned)((a.m + 255) / 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_finalize(const Control* c, int32_t B, uint32_t* sticky, hipStream_t s) {
    k_finalize<<<1, 64, 0, s>>>(c, B, sticky);
    return hipGetLastError();
}

hipError_t launch_clear_words(uint32_t* p, int64_t n, hipStream_t s) {
    if (n < 1) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_fill_u32<<<(unsigned)blocks, 256, 0, s>>>(p, n, 0u);
    return hipGetLastError();
}

hipError_t launch_forest_index(const Forest& f, int64_t m, int64_t n, int32_t* te, int32_t* tv, hipStream_t s) {
    const int64_t work = ((m + 63) >> 6) + ((n + 63) >> 6) + 2;
    int64_t blocks = (work + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_forest_index<<<(unsigned)blocks, 256, 0, s>>>(f, m, n, te, tv);
    return hipGetLastError();
}

hipError_t launch_zero_control(Control* c, int32_t m, int32_t n, int64_t* voff1, hipStream_t s) {
    k_zero_control<<<1, 256, 0, s>>>(c, m, n, voff1);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t value, hipStream_t s) {
    if (n < 1) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_fill_i32<<<(unsigned)blocks, 256, 0, s>>>(p, n, value);
    return hipGetLastError();
}

}  // namespace pandora
