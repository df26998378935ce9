// Stable LSD radix sort with 8- or 9-bit digits for gfx950.
//
// Sorting is the first step of the method (the paper's Section 3.1.1 orders
// the MST edges by weight with a consistent tie order) and it is used again
// to group edges by dendrogram chain (Section 3.3.3).  The paper leaves the
// sort to a library; here it is a one-sweep radix sort:
//
//   * one histogram pass computes the digit counts of every pass at once;
//   * each digit pass loads an 8192-key tile, ranks it stably inside LDS
//     (wave64 ballot matching of digits, per-wave digit counters), publishes
//     the tile's per-digit counts and resolves the global offsets with a
//     decoupled look-back over earlier tiles (dynamic tile ids, so every tile
//     waited on has already started), then scatters from LDS in digit order
//     so that runs of equal digits reach HBM as contiguous writes.
//
// Keys of the first sort are the monotone u32 image of the fp32 weights
// (the value carried is the edge id, generated rather than read); the last
// pass of that sort writes the rank -> edge permutation and scatters its
// inverse, the rank of every edge, so that level 0 can run in input order.
#include "kernels.hpp"

#include <type_traits>

namespace pandora {

namespace {

constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint64_t kFlagMask = 3ull << 62;
constexpr uint64_t kCountMask = ~kFlagMask;
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kLookBatch = 4;   // earlier tiles read per look-back hop
constexpr int kHistBlock = 1024;  // threads of a histogram workgroup

// Waves per SIMD to reserve registers for: the 8192-key, 8-bit pass needs
// 52 KB of LDS, so three 512-thread workgroups fit on a CU if each wave keeps
// to 80 VGPRs.
constexpr int sort_waves_per_eu(int bits, int block, int items) {
    return (bits == 8 && block == 512 && items == 16) ? 6 : 1;
}


// Exclusive scan of one value per thread across a block of BLOCK threads.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_wsum) {
    constexpr int W = BLOCK / kWave;
    const int wave = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(x);
    if (lane_id() == kWave - 1) s_wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int w = 0; w < W; ++w)
        if (w < wave) before += s_wsum[w];
    __syncthreads();
    return before + inc - x;
}

template <int SRC>
__global__ __launch_bounds__(kHistBlock) void k_sort_hist(SortHistArgs a) {
    __shared__ uint32_t s_h[4][kMaxRadix];
    const int radix = 1 << a.bits;
    const uint32_t mask = (uint32_t)radix - 1u;
    for (int i = threadIdx.x; i < 4 * kMaxRadix; i += blockDim.x) (&s_h[0][0])[i] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool nan_seen = false;
    for (int64_t i = t0; i < a.n; i += stride) {
        uint32_t key;
        if (SRC == SRC_WEIGHT) {
            const float w = a.w[i];
            nan_seen |= is_nan_bits(w);
            key = weight_key(w);
        } else {
            key = a.keys[i];
        }
        for (int p = 0; p < a.passes; ++p) atomicAdd(&s_h[p][(key >> (a.bits * p)) & mask], 1u);
    }
    for (int64_t i = t0; i < a.fill_n; i += stride) a.fill64[i] = ~0ull;
    for (int64_t i = t0; i < a.zero_n; i += stride) a.zero32[i] = 0;
    for (int64_t i = t0; i < a.lb_zero_words; i += stride) a.lb_zero[i] = 0;
    if (SRC == SRC_WEIGHT && ballot(nan_seen) != 0 && lane_id() == 0) raise_err(a.ctrl, kErrNaN);
    __syncthreads();
    for (int i = threadIdx.x; i < a.passes * radix; i += blockDim.x) {
        const uint32_t c = s_h[i / radix][i % radix];
        if (c) atomicAdd(&a.ctrl->hist[a.hist_row + i / radix][i % radix], c);
    }
}

template <int BITS, int SRC, int DST, int kSortBlock, int kSortItems>
__global__ __launch_bounds__(kSortBlock, sort_waves_per_eu(BITS, kSortBlock, kSortItems)) void k_sort_pass(SortPassArgs a) {
    constexpr int kRadix = 1 << BITS;
    constexpr int kSortTile = kSortBlock * kSortItems;
    static_assert(kSortBlock >= kRadix, "threads below the radix own one digit each");
    constexpr int W = kSortBlock / kWave;
    __shared__ uint32_t s_cnt[W][kRadix];     // per-wave digit counters, then offsets
    __shared__ uint32_t s_start[kRadix];      // first local slot of each digit
    __shared__ int64_t s_gbase[kRadix];       // global slot of local slot 0 per digit
    using DigitT = typename std::conditional<(BITS <= 8), uint8_t, uint16_t>::type;
    __shared__ uint32_t s_buf[kSortTile];    // keys, then values, in digit order
    __shared__ DigitT s_dig[kSortTile];      // digit of each slot
    __shared__ uint32_t s_wsum[W];
    __shared__ uint32_t s_tile;

    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = lane_id();

    {   // clear the next pass's look-back words (that buffer was used two passes ago)
        const int64_t stride = (int64_t)gridDim.x * kSortBlock;
        for (int64_t i = (int64_t)blockIdx.x * kSortBlock + tid; i < a.lb_zero_words; i += stride)
            a.lb_zero[i] = 0;
    }
    for (int i = tid; i < W * kRadix; i += kSortBlock) (&s_cnt[0][0])[i] = 0;
    if (tid == 0) s_tile = atomicAdd(&a.ctrl->sort_tiles[a.pass], 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t base = tile * kSortTile;
    const int64_t wbase = base + (int64_t)wave * (kWave * kSortItems);

    // Registers are what limits occupancy here: ranks and local slots are
    // packed two per register (both < 2^16), and values are loaded only after
    // the look-back, when the keys are about to leave.
    static_assert(kWave * kSortItems <= 65536 && kSortTile <= 65536, "16-bit ranks and slots");
    static_assert(kSortItems % 2 == 0, "items come in pairs");
    uint32_t key[kSortItems];
    uint32_t rank2[kSortItems / 2];

    // All loads first (past the end the last element is read, then replaced
    // by the sentinel): with the weights' key transform beside each load the
    // compiler waited for every load before issuing the next.
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        int64_t idx = wbase + k * kWave + lane;
        idx = idx < a.n ? idx : a.n - 1;
        key[k] = SRC == SRC_WEIGHT ? __float_as_uint(load_stream(a.w + idx)) : load_stream(a.keys_in + idx);
    }
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = wbase + k * kWave + lane;
        if (SRC == SRC_WEIGHT) key[k] = weight_key(__uint_as_float(key[k]));
        if (idx >= a.n) key[k] = 0xffffffffu;
    }

    // Stable in-wave ranking: lanes holding the same digit find each other with
    // one ballot per digit bit; the lowest such lane bumps the wave's counter.
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const bool valid = wbase + k * kWave + lane < a.n;
        const uint32_t d = (key[k] >> a.shift) & (kRadix - 1);
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t mb = ballot(bit);
            peers &= bit ? mb : ~mb;
        }
        uint32_t rk = 0;
        if (valid) {
            const uint64_t below = peers & lanemask_lt();
            const uint32_t c = s_cnt[wave][d];
            rk = c + (uint32_t)popc64(below);
            if (below == 0) s_cnt[wave][d] = c + (uint32_t)popc64(peers);
        }
        if (k & 1) rank2[k / 2] |= rk << 16;
        else rank2[k / 2] = rk;
    }
    __syncthreads();

    // Thread d < kRadix owns digit d: wave offsets, tile total, look-back.
    const bool owner = tid < kRadix;
    const int d = owner ? tid : 0;
    uint32_t tot = 0;
    uint64_t* my = a.lb + tile * kRadix + d;
    if (owner) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint32_t c = s_cnt[w][d];
            s_cnt[w][d] = tot;
            tot += c;
        }
        st_relaxed(my, (tile == 0 ? kFlagInc : kFlagAgg) | (uint64_t)tot);
    }

    const uint32_t hist_d = owner ? a.ctrl->hist[a.pass][d] : 0u;
    const uint32_t digit_off = block_excl_scan<kSortBlock>(hist_d, s_wsum);
    const uint32_t start = block_excl_scan<kSortBlock>(tot, s_wsum);

    if (owner) {
        s_start[d] = start;
        uint64_t excl = 0;
        if (tile > 0) {
            // Each hop reads kLookBatch earlier tiles at once (independent
            // loads, one latency): consume them newest first up to the first
            // inclusive word, or up to the first tile that has not published.
            int64_t p = tile - 1;
            uint32_t spins = 0;
            bool done = false;
            while (!done) {
                uint64_t wv[kLookBatch];
#pragma unroll
                for (int j = 0; j < kLookBatch; ++j)
                    wv[j] = (p - j >= 0) ? ld_relaxed(a.lb + (p - j) * kRadix + d) : kFlagInc;
                int used = 0;
#pragma unroll
                for (int j = 0; j < kLookBatch; ++j) {
                    if (done || used < j) continue;
                    const uint64_t flag = wv[j] & kFlagMask;
                    if (flag == 0) continue;
                    excl += wv[j] & kCountMask;
                    used = j + 1;
                    if (flag == kFlagInc || p - j <= 0) done = true;
                }
                if (done) break;
                if (used == 0) {
                    if (++spins > kSpinLimit) {
                        raise_err(a.ctrl, kErrSpin);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                spins = 0;
                p -= used;
            }
            st_relaxed(my, kFlagInc | (excl + tot));
        }
        s_gbase[d] = (int64_t)digit_off + (int64_t)excl - (int64_t)start;
    }
    __syncthreads();

    // The tile leaves in digit order, keys first and values second, through
    // one LDS buffer (half the LDS of staging both, so more workgroups fit on
    // a CU); each slot's digit is kept beside it to find its global slot.
    // Consecutive threads take consecutive LDS slots, so each digit's run
    // lands on consecutive global slots.
    // Recompute digits here rather than keep all of them alive across the
    // look-back (an empty asm hides that the keys are unchanged).
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) asm volatile("" : "+v"(key[k]));
#pragma unroll
    for (int k = 0; k < kSortItems / 2; ++k) asm volatile("" : "+v"(rank2[k]));
    uint32_t lp2[kSortItems / 2];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        uint32_t slot = 0;
        if (wbase + k * kWave + lane < a.n) {
            const uint32_t dd = (key[k] >> a.shift) & (kRadix - 1);
            const uint32_t rk = (rank2[k / 2] >> (16 * (k & 1))) & 0xffffu;
            slot = s_start[dd] + s_cnt[wave][dd] + rk;
            s_dig[slot] = (DigitT)dd;
            if (DST == DST_KEYS) s_buf[slot] = key[k];
        }
        if (k & 1) lp2[k / 2] |= slot << 16;
        else lp2[k / 2] = slot;
    }
    // Values of the weight sort are the edge ids themselves, made where used.
    int32_t val[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t idx = wbase + k * kWave + lane;
        val[k] = -1;
        if (SRC == SRC_KEYS && idx < a.n) val[k] = load_stream(a.vals_in + idx);
    }
    __syncthreads();
    const int tile_n = (int)((a.n - base) < kSortTile ? (a.n - base) : kSortTile);
    // A global slot is out of range only after a look-back failure (already
    // reported): never write outside the arrays.
    if (DST == DST_KEYS) {
#pragma unroll 4
        for (int j = 0; j < kSortItems; ++j) {
            const int i = tid + j * kSortBlock;
            if (i < tile_n) {
                const int64_t g = s_gbase[s_dig[i]] + i;
                if (g >= 0 && g < a.n) a.keys_out[g] = s_buf[i];
            }
        }
        __syncthreads();
    }
    int lane_v = lane;   // recomputed below rather than kept from the loads
    asm volatile("" : "+v"(lane_v));
#pragma unroll
    for (int k = 0; k < kSortItems; ++k)
        if (wbase + k * kWave + lane_v < a.n)
            s_buf[(lp2[k / 2] >> (16 * (k & 1))) & 0xffffu] =
                SRC == SRC_WEIGHT ? (uint32_t)(wbase + k * kWave + lane_v) : (uint32_t)val[k];
    __syncthreads();
#pragma unroll 4
    for (int j = 0; j < kSortItems; ++j) {
        const int i = tid + j * kSortBlock;
        if (i >= tile_n) continue;
        const int64_t g = s_gbase[s_dig[i]] + i;
        if (g < 0 || g >= a.n) continue;
        const int32_t id = (int32_t)s_buf[i];
        a.vals_out[g] = id;
        if (DST == DST_RANK && id >= 0 && id < a.n) a.rank[id] = (int32_t)g;
    }
}

}  // namespace

hipError_t launch_sort_hist(int src, const SortHistArgs& a, hipStream_t s) {
    int64_t work = a.n > a.fill_n ? a.n : a.fill_n;
    if (a.zero_n > work) work = a.zero_n;
    // Large workgroups, each flushing one histogram: every workgroup adds its
    // counts to the global histogram with atomics, so fewer and larger ones
    // contend less (measured against 256-thread workgroups).
    int64_t blocks = (work + kHistBlock * 16 - 1) / (kHistBlock * 16);
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    if (src == SRC_WEIGHT)
        k_sort_hist<SRC_WEIGHT><<<dim3((unsigned)blocks), dim3(kHistBlock), 0, s>>>(a);
    else
        k_sort_hist<SRC_KEYS><<<dim3((unsigned)blocks), dim3(kHistBlock), 0, s>>>(a);
    return hipGetLastError();
}

template <int BITS, int BLOCK, int ITEMS>
void launch_pass_cfg(int src, int dst, const SortPassArgs& a, dim3 grid, hipStream_t s) {
    const dim3 block(BLOCK);
    if (src == SRC_WEIGHT && dst == DST_KEYS) k_sort_pass<BITS, SRC_WEIGHT, DST_KEYS, BLOCK, ITEMS><<<grid, block, 0, s>>>(a);
    else if (src == SRC_WEIGHT) k_sort_pass<BITS, SRC_WEIGHT, DST_RANK, BLOCK, ITEMS><<<grid, block, 0, s>>>(a);
    else if (dst == DST_KEYS) k_sort_pass<BITS, SRC_KEYS, DST_KEYS, BLOCK, ITEMS><<<grid, block, 0, s>>>(a);
    else k_sort_pass<BITS, SRC_KEYS, DST_RANK, BLOCK, ITEMS><<<grid, block, 0, s>>>(a);
}

hipError_t launch_sort_pass(int src, int dst, const SortPassArgs& a, hipStream_t s) {
    const int64_t tiles = sort_tiles(a.n, a.cfg);
    if (tiles < 1) return hipSuccess;
    const dim3 grid((unsigned)tiles);
    if (a.bits == 9) {
        switch (a.cfg) {
            case 0: launch_pass_cfg<9, 512, 2>(src, dst, a, grid, s); break;
            case 1: launch_pass_cfg<9, 512, 4>(src, dst, a, grid, s); break;
            case 2: launch_pass_cfg<9, 512, 8>(src, dst, a, grid, s); break;
            default: launch_pass_cfg<9, 512, 16>(src, dst, a, grid, s); break;
        }
    } else {
        switch (a.cfg) {
            case 0: launch_pass_cfg<8, 256, 4>(src, dst, a, grid, s); break;
            case 1: launch_pass_cfg<8, 256, 8>(src, dst, a, grid, s); break;
            case 2: launch_pass_cfg<8, 256, 16>(src, dst, a, grid, s); break;
            default: launch_pass_cfg<8, 512, 16>(src, dst, a, grid, s); break;
        }
    }
    return hipGetLastError();
}

}  // namespace pandora
