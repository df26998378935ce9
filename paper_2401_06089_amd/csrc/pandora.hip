// Host orchestration and C ABI of libpandora.so (see include/pandora.h).
//
// One call runs the whole method (Sections 3.1-3.3) on the device:
//   1. weight sort: one histogram pass and 4 one-sweep radix passes over the
//      u32 image of the weights; the last pass writes perm (rank -> edge id)
//      and scatters rank (edge id -> rank);
//   2. contraction levels, level 0 in the caller's edge order: k_min_incident,
//      k_own, k_classify, k_jump (rounds until converged), k_compact.  Either
//      the host reads one small block back per level and launches exact
//      grids, or every level is launched with capacity-sized grids and nothing
//      is read back (the form a HIP graph captures).  Levels below
//      persist_max_edges may instead run in one persistent launch (k_levels);
//   3. every level small enough for LDS in one workgroup (k_tail);
//   4. expansion: chain keys by the level walk (with the chain-key histogram),
//      radix passes of (chain key, edge id), stitch.
// A forest gets its offsets copied once and a small index (the tree of every
// 64th edge and vertex) for tree lookups.  The plain calls wait for their
// stream and return the status; the stream-ordered calls do not wait and leave
// their status in a per-stream word on the device.
//
// Scratch memory comes from one allocation per (device, stream), kept
// between calls and grown on demand (or the caller's buffer).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "pandora.h"

// Scratch of pandora_dendrogram_noalloc: a fixed array in every GPU's memory
// (see run_noalloc).  Its name stands for a host-side shadow in host code;
// kernels get the device address from noalloc_symbol_address().
static __device__ __align__(256) unsigned char scratch[PANDORA_NOALLOC_SCRATCH_BYTES];

static void* noalloc_symbol_address() {   // for the current device
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

namespace pandora {
namespace {

constexpr int kMaxJumpRounds = 64;
constexpr int kSyncFreeJumpRounds = 3;   // the last one is bounded only by the level size
constexpr int kPersistJumpRounds = 6;    // rounds inside the persistent level kernel (same rule)
constexpr size_t kAlign = 256;
constexpr size_t kCtrlReadback = 32;   // err .. tail_vertices
constexpr size_t kCtrlLevelsReadback = offsetof(Control, hist);   // header + level table

// Process-wide tuning (pandora_set_tuning); read once per call.
std::mutex g_tune_mu;
pandora_tuning_t g_tune = {
    /*sync_free_max_edges=*/0,
    /*jump_steps=*/16,
    /*chain_digit_bits=*/0,
    /*sort_tile_cfg=*/kDefaultSortCfg,
    /*persist_max_edges=*/0,
};

thread_local bool t_has_tune = false;
thread_local pandora_tuning_t t_tune;

pandora_tuning_t current_tuning() {
    if (t_has_tune) return t_tune;
    std::lock_guard<std::mutex> g(g_tune_mu);
    return g_tune;
}

bool tuning_valid(const pandora_tuning_t* t) {
    return t->sync_free_max_edges >= 0 && t->jump_steps >= 1 && t->jump_steps <= 4096 &&
           (t->chain_digit_bits == 0 || t->chain_digit_bits == 8 || t->chain_digit_bits == 9) &&
           t->sort_tile_cfg >= 0 && t->sort_tile_cfg < kNumSortCfg && t->persist_max_edges >= 0;
}

// Compute units of a device (the persistent level kernel sizes its grid by
// them).
int cu_count(int dev) {
    static std::mutex mu;
    static std::map<int, int> cache;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 64;
    cache[dev] = cus;
    return cus;
}

// Digit widths of the chain sort's passes (least significant first).
struct ChainDigits {
    int passes = 1;
    int bits[4] = {8, 8, 8, 8};
    int widest() const {
        int w = 0;
        for (int p = 0; p < passes; ++p) w = std::max(w, bits[p]);
        return w;
    }
};

struct Layout {
    int64_t N = 0, M = 0;
    int32_t B = 0;
    int Lmax = 0;
    std::vector<int64_t> capE, capV;
    int64_t flat_cap = 0;
    ChainDigits chain;
    int sort_cfg = kDefaultSortCfg;
    int64_t lb_words_w = 0, lb_words_c = 0;   // look-back words per pass (weight / chain sort)
    size_t ctrl, voff, tidx, K0, K1, V0, V1, perm, rank, E0, EA, EB, EA_r, EB_r, min64, own, alpha, scan_lb,
        tile_excl, vinfo, ptr, svflat, lb0, lb1;
    size_t total = 0;
};

size_t take(size_t& cursor, size_t bytes) {
    const size_t at = cursor;
    cursor += (bytes + kAlign - 1) / kAlign * kAlign;
    return at;
}

int ceil_log2(int64_t x) {   // smallest L with 2^L >= x (x >= 1)
    int L = 0;
    while ((int64_t(1) << L) < x) ++L;
    return L;
}

// Digit widths of the chain sort for chain keys in [0, key_range): as few
// passes as cover the keys, each of 8 bits, or of 9 bits where 8-bit passes
// alone would need one more (a 9-bit pass is slower); or all of the width the
// tuning fixes.  Widths are listed least significant digit first.
ChainDigits chain_digits(int64_t key_range, int pref) {
    int total = 0;
    while ((int64_t(1) << total) < std::max<int64_t>(key_range, 1)) ++total;
    ChainDigits c;
    if (pref == 8 || pref == 9) {
        c.passes = std::max(1, (total + pref - 1) / pref);
        for (int p = 0; p < c.passes; ++p) c.bits[p] = pref;
        return c;
    }
    c.passes = std::max(1, (total + 8) / 9);             // fewest passes of at most 9 bits
    const int nine = std::max(0, total - 8 * c.passes);  // 9-bit passes those need
    for (int p = 0; p < c.passes; ++p) c.bits[p] = p < nine ? 9 : 8;
    return c;
}

Layout make_layout(int64_t N, int32_t B, int chain_bits_pref = 0, int sort_cfg = kDefaultSortCfg) {
    Layout L;
    L.N = N;
    L.B = B;
    L.M = N - B;
    const int64_t M = L.M;
    // Section 4.2: at most (m-1)/2 alpha edges per level, so at most
    // ceil(log2(m+1)) levels.  A level of a forest has at most m_j + B
    // vertices, and one vertex per leaf edge of the level before.
    L.Lmax = ceil_log2(M + 1) + 2;
    L.capE.assign(L.Lmax + 2, 0);
    L.capV.assign(L.Lmax + 2, 0);
    L.capE[0] = M;
    L.capV[0] = N;
    for (int j = 1; j < (int)L.capE.size(); ++j) {
        L.capE[j] = L.capE[j - 1] / 2;
        L.capV[j] = std::min<int64_t>(std::min<int64_t>(L.capE[j] + B, L.capE[j - 1]), N);
    }
    L.flat_cap = 0;
    for (int64_t c : L.capV) L.flat_cap += c;
    L.chain = chain_digits(L.flat_cap - N, chain_bits_pref);

    const int64_t E1 = std::max<int64_t>(L.capE[1], 1), E2 = std::max<int64_t>(L.capE[2], 1);
    L.sort_cfg = sort_cfg;
    L.lb_words_w = sort_tiles(std::max<int64_t>(M, 1), sort_cfg) * 256;
    // room for 9-bit chain digits whatever the capacity suggests: a call may
    // pick its digits from the level sizes it finds (see enqueue)
    L.lb_words_c = sort_tiles(std::max<int64_t>(M, 1), sort_cfg) * (int64_t(1) << kMaxRadixBits);
    const int64_t sortlb = std::max(L.lb_words_w, L.lb_words_c);
    const int64_t scant = scan_tiles(std::max<int64_t>(M, 1));
    size_t c = 0;
    L.ctrl = take(c, sizeof(Control));
    L.voff = take(c, sizeof(int64_t) * (B + 1));
    // forest index (a single tree has none: its arrays keep their placement)
    L.tidx = take(c, B > 1 ? sizeof(int32_t) * (((M + 63) >> 6) + ((N + 63) >> 6) + 2) : 0);
    L.K0 = take(c, 4 * M);
    L.K1 = take(c, 4 * M);
    L.V0 = take(c, 4 * M);
    L.V1 = take(c, 4 * M);
    L.perm = take(c, 4 * M);
    L.rank = take(c, 4 * M);
    L.E0 = take(c, 8 * M);   // level 0: (u, v); id = position, rank in `rank`
    L.EA = take(c, 8 * E1);
    L.EB = take(c, 8 * E2);
    L.EA_r = take(c, 4 * E1);
    L.EB_r = take(c, 4 * E2);
    L.min64 = take(c, 8 * N);
    L.own = take(c, 2 * M);
    L.alpha = take(c, M);
    L.scan_lb = take(c, 8 * scant);
    L.tile_excl = take(c, 4 * scant);
    L.vinfo = take(c, sizeof(VInfo) * L.flat_cap);
    L.ptr = take(c, 4 * N);
    L.svflat = take(c, 4 * M);
    L.lb0 = take(c, 8 * sortlb);
    L.lb1 = take(c, 8 * sortlb);
    L.total = c;
    return L;
}

// Vertices of all levels share one int32 id space (about 2n ids for one
// tree); larger inputs are rejected up front.
bool ids_fit(int64_t N, int32_t B) {
    if (N <= B) return true;
    return make_layout(N, B).flat_cap <= INT32_MAX;
}

// Pinned staging for the offsets of a stream-ordered batched call: the copy
// to the device runs later in stream order, so a slot is reused only once the
// event after its copy has completed.
constexpr int kStageSlots = 4;
struct StageSlot {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};

struct Workspace {
    std::mutex mu;
    void* dev = nullptr;
    size_t bytes = 0;
    bool owned = true;             // false: the caller's buffer (pandora_set_workspace)
    void* host = nullptr;          // pinned: Control readback + voff staging
    size_t host_bytes = 0;
    uint32_t* sticky = nullptr;    // device: deferred status of stream-ordered calls
    StageSlot stage[kStageSlots];
    int next_stage = 0;
    hipStream_t stream = nullptr;
    hipEvent_t readback = nullptr; // marks a level's Control readback (the host waits for it alone)
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;

struct Stats {
    int64_t levels = 0, sum_edges = 0, jump_launches = 0, tail_levels = 0, tail_entry_edges = 0,
            sync_free = 0, persistent = 0;
    int chain_passes = 0;   // passes the chain sort ran (its output ends in K1/V1 when odd, else K0/V0)
};
thread_local Stats g_last;

// ---- per-kernel profiler: HIP events around selected launches -------------------
// Algorithmic bytes per launch are the minimum traffic of each kernel (every
// array element it must read or write once; gathers count 4 bytes).
// Level kernels are split into their level-0 and deeper-level instantiations
// (different templates, different sizes per launch).
enum ProfKind {
    PK_ZERO, PK_SORT_HIST, PK_SORT_W_FIRST, PK_SORT_W_MID, PK_SORT_W_LAST, PK_MIN_INC,
    PK_OWN, PK_CLASSIFY, PK_JUMP, PK_COMPACT, PK_TAIL, PK_WALK_HIST, PK_SORT_C_PASS, PK_STITCH,
    PK_MIN_INC_N, PK_OWN_N, PK_CLASSIFY_N, PK_JUMP_N, PK_COMPACT_N, PK_LEVELS,
    PK_FC_PREPARE, PK_FC_SIZES, PK_FC_CLUSTERS, PK_FC_STAB, PK_FC_SELECT, PK_FC_LABEL,
    PK_EM_CORE, PK_EM_SEARCH, PK_EM_MERGE, PK_EM_SORT,
    PK_COUNT
};
const char* const kProfNames[PK_COUNT] = {
    "zero_control", "sort_hist", "sort_pass_weight_first", "sort_pass_weight_mid",
    "sort_pass_weight_last", "min_incident_l0", "own_l0", "classify_l0", "jump_l0", "compact_l0",
    "tail", "walk_hist", "sort_pass_chain", "stitch", "min_incident_ln", "own_ln", "classify_ln",
    "jump_ln", "compact_ln", "levels_persistent", "flat_prepare", "flat_sizes", "flat_clusters",
    "flat_stability", "flat_select", "flat_label", "emst_core", "emst_search", "emst_merge", "emst_sort"};

struct Prof {
    std::mutex mu;
    uint32_t mask = 0;                // kinds being timed (0 = profiling off)
    double ms[PK_COUNT] = {};
    double bytes[PK_COUNT] = {};
    int64_t launches[PK_COUNT] = {};
};
Prof g_prof;

struct PendingEvent {
    hipEvent_t a, b;
    int kind;
    double bytes;
};
thread_local std::vector<PendingEvent> t_pending;
thread_local std::vector<hipEvent_t> t_event_pool;

hipEvent_t pooled_event() {
    if (!t_event_pool.empty()) {
        hipEvent_t e = t_event_pool.back();
        t_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

thread_local bool t_capturing = false;   // no profiler events inside a graph capture

template <class F>
hipError_t timed(int kind, double bytes, hipStream_t s, F&& launch) {
    uint32_t mask;
    {
        std::lock_guard<std::mutex> g(g_prof.mu);
        mask = t_capturing ? 0u : g_prof.mask;
    }
    if (!(mask & (1u << kind))) return launch();
    hipEvent_t a = pooled_event(), b = pooled_event();
    if (!a || !b) return launch();
    (void)hipEventRecord(a, s);
    const hipError_t e = launch();
    (void)hipEventRecord(b, s);
    t_pending.push_back({a, b, kind, bytes});
    return e;
}

// Adds work counted on the device to a kind's algorithmic total (its
// launches are timed separately).
void profile_add(int kind, double amount) {
    std::lock_guard<std::mutex> g(g_prof.mu);
    if (!t_capturing && (g_prof.mask & (1u << kind))) g_prof.bytes[kind] += amount;
}

bool profiling(int kind) {
    std::lock_guard<std::mutex> g(g_prof.mu);
    return !t_capturing && (g_prof.mask & (1u << kind));
}

// Sets the algorithmic bytes of the latest timed launch of `kind`, for
// launches enqueued before the host knew their size.
void set_last_bytes(int kind, double bytes) {
    for (auto it = t_pending.rbegin(); it != t_pending.rend(); ++it)
        if (it->kind == kind) {
            it->bytes = bytes;
            return;
        }
}

// Called once the stream has been synchronized.
void drain_profile() {
    if (t_pending.empty()) return;
    std::lock_guard<std::mutex> g(g_prof.mu);
    for (const PendingEvent& p : t_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_prof.ms[p.kind] += ms;
            g_prof.bytes[p.kind] += p.bytes;
            g_prof.launches[p.kind] += 1;
        }
        t_event_pool.push_back(p.a);
        t_event_pool.push_back(p.b);
    }
    t_pending.clear();
}

#define PD_TIMED(kind, bytes, expr) PD_TRY(timed((kind), (double)(bytes), s, [&]() { return (expr); }))

Workspace* workspace_for(int dev, hipStream_t s) {
    std::lock_guard<std::mutex> g(g_mu);
    auto& slot = g_ws[{dev, s}];
    if (!slot) {
        slot.reset(new Workspace);
        slot->stream = s;
    }
    return slot.get();
}

int status_from_err(uint32_t err) {
    if (err & kErrBadVertex) return PANDORA_ERR_BAD_VERTEX;
    if (err & kErrNaN) return PANDORA_ERR_NAN_WEIGHT;
    if (err & (kErrNotTree | kErrOverflow)) return PANDORA_ERR_NOT_A_TREE;
    if (err) return PANDORA_ERR_HIP;
    return PANDORA_OK;
}

#define PD_TRY(expr)                                 \
    do {                                             \
        if ((expr) != hipSuccess) return PANDORA_ERR_HIP; \
    } while (0)

int ensure(Workspace& ws, size_t dev_bytes, size_t host_bytes) {
    if (!ws.owned && ws.bytes < dev_bytes) return PANDORA_ERR_OUT_OF_MEMORY;   // the caller's buffer is too small
    if (ws.bytes < dev_bytes) {
        if (ws.dev) {
            if (hipStreamSynchronize(ws.stream) != hipSuccess) return PANDORA_ERR_HIP;
            (void)hipFree(ws.dev);
            ws.dev = nullptr;
            ws.bytes = 0;
        }
        if (hipMalloc(&ws.dev, dev_bytes) != hipSuccess) {
            ws.dev = nullptr;
            (void)hipGetLastError();
            return PANDORA_ERR_OUT_OF_MEMORY;
        }
        ws.bytes = dev_bytes;
        // No initial clearing: every look-back buffer is cleared on the call's
        // stream by the kernel that runs before its first user.  (A blocking
        // memset here would run on the null stream, unordered with respect to
        // non-blocking streams that may already be computing.)
    }
    if (!ws.readback && hipEventCreateWithFlags(&ws.readback, hipEventDisableTiming) != hipSuccess) {
        ws.readback = nullptr;
        (void)hipGetLastError();
        return PANDORA_ERR_HIP;
    }
    if (ws.host_bytes < host_bytes) {
        if (ws.host) (void)hipHostFree(ws.host);
        ws.host = nullptr;
        ws.host_bytes = 0;
        if (hipHostMalloc(&ws.host, host_bytes, hipHostMallocDefault) != hipSuccess) {
            ws.host = nullptr;
            (void)hipGetLastError();
            return PANDORA_ERR_OUT_OF_MEMORY;
        }
        ws.host_bytes = host_bytes;
    }
    return PANDORA_OK;
}

template <class T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

int read_ctrl(Control* dctrl, Control* hctrl, hipStream_t s, size_t bytes = kCtrlReadback) {
    PD_TRY(hipMemcpyAsync(hctrl, dctrl, bytes, hipMemcpyDeviceToHost, s));
    PD_TRY(hipStreamSynchronize(s));
    return PANDORA_OK;
}

// One call's memory: the device scratch block and the pinned host block
// (Control readback, then voff staging).
struct Scratch {
    void* dev;
    void* host;
    hipEvent_t readback = nullptr;   // null: wait for the whole stream at every readback
};

size_t host_bytes_for(int32_t B) { return sizeof(Control) + sizeof(int64_t) * (B + 1); }

// Enqueues the whole method for a forest given by host offsets voff[0..B]
// (M >= 1 edges).  With sync_free nothing waits for the device before the
// final readback in finish(), so the sequence can be captured in a graph.
int enqueue(const Scratch& sc, const Layout& L, const pandora_tuning_t& tune, bool sync_free,
            const int64_t* staged_voff, int32_t B, const int32_t* u, const int32_t* v, const float* w,
            int32_t* edge_parent, int32_t* vertex_parent, hipStream_t s, Stats& st) {
    const int64_t N = L.N;
    const int64_t M = L.M;
    int rc = PANDORA_OK;
    void* d = sc.dev;
    Control* ctrl = at<Control>(d, L.ctrl);
    Control* hctrl = static_cast<Control*>(sc.host);
    // Tree offsets on the device: a single tree's are written by the first
    // kernel; a forest's are copied from pinned staging that stays valid
    // until the copy has run.
    int64_t* dvoff = at<int64_t>(d, L.voff);
    if (B > 1) PD_TRY(hipMemcpyAsync(dvoff, staged_voff, sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice, s));
    int32_t* tidx_e = B > 1 ? at<int32_t>(d, L.tidx) : nullptr;
    int32_t* tidx_v = B > 1 ? tidx_e + ((M + 63) >> 6) + 1 : nullptr;
    const Forest forest{dvoff, B, tidx_e, tidx_v};
    if (B > 1) PD_TRY(launch_forest_index(forest, M, N, tidx_e, tidx_v, s));

    uint32_t* K[2] = {at<uint32_t>(d, L.K0), at<uint32_t>(d, L.K1)};
    int32_t* V[2] = {at<int32_t>(d, L.V0), at<int32_t>(d, L.V1)};
    uint64_t* LB[2] = {at<uint64_t>(d, L.lb0), at<uint64_t>(d, L.lb1)};
    int32_t* perm = at<int32_t>(d, L.perm);
    VInfo* vinfo_all = at<VInfo>(d, L.vinfo);
    int32_t* svflat = at<int32_t>(d, L.svflat);
    const int64_t lb_words = L.lb_words_w;

    PD_TIMED(PK_ZERO, sizeof(Control), launch_zero_control(ctrl, (int32_t)M, (int32_t)N, B == 1 ? dvoff : nullptr, s));

    // ---- 1. weight sort --------------------------------------------------------
    uint64_t* min64 = at<uint64_t>(d, L.min64);
    uint16_t* own = at<uint16_t>(d, L.own);
    int32_t* rank = at<int32_t>(d, L.rank);
    {
        SortHistArgs h{};
        h.n = M;
        h.bits = 8;
        h.hist_row = 0;
        h.passes = 4;
        h.w = w;
        h.fill64 = min64;           // level 0 starts with no lightest edge
        h.fill_n = N;
        h.zero32 = reinterpret_cast<uint32_t*>(own);
        h.zero_n = (2 * M + 3) / 4;
        h.lb_zero = LB[0];
        h.lb_zero_words = lb_words;
        h.ctrl = ctrl;
        PD_TIMED(PK_SORT_HIST, 4.0 * M + 8.0 * N + 2.0 * M, launch_sort_hist(SRC_WEIGHT, h, s));
        const uint32_t* kin = nullptr;
        const int32_t* vin = nullptr;
        for (int p = 0; p < 4; ++p) {
            SortPassArgs a{};
            a.n = M;
            a.cfg = L.sort_cfg;
            a.bits = 8;
            a.shift = 8 * p;
            a.pass = p;
            a.w = w;
            a.keys_in = kin;
            a.vals_in = vin;
            a.keys_out = K[p & 1];
            a.vals_out = (p == 3) ? perm : V[p & 1];
            a.rank = rank;
            a.lb = LB[p & 1];
            a.lb_zero = LB[(p + 1) & 1];
            a.lb_zero_words = lb_words;
            a.ctrl = ctrl;
            const int kind = p == 0 ? PK_SORT_W_FIRST : (p == 3 ? PK_SORT_W_LAST : PK_SORT_W_MID);
            const double by = (p == 0 ? 12.0 : 16.0) * M;
            PD_TIMED(kind, by, launch_sort_pass(p == 0 ? SRC_WEIGHT : SRC_KEYS, p == 3 ? DST_RANK : DST_KEYS, a, s));
            kin = K[p & 1];
            vin = V[p & 1];
        }
    }

    // ---- 2. contraction levels --------------------------------------------------
    i32x2* E0 = at<i32x2>(d, L.E0);
    i32x2* EA = at<i32x2>(d, L.EA);
    i32x2* EB = at<i32x2>(d, L.EB);
    int32_t* EA_r = at<int32_t>(d, L.EA_r);
    int32_t* EB_r = at<int32_t>(d, L.EB_r);
    const int jump_steps = tune.jump_steps > 0 ? tune.jump_steps : 16;
    auto level_args = [&](int j) {
        LevelArgs a{};
        a.level = j;
        a.cap_m = (int32_t)L.capE[j];
        a.cap_n = (int32_t)L.capV[j];
        a.in_u = u;
        a.in_v = v;
        a.rank = rank;
        a.forest = forest;
        a.E = j == 0 ? E0 : (j % 2 == 1 ? EA : EB);
        a.Er = j == 0 ? rank : (j % 2 == 1 ? EA_r : EB_r);
        a.out = j % 2 == 0 ? EA : EB;
        a.out_r = j % 2 == 0 ? EA_r : EB_r;
        a.min64 = min64;
        a.vinfo_all = vinfo_all;
        // level 0's minima and labels live in its part of the flat table
        // (2 x 4 bytes per vertex), as two plain arrays
        a.min0 = reinterpret_cast<int32_t*>(vinfo_all);
        a.lab0 = a.min0 + N;
        a.ptr = at<int32_t>(d, L.ptr);
        a.own = own;
        a.alpha = at<uint8_t>(d, L.alpha);
        a.scan_lb = at<uint64_t>(d, L.scan_lb);
        a.tile_alpha_excl = at<int32_t>(d, L.tile_excl);
        a.cap_next_e = (int32_t)L.capE[j + 1];
        a.cap_next_v = (int32_t)L.capV[j + 1];
        a.svflat = svflat;
        a.vertex_parent = vertex_parent;
        a.ctrl = ctrl;
        a.jump_steps = jump_steps;
        // measured on 4,096 trees of lognormal sizes: level 0's minima 1.88 -> 1.28 ms,
        // the deeper levels' 0.93 -> 0.75 ms; forests of a few large trees are a little
        // faster without
        a.spread = B > 1 && M <= (int64_t)B * kSpreadMaxMeanEdges;
        return a;
    };
    // Levels of at most persist_max_edges edges run in one persistent launch
    // (from level j on, until a level fits the LDS tail).
    int dev = 0;
    PD_TRY(hipGetDevice(&dev));
    auto persistent_from = [&](int j) {
        PersistArgs p{};
        p.a = level_args(j);
        p.E0 = E0;
        p.EA = EA;
        p.EB = EB;
        p.EA_r = EA_r;
        p.EB_r = EB_r;
        p.first_level = j;
        p.last_level = L.Lmax;
        p.jump_rounds = kPersistJumpRounds;
        for (int k = 0; k <= kMaxLevels; ++k) {
            p.capE[k] = k < (int)L.capE.size() ? (int32_t)L.capE[k] : 0;
            p.capV[k] = k < (int)L.capV.size() ? (int32_t)L.capV[k] : 0;
        }
        st.persistent = 1;
        // a quarter of the CUs: fewer arrivals per grid barrier, enough
        // workgroups for levels of this size (measured best of 1/1 to 1/8)
        return launch_levels(p, std::max(1, cu_count(dev) / 4), s);
    };
    const int64_t persist_max = tune.persist_max_edges;
    st.sync_free = sync_free ? 1 : 0;
    ChainDigits chain = L.chain;
    if (!sync_free) {
        // Host-driven: exact grids, pointer jumping relaunched until it converges.
        int64_t m = M, n = N, off = 0;
        int j = 0;
        while (!tail_level(m, n, kTailE, kTailV)) {
            if (j >= L.Lmax) return PANDORA_ERR_NOT_A_TREE;
            const bool l0 = j == 0;
            LevelArgs a = level_args(j);
            a.cap_m = (int32_t)m;
            a.cap_n = (int32_t)n;
            PD_TIMED(l0 ? PK_MIN_INC : PK_MIN_INC_N, (l0 ? 20.0 : 12.0) * m + 16.0 * n,
                     launch_min_incident(l0, a, s));
            if (m <= persist_max) {
                PD_TIMED(PK_LEVELS, 60.0 * m, persistent_from(j));
                break;
            }
            PD_TIMED(l0 ? PK_OWN : PK_OWN_N, (l0 ? 29.0 : 25.0) * n, launch_own(l0, a, s));
            // classification and the first jumping round: bytes set once the
            // next level's size is read back (below)
            PD_TIMED(l0 ? PK_CLASSIFY : PK_CLASSIFY_N, 3.0 * m, launch_classify(a, s));
            // The compaction is queued behind the first jumping round before the
            // host waits for the readback, guarded by that round's convergence
            // bit, so the device does not idle during the round trip; if the
            // round left work, it returns at once and runs again after the
            // further rounds.
            const int kc = l0 ? PK_COMPACT : PK_COMPACT_N;
            bool compacted = false;
            for (int round = 0;; ++round) {
                if (round >= kMaxJumpRounds) return PANDORA_ERR_NOT_A_TREE;
                a.round = round;
                PD_TIMED(l0 ? PK_JUMP : PK_JUMP_N, (round == 0 ? 18.0 : 4.0) * n, launch_jump(a, s));
                ++st.jump_launches;
                if (round == 0 && sc.readback) {
                    PD_TRY(hipMemcpyAsync(hctrl, ctrl, kCtrlReadback, hipMemcpyDeviceToHost, s));
                    PD_TRY(hipEventRecord(sc.readback, s));
                    a.compact_guard = 1u;
                    PD_TIMED(kc, 0.0, launch_compact(a, s));
                    PD_TRY(hipEventSynchronize(sc.readback));
                    compacted = true;
                } else {
                    rc = read_ctrl(ctrl, hctrl, s);
                    if (rc != PANDORA_OK) return rc;
                }
                if (hctrl->err) {
                    PD_TRY(hipStreamSynchronize(s));
                    return status_from_err(hctrl->err);
                }
                if (round == 0) {
                    // n_next leaf edges: their endpoints are labelled by the
                    // classification, which reads only those edges' records
                    const double nn = (double)hctrl->n_next;
                    set_last_bytes(l0 ? PK_CLASSIFY : PK_CLASSIFY_N, 3.0 * m + 16.0 * nn);
                    set_last_bytes(l0 ? PK_JUMP : PK_JUMP_N, 24.0 * n - 12.0 * nn);
                }
                if (!(hctrl->not_converged & (1u << (round & 31)))) break;
                compacted = false;   // the guarded compaction returned at once
            }
            const int64_t m_next = hctrl->m_next, n_next = hctrl->n_next;
            if (m_next > L.capE[j + 1] || n_next > L.capV[j + 1] || m_next >= m) {
                PD_TRY(hipStreamSynchronize(s));
                return PANDORA_ERR_NOT_A_TREE;
            }
            if (compacted) {
                set_last_bytes(kc, 1.0 * m + 32.0 * m_next);
            } else {
                a.compact_guard = 0;
                PD_TIMED(kc, 1.0 * m + 32.0 * m_next, launch_compact(a, s));
            }
            off += n;
            n = n_next;
            m = m_next;
            ++j;
        }
        // Chain keys are flat ids above level 0.  The levels from here on
        // (persistent kernel, LDS tail) hold fewer than 2(n + B) + 2 vertices
        // in all: a level has at most (m + B) / 2 leaf edges, one vertex each
        // above it.  So the keys lie below this bound, usually far below the
        // capacity-based one, and the chain sort may need fewer or narrower
        // digits.
        const int64_t bound = std::max<int64_t>(off - N, 0) + 2 * (n + B) + 66;
        if (bound < L.flat_cap - N) chain = chain_digits(bound, tune.chain_digit_bits);
    } else {
        // Sync-free: every level that could exceed the LDS tail is launched with
        // capacity-sized grids; levels that turn out small or empty return at
        // once.  Nothing is read back until the end, so the whole call can be
        // captured in a graph.
        for (int j = 0; j < L.Lmax && !tail_level(L.capE[j], L.capV[j], kTailE, kTailV); ++j) {
            const bool l0 = j == 0;
            LevelArgs a = level_args(j);
            const double mj = (double)L.capE[j], nj = (double)L.capV[j];
            PD_TIMED(l0 ? PK_MIN_INC : PK_MIN_INC_N, (l0 ? 20.0 : 12.0) * mj + 16.0 * nj,
                     launch_min_incident(l0, a, s));
            if (L.capE[j] <= persist_max) {
                PD_TIMED(PK_LEVELS, 60.0 * mj, persistent_from(j));
                break;
            }
            PD_TIMED(l0 ? PK_OWN : PK_OWN_N, (l0 ? 29.0 : 25.0) * nj, launch_own(l0, a, s));
            PD_TIMED(l0 ? PK_CLASSIFY : PK_CLASSIFY_N, 3.0 * mj, launch_classify(a, s));
            for (int round = 0; round < kSyncFreeJumpRounds; ++round) {
                a.round = round;
                a.jump_steps = round + 1 < kSyncFreeJumpRounds ? jump_steps : (int)std::max<int64_t>(L.capV[j], 16);
                PD_TIMED(l0 ? PK_JUMP : PK_JUMP_N, round == 0 ? 18.0 * nj : 0.0, launch_jump(a, s));
                ++st.jump_launches;
            }
            // sizes are capacities here; about a third of a level's edges are alpha
            PD_TIMED(l0 ? PK_COMPACT : PK_COMPACT_N, (1.0 + 32.0 / 3.0) * mj, launch_compact(a, s));
        }
    }

    // ---- 3. remaining levels in LDS -------------------------------------------------
    {
        TailArgs t{};
        t.EA = EA;
        t.EB = EB;
        t.EA_r = EA_r;
        t.EB_r = EB_r;
        t.in_u = u;
        t.in_v = v;
        t.rank = rank;
        t.flat_cap = L.flat_cap;
        t.vinfo_all = vinfo_all;
        t.svflat = svflat;
        t.perm = perm;
        t.vertex_parent = vertex_parent;
        t.forest = forest;
        t.ctrl = ctrl;
        PD_TIMED(PK_TAIL, 16.0 * kTailE, launch_tail(t, s));
    }

    // ---- 4. expansion -----------------------------------------------------------------
    {
        WalkArgs wa{};
        wa.m = M;
        wa.n0 = N;
        wa.flat_cap = L.flat_cap;
        wa.svflat = svflat;
        wa.vinfo_all = vinfo_all;
        for (int p = 0; p < 4; ++p) wa.bits[p] = chain.bits[p];
        wa.ckey = K[0];
        wa.hist_row = 4;
        wa.passes = chain.passes;
        wa.lb_zero = LB[0];
        const int64_t lbw_c = sort_tiles(M, L.sort_cfg) << chain.widest();
        wa.lb_zero_words = lbw_c;
        wa.ctrl = ctrl;
        PD_TIMED(PK_WALK_HIST, 8.0 * M, launch_walk_hist(wa, s));   // lookups added once counted
        const uint32_t* kin = K[0];
        const int32_t* vin = perm;
        st.chain_passes = chain.passes;
        for (int p = 0, shift = 0; p < chain.passes; shift += chain.bits[p], ++p) {
            SortPassArgs a{};
            a.n = M;
            a.cfg = L.sort_cfg;
            a.bits = chain.bits[p];
            a.shift = shift;
            a.pass = 4 + p;
            a.keys_in = kin;
            a.vals_in = vin;
            a.keys_out = K[(p + 1) & 1];
            a.vals_out = V[(p + 1) & 1];
            a.lb = LB[p & 1];
            a.lb_zero = LB[(p + 1) & 1];
            a.lb_zero_words = lbw_c;
            a.ctrl = ctrl;
            PD_TIMED(PK_SORT_C_PASS, 16.0 * M, launch_sort_pass(SRC_KEYS, DST_KEYS, a, s));
            kin = K[(p + 1) & 1];
            vin = V[(p + 1) & 1];
        }
        StitchArgs sa{};
        sa.m = M;
        sa.n0 = N;
        sa.flat_cap = L.flat_cap;
        sa.skey = kin;
        sa.sid = vin;
        sa.vinfo_all = vinfo_all;
        sa.perm = perm;
        sa.edge_parent = edge_parent;
        sa.forest = forest;
        PD_TIMED(PK_STITCH, 12.0 * M, launch_stitch(sa, s));
    }
    return PANDORA_OK;
}

// Waits for the enqueued call, reads its control block back and checks it.
int finish(const Scratch& sc, const Layout& L, int32_t B, hipStream_t s, Stats& st) {
    Control* ctrl = at<Control>(sc.dev, L.ctrl);
    Control* hctrl = static_cast<Control*>(sc.host);
    const int rc = read_ctrl(ctrl, hctrl, s, kCtrlLevelsReadback);
    if (rc != PANDORA_OK) return rc;
    if (hctrl->err) return status_from_err(hctrl->err);
    if ((int64_t)hctrl->isolated != B) return PANDORA_ERR_NOT_A_TREE;
    int entry = 0;
    while (entry + 1 < kMaxLevels && !tail_level(hctrl->lv[entry].m, hctrl->lv[entry].n, kTailE, kTailV)) {
        st.sum_edges += hctrl->lv[entry].m;
        ++entry;
    }
    st.tail_entry_edges = hctrl->lv[entry].m;
    st.sum_edges += hctrl->lv[entry].m;
    st.tail_levels = hctrl->tail_levels;
    st.levels = entry + hctrl->tail_levels;
    // The walk looks up a record for every edge but the leaf edges, one per
    // vertex above level 0 (those of the levels up to the tail's entry are
    // known here; the tail's few further ones are counted as lookups).
    int64_t leaf = 0;
    for (int j = 1; j <= entry; ++j) leaf += hctrl->lv[j].n;
    set_last_bytes(PK_WALK_HIST, 8.0 * (double)L.M + 8.0 * (double)std::max<int64_t>(0, L.M - leaf));
    return PANDORA_OK;
}

// The whole path for a forest described by host offsets voff[0..B].
int run(const int64_t* voff, int32_t B, const int32_t* u, const int32_t* v, const float* w,
        int32_t* edge_parent, int32_t* vertex_parent, hipStream_t s) {
    const int64_t N = voff[B];
    const int64_t M = N - B;
    Stats st;
    if (M == 0) {   // only single-vertex trees: every vertex is a root
        PD_TRY(launch_fill_i32(vertex_parent, N, -1, s));
        PD_TRY(hipStreamSynchronize(s));
        g_last = st;
        return PANDORA_OK;
    }
    int dev = 0;
    PD_TRY(hipGetDevice(&dev));
    Workspace& ws = *workspace_for(dev, s);
    std::lock_guard<std::mutex> lock(ws.mu);
    const pandora_tuning_t tune = current_tuning();
    const Layout L = make_layout(N, B, tune.chain_digit_bits, tune.sort_tile_cfg);
    int rc = ensure(ws, L.total, host_bytes_for(B));
    if (rc != PANDORA_OK) return rc;
    const Scratch sc{ws.dev, ws.host, ws.readback};
    // this call waits for its stream before returning, so the pinned block's
    // staging area is free again by the next call
    int64_t* hv = reinterpret_cast<int64_t*>(static_cast<char*>(ws.host) + sizeof(Control));
    std::memcpy(hv, voff, sizeof(int64_t) * (B + 1));
    rc = enqueue(sc, L, tune, M <= (int64_t)tune.sync_free_max_edges, hv, B, u, v, w, edge_parent,
                 vertex_parent, s, st);
    if (rc != PANDORA_OK) return rc;
    rc = finish(sc, L, B, s, st);
    if (rc == PANDORA_OK) g_last = st;
    return rc;
}

int run_and_drain(const int64_t* voff, int32_t B, const int32_t* u, const int32_t* v, const float* w,
                  int32_t* edge_parent, int32_t* vertex_parent, hipStream_t s) {
    const int rc = run(voff, B, u, v, w, edge_parent, vertex_parent, s);
    if (!t_pending.empty()) {
        (void)hipStreamSynchronize(s);
        drain_profile();
    }
    return rc;
}

// ---- stream-ordered calls -----------------------------------------------------------

int ensure_sticky(Workspace& ws, hipStream_t s) {
    if (ws.sticky) return PANDORA_OK;
    void* p = nullptr;
    if (hipMalloc(&p, kAlign) != hipSuccess) {
        (void)hipGetLastError();
        return PANDORA_ERR_OUT_OF_MEMORY;
    }
    ws.sticky = static_cast<uint32_t*>(p);
    PD_TRY(launch_clear_words(ws.sticky, 1, s));
    return PANDORA_OK;
}

// Copies voff into the next staging slot (waiting, if that slot's previous
// copy has not run yet).
int stage_voff(Workspace& ws, const int64_t* voff, int32_t B, const int64_t** staged, int* slot) {
    const size_t need = sizeof(int64_t) * (B + 1);
    StageSlot& sl = ws.stage[ws.next_stage];
    if (sl.pending) {
        if (hipEventSynchronize(sl.done) != hipSuccess) return PANDORA_ERR_HIP;
        sl.pending = false;
    }
    if (!sl.done && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
        sl.done = nullptr;
        return PANDORA_ERR_HIP;
    }
    if (sl.bytes < need) {
        if (sl.host) (void)hipHostFree(sl.host);
        sl.host = nullptr;
        sl.bytes = 0;
        if (hipHostMalloc(&sl.host, need, hipHostMallocDefault) != hipSuccess) {
            sl.host = nullptr;
            (void)hipGetLastError();
            return PANDORA_ERR_OUT_OF_MEMORY;
        }
        sl.bytes = need;
    }
    std::memcpy(sl.host, voff, need);
    *staged = static_cast<const int64_t*>(sl.host);
    *slot = ws.next_stage;
    ws.next_stage = (ws.next_stage + 1) % kStageSlots;
    return PANDORA_OK;
}

// The whole path enqueued on s with no host round trip (the sync-free level
// loop); input errors land in the stream's sticky status word.
int run_async(const int64_t* voff, int32_t B, const int32_t* u, const int32_t* v, const float* w,
              int32_t* edge_parent, int32_t* vertex_parent, hipStream_t s) {
    const int64_t N = voff[B];
    const int64_t M = N - B;
    int dev = 0;
    PD_TRY(hipGetDevice(&dev));
    Workspace& ws = *workspace_for(dev, s);
    std::lock_guard<std::mutex> lock(ws.mu);
    if (M == 0) {   // only single-vertex trees: every vertex is a root
        PD_TRY(launch_fill_i32(vertex_parent, N, -1, s));
        return PANDORA_OK;
    }
    const pandora_tuning_t tune = current_tuning();
    const Layout L = make_layout(N, B, tune.chain_digit_bits, tune.sort_tile_cfg);
    int rc = ensure(ws, L.total, host_bytes_for(1));
    if (rc == PANDORA_OK) rc = ensure_sticky(ws, s);
    if (rc != PANDORA_OK) return rc;
    const int64_t* staged = nullptr;
    int slot = -1;
    if (B > 1) {
        rc = stage_voff(ws, voff, B, &staged, &slot);
        if (rc != PANDORA_OK) return rc;
    }
    Stats st;
    const Scratch sc{ws.dev, ws.host};
    t_capturing = true;   // no profiler events: nothing would wait for them
    rc = enqueue(sc, L, tune, true, staged, B, u, v, w, edge_parent, vertex_parent, s, st);
    t_capturing = false;
    if (rc == PANDORA_OK && launch_finalize(at<Control>(ws.dev, L.ctrl), B, ws.sticky, s) != hipSuccess)
        rc = PANDORA_ERR_HIP;
    if (slot >= 0 && hipEventRecord(ws.stage[slot].done, s) == hipSuccess) ws.stage[slot].pending = true;
    return rc;
}

// ---- the entry point that allocates nothing --------------------------------------
//
// pandora_dendrogram_noalloc keeps every byte of its scratch in the fixed
// device array `scratch` (file scope, below the namespaces).  Each GPU holds its
// own copy at its own address; host code never passes the array's name to a
// kernel (that is a host-side stand-in), only the address hipGetSymbolAddress
// returns for the current device, fetched once per device.  One lock per
// device covers the whole blocking call, so two calls never share the array
// at the same time.
struct NoAllocDevice {
    std::mutex mu;
    void* ptr = nullptr;   // device address of `scratch` on this GPU
};
constexpr int kNoAllocMaxDevices = 64;
NoAllocDevice g_noalloc[kNoAllocMaxDevices];

int run_noalloc(int64_t N, const int32_t* u, const int32_t* v, const float* w, int32_t* edge_parent,
                int32_t* vertex_parent, hipStream_t s) {
    int dev = 0;
    PD_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices) return PANDORA_ERR_HIP;
    NoAllocDevice& nd = g_noalloc[dev];
    std::lock_guard<std::mutex> lock(nd.mu);
    if (!nd.ptr) {
        nd.ptr = noalloc_symbol_address();
        if (!nd.ptr) return PANDORA_ERR_HIP;
    }
    const int64_t M = N - 1;
    if (M == 0) {
        PD_TRY(launch_fill_i32(vertex_parent, 1, -1, s));
        PD_TRY(hipStreamSynchronize(s));
        g_last = Stats{};
        return PANDORA_OK;
    }
    const pandora_tuning_t tune = current_tuning();
    const Layout L = make_layout(N, 1, tune.chain_digit_bits, tune.sort_tile_cfg);
    if (L.total > PANDORA_NOALLOC_SCRATCH_BYTES) return PANDORA_ERR_OUT_OF_MEMORY;
    // The control block is read back into this host copy (plain pageable
    // memory); the level loop is the same as pandora_dendrogram's.
    static thread_local Control hctrl;
    const Scratch sc{nd.ptr, &hctrl};
    Stats st;
    struct NoEvents {   // no profiler events: creating them may allocate
        NoEvents() { t_capturing = true; }
        ~NoEvents() { t_capturing = false; }
    } no_events;
    int rc = enqueue(sc, L, tune, M <= (int64_t)tune.sync_free_max_edges, nullptr, 1, u, v, w, edge_parent,
                     vertex_parent, s, st);
    if (rc == PANDORA_OK) rc = finish(sc, L, 1, s, st);
    else (void)hipStreamSynchronize(s);   // nothing may still use the array when the lock drops
    if (rc == PANDORA_OK) g_last = st;
    return rc;
}

// ---- HDBSCAN* flat clusters ------------------------------------------------------

struct FlatLayout {
    size_t ext, size, bigcnt, bigmax, T, cpar, stab, acc, cidx, clist, cparD, heavy, up0, up1, dist0, dist1, plen,
        poff, posof, lay, s_lay, b_lay, pending, ready, sel, jp0, jp1, tp0, tp1, minv, cnum, lb0, lb1, scan_ctr,
        keys, pos, count, counters;
    int64_t lb_words = 0;
    size_t total = 0;
};

// Born clusters come in sibling pairs of >= mcs vertices each, so there are
// at most 2n / mcs of them.
FlatLayout make_flat_layout(int64_t N, int32_t mcs) {
    const int64_t M = N - 1;
    const int64_t K = std::min<int64_t>(M, 2 * (N / std::max<int32_t>(mcs, 2)) + 2), K1 = K + 1;
    const int64_t tiles = (std::max(N, M) + 4 * kFcBlock - 1) / (4 * kFcBlock) + 1;
    FlatLayout F;
    size_t c = 0;
    F.ext = take(c, 4 * M);
    F.size = take(c, 4 * M);
    F.bigcnt = take(c, 4 * M);
    F.bigmax = take(c, 4 * M);
    F.T = take(c, 4 * M);
    F.cpar = take(c, 4 * M);
    F.stab = take(c, 8 * M);
    F.acc = take(c, 8 * kAccChunks * K);
    F.cidx = take(c, 4 * M);
    F.clist = take(c, 4 * K);
    F.cparD = take(c, 4 * K);
    F.heavy = take(c, 8 * K);
    F.up0 = take(c, 4 * K);
    F.up1 = take(c, 4 * K);
    F.dist0 = take(c, 4 * K);
    F.dist1 = take(c, 4 * K);
    F.plen = take(c, 4 * K);
    F.poff = take(c, 4 * K);
    F.posof = take(c, 4 * K);
    F.lay = take(c, 4 * K);
    F.s_lay = take(c, 8 * K);
    F.b_lay = take(c, 8 * K);
    F.pending = take(c, 4 * K);
    F.ready = take(c, 4 * K);
    F.sel = take(c, K1);
    F.jp0 = take(c, 4 * K1);
    F.jp1 = take(c, 4 * K1);
    F.tp0 = take(c, 4 * K1);
    F.tp1 = take(c, 4 * K1);
    F.minv = take(c, 4 * K);
    F.cnum = take(c, 4 * K);
    F.lb_words = tiles;
    F.lb0 = take(c, 8 * tiles);
    F.lb1 = take(c, 8 * tiles);
    F.scan_ctr = take(c, 8);
    F.keys = take(c, 8 * (kMaxLevels + 2));
    F.pos = take(c, 8 * (kMaxLevels + 2));
    F.count = take(c, 16);
    F.counters = take(c, 16);
    F.total = c;
    return F;
}

int rounds_for(int64_t k) {   // pointer-jumping rounds that cover a depth of k
    int r = 1;
    while ((int64_t(1) << (r - 1)) <= k) ++r;
    return r;
}

// The dendrogram of one tree, then its flat clusters from the chains the
// expansion left sorted in the workspace.  Synchronous.
int run_flat(int64_t n, const int32_t* u, const int32_t* v, const float* w, int32_t mcs, int32_t* edge_parent,
             int32_t* vertex_parent, int32_t* labels, double* stability, int64_t* num_clusters, hipStream_t s) {
    const int64_t N = n, M = n - 1;
    if (M == 0) {
        PD_TRY(launch_fill_i32(vertex_parent, 1, -1, s));
        PD_TRY(launch_fill_i32(labels, 1, -1, s));
        PD_TRY(hipStreamSynchronize(s));
        if (num_clusters) *num_clusters = 0;
        g_last = Stats{};
        return PANDORA_OK;
    }
    int dev = 0;
    PD_TRY(hipGetDevice(&dev));
    Workspace& ws = *workspace_for(dev, s);
    std::lock_guard<std::mutex> lock(ws.mu);
    const pandora_tuning_t tune = current_tuning();
    const Layout L = make_layout(N, 1, tune.chain_digit_bits, tune.sort_tile_cfg);
    const FlatLayout FL = make_flat_layout(N, mcs);
    int rc = ensure(ws, L.total + FL.total, host_bytes_for(1));
    if (rc != PANDORA_OK) return rc;
    const Scratch sc{ws.dev, ws.host, ws.readback};
    int64_t* hv = reinterpret_cast<int64_t*>(static_cast<char*>(ws.host) + sizeof(Control));
    hv[0] = 0;
    hv[1] = N;
    Stats st;
    rc = enqueue(sc, L, tune, M <= (int64_t)tune.sync_free_max_edges, hv, 1, u, v, w, edge_parent, vertex_parent,
                 s, st);
    if (rc != PANDORA_OK) return rc;
    rc = finish(sc, L, 1, s, st);
    if (rc != PANDORA_OK) return rc;
    g_last = st;

    // Levels 1..J hold chain keys; J is the last (edgeless) level.
    const Control* hctrl = static_cast<const Control*>(sc.host);
    const int J = (int)st.levels;
    if (J < 1 || J + 1 >= kMaxLevels) return PANDORA_ERR_HIP;
    std::vector<int64_t> keys(J, 0), pos(J + 1, M);
    for (int j = 1; j <= J; ++j) keys[j - 1] = hctrl->lv[j].off - N;

    char* fb = static_cast<char*>(ws.dev) + L.total;
    FlatArgs a{};
    a.n = N;
    a.m = M;
    a.mcs = mcs;
    a.skey = at<uint32_t>(ws.dev, (st.chain_passes & 1) ? L.K1 : L.K0);
    a.sid = at<int32_t>(ws.dev, (st.chain_passes & 1) ? L.V1 : L.V0);
    a.ep = edge_parent;
    a.vp = vertex_parent;
    a.w = w;
    a.ext = at<int32_t>(fb, FL.ext);
    a.size = at<int32_t>(fb, FL.size);
    a.bigcnt = at<uint32_t>(fb, FL.bigcnt);
    a.bigmax = at<int32_t>(fb, FL.bigmax);
    a.T = at<int32_t>(fb, FL.T);
    a.cpar = at<int32_t>(fb, FL.cpar);
    a.stab = at<double>(fb, FL.stab);
    a.acc = at<unsigned long long>(fb, FL.acc);
    a.K = std::min<int64_t>(M, 2 * (N / std::max<int32_t>(mcs, 2)) + 2);   // bound until counted
    a.cidx = at<int32_t>(fb, FL.cidx);
    a.clist = at<int32_t>(fb, FL.clist);
    a.cparD = at<int32_t>(fb, FL.cparD);
    a.heavy = at<uint64_t>(fb, FL.heavy);
    a.up[0] = at<int32_t>(fb, FL.up0);
    a.up[1] = at<int32_t>(fb, FL.up1);
    a.dist[0] = at<int32_t>(fb, FL.dist0);
    a.dist[1] = at<int32_t>(fb, FL.dist1);
    a.plen = at<int32_t>(fb, FL.plen);
    a.poff = at<int32_t>(fb, FL.poff);
    a.posof = at<int32_t>(fb, FL.posof);
    a.lay = at<int32_t>(fb, FL.lay);
    a.s_lay = at<double>(fb, FL.s_lay);
    a.b_lay = at<double>(fb, FL.b_lay);
    a.pending = at<int32_t>(fb, FL.pending);
    a.ready = at<int32_t>(fb, FL.ready);
    a.sel = at<uint8_t>(fb, FL.sel);
    a.jp[0] = at<int32_t>(fb, FL.jp0);
    a.jp[1] = at<int32_t>(fb, FL.jp1);
    a.tp[0] = at<int32_t>(fb, FL.tp0);
    a.tp[1] = at<int32_t>(fb, FL.tp1);
    a.minv = at<int32_t>(fb, FL.minv);
    a.cnum = at<int32_t>(fb, FL.cnum);
    a.labels = labels;
    a.stab_out = stability;
    a.count = at<int64_t>(fb, FL.count);
    a.counters = at<uint32_t>(fb, FL.counters);
    a.lb[0] = at<uint64_t>(fb, FL.lb0);
    a.lb[1] = at<uint64_t>(fb, FL.lb1);
    a.lb_words = FL.lb_words;
    a.scan_ctr = at<uint32_t>(fb, FL.scan_ctr);
    int scan_seq = 0;
    a.scan_seq = &scan_seq;

    int64_t* dkeys = at<int64_t>(fb, FL.keys);
    int64_t* dpos = at<int64_t>(fb, FL.pos);
    PD_TRY(hipMemcpyAsync(dkeys, keys.data(), sizeof(int64_t) * J, hipMemcpyHostToDevice, s));
    PD_TRY(launch_fc_bounds(a.skey, M, dkeys, dpos, J, s));
    PD_TRY(hipMemcpyAsync(pos.data(), dpos, sizeof(int64_t) * J, hipMemcpyDeviceToHost, s));
    PD_TRY(hipStreamSynchronize(s));
    for (int j = 0; j <= J; ++j)
        if (pos[j] < 0 || pos[j] > M || (j > 0 && pos[j] < pos[j - 1])) return PANDORA_ERR_HIP;

    // Algorithmic bytes: every array element read or written once (gathers
    // count their element size).  pos[j-1] .. pos[j] holds the runs of level j.
    const double Md = (double)M, Nd = (double)N;
    PD_TIMED(PK_FC_PREPARE, 16.0 * Md + 8.0 * Nd + 4.0 * Md, launch_fc_prepare(a, s));
    for (int j = 1; j <= J; ++j)
        PD_TIMED(PK_FC_SIZES, 20.0 * (double)(pos[j] - pos[j - 1]), launch_fc_sizes(a, pos[j - 1], pos[j], s));
    for (int j = J; j >= 1; --j)
        PD_TIMED(PK_FC_CLUSTERS, 24.0 * (double)(pos[j] - pos[j - 1]),
                 launch_fc_clusters(a, pos[j - 1], pos[j], s));
    PD_TIMED(PK_FC_STAB, 24.0 * Md, launch_fc_stab(a, s));
    uint32_t hc[4] = {0, 0, 0, 0};
    int64_t hk[2] = {0, 0};
    PD_TRY(hipMemcpyAsync(hc, a.counters, sizeof(hc), hipMemcpyDeviceToHost, s));
    PD_TRY(hipMemcpyAsync(hk, a.count, sizeof(hk), hipMemcpyDeviceToHost, s));
    PD_TRY(hipStreamSynchronize(s));
    if (hc[1] & 1u) return PANDORA_ERR_INVALID_ARG;      // a weight <= 0
    if (hc[1]) return PANDORA_ERR_HIP;
    const int64_t K = hk[0];
    if (K != (int64_t)hc[0] || K > (int64_t)std::min<int64_t>(M, 2 * (N / mcs) + 2)) return PANDORA_ERR_HIP;
    if (K == 0) {                                         // no true split: every vertex is noise
        PD_TRY(launch_fill_i32(labels, N, -1, s));
        PD_TRY(hipStreamSynchronize(s));
        if (num_clusters) *num_clusters = 0;
        return PANDORA_OK;
    }
    a.K = K;
    const int rounds = rounds_for(K);
    const double Kd = (double)K;
    PD_TIMED(PK_FC_SELECT, 40.0 * Kd + 16.0 * Kd * rounds, launch_fc_tree(a, rounds, s));
    PD_TRY(hipMemcpyAsync(hc, a.counters, sizeof(hc), hipMemcpyDeviceToHost, s));
    PD_TRY(hipStreamSynchronize(s));
    if (hc[1]) return PANDORA_ERR_HIP;
    const uint32_t heads = hc[3];
    for (int round = 0;; ++round) {
        if (round > 64) return PANDORA_ERR_HIP;           // light depth is below log2 n
        PD_TIMED(PK_FC_SELECT, 8.0 * Kd, launch_fc_eval(a, round, s));
        PD_TRY(hipMemcpyAsync(hc, a.counters, sizeof(hc), hipMemcpyDeviceToHost, s));
        PD_TRY(hipStreamSynchronize(s));
        if (hc[2] >= heads) break;
    }
    PD_TIMED(PK_FC_LABEL, 24.0 * Nd + 16.0 * Kd * rounds, launch_fc_label(a, rounds, s));
    PD_TRY(hipMemcpyAsync(hc, a.counters, sizeof(hc), hipMemcpyDeviceToHost, s));
    PD_TRY(hipMemcpyAsync(hk, a.count, sizeof(hk), hipMemcpyDeviceToHost, s));
    PD_TRY(hipStreamSynchronize(s));
    if (hc[1]) return PANDORA_ERR_HIP;
    if (num_clusters) *num_clusters = hk[1];
    return PANDORA_OK;
}

// ---- mutual-reachability MST of a point cloud -------------------------------------

struct EmstLayout {
    size_t core2, comp, comp2, best_w, best_j, active, cmin_w, cmin_e, par0, par1, ew, ea, eb, counters, pairs, bbox,
        sctrl, skey[2], sval[2], slb[2], roots[2],
        cellof, cstart, cfill, sorted, slotof, spts, partial, fallback, scan_agg;
    int64_t len = 0;        // edge-list length (n - 1, at least 1)
    int64_t slb_words = 0;  // look-back words of one radix pass
    int64_t max_cells = 0;  // grid cells allowed
    size_t total = 0;
};

constexpr int64_t kEmstGridMin = 2048;
constexpr size_t kPairsHostAt = 256;     // pinned readback of the pair counts, after the counters   // clouds at least this large use the grid

EmstLayout make_emst_layout(int64_t n) {
    EmstLayout E;
    E.len = std::max<int64_t>(n - 1, 1);
    E.slb_words = sort_tiles(E.len, kDefaultSortCfg) << 8;
    E.max_cells = n >= kEmstGridMin ? 4 * n + 16 : 0;
    const bool grid = E.max_cells > 0;
    size_t c = 0;
    E.core2 = take(c, 8 * n);
    E.comp = take(c, 4 * n);
    E.comp2 = take(c, 4 * n);
    E.best_w = take(c, 8 * n);
    E.best_j = take(c, 4 * n);
    E.active = take(c, 4 * n);
    E.cmin_w = take(c, 8 * n);
    E.cmin_e = take(c, 8 * n);
    E.par0 = take(c, 4 * n);
    E.par1 = take(c, 4 * n);
    E.ew = take(c, 8 * E.len);
    E.ea = take(c, 4 * E.len);
    E.eb = take(c, 4 * E.len);
    E.counters = take(c, 32);
    E.pairs = take(c, 8 * kEmstPairSlots);
    E.roots[0] = take(c, 4 * n);
    E.roots[1] = take(c, 4 * n);
    E.sctrl = take(c, sizeof(Control));
    for (int k = 0; k < 2; ++k) {
        E.skey[k] = take(c, 4 * E.len);
        E.sval[k] = take(c, 4 * E.len);
        E.slb[k] = take(c, 8 * E.slb_words);
    }
    E.bbox = take(c, 8 * kEmstMaxDim);
    E.cellof = take(c, grid ? 4 * n : 0);
    E.cstart = take(c, grid ? 4 * (E.max_cells + 1) : 0);
    E.cfill = take(c, grid ? 4 * E.max_cells : 0);
    E.sorted = take(c, grid ? 4 * n : 0);
    E.spts = take(c, grid ? 4 * kEmstMaxDim * n : 0);
    E.slotof = take(c, grid ? 4 * n : 0);
    E.partial = take(c, grid ? n : 0);
    E.fallback = take(c, grid ? 4 * n : 0);
    E.scan_agg = take(c, grid ? 8 * ((E.max_cells + 4095) / 4096 + 1) : 0);
    E.total = c;
    return E;
}

float from_order_bits(uint32_t b) {
    const uint32_t f = (b & 0x80000000u) ? (b & 0x7fffffffu) : ~b;
    float x;
    std::memcpy(&x, &f, 4);
    return x;
}

// Grid over the bounding box: about one point per cell, at most max_cells.
// False when every point coincides (no extent to divide).
bool plan_grid(EmstArgs& a, const uint32_t* bbox, int64_t max_cells) {
    double lo[kEmstMaxDim], ext[kEmstMaxDim], mag = 0.0, vol = 1.0;
    int live = 0;
    for (int k = 0; k < a.dim; ++k) {
        lo[k] = (double)from_order_bits(bbox[2 * k]);
        const double hi = (double)from_order_bits(~bbox[2 * k + 1]);
        ext[k] = hi - lo[k];
        mag = std::max(mag, std::max(std::fabs(lo[k]), std::fabs(hi)));
        if (ext[k] > 0.0) {
            vol *= ext[k];
            ++live;
        }
    }
    if (live == 0) return false;
    // about one point per cell: the ring walks are bound by their dependent
    // loads, and of 0.35 to 8 points per cell, one was fastest on 10^7
    // uniform points in 3D (sparser grids send more points past the ring
    // cap to full sweeps)
    double h = std::pow(vol / std::max(1.0, (double)a.n), 1.0 / live);
    for (int attempt = 0; attempt < 64; ++attempt) {
        int64_t cells = 1;
        bool fits = true;
        for (int k = 0; k < a.dim; ++k) {
            const double g = ext[k] > 0.0 ? std::floor(ext[k] / h) + 1.0 : 1.0;
            if (g > (double)max_cells) fits = false;
            a.gdim[k] = fits ? (int32_t)g : 1;
            cells = fits ? cells * a.gdim[k] : cells;
            if (cells > max_cells) fits = false;
        }
        if (fits) {
            a.ncells = cells;
            break;
        }
        h *= 1.25;
        if (attempt == 63) return false;
    }
    int64_t stride = 1;
    for (int k = 0; k < kEmstMaxDim; ++k) {
        a.gmin[k] = k < a.dim ? lo[k] : 0.0;
        if (k >= a.dim) a.gdim[k] = 1;
        a.gstride[k] = stride;
        stride *= a.gdim[k];
    }
    a.h = h;
    a.inv_h = 1.0 / h;
    // a rounded floor misplaces a point across a boundary only within a few
    // rounding units of the coordinates' magnitude
    a.gslack = 16.0 * (mag + h) * std::ldexp(1.0, -52);
    return true;
}

// Synchronous: Borůvka rounds until one component, then the sorted tree.
int run_emst(int64_t n, int32_t dim, const float* points, int32_t min_pts, int32_t* u, int32_t* v, double* w64,
             float* w32, hipStream_t s) {
    if (n == 1) return PANDORA_OK;
    int dev = 0;
    PD_TRY(hipGetDevice(&dev));
    Workspace& ws = *workspace_for(dev, s);
    std::lock_guard<std::mutex> lock(ws.mu);
    const EmstLayout E = make_emst_layout(n);
    int rc = ensure(ws, E.total, std::max<size_t>(host_bytes_for(1), kPairsHostAt + 8 * kEmstPairSlots));
    if (rc != PANDORA_OK) return rc;
    void* d = ws.dev;
    EmstArgs a{};
    a.n = n;
    a.dim = dim;
    a.min_pts = min_pts;
    a.pts = points;
    a.core2 = at<double>(d, E.core2);
    a.comp = at<int32_t>(d, E.comp);
    a.comp2 = at<int32_t>(d, E.comp2);
    a.best_w = at<double>(d, E.best_w);
    a.best_j = at<int32_t>(d, E.best_j);
    a.active = at<int32_t>(d, E.active);
    a.cmin_w = at<uint64_t>(d, E.cmin_w);
    a.cmin_e = at<uint64_t>(d, E.cmin_e);
    a.parent[0] = at<int32_t>(d, E.par0);
    a.parent[1] = at<int32_t>(d, E.par1);
    a.ew = at<uint64_t>(d, E.ew);
    a.ea = at<int32_t>(d, E.ea);
    a.eb = at<int32_t>(d, E.eb);
    a.u = u;
    a.v = v;
    a.w64 = w64;
    a.w32 = w32;
    a.counters = at<uint32_t>(d, E.counters);
    a.bbox = at<uint32_t>(d, E.bbox);
    uint32_t* hc = static_cast<uint32_t*>(ws.host);       // pinned readback of the counters
    auto read_counters = [&]() -> int {
        PD_TRY(hipMemcpyAsync(hc, a.counters, 32, hipMemcpyDeviceToHost, s));
        PD_TRY(hipStreamSynchronize(s));
        return PANDORA_OK;
    };
    PD_TRY(launch_clear_words(a.counters, 8, s));

    // The searches are dense fp64 work: their "bytes" in the profiler are
    // fp64 operations, 3 per coordinate and 2 more per point pair examined.
    // The sweeps examine every pair; the grid searches count theirs on the
    // device while the profiler watches them.
    const double ops_per_pair = 3.0 * dim + 2.0;
    const double pair_ops = (double)n * (double)n * ops_per_pair;
    a.pairs = at<uint64_t>(d, E.pairs);
    a.count_pairs = (profiling(PK_EM_CORE) || profiling(PK_EM_SEARCH)) ? 1 : 0;
    auto counted_pairs = [&](int kind) -> int {
        if (!a.count_pairs) return PANDORA_OK;
        uint64_t* hp = reinterpret_cast<uint64_t*>(static_cast<char*>(ws.host) + kPairsHostAt);
        PD_TRY(hipMemcpyAsync(hp, a.pairs, 8 * kEmstPairSlots, hipMemcpyDeviceToHost, s));
        PD_TRY(hipStreamSynchronize(s));
        double total = 0.0;
        for (int k = 0; k < kEmstPairSlots; ++k) total += (double)hp[k];
        profile_add(kind, total * ops_per_pair);
        PD_TRY(launch_clear_words(reinterpret_cast<uint32_t*>(a.pairs), 2 * kEmstPairSlots, s));
        return PANDORA_OK;
    };
    if (a.count_pairs) PD_TRY(launch_clear_words(reinterpret_cast<uint32_t*>(a.pairs), 2 * kEmstPairSlots, s));
    if (E.max_cells > 0) {
        PD_TRY(launch_fill_i32(reinterpret_cast<int32_t*>(a.bbox), 2 * kEmstMaxDim, -1, s));
        PD_TRY(launch_em_bbox(a, s));
        PD_TRY(hipMemcpyAsync(hc, a.bbox, 8 * kEmstMaxDim, hipMemcpyDeviceToHost, s));
        PD_TRY(hipStreamSynchronize(s));
        uint32_t bb[2 * kEmstMaxDim];
        std::memcpy(bb, hc, sizeof(bb));
        a.use_grid = plan_grid(a, bb, E.max_cells) ? 1 : 0;
    }
    if (a.use_grid) {
        a.cellof = at<int32_t>(d, E.cellof);
        a.cstart = at<int32_t>(d, E.cstart);
        a.cfill = at<int32_t>(d, E.cfill);
        a.sorted = at<int32_t>(d, E.sorted);
        a.spts = at<float>(d, E.spts);
        a.slotof = at<int32_t>(d, E.slotof);
        a.partial = at<uint8_t>(d, E.partial);
        a.fallback = at<int32_t>(d, E.fallback);
        a.scan_agg = at<uint64_t>(d, E.scan_agg);
        PD_TRY(launch_clear_words(reinterpret_cast<uint32_t*>(a.cfill), a.ncells, s));
        PD_TRY(launch_em_grid(a, s));
        PD_TIMED(PK_EM_CORE, 0.0, launch_em_core_grid(a, s));
        int rc2 = read_counters();
        if (rc2 != PANDORA_OK) return rc2;
        if (hc[2]) return (hc[2] & 1u) ? PANDORA_ERR_INVALID_ARG : PANDORA_ERR_HIP;
        rc2 = counted_pairs(PK_EM_CORE);
        if (rc2 != PANDORA_OK) return rc2;
        PD_TIMED(PK_EM_CORE, (double)hc[4] * pair_ops / (double)n, launch_em_core(a, a.fallback, hc[4], s));
    } else {
        PD_TIMED(PK_EM_CORE, pair_ops, launch_em_core(a, nullptr, 0, s));
    }
    int64_t comps = n;
    // component roots: every point in the first round, then the list the
    // relabelling appends (two buffers in turn)
    int32_t* RL[2] = {at<int32_t>(d, E.roots[0]), at<int32_t>(d, E.roots[1])};
    int rcur = -1;
    a.roots = nullptr;
    a.nroots = n;
    for (int round = 0; comps > 1; ++round) {
        if (round > 64) return PANDORA_ERR_HIP;           // every round at least halves the components
        PD_TRY(launch_clear_words(a.counters + 3, 2, s));
        PD_TRY(launch_em_active(a, s));
        int rc2 = read_counters();
        if (rc2 != PANDORA_OK) return rc2;
        if (hc[2]) return (hc[2] & 1u) ? PANDORA_ERR_INVALID_ARG : PANDORA_ERR_HIP;
        const int64_t active = hc[3];
        if (active > n) return PANDORA_ERR_HIP;
        if (a.use_grid) {
            PD_TIMED(PK_EM_SEARCH, 0.0, launch_em_search_grid(a, active, s));
            rc2 = read_counters();
            if (rc2 != PANDORA_OK) return rc2;
            const int64_t left = hc[4];
            if (left > active) return PANDORA_ERR_HIP;
            rc2 = counted_pairs(PK_EM_SEARCH);
            if (rc2 != PANDORA_OK) return rc2;
            PD_TIMED(PK_EM_SEARCH, (double)left * pair_ops / (double)n, launch_em_search(a, a.fallback, left, s));
        } else {
            PD_TIMED(PK_EM_SEARCH, (double)active * (double)n * (3.0 * dim + 2.0),
                     launch_em_search(a, a.active, active, s));
        }
        PD_TIMED(PK_EM_MERGE, 16.0 * (double)n, launch_em_merge_edges(a, s));
        int src = 0;
        for (int jr = 0;; ++jr) {
            if (jr > 64) return PANDORA_ERR_HIP;
            PD_TRY(launch_clear_words(a.counters + 3, 1, s));
            PD_TIMED(PK_EM_MERGE, 12.0 * (double)comps, launch_em_jump(a, src, s));
            src ^= 1;
            rc2 = read_counters();
            if (rc2 != PANDORA_OK) return rc2;
            if (hc[2]) return PANDORA_ERR_HIP;
            if (hc[3] == 0) break;
        }
        PD_TRY(launch_clear_words(a.counters + 1, 1, s));
        a.roots_next = RL[rcur == 0 ? 1 : 0];
        PD_TIMED(PK_EM_MERGE, 40.0 * (double)n, launch_em_relabel(a, src, s));
        rc2 = read_counters();
        if (rc2 != PANDORA_OK) return rc2;
        if (hc[2]) return PANDORA_ERR_HIP;
        if ((int64_t)hc[1] >= comps) return PANDORA_ERR_HIP;   // no progress: cannot happen
        comps = hc[1];
        rcur = rcur == 0 ? 1 : 0;
        a.roots = RL[rcur];
        a.nroots = comps;
    }
    if ((int64_t)hc[0] != n - 1) return PANDORA_ERR_HIP;

    // The tree in the total order: stable LSD radix sorts of the edge order,
    // one 32-bit key word at a time from the least significant (endpoint
    // ids take 3 digits, being below 2^24; the mrd2 halves 4 each).
    const int64_t m = n - 1;
    Control* sc = at<Control>(d, E.sctrl);
    uint32_t* SK[2] = {at<uint32_t>(d, E.skey[0]), at<uint32_t>(d, E.skey[1])};
    int32_t* SV[2] = {at<int32_t>(d, E.sval[0]), at<int32_t>(d, E.sval[1])};
    uint64_t* SL[2] = {at<uint64_t>(d, E.slb[0]), at<uint64_t>(d, E.slb[1])};
    int kc = 0, vc = 0;
    for (int word = 0; word < 4; ++word) {
        const int passes = word < 2 ? 3 : 4;
        PD_TRY(launch_clear_words(reinterpret_cast<uint32_t*>(sc), sizeof(Control) / 4, s));
        PD_TIMED(PK_EM_SORT, 20.0 * (double)m,
                 launch_em_sort_key(a, word, word == 0 ? nullptr : SV[vc], SK[kc], SV[vc], s));
        SortHistArgs h{};
        h.n = m;
        h.bits = 8;
        h.hist_row = 0;
        h.passes = passes;
        h.keys = SK[kc];
        h.lb_zero = SL[0];
        h.lb_zero_words = E.slb_words;
        h.ctrl = sc;
        PD_TIMED(PK_EM_SORT, 4.0 * (double)m, launch_sort_hist(SRC_KEYS, h, s));
        for (int p = 0; p < passes; ++p) {
            SortPassArgs pa{};
            pa.n = m;
            pa.cfg = kDefaultSortCfg;
            pa.bits = 8;
            pa.shift = 8 * p;
            pa.pass = p;
            pa.keys_in = SK[kc];
            pa.vals_in = SV[vc];
            pa.keys_out = SK[kc ^ 1];
            pa.vals_out = SV[vc ^ 1];
            pa.lb = SL[p & 1];
            pa.lb_zero = SL[(p + 1) & 1];
            pa.lb_zero_words = E.slb_words;
            pa.ctrl = sc;
            PD_TIMED(PK_EM_SORT, 16.0 * (double)m, launch_sort_pass(SRC_KEYS, DST_KEYS, pa, s));
            kc ^= 1;
            vc ^= 1;
        }
        PD_TRY(hipMemcpyAsync(hc, &sc->err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        PD_TRY(hipStreamSynchronize(s));
        if (hc[0]) return PANDORA_ERR_HIP;
    }
    PD_TIMED(PK_EM_SORT, 32.0 * (double)m, launch_em_out(a, SV[vc], s));
    PD_TRY(hipStreamSynchronize(s));
    return PANDORA_OK;
}

}  // namespace
}  // namespace pandora

using namespace pandora;

extern "C" {

int pandora_dendrogram(int64_t n, const int32_t* u, const int32_t* v, const float* w,
                       int32_t* edge_parent, int32_t* vertex_parent, void* hip_stream) {
    if (n < 1 || n > INT32_MAX || !vertex_parent) return PANDORA_ERR_INVALID_ARG;
    if (n > 1 && (!u || !v || !w || !edge_parent)) return PANDORA_ERR_INVALID_ARG;
    if (!ids_fit(n, 1)) return PANDORA_ERR_INVALID_ARG;
    const int64_t voff[2] = {0, n};
    return run_and_drain(voff, 1, u, v, w, edge_parent, vertex_parent, static_cast<hipStream_t>(hip_stream));
}

int pandora_dendrogram_noalloc(int64_t n, const int32_t* u, const int32_t* v, const float* w,
                               int32_t* edge_parent, int32_t* vertex_parent, void* hip_stream) {
    if (n < 1 || n > INT32_MAX || !vertex_parent) return PANDORA_ERR_INVALID_ARG;
    if (n > 1 && (!u || !v || !w || !edge_parent)) return PANDORA_ERR_INVALID_ARG;
    if (!ids_fit(n, 1)) return PANDORA_ERR_INVALID_ARG;
    // the limit does not depend on the tuning
    if (n > 1 && pandora_workspace_bytes(n, 1) > PANDORA_NOALLOC_SCRATCH_BYTES) return PANDORA_ERR_OUT_OF_MEMORY;
    return run_noalloc(n, u, v, w, edge_parent, vertex_parent, static_cast<hipStream_t>(hip_stream));
}

int pandora_dendrogram_batched(int32_t B, const int64_t* voff, const int32_t* u, const int32_t* v,
                               const float* w, int32_t* edge_parent, int32_t* vertex_parent,
                               void* hip_stream) {
    if (B < 1 || !voff || !vertex_parent || voff[0] != 0) return PANDORA_ERR_INVALID_ARG;
    for (int32_t b = 0; b < B; ++b)
        if (voff[b + 1] <= voff[b]) return PANDORA_ERR_INVALID_ARG;
    if (voff[B] > INT32_MAX || !ids_fit(voff[B], B)) return PANDORA_ERR_INVALID_ARG;
    if (voff[B] > B && (!u || !v || !w || !edge_parent)) return PANDORA_ERR_INVALID_ARG;
    return run_and_drain(voff, B, u, v, w, edge_parent, vertex_parent, static_cast<hipStream_t>(hip_stream));
}

int pandora_dendrogram_async(int64_t n, const int32_t* u, const int32_t* v, const float* w,
                             int32_t* edge_parent, int32_t* vertex_parent, void* hip_stream) {
    if (n < 1 || n > INT32_MAX || !vertex_parent) return PANDORA_ERR_INVALID_ARG;
    if (n > 1 && (!u || !v || !w || !edge_parent)) return PANDORA_ERR_INVALID_ARG;
    if (!ids_fit(n, 1)) return PANDORA_ERR_INVALID_ARG;
    const int64_t voff[2] = {0, n};
    return run_async(voff, 1, u, v, w, edge_parent, vertex_parent, static_cast<hipStream_t>(hip_stream));
}

int pandora_dendrogram_batched_async(int32_t B, const int64_t* voff, const int32_t* u, const int32_t* v,
                                     const float* w, int32_t* edge_parent, int32_t* vertex_parent,
                                     void* hip_stream) {
    if (B < 1 || !voff || !vertex_parent || voff[0] != 0) return PANDORA_ERR_INVALID_ARG;
    for (int32_t b = 0; b < B; ++b)
        if (voff[b + 1] <= voff[b]) return PANDORA_ERR_INVALID_ARG;
    if (voff[B] > INT32_MAX || !ids_fit(voff[B], B)) return PANDORA_ERR_INVALID_ARG;
    if (voff[B] > B && (!u || !v || !w || !edge_parent)) return PANDORA_ERR_INVALID_ARG;
    return run_async(voff, B, u, v, w, edge_parent, vertex_parent, static_cast<hipStream_t>(hip_stream));
}

int pandora_stream_status(void* hip_stream) {
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PANDORA_ERR_HIP;
    Workspace& ws = *workspace_for(dev, s);
    std::lock_guard<std::mutex> lock(ws.mu);
    if (hipStreamSynchronize(s) != hipSuccess) return PANDORA_ERR_HIP;
    if (!ws.sticky) return PANDORA_OK;
    uint32_t e = 0;
    if (hipMemcpyAsync(&e, ws.sticky, sizeof(e), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PANDORA_ERR_HIP;
    if (e == 0) return PANDORA_OK;
    if (launch_clear_words(ws.sticky, 1, s) != hipSuccess) return PANDORA_ERR_HIP;
    return status_from_err(e);
}

int pandora_set_workspace(void* hip_stream, void* dev_ptr, size_t bytes) {
    if (dev_ptr && (reinterpret_cast<uintptr_t>(dev_ptr) % kAlign != 0 || bytes == 0))
        return PANDORA_ERR_INVALID_ARG;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PANDORA_ERR_HIP;
    Workspace& ws = *workspace_for(dev, s);
    std::lock_guard<std::mutex> lock(ws.mu);
    // earlier calls on the stream may still use the current buffer
    if (hipStreamSynchronize(s) != hipSuccess) return PANDORA_ERR_HIP;
    if (ws.owned && ws.dev) (void)hipFree(ws.dev);
    ws.dev = dev_ptr;
    ws.bytes = dev_ptr ? bytes : 0;
    ws.owned = dev_ptr == nullptr;
    return PANDORA_OK;
}

int pandora_flat_clusters(int64_t n, const int32_t* u, const int32_t* v, const float* w, int32_t min_cluster_size,
                          int32_t* edge_parent, int32_t* vertex_parent, int32_t* labels, double* stability,
                          int64_t* num_clusters, void* hip_stream) {
    if (n < 1 || n > INT32_MAX || min_cluster_size < 2 || !vertex_parent || !labels) return PANDORA_ERR_INVALID_ARG;
    if (n > 1 && (!u || !v || !w || !edge_parent)) return PANDORA_ERR_INVALID_ARG;
    if (!ids_fit(n, 1)) return PANDORA_ERR_INVALID_ARG;
    const int rc = run_flat(n, u, v, w, min_cluster_size, edge_parent, vertex_parent, labels, stability,
                            num_clusters, static_cast<hipStream_t>(hip_stream));
    if (!t_pending.empty()) {
        (void)hipStreamSynchronize(static_cast<hipStream_t>(hip_stream));
        drain_profile();
    }
    return rc;
}

int pandora_emst(int64_t n, int32_t dim, const float* points, int32_t min_pts, int32_t* u, int32_t* v, double* w64,
                 float* w32, void* hip_stream) {
    if (n < 1 || n > (int64_t(1) << 24) || dim < 1 || dim > kEmstMaxDim || min_pts < 1 ||
        min_pts > kEmstMaxMinPts || min_pts > n || !points)
        return PANDORA_ERR_INVALID_ARG;
    if (n > 1 && (!u || !v || !w32)) return PANDORA_ERR_INVALID_ARG;
    const int rc = run_emst(n, dim, points, min_pts, u, v, w64, w32, static_cast<hipStream_t>(hip_stream));
    if (!t_pending.empty()) {
        (void)hipStreamSynchronize(static_cast<hipStream_t>(hip_stream));
        drain_profile();
    }
    return rc;
}

size_t pandora_flat_clusters_workspace_bytes(int64_t n) {
    if (n < 2 || n > INT32_MAX || !ids_fit(n, 1)) return 0;
    size_t most = 0;
    for (int cfg = 0; cfg < kNumSortCfg; ++cfg)
        for (int bits : {8, 9}) most = std::max(most, make_layout(n, 1, bits, cfg).total);
    return most + make_flat_layout(n, 2).total;
}

size_t pandora_workspace_bytes(int64_t n_total_vertices, int32_t B) {
    if (B < 1 || n_total_vertices < B || n_total_vertices > INT32_MAX) return 0;
    if (n_total_vertices == B || !ids_fit(n_total_vertices, B)) return 0;
    // enough for every tuning: the radix tile and digit width change the size
    // of the look-back buffers
    size_t most = 0;
    for (int cfg = 0; cfg < kNumSortCfg; ++cfg)
        for (int bits : {8, 9}) most = std::max(most, make_layout(n_total_vertices, B, bits, cfg).total);
    return most;
}

int pandora_last_stats(int64_t* out, int cap) {
    const int64_t vals[7] = {g_last.levels, g_last.sum_edges, g_last.jump_launches, g_last.tail_levels,
                             g_last.tail_entry_edges, g_last.sync_free, g_last.persistent};
    if (!out || cap < 0) return -PANDORA_ERR_INVALID_ARG;
    int k = 0;
    for (; k < cap && k < 7; ++k) out[k] = vals[k];
    return k;
}

int pandora_set_tuning(const pandora_tuning_t* t) {
    if (!t || !tuning_valid(t)) return PANDORA_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune = *t;
    return PANDORA_OK;
}

int pandora_set_thread_tuning(const pandora_tuning_t* t) {
    if (!t) {
        t_has_tune = false;
        return PANDORA_OK;
    }
    if (!tuning_valid(t)) return PANDORA_ERR_INVALID_ARG;
    t_tune = *t;
    t_has_tune = true;
    return PANDORA_OK;
}

int pandora_get_tuning(pandora_tuning_t* t) {
    if (!t) return PANDORA_ERR_INVALID_ARG;
    *t = current_tuning();
    return PANDORA_OK;
}

int pandora_profile_enable(uint32_t kind_mask) {
    std::lock_guard<std::mutex> g(g_prof.mu);
    g_prof.mask = kind_mask;
    for (int k = 0; k < PK_COUNT; ++k) {
        g_prof.ms[k] = 0;
        g_prof.bytes[k] = 0;
        g_prof.launches[k] = 0;
    }
    return PK_COUNT;
}

int pandora_profile_read(double* ms, double* bytes, int64_t* launches, int cap) {
    std::lock_guard<std::mutex> g(g_prof.mu);
    int k = 0;
    for (; k < cap && k < PK_COUNT; ++k) {
        if (ms) ms[k] = g_prof.ms[k];
        if (bytes) bytes[k] = g_prof.bytes[k];
        if (launches) launches[k] = g_prof.launches[k];
    }
    return k;
}

const char* pandora_profile_name(int kind) {
    return (kind >= 0 && kind < PK_COUNT) ? kProfNames[kind] : "";
}

struct pandora_graph {
    Layout L;
    int32_t B = 0;
    int64_t M = 0;
    void* dev = nullptr;
    void* host = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void graph_free(pandora_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->dev) (void)hipFree(g->dev);
    if (g->host) (void)hipHostFree(g->host);
    delete g;
}

static int graph_create(int32_t B, const int64_t* voff, const int32_t* u, const int32_t* v,
                        const float* w, int32_t* edge_parent, int32_t* vertex_parent,
                        pandora_graph** out) {
    *out = nullptr;
    const int64_t N = voff[B];
    const int64_t M = N - B;
    pandora_graph* g = new pandora_graph;
    g->B = B;
    g->M = M;
    const pandora_tuning_t tune = current_tuning();
    if (M > 0) {
        g->L = make_layout(N, B, tune.chain_digit_bits, tune.sort_tile_cfg);
        if (hipMalloc(&g->dev, g->L.total) != hipSuccess) {
            (void)hipGetLastError();
            g->dev = nullptr;
            graph_free(g);
            return PANDORA_ERR_OUT_OF_MEMORY;
        }
    }
    if (hipHostMalloc(&g->host, host_bytes_for(B), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        g->host = nullptr;
        graph_free(g);
        return PANDORA_ERR_OUT_OF_MEMORY;
    }
    // Capture on a private stream: the legacy default stream cannot be captured.
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        graph_free(g);
        return PANDORA_ERR_HIP;
    }
    int rc = PANDORA_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = PANDORA_ERR_HIP;
    } else {
        t_capturing = true;
        Stats st;
        if (M == 0) {
            if (launch_fill_i32(vertex_parent, N, -1, cs) != hipSuccess) rc = PANDORA_ERR_HIP;
        } else {
            const Scratch sc{g->dev, g->host};
            int64_t* hv = reinterpret_cast<int64_t*>(static_cast<char*>(g->host) + sizeof(Control));
            std::memcpy(hv, voff, sizeof(int64_t) * (B + 1));
            rc = enqueue(sc, g->L, tune, true, hv, B, u, v, w, edge_parent, vertex_parent, cs, st);
        }
        t_capturing = false;
        if (hipStreamEndCapture(cs, &g->graph) != hipSuccess && rc == PANDORA_OK) rc = PANDORA_ERR_HIP;
    }
    (void)hipStreamDestroy(cs);
    if (rc == PANDORA_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
        rc = PANDORA_ERR_HIP;
    if (rc != PANDORA_OK) {
        (void)hipGetLastError();
        graph_free(g);
        return rc;
    }
    *out = g;
    return PANDORA_OK;
}

int pandora_graph_create(int64_t n, const int32_t* u, const int32_t* v, const float* w,
                         int32_t* edge_parent, int32_t* vertex_parent, pandora_graph_t** out) {
    if (!out) return PANDORA_ERR_INVALID_ARG;
    *out = nullptr;
    if (n < 1 || n > INT32_MAX || !vertex_parent) return PANDORA_ERR_INVALID_ARG;
    if (n > 1 && (!u || !v || !w || !edge_parent)) return PANDORA_ERR_INVALID_ARG;
    if (!ids_fit(n, 1)) return PANDORA_ERR_INVALID_ARG;
    const int64_t voff[2] = {0, n};
    return graph_create(1, voff, u, v, w, edge_parent, vertex_parent, out);
}

int pandora_graph_create_batched(int32_t B, const int64_t* voff, const int32_t* u, const int32_t* v,
                                 const float* w, int32_t* edge_parent, int32_t* vertex_parent,
                                 pandora_graph_t** out) {
    if (!out) return PANDORA_ERR_INVALID_ARG;
    *out = nullptr;
    if (B < 1 || !voff || !vertex_parent || voff[0] != 0) return PANDORA_ERR_INVALID_ARG;
    for (int32_t b = 0; b < B; ++b)
        if (voff[b + 1] <= voff[b]) return PANDORA_ERR_INVALID_ARG;
    if (voff[B] > INT32_MAX || !ids_fit(voff[B], B)) return PANDORA_ERR_INVALID_ARG;
    if (voff[B] > B && (!u || !v || !w || !edge_parent)) return PANDORA_ERR_INVALID_ARG;
    return graph_create(B, voff, u, v, w, edge_parent, vertex_parent, out);
}

int pandora_graph_launch(pandora_graph_t* g, void* hip_stream) {
    if (!g || !g->exec) return PANDORA_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (hipGraphLaunch(g->exec, s) != hipSuccess) return PANDORA_ERR_HIP;
    if (g->M == 0) return hipStreamSynchronize(s) == hipSuccess ? PANDORA_OK : PANDORA_ERR_HIP;
    Stats st;
    st.sync_free = 1;
    const int rc = finish(Scratch{g->dev, g->host}, g->L, g->B, s, st);
    if (rc == PANDORA_OK) g_last = st;
    return rc;
}

void pandora_graph_destroy(pandora_graph_t* g) { graph_free(g); }

void pandora_release_workspaces(void) {
    std::lock_guard<std::mutex> g(g_mu);
    for (auto& kv : g_ws) {
        Workspace& ws = *kv.second;
        std::lock_guard<std::mutex> l(ws.mu);
        (void)hipStreamSynchronize(ws.stream);
        if (ws.dev && ws.owned) (void)hipFree(ws.dev);
        if (ws.host) (void)hipHostFree(ws.host);
        if (ws.sticky) (void)hipFree(ws.sticky);
        if (ws.readback) (void)hipEventDestroy(ws.readback);
        ws.readback = nullptr;
        for (StageSlot& sl : ws.stage) {
            if (sl.host) (void)hipHostFree(sl.host);
            if (sl.done) (void)hipEventDestroy(sl.done);
            sl = StageSlot{};
        }
        ws.dev = nullptr;
        ws.host = nullptr;
        ws.sticky = nullptr;
        ws.bytes = ws.host_bytes = 0;
    }
    g_ws.clear();
}

const char* pandora_status_string(int status) {
    switch (status) {
        case PANDORA_OK: return "ok";
        case PANDORA_ERR_INVALID_ARG: return "invalid argument";
        case PANDORA_ERR_NOT_A_TREE: return "input is not a tree (cycle or disconnected)";
        case PANDORA_ERR_NAN_WEIGHT: return "NaN edge weight";
        case PANDORA_ERR_OUT_OF_MEMORY: return "out of device memory";
        case PANDORA_ERR_HIP: return "HIP runtime error";
        case PANDORA_ERR_BAD_VERTEX: return "vertex id out of range";
        default: return "unknown status";
    }
}

}  // extern "C"
