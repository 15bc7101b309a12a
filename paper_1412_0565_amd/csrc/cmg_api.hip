// libcmg host driver: the C ABI declared in include/cmg.h.
//
// The host sequences kernel launches on one stream and reads back only the
// sizes it needs to allocate the next level (aggregate count, coarse nnz)
// and the HEC round flag.  All arithmetic of the method runs in the
// kernels of setup.hip and refine.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "cmg.h"
#include "cmg_internal.h"

using namespace cmg;

namespace {

// roctx range around a phase (named in rocprofv3 --marker-trace output);
// a no-op without a tool attached
struct Range {
    explicit Range(const char* fmt, int a = 0) {
        char buf[64];
        std::snprintf(buf, sizeof(buf), fmt, a);
        roctxRangePushA(buf);
    }
    ~Range() { roctxRangePop(); }
};

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

void* default_alloc(size_t bytes, void*, void*) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes == 0 ? 1 : bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void default_free(void* p, void*, void*) { (void)hipFree(p); }

const cmg_allocator kDefaultAllocator = {default_alloc, default_free, nullptr};

struct HostLevel {
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t* rp = nullptr;
    int32_t* col = nullptr;
    double* w64 = nullptr;
    float* w32 = nullptr;
    uint8_t* w8 = nullptr;  // 8-bit copy of the weights (kWU8)
    uint16_t* w16 = nullptr;  // 16-bit copy of the weights (kWU16)
    int32_t* agg = nullptr;
    double g = 0.0, wmax = 0.0;
    int w32exact = 0;
    int wunit = 0;  // every weight is 1 (checked on the input level)
    int wk = kWNative;  // weight storage read by the grid and step kernels
    int64_t maxlen = 0;
    int fp32 = 0, in_block = 0, lanes = 8, grid = 0, variant = 1;
    int stage = 1;  // grid levels: a workgroup's rows may be staged in LDS
    void* buf0 = nullptr;
    void* buf1 = nullptr;
    int32_t* part = nullptr;
    int bwaves = 0, bregs = 0, bslots = 0;  // single-workgroup level: waves, register rows, slots
    int step = 0;              // 1: refined with one launch per PI step
    int kfix = 0;              // fixed schedule: PI steps of this level (0: stopping test)
    int fgrid = 0;             // level 0 in step mode: finishing pass grid
    int32_t* fpart = nullptr;  // ... and its row split
    int fbgrid = 0;            // persistent level: workgroups of its step-mode fallback
    int32_t* fbpart = nullptr; // ... and their row split
    int lmin = 0x7fffffff;     // rows traversal: rows with more entries are long
    int32_t* lrows = nullptr;  // ... their count and the list (nullptr: none)
    int k = 0;
    double margin = 0.0;
    double pi_ms = 0.0;
};

// Lanes per row: about 3 entries per lane (measured best for degree 6
// to 16 meshes and geometric graphs: fewer lanes leave the loads of a row
// serialised, more leave lanes idle).
int pick_lanes(double avg_deg) {
    double t = avg_deg / 3.0;
    int g = 1;
    while (g < t && g < 64) g <<= 1;
    return g;
}

// Lanes per row on a level refined inside one workgroup, where a step is
// one latency chain: G minimises the critical path of the slowest lane
// group, (rows per group - 1) (avg/G + c) + maxlen/G + c, with c = 8 entry
// visits standing for the per-row reduction and bookkeeping (threads = 64
// for the one-wavefront mode of levels up to 256 vertices, else the
// workgroup).  Meshes get 1-2 lanes; levels with hub rows get more.
int pick_lanes_block(int n, double avg_deg, int maxlen, int block_threads) {
    const int threads = n <= 256 ? 64 : block_threads;
    const double c = 8.0;
    int best = 1;
    double best_cost = 0.0;
    for (int g = 1; g <= 64; g <<= 1) {
        const double groups = threads / g;
        const double rows = std::ceil(n / groups);
        const double cost = (rows - 1.0) * (avg_deg / g + c) + (double)maxlen / g + c;
        if (g == 1 || cost < best_cost) {
            best = g;
            best_cost = cost;
        }
    }
    return best;
}

int bitlen(unsigned long long x) {
    int b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

// Register-row layout of a single-workgroup level (kernels of
// kBlockRegsThreads threads): W wavefronts run the steps; layout l gives G
// lanes per row and E entry slots per lane and row; R rows per lane group;
// one wavefront only with G = R = 1; weights exact in FP32.  Rows of up to
// 2 G E entries are allowed: the entries beyond G E go to an LDS list
// after the two vectors, which must hold n (maxlen - G E) of them (or nnz,
// if fewer).  The layout of least modelled step time wins: a cost per wave
// count (barrier and cross-wave sums; none for one wave), the latency of
// R E gathers, their LDS bandwidth (W R E 64 gathers of 8 bytes), and two
// dependent LDS reads per trip over a long row's list (two entries a
// trip).  Fitted to MI355X measurements: 0.41 us per step for 62 rows on
// one wave (E = 8), 0.64 us for 171 rows on 4 waves, 0.92 us for 400 rows
// of 12 to 16 entries on 4 to 8 waves, 1.46 us for 1536 rows on 8 waves
// (R = 4, E = 8), 2.19 us for 262 rows of up to 34 entries on 8 waves
// (G = 4, R = 4, E = 16); with the list, 1.34 us for those rows (G = 2,
// R = 2, E = 16, one trip), 2.49 us for 895 rows of up to 35 entries
// (G = 2, R = 4, E = 16, one trip), 1.86 us for 1536 rows of up to 11
// entries (G = 1, R = 4, E = 8, two trips) and 1.29 us for 511 rows of up
// to 12 (G = 1, R = 2, E = 8, two trips; 1.04 us with E = 16).
struct BlockPlan {
    int waves = 0, lanes = 1, regs = 0, slots = 0, layout = -1;
};

BlockPlan plan_block_regs(const HostLevel& L, int lds_budget) {
    static const double wave_cost[9] = {0, 0.31, 0.45, 0, 0.52, 0, 0, 0, 0.70};
    const double slot_cost = 0.0125, lds_cost = 0.0012, lane_sum_cost = 0.02, list_trip_cost = 0.25;
    BlockPlan best;
    double best_cost = 0.0;
    if (L.n < 1 || L.n > 65536 || !L.w32exact) return best;
    for (int W : {1, 2, 4, 8}) {
        for (int l = 0; l < kRegLayouts; ++l) {
            const int G = kRegLayoutG[l], E = kRegLayoutE[l];
            const int64_t over = std::max<int64_t>(L.maxlen - (int64_t)G * E, 0);
            if (over > (int64_t)G * E) continue;
            if (over > 0) {
                const int64_t list = std::min<int64_t>((int64_t)L.n * over, L.nnz);
                if (16 * (int64_t)L.n + 8 * list > (int64_t)lds_budget) continue;
            }
            const int groups = 64 * W / G;
            const int need = (L.n + groups - 1) / groups;
            const int R = need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : 0;
            if (R == 0) continue;
            if (W == 1 && (G != 1 || R != 1)) continue;
            const int64_t trips = (over + 2 * G - 1) / (2 * G);
            const double cost = wave_cost[W] + R * E * slot_cost + W * R * E * lds_cost +
                                R * (bitlen((unsigned)G) - 1) * lane_sum_cost +
                                (trips > 0 ? lane_sum_cost + trips * list_trip_cost : 0.0);
            if (best.regs == 0 || cost < best_cost) {
                best.waves = W;
                best.lanes = G;
                best.regs = R;
                best.slots = E;
                best.layout = l;
                best_cost = cost;
            }
        }
    }
    return best;
}

}  // namespace

struct cmg_ctx {
    cmg_options opt{};
    hipStream_t stream = nullptr;
    cmg_allocator alloc = kDefaultAllocator;
    std::vector<void*> owned;
    std::vector<HostLevel> lv;
    size_t footprint = 0;
    LevelDev* d_lv = nullptr;
    LevelState* d_st = nullptr;
    GridSync* d_sync = nullptr;
    GridSlot* d_slots = nullptr;
    int nslots = 0;
    GridJob* d_jobs = nullptr;  // [j] refines level j, [J+1] finishes level 0
    std::vector<GridJob> h_jobs;
    CoarseJob* d_cjob = nullptr;
    BlockJob* d_bruns = nullptr;  // single-workgroup levels: runs of levels, coarsest run first
    CoarseJob h_cjob{};
    // The dense coarsest solve depends on the hierarchy alone and nothing
    // else writes its outputs (the coarsest level's vector and state), so it
    // runs once, at the end of setup (true from then on).
    bool coarse_done = false;
    // every input weight an integer below 2^20: Galerkin sums are exact in
    // any order, and runs of a long coarse entry are summed in pieces
    bool int_weights = false;
    bool gal_int32 = false;  // integer weights summing below 2^32 (set on level 0)
    unsigned maxlen0 = 0;  // longest input row if over 64 entries (else 0)
    std::vector<BlockJob> h_bruns;
    std::vector<int> brun_kind;   // kernel of each run (launch_block_jobs kind)
    int top = 0;       // finest-to-coarsest: levels top .. 0 are refined
    // host staging of the results of the last solve
    FinishOut h_fo{};
    std::vector<LevelState> h_st;
    GridSync h_gs{};
    GridSlot* d_bcast = nullptr;
    FinishOut* d_fo = nullptr;
    double* d_A = nullptr;
    double* d_V = nullptr;
    double* d_ev = nullptr;
    int32_t* d_idx = nullptr;
    double* d_fa = nullptr;
    double* d_fb = nullptr;
    double* d_y = nullptr;
    int coarse_dense = 1;
    double clock_khz = 100000.0;  // constant-clock ticks per ms
    int block_lo = -1;  // levels >= block_lo (and < coarsest or the PI coarsest) run in one workgroup
    int collapsed = 0;
    int hec_rounds = 0;
    double setup_ms = 0.0;
    cmg_stats last{};
    std::vector<hipEvent_t> events;
    // levels refined with one launch per step
    StepJob* d_step = nullptr;  // [J+1]
    StepJob* d_step_fb = nullptr;  // [J+1]: step-mode fallback of the persistent levels
    int fallbacks = 0;          // solves re-run one launch per step after a barrier wait was given up
    StepCtl* d_ctl = nullptr;
    double* d_part = nullptr;   // 4 partial sums per workgroup
    int* h_flags = nullptr;     // pinned: done flag after each chunk of steps
    std::vector<hipEvent_t> chunk_ev;
    bool fixed = false;            // fixed smoothing schedule: every launch count known in advance
    bool noalloc = false;          // cmg_fiedler_noalloc: no events, no host-pinned or stream objects
    // several eigenpairs (cmg_fiedler_block): buffers for blk_p columns
    int blk_p = 0;
    std::vector<BlkJob> blk_jobs;  // per level
    BlkJob* d_blk_jobs = nullptr;
    BlkCtl* d_blk_ctl = nullptr;
    BlkOut* d_blk_out = nullptr;
    double* d_blk_x = nullptr;
    hipGraphExec_t gexec = nullptr;  // captured refinement launches (cmg_options.graph)

    // Device memory of the handle (hierarchy, refinement state, job
    // tables) comes from a bump arena over a few large chunks of the
    // caller's allocator, released by cmg_free: a setup makes a handful of
    // allocator calls instead of about a hundred (each a callback into the
    // caller, e.g. Python).  Transient buffers use dalloc_direct.
    std::vector<void*> chunks;
    char* acur = nullptr;
    size_t aleft = 0;
    size_t achunk = (size_t)4 << 20;  // first chunk; set from the input size by setup
    void* dalloc(size_t bytes) {
        bytes = (std::max<size_t>(bytes, 8) + 255) & ~(size_t)255;
        if (bytes > aleft) {
            const size_t cs = std::max(bytes, chunks.empty() ? achunk : std::max<size_t>(achunk / 4, (size_t)1 << 20));
            void* p = alloc.alloc(cs, (void*)stream, alloc.user);
            if (!p) return nullptr;
            chunks.push_back(p);
            acur = (char*)p;
            aleft = cs;
            footprint += cs;
        }
        void* r = acur;
        acur += bytes;
        aleft -= bytes;
        return r;
    }
    void dfree(void*) {}  // arena memory goes back with the handle
    void* dalloc_direct(size_t bytes) {
        void* p = alloc.alloc(bytes == 0 ? 8 : bytes, (void*)stream, alloc.user);
        if (p) owned.push_back(p);
        return p;
    }
    void dfree_direct(void* p) {
        if (!p) return;
        auto it = std::find(owned.begin(), owned.end(), p);
        if (it != owned.end()) owned.erase(it);
        alloc.free(p, (void*)stream, alloc.user);
    }
    ~cmg_ctx() {
        if (stream || true) (void)hipStreamSynchronize(stream);
        for (void* p : owned) alloc.free(p, (void*)stream, alloc.user);
        for (void* p : chunks) alloc.free(p, (void*)stream, alloc.user);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipEvent_t e : chunk_ev) (void)hipEventDestroy(e);
        if (h_flags) (void)hipHostFree(h_flags);
        if (gexec) (void)hipGraphExecDestroy(gexec);
    }
};

namespace {

thread_local char g_last_error[512] = "";

void set_error(const char* what, hipError_t e, int line) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s (line %d): %s", what, line,
                  e == hipSuccess ? "" : hipGetErrorString(e));
}

#define CK(x)                                                                                      \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) {                                                                    \
            set_error(#x, e_, __LINE__);                                                           \
            (void)hipGetLastError();                                                               \
            return CMG_E_DEVICE;                                                                   \
        }                                                                                          \
    } while (0)

#define ALLOC(ptr, type, count)                                                                    \
    do {                                                                                           \
        ptr = (type*)c->dalloc(sizeof(type) * (size_t)(count));                                    \
        if (!ptr) return CMG_E_OOM;                                                                \
    } while (0)

template <typename T>
cmg_status d2h(cmg_ctx* c, T* host, const T* dev, size_t count) {
    CK(hipMemcpyAsync(host, dev, sizeof(T) * count, hipMemcpyDeviceToHost, c->stream));
    CK(hipStreamSynchronize(c->stream));
    return CMG_OK;
}

// Temporary buffers of the setup phase, sized for level 0 and reused.
struct SetupTmp {
    int32_t* h = nullptr;
    unsigned long long* slot = nullptr;
    uint8_t* live = nullptr;
    uint8_t* state = nullptr;
    int32_t* pairseed = nullptr;
    int32_t* rootseed = nullptr;
    int32_t* flags = nullptr;
    int32_t* rank = nullptr;
    long long* scan_tmp = nullptr;
    unsigned long long* k0 = nullptr;
    unsigned long long* k1 = nullptr;
    double* v0 = nullptr;
    double* v1 = nullptr;
    int32_t* heads = nullptr;
    int32_t* idx = nullptr;
    int32_t* sort_counts = nullptr;
    long long* sort_scan = nullptr;
    unsigned long long* scal = nullptr;  // [0] gbits [1] wmaxbits [2] live count [3] nvalid
    long long* totals = nullptr;         // [0] scan total
    unsigned* vflags = nullptr;
    double* bmax = nullptr;              // per-block maxima of the row pass
    unsigned long long* ri = nullptr;    // row information of level j at ri[4j .. 4j+3]
    double* gpart = nullptr;             // Galerkin pieces of runs that cross workgroups
    unsigned* alive = nullptr;           // HEM: one flag per round
    unsigned long long* rb = nullptr;    // words gathered for one host read
    void* block = nullptr;               // the one allocation all of the above point into
    std::vector<int> ri_pending;         // levels whose row information is still on the device
};

constexpr int kMaxLevels = 64;

// The setup scratch is one allocation, carved into 256-byte aligned pieces.
struct Carver {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(int64_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = (T*)(base ? base + off : nullptr);
        off += sizeof(T) * (size_t)std::max<int64_t>(count, 1);
        return p;
    }
};

void carve_tmp(Carver& cv, SetupTmp& t, int32_t n, int64_t nnz) {
    t.h = cv.take<int32_t>(n);
    t.slot = cv.take<unsigned long long>(n);
    t.live = cv.take<uint8_t>(n);
    t.state = cv.take<uint8_t>(n);
    t.pairseed = cv.take<int32_t>(n);
    t.rootseed = cv.take<int32_t>(n);
    t.flags = cv.take<int32_t>(n);
    t.rank = cv.take<int32_t>(n);
    t.scan_tmp = cv.take<long long>(std::max<int64_t>(scan_tmp_elems(std::max<int64_t>(n, nnz)), 16));
    t.k0 = cv.take<unsigned long long>(nnz);
    t.k1 = cv.take<unsigned long long>(nnz);
    t.v0 = cv.take<double>(nnz);
    t.v1 = cv.take<double>(nnz);
    t.heads = cv.take<int32_t>(nnz);
    t.idx = cv.take<int32_t>(nnz);
    const int64_t nsc = sort_tmp_elems(nnz);
    t.sort_counts = cv.take<int32_t>(nsc);
    t.sort_scan = cv.take<long long>(scan_tmp_elems(nsc) + 4);
    t.scal = cv.take<unsigned long long>(8);
    t.totals = cv.take<long long>(4);
    t.vflags = cv.take<unsigned>(4);
    t.bmax = cv.take<double>(4 * kRowinfoMaxBlocks);
    t.ri = cv.take<unsigned long long>(4 * kMaxLevels);
    t.gpart = cv.take<double>(gal_part_elems(nnz));
    t.alive = cv.take<unsigned>(kHemMaxRounds);
    t.rb = cv.take<unsigned long long>(kPackWordsMax);
}

cmg_status alloc_tmp(cmg_ctx* c, SetupTmp& t, int32_t n, int64_t nnz) {
    Carver size;
    carve_tmp(size, t, n, nnz);
    Carver cv;
    cv.base = (char*)c->dalloc_direct(size.off);
    if (!cv.base) return CMG_E_OOM;
    carve_tmp(cv, t, n, nnz);
    t.block = cv.base;
    return CMG_OK;
}

void free_tmp(cmg_ctx* c, SetupTmp& t) {
    (void)hipStreamSynchronize(c->stream);
    c->dfree_direct(t.block);
    t = SetupTmp{};
}

// Gershgorin shift, heaviest neighbours, largest weight, FP32 exactness and
// longest row of level j: enqueued; the values stay on the device until
// finish_rowinfo reads those of every level at once.
cmg_status level_rowinfo(cmg_ctx* c, SetupTmp& t, int j) {
    HostLevel& L = c->lv[j];
    if (j >= kMaxLevels) return CMG_E_DEVICE;
    CK(launch_rowinfo(L.n, L.lanes, L.rp, L.col, L.w64, L.wunit, t.h, t.bmax, t.ri + 4 * j, t.vflags, c->stream));
    t.ri_pending.push_back(j);
    return CMG_OK;
}

cmg_status finish_rowinfo(cmg_ctx* c, SetupTmp& t) {
    if (t.ri_pending.empty()) return CMG_OK;
    std::vector<unsigned long long> hb(4 * kMaxLevels);
    cmg_status st = d2h(c, hb.data(), t.ri, hb.size());
    if (st != CMG_OK) return st;
    for (int j : t.ri_pending) {
        HostLevel& L = c->lv[j];
        double gv, wm, ex, ml;
        std::memcpy(&gv, &hb[4 * j], 8);
        std::memcpy(&wm, &hb[4 * j + 1], 8);
        std::memcpy(&ex, &hb[4 * j + 2], 8);
        std::memcpy(&ml, &hb[4 * j + 3], 8);
        L.g = gv;
        L.wmax = wm;
        L.w32exact = (ex == 0.0) ? 1 : 0;
        L.maxlen = (int64_t)ml;
    }
    t.ri_pending.clear();
    return CMG_OK;
}

// longest input row for which member lists are built by counting
constexpr unsigned kCountMembersMaxRow = 1024;

// Device words (4 or 8 bytes each) read back with one copy: a launch
// gathers them into the setup scratch, so a host decision waits for one
// transfer instead of one per value.
cmg_status read_words(cmg_ctx* c, SetupTmp& t, std::initializer_list<std::pair<const void*, int>> src,
                      unsigned long long* out) {
    PackWords p{};
    for (const auto& e : src) {
        if (p.n == kPackWordsMax) return CMG_E_ARG;
        p.src[p.n] = e.first;
        p.bytes[p.n] = e.second;
        ++p.n;
    }
    CK(launch_pack_words(p, t.rb, c->stream));
    return d2h(c, out, t.rb, (size_t)p.n);
}

// HEC greedy rounds launched before the first host check of a level (the
// 3D-grid and geometric levels measured need 4 to 6; unused rounds return
// at once)
constexpr int kHecRoundsAhead = 6;

// More HEC rounds, two per host check, until none leaves a live candidate
// edge; *launched counts the rounds launched on the level so far.
cmg_status hec_finish(cmg_ctx* c, SetupTmp& t, int j, int* launched) {
    const HostLevel& L = c->lv[j];
    unsigned long long* hflags = t.scal + 6;
    for (;;) {
        unsigned long long w[2];
        cmg_status st = read_words(c, t, {{t.vflags, 4}, {hflags + ((*launched - 1) & 1), 8}}, w);
        if (st != CMG_OK) return st;
        const unsigned long long iso = w[0], more = w[1];
        if (iso) return CMG_E_ISOLATED;
        if (more == 0) return CMG_OK;
        if (*launched > 100000) return CMG_E_DEVICE;
        for (int r = 0; r < 2; ++r)
            CK(launch_hec_round(L.n, t.h, c->opt.seed, j, t.live, t.state, t.pairseed, t.slot, hflags, *launched + r,
                                c->stream));
        *launched += 2;
        c->hec_rounds += 2;
    }
}

// aggregates of the HEC matching: attach, number the opening vertices, label
hipError_t hec_aggregates(cmg_ctx* c, SetupTmp& t, const HostLevel& L) {
    hipStream_t s = c->stream;
    hipError_t e = launch_hec_attach(L.n, t.h, t.state, t.pairseed, t.rootseed, t.flags, s);
    if (e == hipSuccess) e = launch_scan(t.flags, t.rank, L.n, t.scan_tmp, t.totals, s);  // totals[0]: aggregates
    if (e == hipSuccess) e = launch_hec_label(L.n, t.rootseed, t.rank, L.agg, s);
    return e;
}

// One HEC + Galerkin step from level j; appends level j+1 unless HEC
// collapses (fewer than 2 aggregates).
cmg_status coarsen_once(cmg_ctx* c, SetupTmp& t, int j, bool* stop) {
    Range range("cmg coarsen level %d", j);
    HostLevel& L = c->lv[j];
    hipStream_t s = c->stream;
    const uint64_t seed = c->opt.seed;
    *stop = false;
    CK(launch_fill_u32(t.vflags, 0u, 1, s));  // raised by the row pass if a vertex has no neighbour
    cmg_status st = level_rowinfo(c, t, j);
    if (st != CMG_OK) return st;
    const bool hem = c->opt.coarsen == 1;
    unsigned long long* hflags = t.scal + 6;  // HEC round flags
    int hec_launched = 0;
    if (hem) {
        // heavy edge matching: rounds in batches between host checks; the
        // flag of a batch's last round tells whether any vertex was still
        // unmatched when it began (a round with none changes nothing)
        CK(launch_fill_u32((unsigned*)t.pairseed, 0xFFFFFFFFu, L.n, s));
        CK(launch_fill_u32(t.alive, 0u, kHemMaxRounds, s));
        int round = 0;
        for (int batch = 4;; batch = 4) {
            if (round + batch > kHemMaxRounds) return CMG_E_DEVICE;
            for (int r = 0; r < batch; ++r, ++round)
                CK(launch_hem_round(L.n, L.rp, L.col, L.w64, seed, j, t.pairseed, t.live, t.slot, t.alive, round,
                                    s));
            c->hec_rounds += batch;
            unsigned long long w[2];
            st = read_words(c, t, {{t.vflags, 4}, {t.alive + round - 1, 4}}, w);
            if (st != CMG_OK) return st;
            const unsigned long long iso = w[0], last = w[1];
            if (iso) return CMG_E_ISOLATED;
            if (last == 0) break;
        }
        CK(launch_hem_flags(L.n, t.pairseed, t.flags, s));
        CK(launch_scan(t.flags, t.rank, L.n, t.scan_tmp, t.totals, s));  // totals[0]: aggregates
        ALLOC(L.agg, int32_t, L.n);
        CK(launch_hec_label(L.n, t.pairseed, t.rank, L.agg, s));
    } else {
        CK(launch_hec_init(L.n, t.h, seed, j, t.live, t.state, t.pairseed, t.slot, hflags, s));
        // greedy rounds launched ahead without a host check; whether they
        // were enough is read with the next synchronisation below
        for (int r = 0; r < kHecRoundsAhead; ++r)
            CK(launch_hec_round(L.n, t.h, seed, j, t.live, t.state, t.pairseed, t.slot, hflags, hec_launched + r, s));
        hec_launched += kHecRoundsAhead;
        c->hec_rounds += kHecRoundsAhead;
        if (c->opt.galerkin == 1) {
            st = hec_finish(c, t, j, &hec_launched);
            if (st != CMG_OK) return st;
        }
        ALLOC(L.agg, int32_t, L.n);
        CK(hec_aggregates(c, t, L));
    }
    // Galerkin product by aggregates when no aggregate's member rows hold
    // more than kGalWaveCap entries: the aggregate count and the largest
    // aggregate are read back in one synchronisation, the coarse rows are
    // formed in fine CSR order; else the radix-sort path below.
    const int64_t ncmax = hem ? (int64_t)L.n : (int64_t)L.n / 2 + 1;
    if (c->opt.galerkin != 1) {
        int32_t* members = t.rootseed;
        int32_t* mdeg = t.flags;
        int32_t* mstart = t.pairseed;
        int32_t* moff = t.rank;
        long long nc0 = 0;
        unsigned long long emax = 0;
        for (;;) {
            // counted lists where the input has no long rows: an
            // aggregate's members (at most one plus the vertices naming the
            // same heaviest neighbour) then contend for its counter only a
            // few at a time; power-law hubs keep the radix sort
            if (c->int_weights && !hem && c->maxlen0 <= kCountMembersMaxRow)
                CK(launch_gal_members_count(L.n, (int)ncmax, L.agg, L.rp, t.idx, t.scan_tmp, t.totals + 3, members,
                                            mdeg, mstart, s));
            else
                CK(launch_gal_members(L.n, L.agg, L.rp, t.k0, t.k1, bitlen((unsigned long long)ncmax),
                                      t.sort_counts, t.sort_scan, members, mdeg, mstart, s));
            CK(launch_scan(mdeg, moff, L.n, t.scan_tmp, t.totals + 2, s));
            CK(launch_fill_u32((unsigned*)(t.scal + 4), 0u, 2, s));
            CK(launch_gal_agg_len((int)ncmax, t.totals, L.n, L.nnz, mstart, moff, t.scal + 4, s));
            // flag of a coarse vertex without neighbours, aggregate count,
            // largest input weight (level 0), live candidates after the
            // rounds launched (HEC), entries of the largest aggregate
            unsigned long long w[5];
            st = read_words(c, t,
                            {{t.vflags, 4}, {t.totals, 8}, {t.ri + 1, 8}, {hflags + ((hec_launched - 1) & 1), 8},
                             {t.scal + 4, 8}},
                            w);
            if (st != CMG_OK) return st;
            const unsigned long long iso = w[0], wmax0 = j == 0 ? w[2] : 0ull, more = hem ? 0ull : w[3];
            nc0 = (long long)w[1];
            emax = w[4];
            if (iso) return CMG_E_ISOLATED;  // a component of the graph became one aggregate
            if (j == 0) {
                // every coarse weight is a sum of input weights: with
                // integer weights whose total (at most nnz times the
                // largest) stays below 2^32, 32-bit integer sums are exact
                double wm = 0.0;
                std::memcpy(&wm, &wmax0, sizeof(wm));
                c->gal_int32 = c->int_weights && (double)L.nnz * wm < 4294967295.0;
            }
            if (more == 0) break;
            // the rounds launched ahead left live candidate edges.  The
            // member lists reused the matching's pair array, so the matching
            // is formed again from the start (the rounds are deterministic)
            // with two more rounds, then finished, and the aggregates and
            // their members formed again.
            CK(launch_hec_init(L.n, t.h, seed, j, t.live, t.state, t.pairseed, t.slot, hflags, s));
            const int redo = hec_launched + 2;
            for (int r = 0; r < redo; ++r)
                CK(launch_hec_round(L.n, t.h, seed, j, t.live, t.state, t.pairseed, t.slot, hflags, r, s));
            c->hec_rounds += 2;
            hec_launched = redo;
            st = hec_finish(c, t, j, &hec_launched);
            if (st != CMG_OK) return st;
            CK(hec_aggregates(c, t, L));
        }
        if (nc0 < 2) {
            c->dfree(L.agg);
            L.agg = nullptr;
            c->collapsed = 1;
            *stop = true;
            return CMG_OK;
        }
        if (emax <= (unsigned long long)kGalWaveCap) {
            const int nc = (int)nc0;
            int32_t* rowlen = t.h;
            int32_t* tcol = t.idx;
            double* tw = t.v1;
            // a lane per aggregate with 16 register slots where fine rows are
            // short (coarse rows rarely exceed 16 columns), 24 where they
            // hold up to 16 entries on average, else 32 (a row with more
            // columns goes to the wave sort); on levels with few aggregates
            // (a lane's walk would be one long chain of loads on a mostly
            // idle device) every row by the wave sort
            const int slots = (c->opt.galerkin == 2 || nc < kGalLaneMinRows) ? 0
                              : L.nnz <= 7 * (int64_t)L.n                    ? 16
                              : L.nnz <= 16 * (int64_t)L.n                   ? 24
                                                                             : 32;
            CK(launch_gal_gather(nc, L.n, L.nnz, slots, L.wunit, c->gal_int32, members, mstart, moff, L.rp, L.col,
                                 L.w64, L.agg,
                                 tcol, tw, rowlen, t.heads, (unsigned*)(t.scal + 5), s));
            HostLevel C;
            C.n = nc;
            ALLOC(C.rp, int32_t, nc + 1);
            CK(launch_scan(rowlen, C.rp, nc, t.scan_tmp, t.totals + 1, s));
            long long zc = 0;
            st = d2h(c, &zc, t.totals + 1, 1);
            if (st != CMG_OK) return st;
            CK(launch_fill_u32((unsigned*)(C.rp + nc), (unsigned)zc, 1, s));
            C.nnz = zc;
            ALLOC(C.col, int32_t, std::max<long long>(zc, 1));
            ALLOC(C.w64, double, std::max<long long>(zc, 1));
            if (zc > 0)
                CK(launch_gal_compact(nc, mstart, moff, C.rp, tcol, tw, t.heads, (const unsigned*)(t.scal + 5), C.col,
                                      C.w64, s));
            C.lanes = pick_lanes(C.nnz / (double)C.n);
            c->lv.push_back(C);
            return CMG_OK;
        }
    }
    // Radix-sort path, with the aggregate count left on the device: keys
    // a * mult + b with mult >= the count (HEC aggregates have two vertices
    // or more: n/2 + 1; HEM's one or two: n), sorted on enough bits that
    // the sentinel's low bits exceed every key
    const int64_t mult = ncmax;
    const int bits = bitlen((unsigned long long)mult * (unsigned long long)mult);
    // packed words (key << pbits | fine position) when they fit 64 bits:
    // the sort then moves 8 bytes per entry instead of 16
    const int pbits = std::max(1, bitlen((unsigned long long)std::max<int64_t>(L.nnz - 1, 1)));
    const bool packed = bits + pbits <= 64;
    const int pshift = packed ? pbits : 0;
    const unsigned long long sent = packed ? (~0ull >> (64 - bits)) : kGalSentinel;
    if (j == 0 && c->maxlen0 > 64u * (unsigned)L.lanes) {  // a row of many lane-group trips
        CK(launch_gal_emit_entries(L.n, L.nnz, L.rp, L.col, L.w64, L.agg, mult, pshift, sent, t.k0,
                                   packed ? nullptr : t.v0, s));
    } else {
        CK(launch_gal_emit(L.n, L.lanes, L.rp, L.col, L.w64, L.agg, mult, pshift, sent, t.k0,
                           packed ? nullptr : t.v0, s));
    }
    int second = 0;
    CK(launch_sort(t.k0, packed ? nullptr : t.v0, t.k1, packed ? nullptr : t.v1, L.nnz, pshift, bits,
                   t.sort_counts, t.sort_scan, &second, s));
    const unsigned long long* ks = second ? t.k1 : t.k0;
    const double* vs = packed ? nullptr : (second ? t.v1 : t.v0);
    CK(launch_count_below(ks, L.nnz, packed ? (sent << pshift) : kGalSentinel, t.scal + 3, s));
    CK(launch_gal_heads(L.nnz, t.scal + 3, ks, pshift, t.heads, s));
    CK(launch_scan(t.heads, t.idx, L.nnz, t.scan_tmp, t.totals + 1, s));  // totals[1]: coarse entries
    unsigned long long w[3];
    st = read_words(c, t, {{t.totals, 8}, {t.totals + 1, 8}, {t.scal + 3, 8}}, w);
    if (st != CMG_OK) return st;
    const long long nc = (long long)w[0], zc = (long long)w[1];
    const unsigned long long nvalid = w[2];
    if (nc < 2) {
        c->dfree(L.agg);
        L.agg = nullptr;
        c->collapsed = 1;
        *stop = true;
        return CMG_OK;
    }
    HostLevel C;
    C.n = (int32_t)nc;
    C.nnz = zc;
    ALLOC(C.rp, int32_t, C.n + 1);
    ALLOC(C.col, int32_t, std::max<long long>(zc, 1));
    ALLOC(C.w64, double, std::max<long long>(zc, 1));
    if (zc == 0) {
        CK(hipMemsetAsync(C.rp, 0, sizeof(int32_t) * (C.n + 1), s));
    } else {
        CK(launch_gal_reduce((int64_t)nvalid, ks, vs, L.w64, pshift, t.heads, t.idx, mult, (int)nc, zc, C.rp,
                             C.col, C.w64, c->int_weights ? t.gpart : nullptr, s));
    }
    C.lanes = pick_lanes(C.nnz / (double)C.n);
    c->lv.push_back(C);
    return CMG_OK;
}

// ---- small levels: one launch for the rest of the hierarchy
bool chain_level(const HostLevel& L) { return L.n <= kChainMaxN && L.nnz <= kChainMaxNnz; }

// Coarsens level j0 and the levels below it in one workgroup.  *next = -1
// if the hierarchy is complete, else the index of a level left to the grid
// kernels (a coarse row too long for the single-workgroup Galerkin step).
cmg_status coarsen_chain(cmg_ctx* c, SetupTmp& t, int j0, int* next) {
    Range range("cmg coarsen levels from %d in one workgroup", j0);
    HostLevel L = c->lv[j0];
    hipStream_t s = c->stream;
    const int max_levels = 61 - j0;  // coarsening stops at level index 60
    // arena bounds: n_{k+1} <= n_k / 2; nnz_{k+1} <= min(nnz_k, n_{k+1} (n_{k+1} - 1))
    int64_t cw = 0;
    {
        int64_t prev = L.nnz, nk = L.n;
        for (int k = 1; k < max_levels; ++k) {
            nk /= 2;
            if (nk < 2) break;
            const int64_t b = std::min<int64_t>(prev, nk * (nk - 1));
            cw += b;
            prev = b;
        }
    }
    cw = std::max<int64_t>(cw, 1);
    const int64_t i32cap = 4 * (int64_t)L.n + 2 * (int64_t)max_levels + 64;
    ChainJob job{};
    job.n0 = L.n;
    job.level0 = j0;
    job.nnz0 = L.nnz;
    job.rp0 = L.rp;
    job.col0 = L.col;
    job.w0 = L.w64;
    job.seed = c->opt.seed;
    job.coarsest_n = c->opt.coarsest_n;
    job.max_levels = max_levels;
    // scratch: the level-0 setup buffers (n0 >= n and nnz0 >= nnz, and
    // nnz0 >= n0 since every vertex has a neighbour)
    job.h = t.h;
    job.pairseed = t.pairseed;
    job.rootseed = t.rootseed;
    job.rank = t.rank;
    job.members = t.idx;
    job.astart = (int32_t*)t.k0;  // 2 nnz0 ints
    job.soff = job.astart + L.n;
    job.rcount = (int32_t*)t.v1;  // 2 nnz0 ints
    job.mb = (int32_t*)t.k1;
    job.bcol = t.heads;
    job.slot = t.slot;
    job.live = t.live;
    job.state = t.state;
    job.mw = t.v0;
    ALLOC(job.ai32, int32_t, i32cap);
    job.ai32_cap = i32cap;
    ALLOC(job.acol, int32_t, cw);
    ALLOC(job.aw, double, cw);
    job.acw_cap = cw;
    const size_t hbytes = sizeof(ChainHdr) * max_levels + 16;
    char* hd_dev = (char*)c->dalloc_direct(hbytes);
    if (!hd_dev) return CMG_E_OOM;
    job.hdr = (ChainHdr*)hd_dev;
    job.out = (int32_t*)(hd_dev + sizeof(ChainHdr) * max_levels);
    CK(launch_coarsen_chain(job, s));
    std::vector<char> hb(hbytes);
    cmg_status st = d2h(c, hb.data(), hd_dev, hbytes);
    c->dfree_direct(hd_dev);
    if (st != CMG_OK) return st;
    const ChainHdr* hdr = (const ChainHdr*)hb.data();
    const int32_t* out = (const int32_t*)(hb.data() + sizeof(ChainHdr) * max_levels);
    const int K = out[0], reason = out[2];
    if (K < 1 || K > max_levels) return CMG_E_DEVICE;
    if (reason == 6) return CMG_E_ISOLATED;  // a component of the graph became one aggregate
    for (int k = 0; k < K; ++k) {
        const ChainHdr& h = hdr[k];
        if (k > 0) {
            HostLevel C;
            C.n = h.n;
            C.nnz = h.nnz;
            C.rp = job.ai32 + h.rp_off;
            C.col = job.acol + h.cw_off;
            C.w64 = job.aw + h.cw_off;
            C.lanes = pick_lanes(C.nnz / (double)std::max(C.n, 1));
            c->lv.push_back(C);
        }
        HostLevel& Lk = c->lv[j0 + k];
        Lk.g = h.g;
        Lk.wmax = h.wmax;
        Lk.w32exact = (h.w32err == 0.0) ? 1 : 0;
        Lk.maxlen = (int64_t)h.maxlen;
        if (h.agg_off >= 0) {
            Lk.agg = job.ai32 + h.agg_off;
            c->hec_rounds += h.rounds;
        }
    }
    if (out[1]) c->collapsed = 1;
    *next = (reason == 3 || reason == 4) ? j0 + K - 1 : -1;
    return CMG_OK;
}

LevelDev level_dev(const HostLevel& L) {
    LevelDev d{};
    d.n = L.n;
    d.lanes = L.lanes;
    d.nnz = L.nnz;
    d.rp = L.rp;
    d.col = L.col;
    d.w64 = L.w64;
    d.w32 = L.w32;
    d.w8 = L.w8;
    d.w16 = L.w16;
    d.agg = L.agg;
    d.g = L.g;
    d.fp32 = L.fp32;
    d.variant = L.variant;
    d.buf0 = L.buf0;
    d.buf1 = L.buf1;
    d.part = L.part;
    d.mpart = nullptr;
    d.grid = L.grid;
    d.w32exact = L.w32exact;
    d.bwaves = L.bwaves;
    d.bregs = L.bregs;
    d.bslots = L.bslots;
    d.stage = L.stage;
    // workgroup parts of more than four times the rows the LDS stage holds:
    // the steps walk the XCD's rows in chunks taken in turn by its
    // workgroups, so they sweep it together and their gathers share that
    // XCD's L2 (256^3 grid levels 0 and 1 2% faster; parts of ~1300 rows
    // 13% slower)
    d.ileave = (L.variant == 1 && L.grid >= 8 && (int64_t)L.n > 4LL * kGridStageRows * L.grid) ? 1 : 0;
    d.kfix = L.kfix;
    d.wk = L.wk;
    d.lmin = L.lrows ? L.lmin : 0x7fffffff;
    d.lrows = L.lrows;
    return d;
}

// SpMV traversal of a grid level: rows per lane group (rows far longer than
// the lanes' share summed by whole workgroups), unless the longest row
// dwarfs the mean (skewed degrees) on a level of short rows, then the merge
// path: there many rows of a few hundred entries would each hold a small
// lane group (measured on 4M-vertex Chung-Lu graphs: merge path faster at
// 8 lanes per row, rows traversal at 64).
int choose_variant(const HostLevel& L, int requested) {
    if (requested == 1 || requested == 2) return requested;
    const double avg = L.nnz / (double)std::max(L.n, 1);
    const bool skewed = L.maxlen > 256 && L.maxlen > 32.0 * avg;
    return (skewed && pick_lanes(avg) < 32) ? 2 : 1;
}

size_t align8h(size_t b) { return (b + 7) & ~(size_t)7; }

// A level is refined inside one workgroup if it has at most block_rows
// vertices and its steps stay cheap there: its LDS image (two vectors,
// weights, row pointers, columns; FP32 weights when exact, uint16 columns
// when n <= 65536) fits the LDS budget, or it has at most kBlockGlobalNnz
// entries to stream from L2 (one CU streaming more is slower than the grid
// kernels).  A dense coarse level (hub rows of a power-law graph) is left
// to the grid kernels, whose bandwidth it needs.
constexpr int64_t kBlockGlobalNnz = 8192;

bool block_level(const HostLevel& L, int block_rows) {
    if (L.n > block_rows) return false;
    if (L.nnz <= kBlockGlobalNnz) return true;
    const size_t wb = L.w32exact ? 4 : 8;
    const size_t cb = L.n <= 65536 ? 2 : 4;
    const size_t img = align8h(16 * (size_t)L.n) + align8h((size_t)L.nnz * wb) +
                       align8h(4 * ((size_t)L.n + 1)) + align8h((size_t)L.nnz * cb);
    return img <= (size_t)refine_block_lds_budget();
}

// Largest co-resident workgroup count of the level's kernels (a multiple
// of 8, at least 8); level 0 also runs the finishing kernel on its grid.
int grid_cap(const HostLevel& L, int j, int lanes) {
    const int kind = job_kind(L.variant, lanes, L.fp32, L.wk);
    int cap = refine_jobs_max_blocks(kind);
    if (j == 0) cap = std::min(cap, finish_jobs_max_blocks(kind));
    return std::max(8, (cap / 8) * 8);
}

// Bytes of a PI step with FP64 values and vectors: the measure of a level's
// size for the choice of step mode, the same whatever storage it gets (a
// mixed-precision level would otherwise fall below the threshold its FP64
// form passes and run one barrier per step: 4M Chung-Lu level 2, 1940
// steps, 16.7 MB in FP32, 42.7 ms against 31.1 ms in step mode).
int64_t step_bytes(const HostLevel& L) {
    return 4 * ((int64_t)L.n + 1) + L.nnz * 12 + 16 * (int64_t)L.n;
}

// Levels at depth >= kStepModeDepth whose PI step streams at least
// kStepModeBytes (counted in FP64) are refined with one launch per step
// (kernel boundaries and a one-workgroup reduction in place of the grid
// barrier), with a workgroup of kStepBlock threads per kStepWork rows +
// entries.  A step there costs less than with the barrier, but the level
// pays about 70-100 us of fixed launches and host checks, which only
// levels with enough steps recover; in a cascadic cycle those are all but
// the finest (256^3 grid level 1, 18 steps: 4.33 -> 4.17 ms; 4M Chung-Lu
// level 1, 197 steps: 38.3 -> 36.6 ms).
constexpr int64_t kStepModeBytes = (int64_t)16 << 20;
// rows traversal: rows longer than max(kLongRowMin, 32 lanes) are long
// (summed by a whole workgroup)
constexpr int kLongRowMin = 256;
constexpr int kStepModeDepth = 1;
constexpr int64_t kStepWork = 4096;
// Levels of at least this many rows + entries take twice kStepWork per
// workgroup (measured on MI355X: 256^3 grid level 1, 58M, 4.19 -> 3.77 ms;
// 4M Chung-Lu level 1, 29M, 36.5 -> 32.9 ms; but at 2M, grid level 4 and
// Chung-Lu level 2, fewer workgroups were 15% and 5% slower).
constexpr int64_t kStepWorkLargeMin = (int64_t)16 << 20;

// Workgroups of a level refined one launch per step.
int step_grid(const HostLevel& L) {
    const int64_t work = (int64_t)L.n + L.nnz;
    const int64_t per = work >= kStepWorkLargeMin ? 2 * kStepWork : kStepWork;
    return (int)std::min<int64_t>(std::max<int64_t>((work + per - 1) / per, 8), 65535);
}
constexpr int kStepChunk = 8;
constexpr int kChunkEvents = 16;

// Default workgroup count: about 2k rows+entries per workgroup (short
// per-group latency chains on mid-size levels), a multiple of 8, at most
// 3 per CU (on levels whose step fits the 256 MB last-level cache the cost
// of the grid barrier, which grows with the workgroup count, outweighs
// more waves; on the streaming levels of a 256^3 grid 3 per CU also beat 4:
// level 0 2.46 against 3.04 ms for 5 steps) and at most what can be
// co-resident.
int default_grid(const HostLevel& L, int j, int ncu) {
    int cap = std::min(grid_cap(L, j, L.lanes), 3 * ncu);
    // about 2k rows + entries per workgroup; on mid-size levels (up to 4M
    // rows + entries) no more than sqrt(work)/4.5 workgroups, since there the
    // barrier's cost, which grows with the count, outweighs the step's work
    // (measured on MI355X: level 1 of a 1M-point random geometric graph,
    // 2.9M rows + entries, 73 us per step on 384 workgroups against 90 on
    // 768; level 3 of a 128^3 grid, 0.93M: 17.9 us on 216 against 21.2 on
    // 456; at 8M, 768 workgroups beat 600)
    const int64_t work = (int64_t)L.n + L.nnz;
    int64_t want = (work + 2047) / 2048;
    if (work <= ((int64_t)4 << 20))
        want = std::min<int64_t>(want, std::max<int64_t>((int64_t)(std::sqrt((double)work) / 4.5), 8));
    want = ((want + 7) / 8) * 8;
    return (int)std::min<int64_t>(std::max<int64_t>(want, 8), cap);
}

// ---- autotuner: lanes per row and workgroup count of a grid level
//
// Candidates: lanes G/2, G, 2G around the rule's G (G only for the merge
// path) and, for each, the default workgroup count and the co-resident
// maximum (and 3/4 of it).  Each candidate runs kTuneSteps power-iteration
// steps of the real refinement kernel from the hashed uniform start with
// the stopping test disabled (tol = -1), twice; the faster run counts.
// The choice is cached per process by level shape.
constexpr int kTuneSteps = 4;

struct TuneKey {
    int variant, fp32, finest, n2, deg2, ml;
    bool operator<(const TuneKey& o) const {
        return std::tie(variant, fp32, finest, n2, deg2, ml) <
               std::tie(o.variant, o.fp32, o.finest, o.n2, o.deg2, o.ml);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;  // -> (lanes, grid)

cmg_status tune_level(cmg_ctx* c, int j, int maxgrid) {
    HostLevel& L = c->lv[j];
    const double avg = L.nnz / (double)std::max(L.n, 1);
    const TuneKey key{L.variant, L.fp32, j == 0 ? 1 : 0, (int)std::lround(2.0 * std::log2((double)L.n)),
                      (int)std::lround(2.0 * avg), bitlen((unsigned long long)L.maxlen)};
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            L.lanes = it->second.first;
            L.grid = it->second.second;
            return CMG_OK;
        }
    }
    std::vector<std::pair<int, int>> cand;
    std::vector<int> lanes_c;
    if (L.variant == 2) lanes_c.push_back(L.lanes);
    else
        for (int g : {L.lanes / 2, L.lanes, 2 * L.lanes})
            if (g >= 1 && g <= 64) lanes_c.push_back(g);
    int64_t want = ((int64_t)L.n + L.nnz + 2047) / 2048;
    want = std::max<int64_t>(8, ((want + 7) / 8) * 8);
    for (int g : lanes_c) {
        const int cap = std::min(grid_cap(L, j, g), maxgrid);
        for (int64_t nb : {want, (int64_t)cap, (int64_t)(cap * 3 / 4 / 8 * 8)}) {
            const int gb = (int)std::max<int64_t>(8, std::min<int64_t>(nb, cap));
            if (std::find(cand.begin(), cand.end(), std::make_pair(g, gb)) == cand.end())
                cand.push_back({g, gb});
        }
    }
    hipStream_t s = c->stream;
    int32_t* part = nullptr;
    LevelState* st = nullptr;
    GridJob* dj = nullptr;
    ALLOC(part, int32_t, maxgrid + 1);
    ALLOC(st, LevelState, 1);
    ALLOC(dj, GridJob, 1);
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    float best_ms = 0.f;
    std::pair<int, int> best{L.lanes, L.grid};
    bool have = false;
    for (const auto& cg : cand) {
        HostLevel T = L;
        T.lanes = cg.first;
        T.grid = cg.second;
        T.part = part;
        CK(launch_partition(L.n, L.nnz, L.rp, T.grid, part, s));
        GridJob g{};
        g.L = level_dev(T);
        g.C = g.L;
        g.st = st;
        g.stc = nullptr;
        g.gs = c->d_sync;
        g.slots = c->d_slots;
        g.bcast = c->d_bcast;
        g.tol = -1.0;  // never converges: exactly maxit steps
        g.seed = c->opt.seed;
        g.maxit = kTuneSteps;
        g.uniform = 1;
        g.tag = j;
        CK(hipMemcpyAsync(dj, &g, sizeof(GridJob), hipMemcpyHostToDevice, s));
        const int kind = job_kind(T.variant, T.lanes, T.fp32, T.wk);
        float ms_min = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
            CK(hipEventRecord(e0, s));
            CK(launch_refine_jobs(dj, 1, T.grid, kind, s));
            CK(hipEventRecord(e1, s));
            CK(hipEventSynchronize(e1));
            float ms = 0.f;
            CK(hipEventElapsedTime(&ms, e0, e1));
            if (rep == 0 || ms < ms_min) ms_min = ms;
        }
        if (!have || ms_min < best_ms) {
            best_ms = ms_min;
            best = cg;
            have = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    GridSync hg{};
    CK(hipMemcpyAsync(&hg, c->d_sync, sizeof(GridSync), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    c->dfree(dj);
    c->dfree(st);
    c->dfree(part);
    if (hg.abort) {
        // a trial did not complete its barriers: keep the rules' choice
        CK(launch_reset_sync(c->d_sync, c->d_slots, c->nslots, c->d_bcast, s));
        return CMG_OK;
    }
    L.lanes = best.first;
    L.grid = best.second;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[key] = best;
    return CMG_OK;
}

// Fixed smoothing schedule of the geometric cascadic method (Algorithm 4;
// Section 3, main theorem): level j runs the smallest integer number of
// steps >= k0 beta^j, beta^j formed by j multiplications, at most cap.
int fixed_steps(int k0, double beta, int j, int cap) {
    double p = (double)k0;
    for (int t = 0; t < j; ++t) p *= beta;
    const double c = std::ceil(p);
    return c > (double)cap ? cap : (int)c;
}

cmg_status build_refine_plan(cmg_ctx* c) {
    Range range("cmg refinement plan");
    const int J = (int)c->lv.size() - 1;
    const cmg_options& o = c->opt;
    HostLevel& CJ = c->lv[J];
    c->coarse_dense = (CJ.n <= o.dense_max) ? 1 : 0;
    const int block_rows = o.block_rows > 0 ? o.block_rows : 4096;
    const int64_t mixed_min = o.mixed_min_nnz > 0 ? o.mixed_min_nnz : (int64_t)1 << 20;
    // refinement levels: 0..J-1, plus J if the coarsest uses power iteration
    int top = c->coarse_dense ? J - 1 : J;
    c->fixed = o.fixed_k0 > 0;
    for (int j = 0; j <= J; ++j)
        c->lv[j].kfix = (c->fixed && j <= top) ? fixed_steps(o.fixed_k0, o.fixed_beta, j, o.max_iters_per_level) : 0;
    c->block_lo = top + 1;
    for (int j = top; j >= 0; --j) {
        const bool in = o.block_rows > 0 ? c->lv[j].n <= o.block_rows : block_level(c->lv[j], block_rows);
        if (in) c->block_lo = j;
        else break;
    }
    // barrier state first: the autotuner launches the refinement kernel
    int ncu = 256;
    {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    }
    const int maxgrid = std::max(8, 4 * ncu);  // 4 workgroups of 512 threads fill a CU
    ALLOC(c->d_sync, GridSync, 1);
    c->nslots = maxgrid;
    ALLOC(c->d_slots, GridSlot, 2 * maxgrid);
    c->d_bcast = (GridSlot*)c->dalloc(kBcastBytes);
    if (!c->d_bcast) return CMG_E_OOM;
    CK(launch_reset_sync(c->d_sync, c->d_slots, c->nslots, c->d_bcast, c->stream));
    // single-workgroup levels: rows in registers where a layout fits, else
    // the CSR traversal
    for (int j = 0; j <= J; ++j) {
        HostLevel& L = c->lv[j];
        L.in_block = (j >= c->block_lo && j <= top) ? 1 : 0;
        L.stage = o.grid_stage != 0 ? 1 : 0;
        L.bwaves = L.bregs = L.bslots = 0;
        if (!L.in_block) continue;
        const BlockPlan p = o.block_regs < 0 ? BlockPlan{} : plan_block_regs(L, refine_block_lds_budget());
        if (p.regs > 0) {
            L.bwaves = p.waves;
            L.lanes = p.lanes;
            L.bregs = p.regs;
            L.bslots = p.slots;
        } else {
            L.lanes = pick_lanes_block(L.n, L.nnz / (double)std::max(L.n, 1), (int)L.maxlen, kBlockKernelThreads);
        }
    }
    // the dense coarsest solve depends on the hierarchy alone: it is
    // launched now and runs while the rest of the plan is built
    ALLOC(c->d_st, LevelState, J + 1);
    ALLOC(c->d_fo, FinishOut, 1);
    if (c->coarse_dense) {
        HostLevel& LJ = c->lv[J];
        LJ.buf0 = c->dalloc(sizeof(double) * (size_t)LJ.n);
        LJ.buf1 = c->dalloc(sizeof(double) * (size_t)LJ.n);
        if (!LJ.buf0 || !LJ.buf1) return CMG_E_OOM;
        const int dm = std::max(CJ.n, 2);
        ALLOC(c->d_A, double, (size_t)dm * dm);
        ALLOC(c->d_V, double, (size_t)dm * dm);
        ALLOC(c->d_ev, double, 2 * (size_t)dm);
        ALLOC(c->d_idx, int32_t, dm);
        CoarseJob cj{};
        cj.L = level_dev(LJ);  // the kernel reads n, rp, col, w64 and buf0
        cj.st = c->d_st + J;
        cj.A = c->d_A;
        cj.V = c->d_V;
        cj.ev = c->d_ev;
        cj.idx = c->d_idx;
        cj.fo = c->d_fo;
        cj.seed = o.seed;
        c->h_cjob = cj;
        ALLOC(c->d_cjob, CoarseJob, 1);
        CK(hipMemcpyAsync(c->d_cjob, &cj, sizeof(cj), hipMemcpyHostToDevice, c->stream));
        CK(launch_coarse_jobs(c->d_cjob, 1, c->stream));
        c->coarse_done = true;
    }
    int max_step_grid = 0;
    int32_t* lt_flags = nullptr;  // long-row list scratch (freed once the plan is built)
    for (int j = 0; j <= J; ++j) {
        HostLevel& L = c->lv[j];
        L.fp32 = 0;
        if (o.precision == CMG_MIXED && !L.in_block && j <= top && L.nnz >= mixed_min &&
            L.wmax < 16777216.0 && !(j == J && c->coarse_dense))
            L.fp32 = 1;
        L.variant = choose_variant(L, o.spmv_variant);
        // weights as the grid and step kernels read them: none where all are
        // 1; an 8- or 16-bit copy where every weight is an integer up to 255
        // or 65535 (every input weight an integer: coarse weights are their
        // sums), else beside FP64 iterates an FP32 copy where every weight
        // is exact in FP32 (the same values, fewer bytes per entry); FP32
        // iterates otherwise read FP32 weights
        L.wk = kWNative;
        if (o.weight_storage == 0 && !L.in_block && j <= top && !(j == J && c->coarse_dense)) {
            if (L.wunit) L.wk = kWUnit;
            else if (c->int_weights && L.wmax <= 255.0) L.wk = kWU8;
            else if (c->int_weights && L.wmax <= 65535.0) L.wk = kWU16;
            else if (!L.fp32 && L.w32exact) L.wk = kWF32;
        }
        const size_t vb = L.fp32 ? 4 : 8;
        if (!(j == J && c->coarse_dense)) {  // else allocated above
            L.buf0 = c->dalloc(vb * (size_t)L.n);
            L.buf1 = c->dalloc(vb * (size_t)L.n);
            if (!L.buf0 || !L.buf1) return CMG_E_OOM;
        }
        if ((L.fp32 && L.wk == kWNative) || L.wk == kWF32) {
            ALLOC(L.w32, float, std::max<int64_t>(L.nnz, 1));
            CK(launch_to_f32(L.nnz, L.w64, L.w32, c->stream));
        }
        if (L.wk == kWU8) {
            ALLOC(L.w8, uint8_t, std::max<int64_t>(L.nnz, 1));
            CK(launch_to_u8(L.nnz, L.w64, L.w8, c->stream));
        }
        if (L.wk == kWU16) {
            ALLOC(L.w16, uint16_t, std::max<int64_t>(L.nnz, 1));
            CK(launch_to_u16(L.nnz, L.w64, L.w16, c->stream));
        }
        L.grid = default_grid(L, j, ncu);
        const bool auto_step = j >= kStepModeDepth && step_bytes(L) >= kStepModeBytes;
        L.step = (!L.in_block && j <= top && L.variant != 2 &&
                  (o.step_mode > 0 || (o.step_mode == 0 && auto_step))) ? 1 : 0;
        if (o.autotune && !L.in_block && !L.step && j <= top) {
            cmg_status st = tune_level(c, j, maxgrid);
            if (st != CMG_OK) return st;
        }
        // hub rows of a rows-traversal level are summed by whole workgroups
        L.lrows = nullptr;
        L.lmin = std::max(kLongRowMin, 32 * L.lanes);
        if (!L.in_block && j <= top && L.variant == 1 && L.maxlen > L.lmin) {
            // flags and positions (n0 ints each, n0 rounded up to even), scan
            // scratch and the total, for any level
            const int64_t n0e = ((int64_t)c->lv[0].n + 1) & ~(int64_t)1;
            if (!lt_flags) {
                const size_t nb = sizeof(int32_t) * 2 * (size_t)n0e +
                                  sizeof(long long) * (size_t)(scan_tmp_elems(c->lv[0].n) + 8);
                lt_flags = (int32_t*)c->dalloc_direct(nb);
                if (!lt_flags) return CMG_E_OOM;
            }
            int32_t* lt_pos = lt_flags + n0e;
            long long* lt_scan = (long long*)(lt_pos + n0e);
            long long* lt_total = lt_scan + scan_tmp_elems(c->lv[0].n) + 4;
            ALLOC(L.lrows, int32_t, 1 + L.nnz / ((int64_t)L.lmin + 1));
            CK(launch_long_rows(L.n, L.rp, L.lmin, lt_flags, lt_pos, lt_scan, lt_total, L.lrows, c->stream));
        }
        if (L.step) {
            if (j == 0) {  // the finishing pass keeps a co-resident grid
                L.fgrid = L.grid;
                ALLOC(L.fpart, int32_t, L.fgrid + 1);
                CK(launch_partition(L.n, L.nnz, L.rp, L.fgrid, L.fpart, c->stream));
            }
            L.grid = step_grid(L);
            max_step_grid = std::max(max_step_grid, L.grid);
        }
        ALLOC(L.part, int32_t, L.grid + 1);
        CK(launch_partition(L.n, L.nnz, L.rp, L.grid, L.part, c->stream));
        // a persistent rows-traversal level can be re-run one launch per step
        // (no inter-workgroup waits) if a barrier wait is given up
        L.fbgrid = 0;
        if (!c->noalloc && !L.in_block && j <= top && L.variant != 2 && !L.step) {
            L.fbgrid = step_grid(L);
            ALLOC(L.fbpart, int32_t, L.fbgrid + 1);
            CK(launch_partition(L.n, L.nnz, L.rp, L.fbgrid, L.fbpart, c->stream));
            max_step_grid = std::max(max_step_grid, L.fbgrid);
        }
    }
    if (max_step_grid > 0) {
        ALLOC(c->d_ctl, StepCtl, 1);
        ALLOC(c->d_part, double, 4 * (size_t)max_step_grid);
        ALLOC(c->d_step, StepJob, J + 1);
        ALLOC(c->d_step_fb, StepJob, J + 1);
    }
    std::vector<LevelDev> ld(J + 1);
    for (int j = 0; j <= J; ++j) ld[j] = level_dev(c->lv[j]);
    ALLOC(c->d_lv, LevelDev, J + 1);
    CK(hipMemcpyAsync(c->d_lv, ld.data(), sizeof(LevelDev) * (J + 1), hipMemcpyHostToDevice, c->stream));
    const int32_t n0 = c->lv[0].n;
    ALLOC(c->d_y, double, n0);
    if (c->lv[0].fp32 && o.fp64_final_sweeps > 0) {
        ALLOC(c->d_fa, double, n0);
        ALLOC(c->d_fb, double, 8);
    }
    // static job table: one refinement job per level, one finishing job
    std::vector<GridJob> jobs(J + 2);
    for (int j = 0; j <= J; ++j) {
        GridJob g{};
        g.L = ld[j];
        g.C = (j < J) ? ld[j + 1] : ld[j];
        g.st = c->d_st + j;
        g.stc = (j < J) ? c->d_st + j + 1 : nullptr;
        g.gs = c->d_sync;
        g.slots = c->d_slots;
        g.bcast = c->d_bcast;
        g.uniform = (j == J) ? 1 : 0;
        g.tol = c->lv[j].kfix > 0 ? -1.0 : o.tol;  // a fixed schedule never passes the test
        g.seed = o.seed;
        g.maxit = c->lv[j].kfix > 0 ? c->lv[j].kfix : o.max_iters_per_level;
        g.b0 = 0;
        g.tag = j;
        jobs[j] = g;
    }
    {
        GridJob g{};
        g.L = ld[0];
        if (c->lv[0].step) {
            g.L.grid = c->lv[0].fgrid;
            g.L.part = c->lv[0].fpart;
        }
        g.C = ld[0];
        g.st = nullptr;
        g.stc = c->d_st;
        g.gs = c->d_sync;
        g.slots = c->d_slots;
        g.bcast = c->d_bcast;
        g.fa = c->d_fa;
        g.yout = c->d_y;
        g.fo = c->d_fo;
        g.redo = (c->lv[0].fp32 && c->d_fa && o.fp64_final_sweeps > 0) ? 1 : 0;
        g.b0 = 0;
        g.tag = -1;
        jobs[J + 1] = g;
    }
    c->h_jobs = jobs;
    ALLOC(c->d_jobs, GridJob, J + 2);
    CK(hipMemcpyAsync(c->d_jobs, jobs.data(), sizeof(GridJob) * (J + 2), hipMemcpyHostToDevice, c->stream));
    if (c->d_step) {
        std::vector<StepJob> sj(J + 1);
        for (int j = 0; j <= J; ++j) {
            StepJob t{};
            t.L = ld[j];
            t.C = (j < J) ? ld[j + 1] : ld[j];
            t.stc = (j < J) ? c->d_st + j + 1 : nullptr;
            t.st = c->d_st + j;
            t.ctl = c->d_ctl;
            t.part = c->d_part;
            t.tol = c->lv[j].kfix > 0 ? -1.0 : o.tol;
            t.seed = o.seed;
            t.maxit = c->lv[j].kfix > 0 ? c->lv[j].kfix : o.max_iters_per_level;
            t.uniform = (j == J) ? 1 : 0;
            sj[j] = t;
        }
        CK(hipMemcpyAsync(c->d_step, sj.data(), sizeof(StepJob) * (J + 1), hipMemcpyHostToDevice, c->stream));
        // the fallback table: the same jobs on the step-mode row splits
        for (int j = 0; j <= J; ++j)
            if (c->lv[j].fbgrid > 0) {
                sj[j].L.grid = c->lv[j].fbgrid;
                sj[j].L.part = c->lv[j].fbpart;
            }
        CK(hipMemcpyAsync(c->d_step_fb, sj.data(), sizeof(StepJob) * (J + 1), hipMemcpyHostToDevice, c->stream));
    }
    c->top = top;
    // single-workgroup levels: maximal runs of levels on the same kernel,
    // coarsest first; each run starts from the state its coarser level left
    c->h_bruns.clear();
    c->brun_kind.clear();
    auto block_kind = [&](int j) {
        const HostLevel& L = c->lv[j];
        if (L.bregs <= 0) return 0;
        int l = 0;
        while (l < kRegLayouts && !(kRegLayoutG[l] == L.lanes && kRegLayoutE[l] == L.bslots)) ++l;
        return 1 + 3 * l + (bitlen((unsigned)L.bregs) - 1);
    };
    for (int j = top; top >= 0 && j >= c->block_lo;) {
        const int kind = block_kind(j);
        int lo = j;
        while (lo - 1 >= c->block_lo && block_kind(lo - 1) == kind) --lo;
        BlockJob bj{};
        bj.lv = c->d_lv;
        bj.st = c->d_st;
        bj.tol = o.tol;
        bj.seed = o.seed;
        bj.maxit = o.max_iters_per_level;
        bj.jhi = j;
        bj.jlo = lo;
        bj.uniform = (!c->coarse_dense && j == J) ? 1 : 0;
        c->h_bruns.push_back(bj);
        c->brun_kind.push_back(kind);
        j = lo - 1;
    }
    if (!c->h_bruns.empty()) {
        ALLOC(c->d_bruns, BlockJob, c->h_bruns.size());
        CK(hipMemcpyAsync(c->d_bruns, c->h_bruns.data(), sizeof(BlockJob) * c->h_bruns.size(), hipMemcpyHostToDevice,
                          c->stream));
    }
    c->h_st.resize(J + 1);
    {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            c->clock_khz = khz;
    }
    if (!c->noalloc) {
        c->events.resize(2 * (J + 1));
        for (auto& e : c->events) CK(hipEventCreate(&e));
    }
    CK(hipStreamSynchronize(c->stream));
    if (lt_flags) c->dfree_direct(lt_flags);
    return CMG_OK;
}

cmg_status setup_impl(cmg_ctx* c, int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                      const void* w, cmg_valtype wtype, cmg_memspace where) {
    Range range("cmg_setup");
    hipStream_t s = c->stream;
    // first arena chunk: level 0's CSR copy, vectors and refinement state
    // plus the coarser levels (together about half of level 0)
    c->achunk = (size_t)(12 * nnz + 48 * (int64_t)n) + ((size_t)2 << 20);
    HostLevel L0;
    L0.n = n;
    L0.nnz = nnz;
    ALLOC(L0.rp, int32_t, n + 1);
    ALLOC(L0.col, int32_t, nnz);
    ALLOC(L0.w64, double, nnz);
    const hipMemcpyKind kind = (where == CMG_MEM_HOST) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    CK(hipMemcpyAsync(L0.rp, row_ptr, sizeof(int32_t) * (n + 1), kind, s));
    CK(hipMemcpyAsync(L0.col, col, sizeof(int32_t) * nnz, kind, s));
    const int wf32 = (wtype == CMG_VAL_F32);
    const void* wdev = w;
    void* wtmp = nullptr;
    if (wf32) {
        if (where == CMG_MEM_HOST) {
            wtmp = c->dalloc_direct(sizeof(float) * nnz);
            if (!wtmp) return CMG_E_OOM;
            CK(hipMemcpyAsync(wtmp, w, sizeof(float) * nnz, hipMemcpyHostToDevice, s));
            wdev = wtmp;
        }
        CK(launch_convert_w(nnz, wdev, 1, L0.w64, s));
    } else {
        CK(hipMemcpyAsync(L0.w64, w, sizeof(double) * nnz, kind, s));
    }
    // validation (on the handle's copy)
    unsigned* vf = (unsigned*)c->dalloc_direct(sizeof(unsigned) * 4);
    if (!vf) return CMG_E_OOM;
    CK(hipMemsetAsync(vf, 0, 2 * sizeof(unsigned), s));
    CK(launch_validate(n, nnz, L0.rp, L0.col, L0.w64, 0, c->opt.validate_full, vf, s));
    unsigned vres[2] = {0u, 0u};
    cmg_status st = d2h(c, vres, vf, 2);
    const unsigned flags = vres[0];
    c->maxlen0 = vres[1];
    c->dfree_direct(vf);
    if (wtmp) c->dfree_direct(wtmp);
    if (st != CMG_OK) return st;
    if (flags & (kBadGraph | kAsym)) return CMG_E_GRAPH;
    if (flags & kIsolated) return CMG_E_ISOLATED;
    c->int_weights = (flags & kWideWeight) == 0;
    L0.wunit = (flags & kNonUnit) == 0;
    L0.lanes = pick_lanes(nnz / (double)n);
    c->lv.push_back(L0);
    SetupTmp t;
    st = alloc_tmp(c, t, n, nnz);
    if (st != CMG_OK) return st;
    int j = 0;
    bool grid_only = false;  // a level the single-workgroup chain handed back
    while (c->lv[j].n > c->opt.coarsest_n && j < 63) {
        // the single-workgroup chain implements HEC only
        if (!grid_only && c->opt.coarsen == 0 && chain_level(c->lv[j])) {
            int next = -1;
            st = coarsen_chain(c, t, j, &next);
            if (st != CMG_OK) return st;
            if (next < 0) break;
            j = next;
            grid_only = true;
            continue;
        }
        grid_only = false;
        bool stop = false;
        st = coarsen_once(c, t, j, &stop);
        if (st != CMG_OK) return st;
        if (stop) break;
        ++j;
    }
    // row information of the coarsest level (not yet computed if the loop
    // ended on the size test), then of every level at once
    {
        const int J = (int)c->lv.size() - 1;
        const bool have = c->lv[J].g != 0.0 ||
                          std::find(t.ri_pending.begin(), t.ri_pending.end(), J) != t.ri_pending.end();
        if (!have) {
            st = level_rowinfo(c, t, J);
            if (st != CMG_OK) return st;
        }
        st = finish_rowinfo(c, t);
        if (st != CMG_OK) return st;
    }
    free_tmp(c, t);
    return build_refine_plan(c);
}

void fill_defaults(cmg_options* o) {
    std::memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(cmg_options);
    o->tol = 1e-8;
    o->coarsest_n = 25;
    o->dense_max = 128;
    o->seed = 14120565ull;
    o->precision = CMG_FP64;
    o->fp64_final_sweeps = 1;
    o->max_iters_per_level = 100000;
    o->validate_full = 0;
    o->stream = nullptr;
    o->allocator = nullptr;
    o->block_rows = 0;
    o->mixed_min_nnz = 0;
    o->spmv_variant = 0;
    o->autotune = 0;
    o->block_regs = 0;
    o->grid_stage = 1;
    o->step_mode = 0;
    o->fixed_k0 = 0;
    o->fixed_beta = 2.0;
    o->graph = 0;
    o->coarsen = 0;
    o->galerkin = 0;
    o->test_abort_level = -1;
}

// Device results of the last solve -> host staging (asynchronous).
cmg_status enqueue_readback(cmg_ctx* c, void* x, cmg_memspace where, hipStream_t s) {
    const int J = (int)c->lv.size() - 1;
    CK(hipMemcpyAsync(&c->h_fo, c->d_fo, sizeof(FinishOut), hipMemcpyDeviceToHost, s));
    CK(hipMemcpyAsync(c->h_st.data(), c->d_st, sizeof(LevelState) * (J + 1), hipMemcpyDeviceToHost, s));
    CK(hipMemcpyAsync(&c->h_gs, c->d_sync, sizeof(GridSync), hipMemcpyDeviceToHost, s));
    if (x) {
        CK(hipMemcpyAsync(x, c->d_y, sizeof(double) * c->lv[0].n,
                          where == CMG_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
    }
    return CMG_OK;
}

// After the stream has drained: statistics, status, lambda.
cmg_status finalize(cmg_ctx* c, double t0, bool timed, double* lambda, cmg_stats* stats) {
    const int J = (int)c->lv.size() - 1;
    if (c->h_gs.abort) {
        const int tag = (int)(c->h_gs.where >> 16) - 2;
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "grid barrier timed out (%s %d, %u workgroups, barrier epoch %llu, last %llu)",
                      tag < 0 ? "finishing pass" : "level", tag < 0 ? 0 : tag, c->h_gs.where & 0xffffu,
                      c->h_gs.abort_epoch, c->h_gs.epoch);
        // barrier state is unusable: start the epoch sequence afresh
        CK(launch_reset_sync(c->d_sync, c->d_slots, c->nslots, c->d_bcast, c->stream));
        CK(hipStreamSynchronize(c->stream));
        return CMG_E_DEVICE;
    }
    cmg_status status = CMG_OK;
    for (int j = 0; j <= J; ++j) {
        HostLevel& L = c->lv[j];
        if (j == J && c->coarse_dense) {
            L.k = -1;
            L.margin = 0.0;
        } else {
            L.k = c->h_st[j].k;
            L.margin = c->h_st[j].margin;
            // a fixed schedule ends every level at its step count by design
            if (c->h_st[j].maxit && L.kfix == 0) status = CMG_W_MAXIT;
            if (L.in_block && c->h_st[j].err) {
                if (c->h_st[j].err == 2)
                    std::snprintf(g_last_error, sizeof(g_last_error),
                                  "level %d: register layout (%d lanes, %d rows per group, %d slots, %d waves) does "
                                  "not fit the level",
                                  j, L.lanes, L.bregs, L.bslots, L.bwaves);
                else
                    std::snprintf(g_last_error, sizeof(g_last_error),
                                  "level %d: the entries of rows longer than the register layout (%d slots of %d "
                                  "lanes) do not fit the LDS left",
                                  j, L.bslots, L.lanes);
                return CMG_E_DEVICE;
            }
        }
        L.pi_ms = 0.0;
        if (L.in_block && c->h_st[j].ticks > 0) L.pi_ms = c->h_st[j].ticks / c->clock_khz;
        if (timed && !L.in_block && j <= c->top) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, c->events[2 * j], c->events[2 * j + 1]) == hipSuccess) L.pi_ms = ms;
        }
    }
    const FinishOut& fo = c->h_fo;
    if (lambda) *lambda = fo.lambda;
    cmg_stats& st = c->last;
    std::memset(&st, 0, sizeof(st));
    st.struct_size = sizeof(cmg_stats);
    st.nlevels = J + 1;
    st.collapsed = c->collapsed;
    st.hec_rounds = c->hec_rounds;
    st.lambda = fo.lambda;
    st.residual = fo.residual;
    st.coarse_lambda2 = c->coarse_dense ? fo.coarse_lambda2 : 0.0;
    st.coarse_mult = c->coarse_dense ? fo.coarse_mult : 0;
    st.setup_ms = c->setup_ms;
    st.fiedler_ms = now_ms() - t0;
    st.finest_pi_ms = c->lv[0].pi_ms;
    st.finest_k = c->lv[0].k;
    {
        const HostLevel& L = c->lv[0];
        double sv = L.fp32 ? 4 : 8;
        double bpi = 4.0 * (L.n + 1) + (double)L.nnz * (4 + sv) + 2 * sv * L.n;
        st.finest_bytes = L.k > 0 ? L.k * bpi : 0.0;
    }
    st.status = status;
    if (stats) {
        uint32_t sz = stats->struct_size ? stats->struct_size : (uint32_t)sizeof(cmg_stats);
        std::memcpy(stats, &st, std::min<size_t>(sz, sizeof(cmg_stats)));
    }
    return status;
}

// A level refined with one launch per PI step.  The step count is decided
// on the device, so steps go out in chunks of kStepChunk with one chunk
// queued behind the one whose done flag the host waits for.  Steps
// launched after the stopping test passed return at once.
cmg_status ensure_flags(cmg_ctx* c);

cmg_status run_step_level(cmg_ctx* c, int j, hipStream_t s, bool fallback = false) {
    const HostLevel& L = c->lv[j];
    const bool fb = fallback && !L.step;
    const StepJob* job = (fb ? c->d_step_fb : c->d_step) + j;
    const int grid = fb ? L.fbgrid : L.grid;
    const int kind = job_kind(L.variant, L.lanes, L.fp32, L.wk);
    const int maxit = c->opt.max_iters_per_level;
    CK(launch_step_begin(job, grid, kind, s));
    if (L.kfix > 0) {  // fixed schedule: the step count is known, no host checks
        for (int i = 0; i < L.kfix; ++i) CK(launch_step_pi(job, grid, kind, s));
        return CMG_OK;
    }
    cmg_status fst = ensure_flags(c);
    if (fst != CMG_OK) return fst;
    int launched = 0, chunks = 0;
    const int chunk = kStepChunk;
    auto enqueue = [&]() -> cmg_status {
        const int q = std::min(chunk, maxit - launched);
        for (int i = 0; i < q; ++i) CK(launch_step_pi(job, grid, kind, s));
        launched += q;
        CK(hipMemcpyAsync(c->h_flags + chunks % kChunkEvents, &c->d_ctl->done, sizeof(int), hipMemcpyDeviceToHost, s));
        CK(hipEventRecord(c->chunk_ev[chunks % kChunkEvents], s));
        ++chunks;
        return CMG_OK;
    };
    // two chunks queued; each one the host sees finish without the stopping
    // test passed is replaced by another, so the device never waits for the
    // host and at most two chunks of steps run empty
    cmg_status st = enqueue();
    if (st != CMG_OK) return st;
    if (launched < maxit) {
        st = enqueue();
        if (st != CMG_OK) return st;
    }
    for (int w = 0;; ++w) {
        CK(hipEventSynchronize(c->chunk_ev[w % kChunkEvents]));
        if (c->h_flags[w % kChunkEvents]) break;  // done at or before chunk w
        if (w + 1 == chunks && launched >= maxit) break;
        if (launched < maxit) {
            st = enqueue();
            if (st != CMG_OK) return st;
        }
    }
    return CMG_OK;
}

// The launches of a solve after the coarsest solve: the single-workgroup
// runs, the grid levels coarse to fine, the finishing pass.  timed: events
// around each grid level (not inside a captured graph).
cmg_status enqueue_refine(cmg_ctx* c, hipStream_t s, bool timed, bool fallback = false) {
    const int J = (int)c->lv.size() - 1;
    for (size_t r = 0; r < c->h_bruns.size(); ++r) CK(launch_block_jobs(c->d_bruns + r, 1, c->brun_kind[r], s));
    // grid levels: one persistent launch per level (one launch per step in
    // step mode, and on the fallback after a barrier wait was given up)
    for (int j = std::min(c->top, c->block_lo - 1); j >= 0; --j) {
        const HostLevel& L = c->lv[j];
        Range range("cmg refine level %d", j);
        if (timed) CK(hipEventRecord(c->events[2 * j], s));
        if (L.step || (fallback && L.fbgrid > 0)) {
            cmg_status st = run_step_level(c, j, s, fallback);
            if (st != CMG_OK) return st;
        } else {
            if (!fallback && j == c->opt.test_abort_level) CK(launch_raise_abort(c->d_sync, s));
            CK(launch_refine_jobs(c->d_jobs + j, 1, L.grid, job_kind(L.variant, L.lanes, L.fp32, L.wk), s));
        }
        if (timed) CK(hipEventRecord(c->events[2 * j + 1], s));
    }
    const HostLevel& L0 = c->lv[0];
    CK(launch_finish_jobs(c->d_jobs + J + 1, 1, L0.step ? L0.fgrid : L0.grid, job_kind(L0.variant, L0.lanes, L0.fp32, L0.wk),
                          s));
    return CMG_OK;
}

// The launch sequence is fixed when no level decides its step count on the
// host: a fixed schedule, or no level refined one launch per step.
bool static_sequence(const cmg_ctx* c) {
    if (c->fixed) return true;
    for (int j = std::min(c->top, c->block_lo - 1); j >= 0; --j)
        if (c->lv[j].step) return false;
    return true;
}

// Records enqueue_refine into c->gexec.  The capture runs on a private
// stream (the null stream cannot be captured); the graph is launched on the
// handle's stream.  Kernels only: no memset or copy nodes.
cmg_status capture_refine(cmg_ctx* c) {
    hipStream_t cs = nullptr;
    CK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    cmg_status st = CMG_OK;
    if (e == hipSuccess) st = enqueue_refine(c, cs, false);
    hipGraph_t g = nullptr;
    if (e == hipSuccess) {
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (st == CMG_OK && e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess && st == CMG_OK) e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (st != CMG_OK) return st;
    if (e != hipSuccess) {
        c->gexec = nullptr;
        set_error("graph capture", e, __LINE__);
        (void)hipGetLastError();
        return CMG_E_DEVICE;
    }
    return CMG_OK;
}

cmg_status fiedler_impl(cmg_ctx* c, double* lambda, void* x, cmg_memspace where, cmg_stats* stats) {
    Range range("cmg_fiedler");
    const double t0 = now_ms();
    hipStream_t s = c->stream;
    if (c->d_cjob && !c->coarse_done) {
        CK(launch_coarse_jobs(c->d_cjob, 1, s));
        c->coarse_done = true;
    }
    const bool graph = c->opt.graph && static_sequence(c);
    if (graph) {
        if (!c->gexec) {
            cmg_status st = capture_refine(c);
            if (st != CMG_OK) return st;
        }
        CK(hipGraphLaunch(c->gexec, s));
    } else {
        cmg_status st = enqueue_refine(c, s, !c->noalloc);
        if (st != CMG_OK) return st;
    }
    cmg_status st = enqueue_readback(c, x, where, s);
    if (st != CMG_OK) return st;
    CK(hipStreamSynchronize(s));
    bool fell_back = false;
    if (c->h_gs.abort && c->d_step_fb) {
        // a grid barrier's bounded wait was given up (workgroups of a
        // persistent level not all resident, e.g. kernels of other streams
        // holding compute units): every launch has exited; re-run the
        // refinement with the persistent rows-traversal levels one launch
        // per step, which needs no inter-workgroup waits
        CK(launch_reset_sync(c->d_sync, c->d_slots, c->nslots, c->d_bcast, s));
        st = enqueue_refine(c, s, !c->noalloc, true);
        if (st != CMG_OK) return st;
        st = enqueue_readback(c, x, where, s);
        if (st != CMG_OK) return st;
        CK(hipStreamSynchronize(s));
        ++c->fallbacks;
        fell_back = true;
    }
    st = finalize(c, t0, !graph && !c->noalloc, lambda, stats);
    if (stats && stats->struct_size >= offsetof(cmg_stats, fallback) + sizeof(int32_t))
        stats->fallback = fell_back ? 1 : 0;
    return st;
}

// ---- several eigenpairs (Remark after Algorithm 4)

cmg_status ensure_flags(cmg_ctx* c) {
    if (c->h_flags) return CMG_OK;
    CK(hipHostMalloc((void**)&c->h_flags, sizeof(int) * kChunkEvents, hipHostMallocDefault));
    c->chunk_ev.resize(kChunkEvents);
    for (auto& e : c->chunk_ev) CK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return CMG_OK;
}

// Buffers and job table of the block refinement for p columns (once per p).
cmg_status blk_plan(cmg_ctx* c, int p) {
    if (c->blk_p == p) return CMG_OK;
    const int J = (int)c->lv.size() - 1;
    hipStream_t s = c->stream;
    std::vector<BlkJob> jobs(J + 1);
    int maxnb = 1;
    ALLOC(c->d_blk_ctl, BlkCtl, J + 1);
    ALLOC(c->d_blk_out, BlkOut, 1);
    ALLOC(c->d_blk_x, double, (size_t)c->lv[0].n * p);
    for (int j = 0; j <= J; ++j) {
        const HostLevel& L = c->lv[j];
        BlkJob b{};
        b.n = L.n;
        const int64_t nb = ((int64_t)L.n + L.nnz + kStepWork - 1) / kStepWork;
        b.nb = (int)std::min<int64_t>(std::max<int64_t>(nb, 1), 65535);
        maxnb = std::max(maxnb, b.nb);
        b.rp = L.rp;
        b.col = L.col;
        b.w = L.w64;
        b.g = L.g;
        b.agg = L.agg;
        ALLOC(b.W0, double, (size_t)L.n * p);
        ALLOC(b.W1, double, (size_t)L.n * p);
        b.ctl = c->d_blk_ctl + j;
        int32_t* rpart = nullptr;
        ALLOC(rpart, int32_t, b.nb + 1);
        CK(launch_partition(L.n, L.nnz, L.rp, b.nb, rpart, s));
        b.rpart = rpart;
        b.out = c->d_blk_out;
        b.tol = c->opt.tol;
        b.seed = c->opt.seed;
        b.maxit = c->opt.max_iters_per_level;
        b.kfix = L.kfix;
        jobs[j] = b;
    }
    double* part = nullptr;
    ALLOC(part, double, (size_t)maxnb * blk_parts(p));
    for (int j = 0; j <= J; ++j) {
        jobs[j].part = part;
        if (j < J) {
            jobs[j].cW0 = jobs[j + 1].W0;
            jobs[j].cW1 = jobs[j + 1].W1;
            jobs[j].cctl = jobs[j + 1].ctl;
        }
    }
    ALLOC(c->d_blk_jobs, BlkJob, J + 1);
    CK(hipMemcpyAsync(c->d_blk_jobs, jobs.data(), sizeof(BlkJob) * (J + 1), hipMemcpyHostToDevice, s));
    c->blk_jobs = jobs;
    c->blk_p = p;
    return CMG_OK;
}

// Steps of block level j: all at once on a fixed schedule, else in chunks
// with one queued ahead while the host reads the done flag (as step mode).
cmg_status blk_steps(cmg_ctx* c, int j, int p, hipStream_t s) {
    const BlkJob& hj = c->blk_jobs[j];
    const BlkJob* dj = c->d_blk_jobs + j;
    if (hj.kfix > 0) {
        for (int i = 0; i < hj.kfix; ++i) CK(launch_blk(kBlkStep, p, dj, hj, nullptr, nullptr, nullptr, nullptr, s));
        return CMG_OK;
    }
    cmg_status st = ensure_flags(c);
    if (st != CMG_OK) return st;
    const int maxit = hj.maxit;
    int launched = 0, chunks = 0;
    auto enqueue = [&]() -> cmg_status {
        const int q = std::min(kStepChunk, maxit - launched);
        for (int i = 0; i < q; ++i) CK(launch_blk(kBlkStep, p, dj, hj, nullptr, nullptr, nullptr, nullptr, s));
        launched += q;
        CK(hipMemcpyAsync(c->h_flags + chunks % kChunkEvents, &hj.ctl->done, sizeof(int), hipMemcpyDeviceToHost,
                          s));
        CK(hipEventRecord(c->chunk_ev[chunks % kChunkEvents], s));
        ++chunks;
        return CMG_OK;
    };
    st = enqueue();
    if (st != CMG_OK) return st;
    if (launched < maxit) {
        st = enqueue();
        if (st != CMG_OK) return st;
    }
    for (int w = 0;; ++w) {
        CK(hipEventSynchronize(c->chunk_ev[w % kChunkEvents]));
        if (c->h_flags[w % kChunkEvents]) break;
        if (w + 1 == chunks && launched >= maxit) break;
        if (launched < maxit) {
            st = enqueue();
            if (st != CMG_OK) return st;
        }
    }
    return CMG_OK;
}

cmg_status block_impl(cmg_ctx* c, int p, double* lambdas, void* X, cmg_memspace where, double* residuals,
                      int32_t* level_steps) {
    const int J = (int)c->lv.size() - 1;
    if (!c->coarse_dense || p < 1 || p > kBlkMaxP || p > c->lv[J].n - 1) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "cmg_fiedler_block: p = %d needs 1 <= p <= %d and p < the coarsest level's %d vertices, "
                      "solved densely (n <= dense_max)",
                      p, kBlkMaxP, c->lv[J].n);
        return CMG_E_ARG;
    }
    hipStream_t s = c->stream;
    if (!c->coarse_done) {
        CK(launch_coarse_jobs(c->d_cjob, 1, s));
        c->coarse_done = true;
    }
    cmg_status st = blk_plan(c, p);
    if (st != CMG_OK) return st;
    CK(launch_blk(kBlkCoarse, p, nullptr, c->blk_jobs[J], nullptr, c->d_V, c->d_ev, c->d_idx, s));
    for (int j = J - 1; j >= 0; --j) {
        CK(launch_blk(kBlkProlong, p, c->d_blk_jobs + j, c->blk_jobs[j], nullptr, nullptr, nullptr, nullptr, s));
        st = blk_steps(c, j, p, s);
        if (st != CMG_OK) return st;
    }
    CK(launch_blk(kBlkOut, p, c->d_blk_jobs, c->blk_jobs[0], c->d_blk_x, nullptr, nullptr, nullptr, s));
    BlkOut out{};
    std::vector<BlkCtl> ctl(J + 1);
    CK(hipMemcpyAsync(&out, c->d_blk_out, sizeof(out), hipMemcpyDeviceToHost, s));
    CK(hipMemcpyAsync(ctl.data(), c->d_blk_ctl, sizeof(BlkCtl) * (J + 1), hipMemcpyDeviceToHost, s));
    if (X)
        CK(hipMemcpyAsync(X, c->d_blk_x, sizeof(double) * (size_t)c->lv[0].n * p,
                          where == CMG_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
    CK(hipStreamSynchronize(s));
    cmg_status status = CMG_OK;
    for (int j = 0; j < J; ++j) {
        if (ctl[j].hit == 2) {
            std::snprintf(g_last_error, sizeof(g_last_error),
                          "cmg_fiedler_block: level %d: the block lost rank (Gram matrix not positive definite)", j);
            return CMG_E_DEVICE;
        }
        if (ctl[j].hit == 1) status = CMG_W_MAXIT;
    }
    for (int q = 0; q < p; ++q) {
        if (lambdas) lambdas[q] = out.lambda[q];
        if (residuals) residuals[q] = out.residual[q];
    }
    if (level_steps)
        for (int j = 0; j <= J; ++j) level_steps[j] = j == J ? -1 : ctl[j].k;
    return status;
}

// ---- recursive spectral bisection

cmg_status bisect_impl(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, const void* w,
                       cmg_valtype wtype, cmg_memspace where, const cmg_options& o, int32_t depth, int32_t* part_out,
                       double* cut) {
    cmg_ctx c;  // allocation helper: its direct allocations go back when it ends
    c.opt = o;
    c.stream = (hipStream_t)o.stream;
    if (o.allocator) c.alloc = *o.allocator;
    hipStream_t s = c.stream;
    const hipMemcpyKind kind = where == CMG_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const int64_t nsc = sort_tmp_elems(n);
    const int maxp = 1 << depth;
    auto take = [&](size_t bytes) { return c.dalloc_direct(bytes); };
    int32_t* rp = (int32_t*)take(sizeof(int32_t) * ((size_t)n + 1));
    int32_t* cl = (int32_t*)take(sizeof(int32_t) * (size_t)nnz);
    double* wd = (double*)take(sizeof(double) * (size_t)nnz);
    void* wtmp = wtype == CMG_VAL_F32 ? take(sizeof(float) * (size_t)nnz) : nullptr;
    unsigned* vf = (unsigned*)take(sizeof(unsigned) * 4);
    int32_t* part = (int32_t*)take(sizeof(int32_t) * (size_t)n);
    int32_t* next = (int32_t*)take(sizeof(int32_t) * (size_t)n);
    int32_t* perm = (int32_t*)take(sizeof(int32_t) * (size_t)n);
    int32_t* pos = (int32_t*)take(sizeof(int32_t) * (size_t)n);
    int32_t* deg = (int32_t*)take(sizeof(int32_t) * (size_t)n);
    int32_t* eoff = (int32_t*)take(sizeof(int32_t) * (size_t)n);
    int32_t* comp = (int32_t*)take(sizeof(int32_t) * (size_t)n);
    int32_t* rpl = (int32_t*)take(sizeof(int32_t) * ((size_t)n + maxp));
    int32_t* colk = (int32_t*)take(sizeof(int32_t) * (size_t)nnz);
    double* wk = (double*)take(sizeof(double) * (size_t)nnz);
    double* X = (double*)take(sizeof(double) * (size_t)n);
    unsigned long long* k0 = (unsigned long long*)take(sizeof(unsigned long long) * (size_t)n);
    unsigned long long* k1 = (unsigned long long*)take(sizeof(unsigned long long) * (size_t)n);
    double* v0 = (double*)take(sizeof(double) * (size_t)n);
    double* v1 = (double*)take(sizeof(double) * (size_t)n);
    int32_t* scounts = (int32_t*)take(sizeof(int32_t) * (size_t)nsc);
    long long* sscan = (long long*)take(sizeof(long long) * (size_t)(scan_tmp_elems(nsc) + 4));
    long long* stmp = (long long*)take(sizeof(long long) * (size_t)(scan_tmp_elems(n) + 4));
    int32_t* meta = (int32_t*)take(sizeof(int32_t) * 6 * (size_t)maxp);  // first, cnt, pnnz, pbase, ncomp, mode
    int* chg = (int*)take(sizeof(int) * 4);
    double* bsum = (double*)take(sizeof(double) * (size_t)rsb_cut_blocks(n));
    if (!rp || !cl || !wd || (wtype == CMG_VAL_F32 && !wtmp) || !vf || !part || !next || !perm || !pos || !deg ||
        !eoff || !comp || !rpl || !colk || !wk || !X || !k0 || !k1 || !v0 || !v1 || !scounts || !sscan || !stmp ||
        !meta || !chg || !bsum)
        return CMG_E_OOM;
    int32_t *first = meta, *cnt = meta + maxp, *pnnz = meta + 2 * maxp, *pbase = meta + 3 * maxp,
            *ncomp = meta + 4 * maxp, *mode = meta + 5 * maxp;
    // the graph, checked as cmg_setup checks it
    CK(hipMemcpyAsync(rp, row_ptr, sizeof(int32_t) * ((size_t)n + 1), kind, s));
    CK(hipMemcpyAsync(cl, col, sizeof(int32_t) * (size_t)nnz, kind, s));
    if (wtype == CMG_VAL_F32) {
        CK(hipMemcpyAsync(wtmp, w, sizeof(float) * (size_t)nnz, kind, s));
        CK(launch_convert_w(nnz, wtmp, 1, wd, s));
    } else {
        CK(hipMemcpyAsync(wd, w, sizeof(double) * (size_t)nnz, kind, s));
    }
    CK(launch_fill_u32(vf, 0u, 2, s));
    CK(launch_validate(n, nnz, rp, cl, wd, 0, o.validate_full, vf, s));
    unsigned vres[2] = {0u, 0u};
    cmg_status st = d2h(&c, vres, vf, 2);
    if (st != CMG_OK) return st;
    if (vres[0] & (kBadGraph | kAsym)) return CMG_E_GRAPH;
    if (vres[0] & kIsolated) return CMG_E_ISOLATED;
    CK(launch_fill_u32((unsigned*)part, 0u, n, s));
    std::vector<int32_t> hm(6 * (size_t)maxp);
    int hchg = 0;
    cmg_options so = o;  // options of every sub-solve
    so.allocator = o.allocator;
    for (int d = 0; d < depth; ++d) {
        const int np = 1 << d;
        // vertices grouped by part, ascending index inside a part
        CK(launch_rsb_keys(n, part, k0, s));
        int second = 0;
        CK(launch_sort(k0, nullptr, k1, nullptr, n, 32, std::max(d, 1), scounts, sscan, &second, s));
        const unsigned long long* ks = second ? k1 : k0;
        CK(launch_fill_u32((unsigned*)meta, 0u, 6 * (int64_t)maxp, s));
        CK(launch_rsb_perm(n, ks, perm, pos, first, comp, s));
        // induced subgraphs: rows in position order, local columns
        CK(launch_rsb_deg(n, rp, cl, part, perm, deg, s));
        CK(launch_scan(deg, eoff, n, stmp, stmp + scan_tmp_elems(n), s));
        CK(launch_rsb_fill(n, rp, cl, wd, part, perm, pos, first, eoff, rpl, colk, wk, cnt, pnnz, pbase, s));
        CK(launch_rsb_components(n, rpl, colk, part, perm, first, eoff, comp, chg, &hchg, s));
        CK(launch_rsb_roots(n, comp, part, perm, ncomp, s));
        st = d2h(&c, hm.data(), meta, 5 * (size_t)maxp);
        if (st != CMG_OK) return st;
        // connected parts of two vertices or more: Fiedler vectors in one batch
        std::vector<cmg_handle> hs;
        std::vector<void*> xs;
        for (int p = 0; p < np; ++p) {
            const int m = hm[maxp + p], comps = hm[4 * maxp + p];
            hm[5 * maxp + p] = m < 2 ? 0 : comps == 1 ? 1 : 2;
        }
        CK(hipMemcpyAsync(mode, hm.data() + 5 * maxp, sizeof(int32_t) * maxp, hipMemcpyHostToDevice, s));
        st = CMG_OK;
        for (int p = 0; p < np && st == CMG_OK; ++p) {
            if (hm[5 * maxp + p] != 1) continue;
            const int f = hm[p], m = hm[maxp + p], z = hm[2 * maxp + p], base = hm[3 * maxp + p];
            cmg_handle h = nullptr;
            st = cmg_setup(m, z, rpl + f + p, colk + base, wk + base, CMG_VAL_F64, CMG_MEM_DEVICE, &so, &h);
            if (st == CMG_OK) {
                hs.push_back(h);
                xs.push_back(X + f);
            }
        }
        if (st == CMG_OK && !hs.empty()) {
            st = cmg_fiedler_batch(hs.data(), (int32_t)hs.size(), nullptr, xs.data(), CMG_MEM_DEVICE, nullptr);
            if (st == CMG_W_MAXIT) st = CMG_OK;
        }
        for (cmg_handle h : hs) cmg_free(h);
        if (st != CMG_OK) return st;
        // split every part at its median: stable sort by key, then by part
        CK(launch_rsb_split_keys(n, X, comp, part, perm, mode, k0, v0, s));
        CK(launch_sort(k0, v0, k1, v1, n, 0, 64, scounts, sscan, &second, s));
        const double* vs = second ? v1 : v0;
        double* vo = second ? v0 : v1;
        unsigned long long* kp = second ? k0 : k1;
        unsigned long long* kq = second ? k1 : k0;
        CK(launch_rsb_part_keys(n, vs, part, perm, kp, s));
        CK(launch_sort(kp, (double*)vs, kq, vo, n, 32, std::max(d, 1), scounts, sscan, &second, s));
        const double* fin = second ? vo : vs;
        CK(launch_rsb_assign(n, fin, part, perm, first, cnt, mode, next, s));
        std::swap(part, next);
    }
    CK(hipMemcpyAsync(part_out, part, sizeof(int32_t) * (size_t)n,
                      where == CMG_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
    if (cut) {
        const int nb = rsb_cut_blocks(n);
        std::vector<double> hb(nb);
        CK(launch_rsb_cut(n, rp, cl, wd, part, bsum, s));
        st = d2h(&c, hb.data(), bsum, nb);
        if (st != CMG_OK) return st;
        double t = 0.0;
        for (double x : hb) t += x;
        *cut = 0.5 * t;
    }
    CK(hipStreamSynchronize(s));
    return CMG_OK;
}

// Several graphs: every stage of all graphs in packed launches (one
// workgroup per graph for the coarsest solve and the coarse levels; for
// the grid levels, round r refines the r-th grid level, counted from the
// coarse end, of every graph that has one, jobs packed up to the
// co-resident capacity).  Each job runs the same code on the same
// workgroup count as a single solve, so results are bitwise identical.
cmg_status batch_impl(cmg_handle* hs, int32_t count, double* lambdas, void** xs, cmg_memspace where,
                      cmg_stats* stats) {
    const double t0 = now_ms();
    cmg_ctx* c0 = hs[0];
    hipStream_t s = c0->stream;
    std::vector<CoarseJob> cj;
    // single-workgroup runs: round q holds the q-th run of every graph,
    // grouped by kernel
    std::vector<BlockJob> bj;
    std::vector<std::pair<int, int>> blaunch;  // (kernel, jobs) in launch order
    int maxrounds = 0;
    size_t maxruns = 0;
    for (int i = 0; i < count; ++i) {
        cmg_ctx* c = hs[i];
        if (c->d_cjob && !c->coarse_done) cj.push_back(c->h_cjob);
        maxruns = std::max(maxruns, c->h_bruns.size());
        maxrounds = std::max(maxrounds, std::min(c->top, c->block_lo - 1) + 1);
    }
    for (size_t q = 0; q < maxruns; ++q) {
        for (int kind = 0; kind < kBlockKinds; ++kind) {
            int nk = 0;
            for (int i = 0; i < count; ++i) {
                const cmg_ctx* c = hs[i];
                if (q < c->h_bruns.size() && c->brun_kind[q] == kind) {
                    bj.push_back(c->h_bruns[q]);
                    ++nk;
                }
            }
            if (nk > 0) blaunch.push_back({kind, nk});
        }
    }
    // device tables: coarse | block | grid rounds | finish
    std::vector<GridJob> gj;
    std::vector<std::pair<size_t, int>> launches;  // (offset in gj, njobs), with kind below
    std::vector<int> launch_blocks;
    std::vector<int> launch_kind;  // 0 refine, 1 finish
    std::vector<int> launch_jk;    // job kernel kind
    auto pack = [&](std::vector<GridJob>& round, int kind) {
        // one launch per job kernel kind, jobs packed up to its co-resident capacity
        for (int jk = 0; jk < kJobKinds; ++jk) {
            std::vector<GridJob> sel;
            for (const GridJob& g : round)
                if (job_kind(g.L.variant, g.L.lanes, g.L.fp32, g.L.wk) == jk) sel.push_back(g);
            const int cap = kind ? finish_jobs_max_blocks(jk) : refine_jobs_max_blocks(jk);
            size_t i = 0;
            while (i < sel.size()) {
                size_t first = gj.size();
                int blocks = 0, nj = 0;
                while (i < sel.size() && (nj == 0 || blocks + sel[i].L.grid <= cap)) {
                    GridJob g = sel[i];
                    g.b0 = blocks;
                    blocks += g.L.grid;
                    gj.push_back(g);
                    ++nj;
                    ++i;
                }
                launches.push_back({first, nj});
                launch_blocks.push_back(blocks);
                launch_kind.push_back(kind);
                launch_jk.push_back(jk);
            }
        }
    };
    // per round: its packed launches, then the step-by-step levels
    std::vector<size_t> round_end;
    std::vector<std::vector<std::pair<int, int>>> step_runs(maxrounds);
    for (int r = 0; r < maxrounds; ++r) {
        std::vector<GridJob> round;
        for (int i = 0; i < count; ++i) {
            cmg_ctx* c = hs[i];
            const int lo = std::min(c->top, c->block_lo - 1);  // coarsest grid level
            const int j = lo - r;
            if (lo < 0 || j < 0) continue;
            if (c->lv[j].step) step_runs[r].push_back({i, j});
            else round.push_back(c->h_jobs[j]);
        }
        pack(round, 0);
        round_end.push_back(launches.size());
    }
    {
        std::vector<GridJob> round;
        for (int i = 0; i < count; ++i) round.push_back(hs[i]->h_jobs[hs[i]->lv.size()]);
        pack(round, 1);
    }
    const size_t bytes = sizeof(CoarseJob) * cj.size() + sizeof(BlockJob) * bj.size() + sizeof(GridJob) * gj.size();
    char* d = (char*)c0->dalloc_direct(bytes + 64);
    if (!d) return CMG_E_OOM;
    std::vector<char> h(bytes);
    size_t off = 0;
    std::memcpy(h.data() + off, cj.data(), sizeof(CoarseJob) * cj.size());
    CoarseJob* d_cj = (CoarseJob*)(d + off);
    off += sizeof(CoarseJob) * cj.size();
    std::memcpy(h.data() + off, bj.data(), sizeof(BlockJob) * bj.size());
    BlockJob* d_bj = (BlockJob*)(d + off);
    off += sizeof(BlockJob) * bj.size();
    std::memcpy(h.data() + off, gj.data(), sizeof(GridJob) * gj.size());
    GridJob* d_gj = (GridJob*)(d + off);
    cmg_status status = CMG_OK;
    hipError_t e = hipMemcpyAsync(d, h.data(), bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !cj.empty()) {
        e = launch_coarse_jobs(d_cj, (int)cj.size(), s);
        if (e == hipSuccess)
            for (int i = 0; i < count; ++i) hs[i]->coarse_done = true;
    }
    {
        const BlockJob* q = d_bj;
        for (const auto& bl : blaunch) {
            if (e == hipSuccess) e = launch_block_jobs(q, bl.second, bl.first, s);
            q += bl.second;
        }
    }
    size_t q = 0;
    for (int r = 0; r <= maxrounds && e == hipSuccess && status == CMG_OK; ++r) {
        const size_t qend = (r < maxrounds) ? round_end[r] : launches.size();
        for (; e == hipSuccess && q < qend; ++q) {
            const GridJob* jp = d_gj + launches[q].first;
            e = launch_kind[q] ? launch_finish_jobs(jp, launches[q].second, launch_blocks[q], launch_jk[q], s)
                               : launch_refine_jobs(jp, launches[q].second, launch_blocks[q], launch_jk[q], s);
        }
        if (r < maxrounds)
            for (const auto& sr : step_runs[r]) {
                if (e != hipSuccess || status != CMG_OK) break;
                status = run_step_level(hs[sr.first], sr.second, s);
            }
    }
    for (int i = 0; e == hipSuccess && i < count && status == CMG_OK; ++i)
        status = enqueue_readback(hs[i], xs ? xs[i] : nullptr, where, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    c0->dfree_direct(d);
    if (e != hipSuccess) {
        set_error("batch launch", e, __LINE__);
        (void)hipGetLastError();
        return CMG_E_DEVICE;
    }
    if (status != CMG_OK) return status;
    cmg_status worst = CMG_OK;
    for (int i = 0; i < count; ++i) {
        cmg_status st = finalize(hs[i], t0, false, lambdas ? lambdas + i : nullptr, stats ? stats + i : nullptr);
        if (st != CMG_OK && st != CMG_W_MAXIT) return st;
        if (st == CMG_W_MAXIT) worst = st;
    }
    return worst;
}

// ---- the entry point that allocates nothing
//
// All device memory of a cmg_fiedler_noalloc call (hierarchy, setup
// temporaries, vectors, job tables, barrier state, and the buffers of a
// first residency count) is carved from `scratch`, a static array that each
// device holds for the life of the process.  Host code must not pass the
// array's name to kernels (it is a host-side stand-in); the device address
// comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
constexpr size_t kNoallocMeasureBytes = 4096;  // residency count buffers at the front
constexpr int kNoallocMaxDevices = 64;

static_assert(256 + sizeof(GridJob) <= kNoallocMeasureBytes, "residency count buffers");

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_noalloc_mu;
unsigned char* g_scratch_dev[kNoallocMaxDevices] = {};

// Scratch a graph of n vertices and nnz entries may need: the handle's
// arena (12 nnz + 48 n + 2 MiB, plus the coarse levels' share), the setup
// temporaries (about 40 nnz + 40 n) and the refinement state.
size_t noalloc_need(int32_t n, int64_t nnz) {
    return (size_t)64 * (size_t)nnz + (size_t)128 * (size_t)n + ((size_t)4 << 20);
}

struct Bump {
    unsigned char* base;
    size_t cap, off;
};

void* bump_alloc(size_t bytes, void*, void* user) {
    Bump* b = (Bump*)user;
    const size_t o = (b->off + 255) & ~(size_t)255;
    if (bytes > b->cap || o > b->cap - bytes) return nullptr;
    b->off = o + bytes;
    return b->base + o;
}

void bump_free(void*, void*, void*) {}

cmg_status noalloc_impl(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, const void* w,
                        cmg_valtype wtype, cmg_memspace where, const cmg_options& o, double* lambda, void* x,
                        cmg_stats* stats) {
    int dev = 0;
    CK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoallocMaxDevices) return CMG_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        CK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_dev[dev] = (unsigned char*)p;
    }
    unsigned char* base = g_scratch_dev[dev];
    Bump bump{base + kNoallocMeasureBytes, kNoallocScratchBytes - kNoallocMeasureBytes, 0};
    const cmg_allocator alloc{bump_alloc, bump_free, &bump};
    const MeasureBuffers mb{(unsigned*)base, (GridJob*)(base + 256), (hipStream_t)o.stream};
    set_measure_buffers(&mb);
    cmg_status st;
    {
        cmg_ctx c;
        c.opt = o;
        c.opt.allocator = nullptr;
        c.stream = (hipStream_t)o.stream;
        c.alloc = alloc;
        c.noalloc = true;
        const double t0 = now_ms();
        st = setup_impl(&c, n, nnz, row_ptr, col, w, wtype, where);
        c.setup_ms = now_ms() - t0;
        if (st == CMG_OK) st = fiedler_impl(&c, lambda, x, where, stats);
    }  // ~cmg_ctx waits for the stream; its frees are no-ops
    set_measure_buffers(nullptr);
    return st;
}

}  // namespace

// ================================================================== C ABI

extern "C" {

void cmg_options_default(cmg_options* o) {
    if (o) fill_defaults(o);
}

const char* cmg_last_error(void) { return g_last_error; }

const char* cmg_status_string(cmg_status s) {
    switch (s) {
        case CMG_OK: return "CMG_OK";
        case CMG_E_ARG: return "CMG_E_ARG: invalid argument";
        case CMG_E_GRAPH: return "CMG_E_GRAPH: invalid graph";
        case CMG_E_ISOLATED: return "CMG_E_ISOLATED: isolated vertex";
        case CMG_E_OOM: return "CMG_E_OOM: out of device memory";
        case CMG_E_DEVICE: return "CMG_E_DEVICE: device error";
        case CMG_W_MAXIT: return "CMG_W_MAXIT: iteration cap reached";
    }
    return "unknown status";
}

cmg_status cmg_setup(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, const void* w,
                     cmg_valtype wtype, cmg_memspace where, const cmg_options* opt, cmg_handle* out) {
    g_last_error[0] = 0;
    if (!out) return CMG_E_ARG;
    *out = nullptr;
    if (n < 2 || nnz < 1 || nnz >= 2147483647LL || !row_ptr || !col || !w) return CMG_E_ARG;
    if (wtype != CMG_VAL_F64 && wtype != CMG_VAL_F32) return CMG_E_ARG;
    if (where != CMG_MEM_HOST && where != CMG_MEM_DEVICE) return CMG_E_ARG;
    cmg_options o;
    fill_defaults(&o);
    if (opt) {
        size_t sz = opt->struct_size ? std::min<size_t>(opt->struct_size, sizeof(o)) : sizeof(o);
        std::memcpy(&o, opt, sz);
        o.struct_size = sizeof(o);
    }
    if (!(o.tol < 1.0) || !std::isfinite(o.tol) || o.coarsest_n < 2 || o.dense_max < 2 || o.dense_max > 128 ||
        o.max_iters_per_level < 1 || (o.precision != CMG_FP64 && o.precision != CMG_MIXED) ||
        o.fp64_final_sweeps < 0 || o.fp64_final_sweeps > 1 || o.coarsest_n > o.dense_max ||
        o.step_mode < -1 || o.step_mode > 1 || o.fixed_k0 < 0 ||
        (o.fixed_k0 > 0 && !(o.fixed_beta >= 1.0 && std::isfinite(o.fixed_beta))) || o.graph < 0 || o.graph > 1 ||
        o.coarsen < 0 || o.coarsen > 1 || o.galerkin < 0 || o.galerkin > 2 || o.weight_storage < 0 ||
        o.weight_storage > 1)
        return CMG_E_ARG;
    const double t0 = now_ms();
    cmg_ctx* c = new (std::nothrow) cmg_ctx;
    if (!c) return CMG_E_OOM;
    c->opt = o;
    c->stream = (hipStream_t)o.stream;
    if (o.allocator) c->alloc = *o.allocator;
    cmg_status st = setup_impl(c, n, nnz, row_ptr, col, w, wtype, where);
    if (st != CMG_OK) {
        delete c;
        return st;
    }
    c->setup_ms = now_ms() - t0;
    *out = c;
    return CMG_OK;
}

cmg_status cmg_fiedler(cmg_handle h, double* lambda, void* x, cmg_memspace where, cmg_stats* stats) {
    g_last_error[0] = 0;
    if (!h) return CMG_E_ARG;
    if (where != CMG_MEM_HOST && where != CMG_MEM_DEVICE) return CMG_E_ARG;
    return fiedler_impl(h, lambda, x, where, stats);
}

cmg_status cmg_fiedler_batch(cmg_handle* hs, int32_t count, double* lambdas, void** xs,
                             cmg_memspace where, cmg_stats* stats) {
    g_last_error[0] = 0;
    if (!hs || count < 0) return CMG_E_ARG;
    if (where != CMG_MEM_HOST && where != CMG_MEM_DEVICE) return CMG_E_ARG;
    if (count == 0) return CMG_OK;
    for (int32_t i = 0; i < count; ++i) {
        if (!hs[i]) return CMG_E_ARG;
        for (int32_t k = 0; k < i; ++k)
            if (hs[k] == hs[i]) return CMG_E_ARG;  // a handle's buffers serve one solve at a time
    }
    return batch_impl(hs, count, lambdas, xs, where, stats);
}

cmg_status cmg_fiedler_block(cmg_handle h, int32_t p, double* lambdas, void* X, cmg_memspace where,
                             double* residuals, int32_t* level_steps) {
    g_last_error[0] = 0;
    if (!h) return CMG_E_ARG;
    if (where != CMG_MEM_HOST && where != CMG_MEM_DEVICE) return CMG_E_ARG;
    return block_impl(h, p, lambdas, X, where, residuals, level_steps);
}

cmg_status cmg_bisect(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, const void* w,
                      cmg_valtype wtype, cmg_memspace where, const cmg_options* opt, int32_t depth, int32_t* part,
                      double* cut) {
    g_last_error[0] = 0;
    if (n < 2 || nnz < 1 || nnz >= 2147483647LL || !row_ptr || !col || !w || !part) return CMG_E_ARG;
    if (wtype != CMG_VAL_F64 && wtype != CMG_VAL_F32) return CMG_E_ARG;
    if (where != CMG_MEM_HOST && where != CMG_MEM_DEVICE) return CMG_E_ARG;
    if (depth < 0 || depth > 16) return CMG_E_ARG;
    cmg_options o;
    fill_defaults(&o);
    if (opt) {
        size_t sz = opt->struct_size ? std::min<size_t>(opt->struct_size, sizeof(o)) : sizeof(o);
        std::memcpy(&o, opt, sz);
        o.struct_size = sizeof(o);
    }
    return bisect_impl(n, nnz, row_ptr, col, w, wtype, where, o, depth, part, cut);
}

cmg_status cmg_level_info(cmg_handle h, cmg_level_stats* out, int32_t cap, int32_t* nlevels) {
    if (!h) return CMG_E_ARG;
    const int nl = (int)h->lv.size();
    if (nlevels) *nlevels = nl;
    if (!out) return CMG_OK;
    for (int j = 0; j < nl && j < cap; ++j) {
        const HostLevel& L = h->lv[j];
        cmg_level_stats li{};
        li.n = L.n;
        li.nnz = L.nnz;
        li.g = L.g;
        li.wmax = L.wmax;
        li.k = L.k;
        li.margin = L.margin;
        li.fp32 = L.fp32;
        li.in_block = L.in_block;
        li.variant = L.variant;
        li.lanes = L.lanes;
        li.grid = L.grid;
        li.pi_ms = L.pi_ms;
        const double sx = L.fp32 ? 4 : 8;
        const int wkr = L.wk == kWUnit ? 2 : L.wk == kWU8 ? 3 : L.wk == kWU16 ? 4 : (L.fp32 || L.wk == kWF32) ? 1 : 0;
        const double sw = wkr == 2 ? 0 : wkr == 3 ? 1 : wkr == 4 ? 2 : wkr == 1 ? 4 : 8;
        li.bytes_per_iter = 4.0 * (L.n + 1) + (double)L.nnz * (4 + sw) + 2 * sx * L.n;
        li.weights = wkr;
        li.block_waves = L.bwaves;
        li.block_regs = L.bregs;
        li.block_slots = L.bslots;
        li.step = L.step;
        out[j] = li;
    }
    return CMG_OK;
}

cmg_status cmg_level_copy(cmg_handle h, int32_t level, int32_t* row_ptr, int32_t* col, double* w,
                          int32_t* agg) {
    if (!h || level < 0 || level >= (int)h->lv.size()) return CMG_E_ARG;
    const HostLevel& L = h->lv[level];
    hipStream_t s = h->stream;
    if (agg && !L.agg) return CMG_E_ARG;
    if (row_ptr) CK(hipMemcpyAsync(row_ptr, L.rp, sizeof(int32_t) * (L.n + 1), hipMemcpyDeviceToHost, s));
    if (col) CK(hipMemcpyAsync(col, L.col, sizeof(int32_t) * L.nnz, hipMemcpyDeviceToHost, s));
    if (w) CK(hipMemcpyAsync(w, L.w64, sizeof(double) * L.nnz, hipMemcpyDeviceToHost, s));
    if (agg) CK(hipMemcpyAsync(agg, L.agg, sizeof(int32_t) * L.n, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    return CMG_OK;
}

cmg_status cmg_set_stream(cmg_handle h, void* stream) {
    if (!h) return CMG_E_ARG;
    h->stream = (hipStream_t)stream;
    h->opt.stream = stream;
    return CMG_OK;
}

cmg_status cmg_footprint(cmg_handle h, size_t* bytes) {
    if (!h || !bytes) return CMG_E_ARG;
    *bytes = h->footprint;
    return CMG_OK;
}

void cmg_free(cmg_handle h) { delete h; }

cmg_status cmg_fiedler_noalloc(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, const void* w,
                               cmg_valtype wtype, cmg_memspace where, const cmg_options* opt, double* lambda,
                               void* x, cmg_stats* stats) {
    g_last_error[0] = 0;
    if (n < 2 || nnz < 1 || nnz >= 2147483647LL || !row_ptr || !col || !w) return CMG_E_ARG;
    if (wtype != CMG_VAL_F64 && wtype != CMG_VAL_F32) return CMG_E_ARG;
    if (where != CMG_MEM_HOST && where != CMG_MEM_DEVICE) return CMG_E_ARG;
    cmg_options o;
    fill_defaults(&o);
    if (opt) {
        size_t sz = opt->struct_size ? std::min<size_t>(opt->struct_size, sizeof(o)) : sizeof(o);
        std::memcpy(&o, opt, sz);
        o.struct_size = sizeof(o);
    }
    if (!(o.tol < 1.0) || !std::isfinite(o.tol) || o.coarsest_n < 2 || o.dense_max < 2 || o.dense_max > 128 ||
        o.max_iters_per_level < 1 || (o.precision != CMG_FP64 && o.precision != CMG_MIXED) ||
        o.fp64_final_sweeps < 0 || o.fp64_final_sweeps > 1 || o.coarsest_n > o.dense_max || o.fixed_k0 < 0 ||
        (o.fixed_k0 > 0 && !(o.fixed_beta >= 1.0 && std::isfinite(o.fixed_beta))) || o.coarsen < 0 ||
        o.coarsen > 1 || o.galerkin < 0 || o.galerkin > 2 || o.weight_storage < 0 || o.weight_storage > 1)
        return CMG_E_ARG;
    const size_t need = noalloc_need(n, nnz);
    if (need > kNoallocScratchBytes - kNoallocMeasureBytes) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "cmg_fiedler_noalloc: a graph of %d vertices and %lld entries needs up to %zu bytes of "
                      "scratch; the static scratch holds %zu",
                      n, (long long)nnz, need, kNoallocScratchBytes - kNoallocMeasureBytes);
        return CMG_E_ARG;
    }
    // launches only: no step-by-step levels (pinned flags, events), no
    // autotuner (events), no graph (a capture stream)
    o.step_mode = -1;
    o.autotune = 0;
    o.graph = 0;
    return noalloc_impl(n, nnz, row_ptr, col, w, wtype, where, o, lambda, x, stats);
}

cmg_status cmg_hash_probe(uint64_t seed, int32_t level, int32_t count, uint64_t* out) {
    if (count < 0 || (count > 0 && !out)) return CMG_E_ARG;
    if (count == 0) return CMG_OK;
    unsigned long long* d = nullptr;
    if (hipMalloc(&d, sizeof(unsigned long long) * count) != hipSuccess) {
        (void)hipGetLastError();
        return CMG_E_OOM;
    }
    hipError_t e = launch_hash_probe(seed, level, count, d, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, d, sizeof(unsigned long long) * count, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return CMG_E_DEVICE;
    }
    return CMG_OK;
}

}  // extern "C"
