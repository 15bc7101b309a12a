// Device-side helpers and structures shared by the libcmg HIP translation
// units (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmg {

constexpr int kWave = 64;

// SplitMix64 output function (Steele, Lea & Flood 2014).
__device__ __host__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// HEC priority of vertex v at level j (ascending key = visit order).
__device__ __forceinline__ uint64_t hec_key(uint64_t seed, int level, int v) {
    return mix64(seed ^ ((uint64_t)(uint32_t)level << 40) ^ (uint64_t)(uint32_t)v);
}

// Hashed uniform in [0,1): start vector for power iteration on a coarsest
// level too large for the dense solve.
__device__ __forceinline__ double hashed_uniform(uint64_t seed, int i) {
    uint64_t h = mix64(seed ^ 0x9E3779B97F4A7C15ull ^ (uint64_t)(uint32_t)i);
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

// Sum over the G-lane group (G power of two <= 64); every lane of the
// group ends with the group sum computed in the same butterfly order as
// its partner lanes, so lane 0 of a group is the canonical value.
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
    for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// A double moved between lanes by DPP (a row of 16 lanes at most): vector
// ALU only, no LDS traffic.  CTRL is the DPP control (0xB1 and 0x4E: quad
// permutations to lane ^ 1 and lane ^ 2; 0x141: mirror within 8 lanes;
// 0x140: mirror within 16 lanes; 0x124 and 0x128: rotation of the 16
// lanes of a row by 4 and by 8).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// x[l] + x[l ^ 16] (ROWS = 16) or x[l] + x[l ^ 32] (ROWS = 32) in every
// lane l of a full wavefront: the gfx950 lane-swap instructions hand each
// lane both values, so the two lanes of a pair hold the same bits.
template <int ROWS>
__device__ __forceinline__ double pair_sum_rows(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)(b & 0xffffffffll), hi = (unsigned)(b >> 32);
    if constexpr (ROWS == 16) {
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        return __longlong_as_double(((long long)h[0] << 32) | (long long)l[0]) +
               __longlong_as_double(((long long)h[1] << 32) | (long long)l[1]);
    } else {
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        return __longlong_as_double(((long long)h[0] << 32) | (long long)l[0]) +
               __longlong_as_double(((long long)h[1] << 32) | (long long)l[1]);
    }
}

// Explicit address spaces.  A pointer read from a descriptor in memory is
// generic to the compiler, and generic (flat) loads make every use of a
// loaded value wait for all outstanding memory operations, so loads that
// could be in flight together are serialised.  gld/gst read and write
// through a global-memory view (loads waited on one by one), sld/sst
// through an LDS view, for pointers known to be of that kind.
#define CMG_AS_GLOBAL __attribute__((address_space(1)))
#define CMG_AS_LDS __attribute__((address_space(3)))
template <typename T, typename I>
__device__ __forceinline__ T gld(const T* p, I i) {
    return ((const CMG_AS_GLOBAL T*)p)[i];
}
template <typename T, typename I>
__device__ __forceinline__ void gst(T* p, I i, T v) {
    ((CMG_AS_GLOBAL T*)p)[i] = v;
}
template <typename T, typename I>
__device__ __forceinline__ T sld(const T* p, I i) {
    return ((const CMG_AS_LDS T*)p)[i];
}
template <typename T, typename I>
__device__ __forceinline__ void sst(T* p, I i, T v) {
    ((CMG_AS_LDS T*)p)[i] = v;
}

// Value of a lane, identical in every lane (needs that lane active).
__device__ __forceinline__ double read_lane(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the aligned G-lane group (G a power of two <= 64; the whole
// group active).  Each step adds a lane's partial to its partner's, so all
// lanes of a group end with bitwise the same sum.  Doubles: quad
// permutations and row mirrors by DPP up to 16 lanes, one shuffle for 32,
// the four row sums by readlane for 64.
template <int G, typename T>
__device__ __forceinline__ T group_sum_t(T v) {
    if constexpr (sizeof(T) == 8) {
        double d = v;
        if constexpr (G >= 2) d += dpp_move<0xB1>(d);
        if constexpr (G >= 4) d += dpp_move<0x4E>(d);
        if constexpr (G >= 8) d += dpp_move<0x141>(d);
        if constexpr (G >= 16) d += dpp_move<0x140>(d);
        if constexpr (G == 32) d += __shfl_xor(d, 16, kWave);
        if constexpr (G == 64) d = (read_lane(d, 0) + read_lane(d, 16)) + (read_lane(d, 32) + read_lane(d, 48));
        return (T)d;
    } else {
#pragma unroll
        for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
        return v;
    }
}

// Deterministic block reduction of NV doubles.  `red` is LDS scratch of at
// least NV * (blockDim/64) doubles.  Result valid in all threads on return.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = group_sum_t<kWave>(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) red[q * 16 + wv] = v[q];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[threadIdx.x * 16 + w];
        red[NV * 16 + threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = red[NV * 16 + q];
    __syncthreads();
}

// Deterministic block reduction with one barrier: waves post their sums to
// a slot chosen by `parity` (flipped on return), every thread then adds the
// posts in wave order.  Two alternating slots make back-to-back calls safe.
// `red` holds 2 * NV * 16 doubles.
template <int NV>
__device__ __forceinline__ void block_sum1(double (&v)[NV], double* red, int& parity) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    double* slot = red + parity * NV * 16;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = group_sum_t<kWave>(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) slot[q * 16 + wv] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += slot[q * 16 + w];
        v[q] = t;
    }
    parity ^= 1;
}

// --------------------------------------------------------------- levels

// One level of the hierarchy as the refinement kernels see it.
// storage of a level's edge weights in the grid and step kernels
constexpr int kWNative = 0;  // the iterates' type (FP64, or FP32 on mixed-precision levels)
constexpr int kWF32 = 1;     // an FP32 copy beside FP64 iterates (every weight exact in FP32)
constexpr int kWUnit = 2;    // every weight is 1: none is read
constexpr int kWU8 = 3;      // an 8-bit copy (every weight an integer in 1..255)
constexpr int kWU16 = 4;     // a 16-bit copy (every weight an integer in 1..65535)

struct LevelDev {
    int32_t n;
    int32_t lanes;       // lanes per row for the row-group SpMV
    int64_t nnz;
    const int32_t* rp;
    const int32_t* col;
    const double* w64;
    const float* w32;
    const uint8_t* w8;   // 8-bit copy of the weights (kWU8 levels)
    const uint16_t* w16; // 16-bit copy of the weights (kWU16 levels)
    const int32_t* agg;  // vertex -> aggregate in level+1 (nullptr on coarsest)
    double g;            // Gershgorin shift
    int32_t fp32;        // 1: FP32 vectors and values
    int32_t variant;     // 1 rows, 2 merge path
    void* buf0;          // two vectors of n entries (double or float)
    void* buf1;
    const int32_t* part; // grid kernel: first row of each workgroup (grid+1 entries)
    const int32_t* mpart;// merge path: diagonal split of each workgroup (2*(grid+1))
    int32_t grid;
    int32_t w32exact;    // 1 if every weight is exactly representable in FP32
    int32_t bwaves;      // single-workgroup refinement: wavefronts that run the PI steps
    int32_t bregs;       // single-workgroup refinement: rows per lane group held in registers (0: CSR)
    int32_t bslots;      // register rows: entry slots per lane and row (E of the layout)
    int32_t stage;       // grid levels: 1 if a workgroup's rows may be staged in LDS
    int32_t kfix;        // > 0: fixed schedule, exactly this many PI steps and no stopping test
    int32_t wk;          // weight storage of the grid and step kernels (kWNative, kWF32, kWUnit, kWU8, kWU16)
    int32_t lmin;        // rows traversal: rows with more entries are long (INT_MAX: none)
    const int32_t* lrows;// ... their count, then the long rows in ascending order (nullptr: none)
    int32_t ileave;      // rows traversal of the persistent grid kernel: 1 if each workgroup's PI
                         // steps take row chunks interleaved over its XCD's workgroups (the
                         // long rows stay with its own part); never staged in LDS
};

// State a refinement launch leaves for the next level (device written).
struct LevelState {
    double mu;      // final vector = (buf[fin] - mu) * s
    double s;
    double mu_prev; // iterate before the last step = (buf[1-fin] - mu_prev) * s_prev
    double s_prev;
    double utv;     // last (u^k, u^{k-1})
    double margin;  // utv - (1 - tol)
    int32_t fin;    // buffer index holding the final vector
    int32_t k;      // PI steps
    int32_t maxit;  // 1 if the cap was hit
    int32_t err;    // device-side failure (barrier timeout)
    long long ticks;  // single-workgroup levels: duration in constant-clock ticks
};

// Result of the finishing pass.
struct FinishOut {
    double lambda;
    double residual;
    double sum_u;
    double sum_uu;
    double edge;
    double coarse_lambda2;
    int32_t coarse_mult;
    int32_t err;
};

// Grid barrier state.  `epoch` counts completed grid barriers over the
// handle's lifetime (never reset while healthy), so per-workgroup slots
// tagged with an epoch need no clearing between launches.
struct GridSync {
    unsigned long long epoch;
    unsigned int abort;
    unsigned int where;             // first timeout: workgroups | (job tag + 2) << 16
    unsigned long long abort_epoch;  // first timeout: the barrier's epoch
};

// One workgroup's contribution to a grid all-reduce: its partial sums and
// the epoch of the barrier they belong to, in one 64-byte line.
struct alignas(64) GridSlot {
    double v[7];
    unsigned long long epoch;
};

// Broadcast of grid all-reduce totals: this many lines, this many bytes
// apart (so they map to different memory channels).
constexpr int kBcastLines = 32;
constexpr int kBcastStride = 4096 + 64;
constexpr size_t kBcastBytes = (size_t)kBcastLines * kBcastStride;

// One unit of a (possibly packed) grid launch: a level of one graph,
// refined (or finished) by workgroups [b0, b0 + L.grid) of the launch.
struct GridJob {
    LevelDev L;             // level processed
    LevelDev C;             // next coarser level (prolongation source)
    LevelState* st;         // refine: state written for L
    const LevelState* stc;  // refine: state of C; finish: state of L
    GridSync* gs;           // barrier state of this graph
    GridSlot* slots;
    GridSlot* bcast;        // kBcastLines lines, kBcastStride bytes apart
    double* fa;             // finish: FP64 scratch of n entries (mixed redo)
    double* yout;           // finish: output vector
    FinishOut* fo;          // finish: scalars out
    double tol;             // refine: stopping tolerance
    uint64_t seed;          // refine: hashed uniform start seed
    int32_t maxit;          // refine: step cap
    int32_t b0;
    int32_t uniform;        // refine: hashed uniform start instead of prolongation
    int32_t redo;           // finish: recompute the last step in FP64
    int32_t tag;            // level index of a refinement job, -1 for finishing,
                            // kResidencyTag for a residency count
    unsigned* count;        // residency count: {live, peak}
    long long hold;         // residency count: wall-clock ticks each workgroup stays
};

// A job with this tag only counts how many of its workgroups are resident
// at once; no workgroup waits for another.
constexpr int32_t kResidencyTag = -100;

// Large levels refined with one launch per power-iteration step: the
// running state between the launches (device written).
struct StepCtl {
    double mu, s;         // current vector = (buf[cur] - mu) * s
    double pmu, ps;       // the same for the previous vector
    double utv;
    int32_t k, cur, done, hit;
};

// One large level refined step by step.
struct StepJob {
    LevelDev L;              // the level (L.grid workgroups, L.part row split)
    LevelDev C;              // next coarser level (prolongation source)
    const LevelState* stc;   // state of C
    LevelState* st;          // written when the level is done
    StepCtl* ctl;
    double* part;            // per-workgroup partial sums, 4 per workgroup
    double tol;
    uint64_t seed;
    int32_t maxit, uniform;
};

// Coarse levels jhi .. jlo of one graph, refined by one workgroup.
struct BlockJob {
    const LevelDev* lv;
    LevelState* st;
    double tol;
    uint64_t seed;
    int32_t maxit;
    int32_t jhi;
    int32_t jlo;
    int32_t uniform;
};

// Dense coarsest solve of one graph, one workgroup.
struct CoarseJob {
    LevelDev L;
    LevelState* st;
    double* A;
    double* V;
    double* ev;
    int32_t* idx;
    FinishOut* fo;
    uint64_t seed;
};

}  // namespace cmg
