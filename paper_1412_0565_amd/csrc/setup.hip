// Setup-phase kernels: input validation, heavy edge coarsening (HEC,
// Algorithm 2) and the Galerkin coarse graph L^{i+1} = I L^i I^T
// (Section 2, Step 1 and the Proposition on restriction).
//
// HEC is defined sequentially: vertices are visited in a random order; an
// unmapped vertex v whose heaviest neighbour h(v) is unmapped opens the
// aggregate {v, h(v)}; otherwise v joins h(v)'s aggregate.  With a fixed
// priority key per vertex (visit order = ascending key) the same result is
// obtained data-parallel:
//   * v can only open an aggregate if key(v) < key(h(v)) ("candidate"),
//     because a vertex visited earlier is always mapped by then;
//   * the opened pairs are exactly the greedy maximal matching of the
//     candidate edges {v, h(v)} taken in key order, which round-synchronous
//     "local minimum" rounds reproduce exactly (an edge holding the smallest
//     live key at both endpoints is accepted; edges touching accepted
//     endpoints die);
//   * an unmatched vertex ends in the aggregate reached by following h until
//     a matched vertex (keys strictly decrease along that chain).
// Aggregates are numbered by ascending index of their opening vertex.
#include <type_traits>

#include "cmg_internal.h"

namespace cmg {

namespace {

constexpr int kBlk = 256;

inline unsigned nblocks(int64_t m, int per) { return (unsigned)((m + per - 1) / per); }

// ------------------------------------------------------------ validation

// One group of kValidateLanes lanes per row (row n: the row-pointer ends);
// each lane checks every kValidateLanes-th entry of the row against the
// entry before it.
constexpr int kValidateLanes = 8;

template <typename W>
__global__ void k_validate(int n, int64_t nnz, const int32_t* __restrict__ rp,
                           const int32_t* __restrict__ col, const W* __restrict__ w, int full,
                           unsigned* flags) {
    const int lane = threadIdx.x & (kValidateLanes - 1);
    const int i = blockIdx.x * (blockDim.x / kValidateLanes) + threadIdx.x / kValidateLanes;
    if (i > n) return;
    unsigned f = 0;
    if (i == n) {
        if (lane == 0 && ((int64_t)rp[n] != nnz || rp[0] != 0)) f |= kBadGraph;
    } else {
        const int a = rp[i], b = rp[i + 1];
        if (a < 0 || b < a || (int64_t)b > nnz) {
            f |= kBadGraph;
        } else if (a == b) {
            f |= kIsolated;
        } else {
            if (lane == 0 && b - a > 64) atomicMax(&flags[1], (unsigned)(b - a));  // long rows only
            for (int e = a + lane; e < b; e += kValidateLanes) {
                const int c = col[e];
                const int prev = e > a ? col[e - 1] : -1;
                const double x = (double)w[e];
                bool bad = c < 0 || c >= n || c == i || c <= prev;
                if (!(x > 0.0) || !isfinite(x)) bad = true;
                if (!bad && (x != floor(x) || x >= 1048576.0)) f |= kWideWeight;
                if (x != 1.0) f |= kNonUnit;
                if (bad) {
                    f |= kBadGraph;
                } else if (full && rp[c] >= 0 && rp[c] <= rp[c + 1] && (int64_t)rp[c + 1] <= nnz) {
                    // binary search i in row c, weights must agree
                    int lo = rp[c], hi = rp[c + 1] - 1;
                    bool found = false;
                    while (lo <= hi) {
                        const int mid = (lo + hi) >> 1;
                        const int cm = col[mid];
                        if (cm == i) {
                            found = ((double)w[mid] == x);
                            break;
                        }
                        if (cm < i) lo = mid + 1;
                        else hi = mid - 1;
                    }
                    if (!found) f |= kAsym;
                }
            }
        }
    }
    if (f) atomicOr(flags, f);
}

template <typename W>
__global__ void k_convert(int64_t nnz, const W* __restrict__ in, double* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < nnz; i += st) out[i] = (double)in[i];
}

__global__ void k_to_f32(int64_t nnz, const double* __restrict__ in, float* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < nnz; i += st) out[i] = (float)in[i];
}

// weights known to be integers in 1..255 (U = uint8_t) or 1..65535
template <typename U>
__global__ void k_to_uint(int64_t nnz, const double* __restrict__ in, U* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < nnz; i += st) out[i] = (U)in[i];
}

// ------------------------------------------------------- row information

// One G-lane group per row: heaviest neighbour (max weight, lowest column
// on ties: the first minimum of the column of L), weighted degree for the
// Gershgorin shift g = 2 max_v d_v, largest weight.  A vertex with no
// neighbour (on a coarse level, a component that became one aggregate)
// raises *iso and names itself as its heaviest neighbour, so the HEC
// kernels that run before the host reads the flag touch only valid
// indices: it is never a candidate, and its aggregate is discarded with
// the level when the setup returns CMG_E_ISOLATED.
template <int G>
__global__ void k_rowinfo(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const double* __restrict__ w, int32_t* __restrict__ h,
                          double* __restrict__ bmax, unsigned* __restrict__ iso) {
    const int lane = threadIdx.x & (G - 1);
    const int gpb = blockDim.x / G;
    int row = blockIdx.x * gpb + threadIdx.x / G;
    double dmax = 0.0, wm = 0.0, ex = 0.0, lmax = 0.0;
    const int stride = gridDim.x * gpb;
    for (; row < n; row += stride) {
        int a = rp[row], b = rp[row + 1];
        lmax = fmax(lmax, (double)(b - a));
        double bw = -1.0;
        int bc = 0x7fffffff;
        double d = 0.0;
        for (int e = a + lane; e < b; e += G) {
            double x = w[e];
            int c = col[e];
            d += x;
            ex = fmax(ex, fabs(x - (double)(float)x));
            if (x > bw || (x == bw && c < bc)) {
                bw = x;
                bc = c;
            }
        }
#pragma unroll
        for (int o = G >> 1; o > 0; o >>= 1) {
            double ow = __shfl_xor(bw, o, kWave);
            int oc = __shfl_xor(bc, o, kWave);
            if (ow > bw || (ow == bw && oc < bc)) {
                bw = ow;
                bc = oc;
            }
        }
        d = group_sum_t<G>(d);
        if (lane == 0) {
            h[row] = b > a ? bc : row;
            if (b == a) atomicOr(iso, 1u);
            dmax = fmax(dmax, 2.0 * d);
            wm = fmax(wm, bw);
        }
    }
    // block maxima (exact, order independent) to bmax[4b .. 4b+3]
    __shared__ double sm[4][kBlk / kWave];
    for (int o = 32; o > 0; o >>= 1) {
        dmax = fmax(dmax, __shfl_xor(dmax, o, kWave));
        wm = fmax(wm, __shfl_xor(wm, o, kWave));
        ex = fmax(ex, __shfl_xor(ex, o, kWave));
        lmax = fmax(lmax, __shfl_xor(lmax, o, kWave));
    }
    if ((threadIdx.x & 63) == 0) {
        sm[0][threadIdx.x >> 6] = dmax;
        sm[1][threadIdx.x >> 6] = wm;
        sm[2][threadIdx.x >> 6] = ex;
        sm[3][threadIdx.x >> 6] = lmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            a = fmax(a, sm[0][q]);
            b = fmax(b, sm[1][q]);
            c = fmax(c, sm[2][q]);
            d = fmax(d, sm[3][q]);
        }
        bmax[4 * blockIdx.x] = a;
        bmax[4 * blockIdx.x + 1] = b;
        bmax[4 * blockIdx.x + 2] = c;
        bmax[4 * blockIdx.x + 3] = d;
    }
}

// The same for a level whose weights are all 1: the heaviest neighbour is
// the lowest column (the row's first entry), the weighted degree the row
// length; the weights are not read.
__global__ void k_rowinfo_unit(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                               int32_t* __restrict__ h, double* __restrict__ bmax, unsigned* __restrict__ iso) {
    double lmax = 0.0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int a = rp[v], b = rp[v + 1];
        h[v] = b > a ? col[a] : v;
        if (b == a) atomicOr(iso, 1u);
        lmax = fmax(lmax, (double)(b - a));
    }
    __shared__ double sm[kBlk / kWave];
    for (int o = 32; o > 0; o >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, o, kWave));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = lmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double d = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) d = fmax(d, sm[q]);
        bmax[4 * blockIdx.x] = 2.0 * d;
        bmax[4 * blockIdx.x + 1] = 1.0;
        bmax[4 * blockIdx.x + 2] = 0.0;
        bmax[4 * blockIdx.x + 3] = d;
    }
}

// one block: maxima over the per-block values; results as double bit
// patterns in out[0] (g), out[1] (largest weight), out[2] (largest FP32
// rounding error of a weight: 0 if all weights are exact in FP32)
__global__ void k_max_reduce(const double* __restrict__ bmax, int nb, unsigned long long* out) {
    __shared__ double sm[4][kBlk / kWave];
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        for (int q = 0; q < 4; ++q) m[q] = fmax(m[q], bmax[4 * i + q]);
    for (int o = 32; o > 0; o >>= 1)
        for (int q = 0; q < 4; ++q) m[q] = fmax(m[q], __shfl_xor(m[q], o, kWave));
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 4; ++q) sm[q][threadIdx.x >> 6] = m[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
            for (int q = 0; q < 4; ++q) m[q] = fmax(m[q], sm[q][w]);
        for (int q = 0; q < 4; ++q) out[q] = (unsigned long long)__double_as_longlong(m[q]);
    }
}

// ------------------------------------------------------------------- HEC

constexpr uint8_t kSeed = 1;     // opened an aggregate (visited vertex)
constexpr uint8_t kPartner = 2;  // heaviest neighbour of a seed
constexpr unsigned long long kNoKey = 0xFFFFFFFFFFFFFFFFull;

// Rounds are launched ahead of the host's check and disable themselves:
// round r runs only if round r - 1 left a live candidate edge
// (flags[(r - 1) & 1]; k_hec_init sets flags[1] for round 0), and k_hec_kill
// of round r raises flags[r & 1] after k_hec_post of round r cleared it.  A
// round after the last live edge changes nothing either way.
__global__ void k_hec_init(int n, const int32_t* __restrict__ h, uint64_t seed, int level,
                           uint8_t* __restrict__ live, uint8_t* __restrict__ state,
                           int32_t* __restrict__ pairseed, unsigned long long* __restrict__ slot,
                           unsigned long long* __restrict__ flags) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0) {
        flags[0] = 0ull;
        flags[1] = 1ull;
    }
    if (v >= n) return;
    pairseed[v] = v;
    uint64_t kv = hec_key(seed, level, v);
    uint64_t km = hec_key(seed, level, h[v]);
    live[v] = (kv < km) ? 1 : 0;
    state[v] = 0;
    slot[v] = kNoKey;
}

// The round kernels run a capped grid whose threads stride over the
// vertices: most vertices of later rounds are settled, and a round launched
// after the matching finished returns at once, so launching a thread per
// vertex would cost more than the work.
constexpr unsigned kHecRoundBlocks = 2048;

// Each live candidate edge {v, h(v)} posts its key at both endpoints.  The
// round's "any live" flag, raised only by k_hec_kill after this kernel, is
// cleared here.
__global__ void k_hec_post(int n, const int32_t* __restrict__ h, uint64_t seed, int level,
                           const uint8_t* __restrict__ live, unsigned long long* slot,
                           unsigned long long* flags, int round) {
    const int v0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (v0 == 0) flags[round & 1] = 0ull;
    if (flags[(round - 1) & 1] == 0ull) return;
    for (int v = v0; v < n; v += gridDim.x * blockDim.x) {
        if (!live[v]) continue;
        unsigned long long k = hec_key(seed, level, v);
        atomicMin(&slot[v], k);
        atomicMin(&slot[h[v]], k);
    }
}

// An edge holding the minimum at both endpoints is accepted.  Two accepted
// edges never share an endpoint, so the writes below never collide.
__global__ void k_hec_accept(int n, const int32_t* __restrict__ h, uint64_t seed, int level,
                             uint8_t* __restrict__ live, uint8_t* __restrict__ state,
                             int32_t* __restrict__ pairseed,
                             const unsigned long long* __restrict__ slot,
                             const unsigned long long* __restrict__ flags, int round) {
    if (flags[(round - 1) & 1] == 0ull) return;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        if (!live[v]) continue;
        unsigned long long k = hec_key(seed, level, v);
        int m = h[v];
        if (slot[v] == k && slot[m] == k) {
            state[v] = kSeed;
            state[m] = kPartner;
            pairseed[v] = v;
            pairseed[m] = v;
            live[v] = 0;
        }
    }
}

// Edges touching a matched endpoint die; survivors re-arm their slots for
// the next round and raise the "any live" flag (a plain store of 1: racing
// writers store the same value).
__global__ void k_hec_kill(int n, const int32_t* __restrict__ h, uint8_t* __restrict__ live,
                           const uint8_t* __restrict__ state, unsigned long long* slot,
                           unsigned long long* flags, int round) {
    if (flags[(round - 1) & 1] == 0ull) return;
    int alive = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        if (!live[v]) continue;
        int m = h[v];
        if (state[v] != 0 || state[m] != 0) {
            live[v] = 0;
        } else {
            slot[v] = kNoKey;
            slot[m] = kNoKey;
            alive = 1;
        }
    }
    if (__syncthreads_or(alive) && threadIdx.x == 0) flags[round & 1] = 1ull;
}

// Unmatched vertices follow h to a matched vertex (keys decrease along the
// chain, so it ends); rootseed = opening vertex of that aggregate.
__global__ void k_hec_attach(int n, const int32_t* __restrict__ h, const uint8_t* __restrict__ state,
                             const int32_t* __restrict__ pairseed, int32_t* __restrict__ rootseed,
                             int32_t* __restrict__ flags) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int r = v;
    for (int guard = 0; guard < n && state[r] == 0 && h[r] != r; ++guard) r = h[r];
    rootseed[v] = pairseed[r];
    flags[v] = (state[v] == kSeed) ? 1 : 0;
}

__global__ void k_hec_label(int n, const int32_t* __restrict__ rootseed,
                            const int32_t* __restrict__ rank, int32_t* __restrict__ agg) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    agg[v] = rank[rootseed[v]];
}

// ------------------------------------------------------------------- HEM
//
// Heavy edge matching (Section 2.1, the coarsening HEC is contrasted with):
// in visit order, an unmatched vertex is matched to its heaviest unmatched
// neighbour (lowest index on ties) or stays alone.  When a vertex's turn
// comes all its earlier neighbours are matched already, so the sequential
// result is the greedy matching over edges ordered by (key of the endpoint
// visited first, decreasing weight, other endpoint), and rounds reproduce
// it exactly: a live vertex whose live neighbours all come later in key
// order proposes to its heaviest live neighbour, and the proposal holds if
// the proposer is that neighbour's earliest live neighbour; a live vertex
// with no live neighbour stays alone.  Each round reads the state its first
// pass recorded, so no decision depends on the order threads run in.
// opener[v] = -1 while v is live, else the vertex that opened its aggregate.

// pass 1: the round's live flags, and the smallest key among each live
// vertex's live neighbours (kNoKey if none); raises alive[round] if any
// vertex is live at the start of the round
__global__ void k_hem_scan(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col, uint64_t seed,
                           int level, const int32_t* __restrict__ opener, uint8_t* __restrict__ live,
                           unsigned long long* __restrict__ mkey, unsigned* __restrict__ alive, int round) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    int lv = 0;
    if (v < n) {
        lv = opener[v] < 0 ? 1 : 0;
        live[v] = (uint8_t)lv;
        if (lv) {
            unsigned long long m = kNoKey;
            for (int e = rp[v]; e < rp[v + 1]; ++e) {
                const int u = col[e];
                if (opener[u] < 0) {
                    const unsigned long long k = hec_key(seed, level, u);
                    m = k < m ? k : m;
                }
            }
            mkey[v] = m;
        }
    }
    if (__syncthreads_or(lv) && threadIdx.x == 0) alive[round] = 1u;
}

// pass 2: proposals of the vertices whose live neighbours all come later
__global__ void k_hem_match(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const double* __restrict__ w, uint64_t seed, int level,
                            const uint8_t* __restrict__ live, const unsigned long long* __restrict__ mkey,
                            int32_t* __restrict__ opener) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || !live[v]) return;
    const unsigned long long mk = mkey[v];
    if (mk == kNoKey) {  // no live neighbour left: a single-vertex aggregate
        opener[v] = v;
        return;
    }
    const unsigned long long kv = hec_key(seed, level, v);
    if (kv > mk) return;  // an earlier live neighbour decides first
    int best = -1;
    double bw = 0.0;
    for (int e = rp[v]; e < rp[v + 1]; ++e) {
        const int u = col[e];
        if (!live[u]) continue;
        const double x = w[e];
        if (best < 0 || x > bw || (x == bw && u < best)) {
            best = u;
            bw = x;
        }
    }
    if (mkey[best] == kv) {  // v is best's earliest live neighbour: no other proposal reaches best
        opener[v] = v;
        opener[best] = v;
    }
}

// opening vertices flagged for the numbering scan
__global__ void k_hem_flags(int n, const int32_t* __restrict__ opener, int32_t* __restrict__ flags) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) flags[v] = opener[v] == v ? 1 : 0;
}

// ------------------------------------------------- Galerkin by aggregates
//
// The coarse row of aggregate a collects, for every member vertex in
// ascending index and every entry of its row in CSR order (that is, in fine
// CSR order), the pair (b = agg(col), w); pairs with b = a are dropped and
// equal b are summed in that order, the distinct b written in ascending
// order.  This is the sorted-key Galerkin product without the sort: the
// same sums in the same order, so coarse graphs are bitwise equal.  Used on
// levels whose aggregates have at most kGalWaveCap entries (else the
// radix-sort path).
//
// Pass 1 forms each row where its columns fit: one lane per aggregate
// walks the member rows and keeps the distinct columns, sorted, with their
// running sums in registers (one add per entry, in fine order).  Aggregates with more than S distinct columns
// are listed for pass 1b: a wavefront per aggregate sorts the entries'
// keys (b, position) in LDS, so equal b stay in fine order, and the first
// lane of each run of equal b adds the run in that order.

// keys (agg << 32 | v) for the stable sort of vertices by aggregate
__global__ void k_gal_member_keys(int n, const int32_t* __restrict__ agg, unsigned long long* __restrict__ keys) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) keys[v] = ((unsigned long long)(uint32_t)agg[v] << 32) | (uint32_t)v;
}

// members in aggregate order, their row lengths, each aggregate's first
// member (mstart[nc] = n is written by the thread of the last member)
__global__ void k_gal_members(int n, const unsigned long long* __restrict__ keys, const int32_t* __restrict__ rp,
                              int32_t* __restrict__ members, int32_t* __restrict__ mdeg,
                              int32_t* __restrict__ mstart) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int v = (int)(keys[k] & 0xffffffffull);
    const int a = (int)(keys[k] >> 32);
    members[k] = v;
    mdeg[k] = rp[v + 1] - rp[v];
    if (k == 0 || (int)(keys[k - 1] >> 32) != a) mstart[a] = k;
    if (k == n - 1) mstart[a + 1] = n;
}

// Member lists by counting, for graphs whose weights are all integers
// below 2^20: every Galerkin sum is then an integer far below 2^53, exact
// in any order, so the members of an aggregate may be listed in any order
// (the coarse graph does not change).  Each aggregate's members are
// counted, the counts scanned into first-member offsets, and every vertex
// placed at the next free slot of its aggregate (counting down); mdeg is
// the degree of each listed member.
__global__ void k_mem_count(int n, const int32_t* __restrict__ agg, int32_t* __restrict__ cnt) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) atomicAdd(&cnt[agg[v]], 1);
}

__global__ void k_mem_place(int n, const int32_t* __restrict__ agg, const int32_t* __restrict__ rp,
                            const int32_t* __restrict__ mstart, int32_t* __restrict__ cnt,
                            int32_t* __restrict__ members, int32_t* __restrict__ mdeg) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int a = agg[v];
    const int k = mstart[a] + atomicSub(&cnt[a], 1) - 1;
    members[k] = v;
    mdeg[k] = rp[v + 1] - rp[v];
}

// entries of aggregate a's member rows and the offset of the first
__device__ __forceinline__ int64_t gal_entries(int a, int n, int64_t nnz, const int32_t* __restrict__ mstart,
                                               const int32_t* __restrict__ moff, int64_t* o0) {
    const int k1 = mstart[a + 1];
    *o0 = moff[mstart[a]];
    return (k1 >= n ? nnz : (int64_t)moff[k1]) - *o0;
}

constexpr int kGalLenBlocks = 1024;

// the largest number of entries of an aggregate's member rows (the
// aggregate count read from the device); a fixed grid striding over the
// aggregates so that only kGalLenBlocks atomics reach the one word
__global__ void k_gal_agg_len(int ncmax, const long long* __restrict__ ncp, int n, int64_t nnz,
                              const int32_t* __restrict__ mstart, const int32_t* __restrict__ moff,
                              unsigned long long* __restrict__ emax) {
    const int nc = (int)min((long long)ncmax, *ncp);
    int e = 0;
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < nc; a += gridDim.x * blockDim.x) {
        int64_t o0;
        e = max(e, (int)gal_entries(a, n, nnz, mstart, moff, &o0));
    }
    for (int o = 32; o > 0; o >>= 1) e = max(e, __shfl_xor(e, o, kWave));
    __shared__ int wm[kBlk / 64];
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kBlk / 64; ++q) e = max(e, wm[q]);
        if (e > 0) atomicMax(emax, (unsigned long long)e);
    }
}

// pass 1: a lane per aggregate, S register slots (UNIT: every weight is 1
// and the weights are not read; INT: every weight is an integer and all of
// them together sum below 2^32, so the sums are kept as 32-bit integers,
// exact and equal to the FP64 sums, with half the register traffic)
template <int S, bool UNIT, bool INT>
__global__ void __launch_bounds__(kBlk) __attribute__((amdgpu_waves_per_eu(4))) k_gal_lane(int nc, const int32_t* __restrict__ members,
                                                   const int32_t* __restrict__ mstart,
                                                   const int32_t* __restrict__ moff, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const double* __restrict__ w,
                                                   const int32_t* __restrict__ agg, int32_t* __restrict__ tcol,
                                                   double* __restrict__ tw, int32_t* __restrict__ rowlen,
                                                   int32_t* __restrict__ big, unsigned* __restrict__ nbig) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nc) return;
    const int k0 = mstart[a], k1 = mstart[a + 1];
    using Acc = typename std::conditional<INT, uint32_t, double>::type;
    int rb[S];
    Acc rw[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        rb[q] = 0x7fffffff;
        rw[q] = (Acc)0;
    }
    int len = 0;
    bool over = false;
    // entries in batches of kGalBatch: their columns and weights, then the
    // columns' aggregates, are loaded together before any is added
    constexpr int kGalBatch = S <= 16 ? 8 : 4;
    for (int k = k0; k < k1 && !over; ++k) {
        const int v = members[k];
        const int e1 = rp[v + 1];
        for (int e = rp[v]; e < e1 && !over; e += kGalBatch) {
            int cb[kGalBatch];
            Acc xb[kGalBatch];
#pragma unroll
            for (int i = 0; i < kGalBatch; ++i) {
                if (e + i < e1) {
                    cb[i] = col[e + i];
                    xb[i] = UNIT ? (Acc)1 : (Acc)w[e + i];
                }
            }
#pragma unroll
            for (int i = 0; i < kGalBatch; ++i)
                if (e + i < e1) cb[i] = agg[cb[i]];
#pragma unroll
            for (int i = 0; i < kGalBatch; ++i) {
                const int b = cb[i];
                const Acc x = xb[i];
                if (e + i >= e1 || over || b == a) continue;
                bool found = false;
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    if (rb[q] == b) {
                        rw[q] += x;
                        found = true;
                    }
                }
                if (found) continue;
                if (len == S) {
                    over = true;
                    continue;
                }
                // insert b at its place: the slots stay sorted ascending
                // (unused ones hold INT_MAX), those above it move up one
#pragma unroll
                for (int q = S - 1; q >= 0; --q) {
                    const int prev = q > 0 ? rb[q - 1] : INT_MIN;
                    const Acc prevw = q > 0 ? rw[q - 1] : (Acc)0;
                    if (rb[q] > b) {
                        if (prev > b) {
                            rb[q] = prev;
                            rw[q] = prevw;
                        } else {
                            rb[q] = b;
                            rw[q] = x;
                        }
                    }
                }
                ++len;
            }
        }
    }
    if (over) {
        big[atomicAdd(nbig, 1u)] = a;
        return;
    }
    const int64_t base = moff[k0];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        if (q < len) {
            tcol[base + q] = rb[q];
            tw[base + q] = (double)rw[q];
        }
    }
    rowlen[a] = len;
}

constexpr int kGalWaveMembers = 256;

// every aggregate listed for pass 1b
__global__ void k_gal_all(int nc, int32_t* __restrict__ big, unsigned* __restrict__ nbig) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < nc) big[a] = a;
    if (a == 0) *nbig = (unsigned)nc;
}

// A wavefront's LDS operations complete in program order: keeping the
// compiler from moving LDS accesses across this point is all the ordering
// the lanes of one wavefront need.
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// pass 1b: the listed aggregates (at most kGalWaveCap entries), a wavefront
// each, wavefronts striding over the list
__global__ void __launch_bounds__(kBlk) k_gal_wave(int n, int64_t nnz, const int32_t* __restrict__ members,
                                                   const int32_t* __restrict__ mstart,
                                                   const int32_t* __restrict__ moff, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const double* __restrict__ w,
                                                   const int32_t* __restrict__ agg,
                                                   const int32_t* __restrict__ big,
                                                   const unsigned* __restrict__ nbig, int32_t* __restrict__ tcol,
                                                   double* __restrict__ tw, int32_t* __restrict__ rowlen) {
    constexpr unsigned long long kNone = ~0ull;
    __shared__ unsigned long long skey[kBlk / kWave][kGalWaveCap];
    __shared__ double sw[kBlk / kWave][kGalWaveCap];
    __shared__ int smrow[kBlk / kWave][kGalWaveMembers];
    __shared__ int smpos[kBlk / kWave][kGalWaveMembers];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    unsigned long long* key = skey[wv];
    double* wt = sw[wv];
    int* mrow = smrow[wv];
    int* mposn = smpos[wv];
    const int count = (int)*nbig;
    for (int q = blockIdx.x * (kBlk / kWave) + wv; q < count; q += gridDim.x * (kBlk / kWave)) {
        const int a = big[q];
        int64_t o0;
        const int E = (int)gal_entries(a, n, nnz, mstart, moff, &o0);
        int P = kWave;
        while (P < E) P <<= 1;
        wave_sync_lds();  // the previous aggregate's LDS reads are done
        // keys (b << 32 | position) in fine order; the own aggregate and
        // the padding sort last as kNone.  With at most kGalWaveMembers
        // members, their row starts and positions go to LDS and every lane
        // loads entries t = lane, lane + 64, ... (its member found by binary
        // search); else member after member.
        const int k0 = mstart[a], k1 = mstart[a + 1];
        const int cnt = k1 - k0;
        if (cnt <= kGalWaveMembers) {
            for (int i = lane; i < cnt; i += kWave) {
                mrow[i] = rp[members[k0 + i]];
                mposn[i] = (int)(moff[k0 + i] - o0);
            }
            wave_sync_lds();
            for (int t = lane; t < E; t += kWave) {
                int lo = 0, hi = cnt - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (mposn[mid] <= t) lo = mid;
                    else hi = mid - 1;
                }
                const int e = mrow[lo] + (t - mposn[lo]);
                const int b = agg[col[e]];
                key[t] = b == a ? kNone : (((unsigned long long)(uint32_t)b << 32) | (uint32_t)t);
                wt[t] = w[e];
            }
        } else {
            for (int k = k0; k < k1; ++k) {
                const int v = members[k];
                const int r0 = rp[v], len = rp[v + 1] - r0;
                const int pos = (int)(moff[k] - o0);
                for (int i = lane; i < len; i += kWave) {
                    const int b = agg[col[r0 + i]];
                    key[pos + i] = b == a ? kNone : (((unsigned long long)(uint32_t)b << 32) | (uint32_t)(pos + i));
                    wt[pos + i] = w[r0 + i];
                }
            }
        }
        for (int i = E + lane; i < P; i += kWave) key[i] = kNone;
        wave_sync_lds();
        // bitonic sort of P keys, ascending
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int p = lane; p < (P >> 1); p += kWave) {
                    const int lo = ((p / j) * 2 * j) + (p % j), hi = lo + j;
                    const unsigned long long x = key[lo], y = key[hi];
                    const bool up = (lo & k) == 0;
                    if ((x > y) == up) {
                        key[lo] = y;
                        key[hi] = x;
                    }
                }
                wave_sync_lds();
            }
        }
        // heads of the runs of equal b, ranked in sorted order; each head
        // adds its run in position (fine) order
        int before = 0;
        for (int p0 = 0; p0 < P; p0 += kWave) {
            const int p = p0 + lane;
            const unsigned long long kp = key[p];
            const bool head = kp != kNone && (p == 0 || (key[p - 1] >> 32) != (kp >> 32));
            const unsigned long long hm = __ballot(head);
            const int rank = before + __popcll(hm & ((1ull << lane) - 1ull));
            if (head) {
                const uint32_t b = (uint32_t)(kp >> 32);
                double sum = 0.0;
                for (int r = p; r < P && key[r] != kNone && (uint32_t)(key[r] >> 32) == b; ++r)
                    sum += wt[key[r] & 0xffffffffull];
                tcol[o0 + rank] = (int32_t)b;
                tw[o0 + rank] = sum;
            }
            before += __popcll(hm);
        }
        if (lane == 0) rowlen[a] = before;
    }
}

// pass 2: the rows into the coarse CSR (row pointers from the scan of
// rowlen).  Rows of at most kGalCompactShort entries (every row the lane
// pass formed) go kGalCompactLanes lanes to a row; the longer ones, all
// among the aggregates listed for pass 1b, a wavefront each.
constexpr int kGalCompactLanes = 4;
constexpr int kGalCompactShort = 32;
constexpr int kGalCompactLongBlocks = 256;
__global__ void k_gal_compact(int nc, const int32_t* __restrict__ mstart, const int32_t* __restrict__ moff,
                              const int32_t* __restrict__ crp, const int32_t* __restrict__ tcol,
                              const double* __restrict__ tw, int32_t* __restrict__ col_out,
                              double* __restrict__ w_out) {
    constexpr int G = kGalCompactLanes;
    const int a = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G);
    const int lane = threadIdx.x & (G - 1);
    if (a >= nc) return;
    const int o = crp[a], len = crp[a + 1] - o;
    if (len > kGalCompactShort) return;
    const int base = moff[mstart[a]];
    for (int t = lane; t < len; t += G) {
        col_out[o + t] = tcol[base + t];
        w_out[o + t] = tw[base + t];
    }
}

__global__ void k_gal_compact_long(const int32_t* __restrict__ mstart, const int32_t* __restrict__ moff,
                                   const int32_t* __restrict__ crp, const int32_t* __restrict__ tcol,
                                   const double* __restrict__ tw, const int32_t* __restrict__ big,
                                   const unsigned* __restrict__ nbig, int32_t* __restrict__ col_out,
                                   double* __restrict__ w_out) {
    const unsigned nb = *nbig;
    const int lane = threadIdx.x & (kWave - 1);
    const unsigned nwaves = (gridDim.x * blockDim.x) / kWave;
    for (unsigned q = (blockIdx.x * blockDim.x + threadIdx.x) / kWave; q < nb; q += nwaves) {
        const int a = big[q];
        const int o = crp[a], len = crp[a + 1] - o;
        if (len <= kGalCompactShort) continue;
        const int base = moff[mstart[a]];
        for (int t = lane; t < len; t += kWave) {
            col_out[o + t] = tcol[base + t];
            w_out[o + t] = tw[base + t];
        }
    }
}

// values the host reads together: a 4- or 8-byte word from each source,
// widened to 64 bits in order
__global__ void k_pack_words(PackWords p, unsigned long long* __restrict__ dst) {
    const int i = threadIdx.x;
    if (i < p.n)
        dst[i] = p.bytes[i] == 4 ? (unsigned long long)*(const unsigned*)p.src[i] : *(const unsigned long long*)p.src[i];
}

// ------------------------------------------------------------------ scan

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlk * kScanItems;

__device__ __forceinline__ long long wave_incl_scan(long long v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        long long t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// exclusive block scan of one value per thread (256 threads); returns the
// block total through *tot
__device__ __forceinline__ long long block_excl_scan(long long v, long long* sh, long long* tot) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    long long inc = wave_incl_scan(v);
    if (lane == 63) sh[wv] = inc;
    __syncthreads();
    long long off = 0, all = 0;
    for (int q = 0; q < kBlk / 64; ++q) {
        if (q < wv) off += sh[q];
        all += sh[q];
    }
    __syncthreads();
    *tot = all;
    return off + inc - v;
}

__global__ void k_scan_reduce(const int32_t* __restrict__ in, int64_t m, long long* __restrict__ bsum) {
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    long long s = 0;
    for (int q = 0; q < kScanItems; ++q) {
        int64_t i = base + q * kBlk + threadIdx.x;
        if (i < m) s += in[i];
    }
    __shared__ long long sh[4];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// single block: exclusive scan of nb block sums in place, total to *total
__global__ void k_scan_top(long long* bsum, int64_t nb, long long* total) {
    __shared__ long long sh[4];
    long long carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kBlk) {
        int64_t i = b0 + threadIdx.x;
        long long v = (i < nb) ? bsum[i] : 0;
        long long tot;
        long long ex = block_excl_scan(v, sh, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_down(const int32_t* __restrict__ in, int32_t* __restrict__ out, int64_t m,
                            const long long* __restrict__ boff) {
    __shared__ int32_t tile[kScanTile];
    __shared__ long long sh[4];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int q = 0; q < kScanItems; ++q) {
        int64_t i = base + q * kBlk + threadIdx.x;
        tile[q * kBlk + threadIdx.x] = (i < m) ? in[i] : 0;
    }
    __syncthreads();
    long long loc[kScanItems];
    long long s = 0;
    for (int q = 0; q < kScanItems; ++q) {
        loc[q] = s;
        s += tile[threadIdx.x * kScanItems + q];
    }
    long long tot;
    long long ex = block_excl_scan(s, sh, &tot);
    long long off = boff[blockIdx.x] + ex;
    __syncthreads();
    for (int q = 0; q < kScanItems; ++q) tile[threadIdx.x * kScanItems + q] = (int32_t)(off + loc[q]);
    __syncthreads();
    for (int q = 0; q < kScanItems; ++q) {
        int64_t i = base + q * kBlk + threadIdx.x;
        if (i < m) out[i] = tile[q * kBlk + threadIdx.x];
    }
}

// -------------------------------------------------------------- Galerkin

// For every fine entry (i, k): key = agg(i) * nc + agg(k), or the sentinel
// nc*nc when both ends are in one aggregate (those entries only feed the
// implicit diagonal).  Keys keep the CSR position, so a stable sort leaves
// equal keys in fine CSR order.
// key of a fine entry: a * mult + b for the coarse entry (a, b), with mult
// at least the coarse vertex count (so keys order by (a, b)); entries
// inside an aggregate get kGalSentinel and sort last
// Packed form (vals == nullptr, pshift > 0): the word is key << pshift | e
// (e the fine entry's position, pshift bits), the sentinel's key part all
// ones; sorting words on the key bits keeps positions in fine CSR order
// within a key, and the weights are read back by position.
template <int G>
__global__ void k_gal_emit(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const double* __restrict__ w, const int32_t* __restrict__ agg, int64_t mult,
                           int pshift, unsigned long long sent,
                           unsigned long long* __restrict__ keys, double* __restrict__ vals) {
    const int lane = threadIdx.x & (G - 1);
    const int gpb = blockDim.x / G;
    for (int row = blockIdx.x * gpb + threadIdx.x / G; row < n; row += gridDim.x * gpb) {
        int a = agg[row];
        int e0 = rp[row], e1 = rp[row + 1];
        for (int e = e0 + lane; e < e1; e += G) {
            int b = agg[col[e]];
            unsigned long long k =
                (a == b) ? sent : (unsigned long long)a * (unsigned long long)mult + (unsigned long long)b;
            if (vals) {
                keys[e] = k;
                vals[e] = w[e];
            } else {
                keys[e] = (k << pshift) | (unsigned long long)e;
            }
        }
    }
}

// k_gal_emit over entries instead of rows, for a level whose longest row
// would keep one lane group busy far longer than the others: each wave
// takes 64 * kEmitPerLane consecutive entries, lane l the entries l, l + 64,
// ...; a lane finds the row of its first entry by binary search on the row
// pointers and follows them from there.  The keys are those of k_gal_emit.
constexpr int kEmitPerLane = 8;

__global__ void k_gal_emit_entries(int n, int64_t nnz, const int32_t* __restrict__ rp,
                                   const int32_t* __restrict__ col, const double* __restrict__ w,
                                   const int32_t* __restrict__ agg, int64_t mult, int pshift,
                                   unsigned long long sent, unsigned long long* __restrict__ keys,
                                   double* __restrict__ vals) {
    const int lane = threadIdx.x & 63;
    const int64_t span = 64 * kEmitPerLane;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * span; c0 < nnz;
         c0 += nwaves * span) {
        int64_t e = c0 + lane;
        if (e >= nnz) continue;
        int lo = 0, hi = n - 1;  // last row r with rp[r] <= e
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rp[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        int r = lo;
        int a = agg[r];
        for (int q = 0; q < kEmitPerLane && e < nnz; ++q, e += 64) {
            if (rp[r + 1] <= e) {
                while (rp[r + 1] <= e) ++r;
                a = agg[r];
            }
            const int b = agg[col[e]];
            const unsigned long long k =
                (a == b) ? sent : (unsigned long long)a * (unsigned long long)mult + (unsigned long long)b;
            if (vals) {
                keys[e] = k;
                vals[e] = w[e];
            } else {
                keys[e] = (k << pshift) | (unsigned long long)e;
            }
        }
    }
}

// number of sorted keys below the sentinel (binary search, one thread)
__global__ void k_count_below(const unsigned long long* __restrict__ keys, int64_t m,
                              unsigned long long sent, unsigned long long* out) {
    if (threadIdx.x != 0) return;
    int64_t lo = 0, hi = m;  // first index with key >= sent
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < sent) lo = mid + 1;
        else hi = mid;
    }
    *out = (unsigned long long)lo;
}

// run heads among the first *nvalid sorted keys (0 beyond), over m entries
__global__ void k_gal_heads(int64_t m, const unsigned long long* __restrict__ nvalid,
                            const unsigned long long* __restrict__ keys, int kshift,
                            int32_t* __restrict__ heads) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int64_t mv = (int64_t)*nvalid;
    heads[t] = (t < mv && (t == 0 || (keys[t] >> kshift) != (keys[t - 1] >> kshift))) ? 1 : 0;
}

// Each run of equal keys is summed in order (fine CSR order); the first
// entry of a run writes the coarse entry and fills the row pointers of the
// coarse rows that start there.
// vals == nullptr: packed words (key << kshift | fine position), weights
// read from the fine level's w by position
// k / mult for keys of the Galerkin sort: a double estimate corrected by
// one (exact below 2^52), else the integer division
__device__ __forceinline__ unsigned long long key_row(unsigned long long k, unsigned long long mult, double inv) {
    if (k >> 52) return k / mult;
    unsigned long long q = (unsigned long long)((double)k * inv);
    if (q * mult > k) --q;
    else if ((q + 1) * mult <= k) ++q;
    return q;
}

// The block's keys and weights are gathered into LDS by all its threads
// first; a run is then summed from LDS, reaching into global memory only
// where it continues past the block.
__global__ void __launch_bounds__(kBlk)
    k_gal_reduce(int64_t m, const unsigned long long* __restrict__ keys, const double* __restrict__ vals,
                 const double* __restrict__ wfine, int kshift, const int32_t* __restrict__ heads,
                 const int32_t* __restrict__ idx, int64_t mult, double inv_mult, int nc, int64_t zc,
                 int32_t* __restrict__ rp, int32_t* __restrict__ col, double* __restrict__ w,
                 double* __restrict__ part) {
    __shared__ unsigned long long sk[kBlk];
    __shared__ double sw[kBlk];
    const int64_t b0 = (int64_t)blockIdx.x * kBlk;
    const int64_t t = b0 + threadIdx.x;
    const unsigned long long pmask = (kshift > 0) ? (~0ull >> (64 - kshift)) : 0ull;
    if (t < m) {
        const unsigned long long kw = keys[t];
        sk[threadIdx.x] = kw >> kshift;
        sw[threadIdx.x] = vals ? vals[t] : wfine[kw & pmask];
    }
    __syncthreads();
    const unsigned long long um = (unsigned long long)mult;
    const int64_t bend = min(b0 + kBlk, m);
    if (part != nullptr && t < m) {
        // pieces: a workgroup that starts inside a run leaves the sum of its
        // entries of that run for k_gal_fix; the last entry's thread ends
        // the row pointers
        if (threadIdx.x == 0 && !heads[t]) {
            double ps = 0.0;
            for (int64_t u = b0; u < bend && sk[u - b0] == sk[0]; ++u) ps += sw[u - b0];
            part[blockIdx.x] = ps;
        }
        if (t == m - 1) {
            const int rl = (int)key_row(sk[threadIdx.x], um, inv_mult);
            for (int r = rl + 1; r <= nc; ++r) rp[r] = (int32_t)zc;
        }
    }
    if (t >= m || !heads[t]) return;
    const unsigned long long k = sk[threadIdx.x];
    const int row = (int)key_row(k, um, inv_mult);
    const int c = (int)(k - (unsigned long long)row * um);
    double s = sw[threadIdx.x];
    int64_t u = t + 1;
    for (; u < bend && sk[u - b0] == k; ++u) s += sw[u - b0];
    if (u == bend && part == nullptr) {
        for (; u < m && (keys[u] >> kshift) == k; ++u) s += vals ? vals[u] : wfine[keys[u] & pmask];
    }
    const int32_t o = idx[t];
    col[o] = c;
    w[o] = s;
    int prow = -1;
    if (t > 0) {
        const unsigned long long kp = (t > b0) ? sk[threadIdx.x - 1] : (keys[t - 1] >> kshift);
        prow = (int)key_row(kp, um, inv_mult);
    }
    for (int r = prow + 1; r <= row; ++r) rp[r] = o;
    if (u == m && part == nullptr) {
        for (int r = row + 1; r <= nc; ++r) rp[r] = (int32_t)zc;
    }
}

// Runs that cross workgroups, pieces mode: the thread of workgroup b whose
// last run goes on into workgroup b + 1 (and starts in b) adds the pieces
// of the following workgroups to the head's sum, in workgroup order.
__global__ void k_gal_fix(int64_t m, int64_t nb, const int32_t* __restrict__ heads,
                          const int32_t* __restrict__ idx, const double* __restrict__ part,
                          double* __restrict__ w) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b + 1 >= nb) return;
    const int64_t e = (b + 1) * kBlk;
    if (heads[e]) return;                        // workgroup b + 1 starts a run
    if (idx[e] - idx[b * kBlk] == 0) return;     // the run's head lies before workgroup b
    const int32_t o = idx[e] - 1;
    double s = w[o];
    for (int64_t bb = b + 1; bb < nb; ++bb) {
        const int64_t eb = bb * kBlk;
        if (heads[eb]) break;
        s += part[bb];
        const int64_t ee = min(eb + kBlk, m);
        if (idx[ee - 1] + heads[ee - 1] - idx[eb] > 0) break;  // the run ends in bb
    }
    w[o] = s;
}

// ------------------------------------------------------------ radix sort

constexpr int kSortItems = 16;
constexpr int kSortTile = kBlk * kSortItems;

__global__ void k_sort_hist(const unsigned long long* __restrict__ keys, int64_t m, int shift,
                            int32_t* __restrict__ counts, int nb) {
    __shared__ int hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int q = 0; q < kSortItems; ++q) {
        int64_t i = base + q * kBlk + threadIdx.x;
        if (i < m) atomicAdd(&hist[(int)((keys[i] >> shift) & 255ull)], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nb + blockIdx.x] = hist[threadIdx.x];
}

// Stable scatter: elements of a tile are ranked in index order; within a
// wave by ballot match on the 8 digit bits, across waves and rounds through
// per-digit running counts in LDS.
template <bool VALS>
__global__ void k_sort_scatter(const unsigned long long* __restrict__ kin,
                               const double* __restrict__ vin, unsigned long long* __restrict__ kout,
                               double* __restrict__ vout, int64_t m, int shift,
                               const int32_t* __restrict__ offs, int nb) {
    __shared__ int wcnt[kBlk / kWave][256];
    __shared__ int run[256];
    __shared__ int base[256];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    base[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
    run[threadIdx.x] = 0;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
    for (int q = 0; q < kSortItems; ++q) {
        for (int w = 0; w < kBlk / kWave; ++w) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        int64_t i = tile0 + q * kBlk + threadIdx.x;
        bool valid = i < m;
        unsigned long long key = valid ? kin[i] : 0ull;
        int d = (int)((key >> shift) & 255ull);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            unsigned long long bal = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bal : ~bal;
        }
        int rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[wv][d] = __popcll(peers);
        __syncthreads();
        {
            int r = run[threadIdx.x];
            for (int w = 0; w < kBlk / kWave; ++w) {
                int t = wcnt[w][threadIdx.x];
                wcnt[w][threadIdx.x] = r;
                r += t;
            }
            run[threadIdx.x] = r;
        }
        __syncthreads();
        if (valid) {
            int64_t pos = (int64_t)base[d] + wcnt[wv][d] + rank;
            kout[pos] = key;
            if constexpr (VALS) vout[pos] = vin[i];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- long rows

// rows with more than lmin entries flagged, then listed in ascending order
// after their count (out[0] = count, out[1 + k] = k-th long row)
__global__ void k_long_flags(int n, const int32_t* __restrict__ rp, int lmin, int32_t* __restrict__ flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = rp[i + 1] - rp[i] > lmin ? 1 : 0;
}

__global__ void k_long_fill(int n, const int32_t* __restrict__ flags, const int32_t* __restrict__ pos,
                            const long long* __restrict__ total, int32_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flags[i]) out[1 + pos[i]] = i;
    if (i == 0) out[0] = (int32_t)*total;
}

// ------------------------------------------------------------- partition

// Row range of each workgroup: boundaries on the merge path of (rows, nnz)
// so every workgroup gets about the same rows + entries.
__global__ void k_partition(int n, int64_t nnz, const int32_t* __restrict__ rp, int nb,
                            int32_t* __restrict__ part) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nb) return;
    if (b == nb) {
        part[b] = n;
        return;
    }
    int64_t total = (int64_t)n + nnz;
    int64_t target = (total * b) / nb;
    // largest r in [0, n] with r + rp[r] <= target
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if ((int64_t)mid + rp[mid] <= target) lo = mid;
        else hi = mid - 1;
    }
    part[b] = lo;
}

__global__ void k_hash_probe(uint64_t seed, int level, int count, unsigned long long* out) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= count) return;
    if (level >= 0) {
        out[v] = hec_key(seed, level, v);
    } else {
        // SplitMix64 sequence: state_v = seed + (v+1) * gamma
        out[v] = mix64(seed + (uint64_t)(v + 1) * 0x9E3779B97F4A7C15ull);
    }
}

__global__ void k_fill_u32(unsigned* p, unsigned v, int64_t m) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = v;
}

}  // namespace

// ================================================================ launchers

hipError_t launch_validate(int n, int64_t nnz, const int32_t* rp, const int32_t* col, const void* w,
                           int wf32, int full, unsigned* flags, hipStream_t s) {
    unsigned nb = nblocks((int64_t)n + 1, kBlk / kValidateLanes);
    if (wf32)
        hipLaunchKernelGGL(k_validate<float>, dim3(nb), dim3(kBlk), 0, s, n, nnz, rp, col,
                           (const float*)w, full, flags);
    else
        hipLaunchKernelGGL(k_validate<double>, dim3(nb), dim3(kBlk), 0, s, n, nnz, rp, col,
                           (const double*)w, full, flags);
    return hipGetLastError();
}

hipError_t launch_convert_w(int64_t nnz, const void* w, int wf32, double* w64, hipStream_t s) {
    unsigned nb = (unsigned)std::min<int64_t>(nblocks(nnz, kBlk), 65536);
    if (nb == 0) return hipSuccess;
    if (wf32)
        hipLaunchKernelGGL(k_convert<float>, dim3(nb), dim3(kBlk), 0, s, nnz, (const float*)w, w64);
    else
        hipLaunchKernelGGL(k_convert<double>, dim3(nb), dim3(kBlk), 0, s, nnz, (const double*)w, w64);
    return hipGetLastError();
}

hipError_t launch_to_f32(int64_t nnz, const double* w64, float* w32, hipStream_t s) {
    unsigned nb = (unsigned)std::min<int64_t>(nblocks(nnz, kBlk), 65536);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_f32, dim3(nb), dim3(kBlk), 0, s, nnz, w64, w32);
    return hipGetLastError();
}

hipError_t launch_to_u8(int64_t nnz, const double* w64, uint8_t* w8, hipStream_t s) {
    unsigned nb = (unsigned)std::min<int64_t>(nblocks(nnz, kBlk), 65536);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_uint<uint8_t>, dim3(nb), dim3(kBlk), 0, s, nnz, w64, w8);
    return hipGetLastError();
}

hipError_t launch_to_u16(int64_t nnz, const double* w64, uint16_t* w16, hipStream_t s) {
    unsigned nb = (unsigned)std::min<int64_t>(nblocks(nnz, kBlk), 65536);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_uint<uint16_t>, dim3(nb), dim3(kBlk), 0, s, nnz, w64, w16);
    return hipGetLastError();
}

hipError_t launch_rowinfo(int n, int lanes, const int32_t* rp, const int32_t* col, const double* w, int unit,
                          int32_t* h, double* bmax, unsigned long long* out, unsigned* iso, hipStream_t s) {
    if (unit) {
        const unsigned nb = (unsigned)std::min<int64_t>(nblocks(n, kBlk), kRowinfoMaxBlocks);
        hipLaunchKernelGGL(k_rowinfo_unit, dim3(nb), dim3(kBlk), 0, s, n, rp, col, h, bmax, iso);
        hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(kBlk), 0, s, bmax, (int)nb, out);
        return hipGetLastError();
    }
    int gpb = kBlk / lanes;
    unsigned nb = (unsigned)std::min<int64_t>(nblocks(n, gpb), kRowinfoMaxBlocks);
    switch (lanes) {
#define CMG_RI(G)                                                                                  \
    case G:                                                                                        \
        hipLaunchKernelGGL(k_rowinfo<G>, dim3(nb), dim3(kBlk), 0, s, n, rp, col, w, h, bmax, iso);  \
        break;
        CMG_RI(1) CMG_RI(2) CMG_RI(4) CMG_RI(8) CMG_RI(16) CMG_RI(32) CMG_RI(64)
#undef CMG_RI
        default:
            return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(kBlk), 0, s, bmax, (int)nb, out);
    return hipGetLastError();
}

hipError_t launch_hec_init(int n, const int32_t* h, uint64_t seed, int level, uint8_t* live,
                           uint8_t* state, int32_t* pairseed, unsigned long long* slot,
                           unsigned long long* flags, hipStream_t s) {
    hipLaunchKernelGGL(k_hec_init, dim3(nblocks(n, kBlk)), dim3(kBlk), 0, s, n, h, seed, level, live,
                       state, pairseed, slot, flags);
    return hipGetLastError();
}

hipError_t launch_hec_round(int n, const int32_t* h, uint64_t seed, int level, uint8_t* live,
                            uint8_t* state, int32_t* pairseed, unsigned long long* slot,
                            unsigned long long* flags, int round, hipStream_t s) {
    const unsigned nb = std::min<unsigned>(nblocks(n, kBlk), kHecRoundBlocks);
    hipLaunchKernelGGL(k_hec_post, dim3(nb), dim3(kBlk), 0, s, n, h, seed, level, live, slot, flags, round);
    hipLaunchKernelGGL(k_hec_accept, dim3(nb), dim3(kBlk), 0, s, n, h, seed, level, live, state,
                       pairseed, slot, flags, round);
    hipLaunchKernelGGL(k_hec_kill, dim3(nb), dim3(kBlk), 0, s, n, h, live, state, slot, flags, round);
    return hipGetLastError();
}

hipError_t launch_hec_attach(int n, const int32_t* h, const uint8_t* state, const int32_t* pairseed,
                             int32_t* rootseed, int32_t* flags, hipStream_t s) {
    hipLaunchKernelGGL(k_hec_attach, dim3(nblocks(n, kBlk)), dim3(kBlk), 0, s, n, h, state, pairseed,
                       rootseed, flags);
    return hipGetLastError();
}

hipError_t launch_hec_label(int n, const int32_t* rootseed, const int32_t* rank, int32_t* agg,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_hec_label, dim3(nblocks(n, kBlk)), dim3(kBlk), 0, s, n, rootseed, rank, agg);
    return hipGetLastError();
}

hipError_t launch_hem_round(int n, const int32_t* rp, const int32_t* col, const double* w, uint64_t seed, int level,
                            int32_t* opener, uint8_t* live, unsigned long long* mkey, unsigned* alive, int round,
                            hipStream_t s) {
    const unsigned nb = nblocks(n, kBlk);
    hipLaunchKernelGGL(k_hem_scan, dim3(nb), dim3(kBlk), 0, s, n, rp, col, seed, level, opener, live, mkey, alive,
                       round);
    hipLaunchKernelGGL(k_hem_match, dim3(nb), dim3(kBlk), 0, s, n, rp, col, w, seed, level, live, mkey, opener);
    return hipGetLastError();
}

hipError_t launch_gal_members(int n, const int32_t* agg, const int32_t* rp, unsigned long long* k0,
                              unsigned long long* k1, int aggbits, int32_t* sort_counts, long long* sort_scan,
                              int32_t* members, int32_t* mdeg, int32_t* mstart, hipStream_t s) {
    hipLaunchKernelGGL(k_gal_member_keys, dim3(nblocks(n, kBlk)), dim3(kBlk), 0, s, n, agg, k0);
    int second = 0;
    hipError_t e = launch_sort(k0, nullptr, k1, nullptr, n, 32, aggbits, sort_counts, sort_scan, &second, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gal_members, dim3(nblocks(n, kBlk)), dim3(kBlk), 0, s, n, second ? k1 : k0, rp, members,
                       mdeg, mstart);
    return hipGetLastError();
}

hipError_t launch_gal_members_count(int n, int ncmax, const int32_t* agg, const int32_t* rp, int32_t* cnt,
                                    long long* scan_tmp, long long* total, int32_t* members, int32_t* mdeg,
                                    int32_t* mstart, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(nblocks(ncmax + 1, kBlk)), dim3(kBlk), 0, s, (unsigned*)cnt, 0u,
                       (int64_t)ncmax + 1);
    hipLaunchKernelGGL(k_mem_count, dim3(nblocks(n, kBlk)), dim3(kBlk), 0, s, n, agg, cnt);
    hipError_t e = launch_scan(cnt, mstart, (int64_t)ncmax + 1, scan_tmp, total, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mem_place, dim3(nblocks(n, kBlk)), dim3(kBlk), 0, s, n, agg, rp, mstart, cnt, members, mdeg);
    return hipGetLastError();
}

hipError_t launch_gal_agg_len(int ncmax, const long long* ncp, int n, int64_t nnz, const int32_t* mstart,
                              const int32_t* moff, unsigned long long* emax, hipStream_t s) {
    const unsigned nb = std::min<unsigned>(nblocks(ncmax, kBlk), (unsigned)kGalLenBlocks);
    hipLaunchKernelGGL(k_gal_agg_len, dim3(nb), dim3(kBlk), 0, s, ncmax, ncp, n, nnz, mstart, moff, emax);
    return hipGetLastError();
}

hipError_t launch_gal_gather(int nc, int n, int64_t nnz, int slots, int unit, int int32sum, const int32_t* members,
                             const int32_t* mstart, const int32_t* moff, const int32_t* rp, const int32_t* col,
                             const double* w, const int32_t* agg, int32_t* tcol, double* tw, int32_t* rowlen,
                             int32_t* big, unsigned* nbig, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kBlk), 0, s, nbig, 0u, (int64_t)1);
    const unsigned nb = nblocks(nc, kBlk);
#define CMG_GAL_LANE(S, U, I)                                                                                     \
    hipLaunchKernelGGL((k_gal_lane<S, U, I>), dim3(nb), dim3(kBlk), 0, s, nc, members, mstart, moff, rp, col, w, agg, \
                       tcol, tw, rowlen, big, nbig)
    switch (slots) {
        case 16:
            if (unit) CMG_GAL_LANE(16, true, true);
            else if (int32sum) CMG_GAL_LANE(16, false, true);
            else CMG_GAL_LANE(16, false, false);
            break;
        case 24:
            if (unit) CMG_GAL_LANE(24, true, true);
            else if (int32sum) CMG_GAL_LANE(24, false, true);
            else CMG_GAL_LANE(24, false, false);
            break;
        case 32:
            if (unit) CMG_GAL_LANE(32, true, true);
            else if (int32sum) CMG_GAL_LANE(32, false, true);
            else CMG_GAL_LANE(32, false, false);
            break;
        case 0: hipLaunchKernelGGL(k_gal_all, dim3(nb), dim3(kBlk), 0, s, nc, big, nbig); break;
        default: return hipErrorInvalidValue;
    }
#undef CMG_GAL_LANE
    hipLaunchKernelGGL(k_gal_wave, dim3(1024), dim3(kBlk), 0, s, n, nnz, members, mstart, moff, rp, col, w, agg,
                       (const int32_t*)big, (const unsigned*)nbig, tcol, tw, rowlen);
    return hipGetLastError();
}

hipError_t launch_pack_words(const PackWords& p, unsigned long long* dst, hipStream_t s) {
    if (p.n < 1 || p.n > kPackWordsMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pack_words, dim3(1), dim3(kWave), 0, s, p, dst);
    return hipGetLastError();
}

hipError_t launch_gal_compact(int nc, const int32_t* mstart, const int32_t* moff, const int32_t* crp,
                              const int32_t* tcol, const double* tw, const int32_t* big, const unsigned* nbig,
                              int32_t* col_out, double* w_out, hipStream_t s) {
    hipLaunchKernelGGL(k_gal_compact, dim3(nblocks((int64_t)nc * kGalCompactLanes, kBlk)), dim3(kBlk), 0, s, nc, mstart,
                       moff, crp, tcol, tw, col_out, w_out);
    hipLaunchKernelGGL(k_gal_compact_long, dim3(kGalCompactLongBlocks), dim3(kBlk), 0, s, mstart, moff, crp, tcol, tw,
                       big, nbig, col_out, w_out);
    return hipGetLastError();
}

hipError_t launch_hem_flags(int n, const int32_t* opener, int32_t* flags, hipStream_t s) {
    hipLaunchKernelGGL(k_hem_flags, dim3(nblocks(n, kBlk)), dim3(kBlk), 0, s, n, opener, flags);
    return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t m) { return (m + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t m, long long* tmp, long long* total,
                       hipStream_t s) {
    int64_t nb = (m + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        return hipMemsetAsync(total, 0, sizeof(long long), s);
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlk), 0, s, in, m, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlk), 0, s, tmp, nb, total);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kBlk), 0, s, in, out, m, tmp);
    return hipGetLastError();
}

hipError_t launch_gal_emit_entries(int n, int64_t nnz, const int32_t* rp, const int32_t* col,
                                   const double* w, const int32_t* agg, int64_t mult, int pshift,
                                   unsigned long long sent, unsigned long long* keys, double* vals,
                                   hipStream_t s) {
    if (nnz == 0) return hipSuccess;
    const unsigned nb = (unsigned)std::min<int64_t>(nblocks(nnz, kBlk / 64 * 64 * kEmitPerLane), 65536);
    hipLaunchKernelGGL(k_gal_emit_entries, dim3(nb), dim3(kBlk), 0, s, n, nnz, rp, col, w, agg, mult, pshift,
                       sent, keys, vals);
    return hipGetLastError();
}

hipError_t launch_gal_emit(int n, int lanes, const int32_t* rp, const int32_t* col, const double* w,
                           const int32_t* agg, int64_t mult, int pshift, unsigned long long sent,
                           unsigned long long* keys, double* vals, hipStream_t s) {
    int gpb = kBlk / lanes;
    unsigned nb = (unsigned)std::min<int64_t>(nblocks(n, gpb), 65536);
    switch (lanes) {
#define CMG_GE(G)                                                                                  \
    case G:                                                                                        \
        hipLaunchKernelGGL(k_gal_emit<G>, dim3(nb), dim3(kBlk), 0, s, n, rp, col, w, agg, mult, pshift, \
                           sent, keys, \
                           vals);                                                                  \
        break;
        CMG_GE(1) CMG_GE(2) CMG_GE(4) CMG_GE(8) CMG_GE(16) CMG_GE(32) CMG_GE(64)
#undef CMG_GE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int64_t sort_tmp_elems(int64_t m) { return 256 * ((m + kSortTile - 1) / kSortTile) + 1; }

hipError_t launch_sort(unsigned long long* k0, double* v0, unsigned long long* k1, double* v1,
                       int64_t m, int shift0, int bits, int32_t* tmp_counts, long long* tmp_scan,
                       int* in_second, hipStream_t s) {
    *in_second = 0;
    if (m <= 1 || bits <= 0) return hipSuccess;
    int nb = (int)((m + kSortTile - 1) / kSortTile);
    int64_t ncounts = 256LL * nb;
    unsigned long long* kin = k0;
    unsigned long long* kout = k1;
    double* vin = v0;
    double* vout = v1;
    long long* scan_tmp = tmp_scan;
    long long* scan_total = tmp_scan + scan_tmp_elems(ncounts);
    for (int shift = shift0; shift < shift0 + bits; shift += 8) {
        hipLaunchKernelGGL(k_sort_hist, dim3(nb), dim3(kBlk), 0, s, kin, m, shift, tmp_counts, nb);
        hipError_t e = launch_scan(tmp_counts, tmp_counts, ncounts, scan_tmp, scan_total, s);
        if (e != hipSuccess) return e;
        if (v0)
            hipLaunchKernelGGL(k_sort_scatter<true>, dim3(nb), dim3(kBlk), 0, s, kin, vin, kout, vout, m,
                               shift, tmp_counts, nb);
        else
            hipLaunchKernelGGL(k_sort_scatter<false>, dim3(nb), dim3(kBlk), 0, s, kin, vin, kout, vout, m,
                               shift, tmp_counts, nb);
        std::swap(kin, kout);
        std::swap(vin, vout);
        *in_second ^= 1;
    }
    return hipGetLastError();
}

hipError_t launch_count_below(const unsigned long long* keys, int64_t m, unsigned long long sent,
                              unsigned long long* out, hipStream_t s) {
    hipLaunchKernelGGL(k_count_below, dim3(1), dim3(64), 0, s, keys, m, sent, out);
    return hipGetLastError();
}

hipError_t launch_gal_heads(int64_t m, const unsigned long long* nvalid, const unsigned long long* keys,
                            int kshift, int32_t* heads, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gal_heads, dim3(nblocks(m, kBlk)), dim3(kBlk), 0, s, m, nvalid, keys, kshift, heads);
    return hipGetLastError();
}

int64_t gal_part_elems(int64_t m) { return (m + kBlk - 1) / kBlk + 1; }

hipError_t launch_gal_reduce(int64_t m, const unsigned long long* keys, const double* vals,
                             const double* wfine, int kshift, const int32_t* heads, const int32_t* idx,
                             int64_t mult, int nc, int64_t zc, int32_t* rp_out, int32_t* col_out,
                             double* w_out, double* part, hipStream_t s) {
    if (m == 0) return hipSuccess;
    const int64_t nb = nblocks(m, kBlk);
    hipLaunchKernelGGL(k_gal_reduce, dim3((unsigned)nb), dim3(kBlk), 0, s, m, keys, vals, wfine, kshift,
                       heads, idx, mult, 1.0 / (double)mult, nc, zc, rp_out, col_out, w_out, part);
    if (part != nullptr && nb > 1)
        hipLaunchKernelGGL(k_gal_fix, dim3(nblocks(nb, kBlk)), dim3(kBlk), 0, s, m, nb, heads, idx, part, w_out);
    return hipGetLastError();
}

hipError_t launch_long_rows(int n, const int32_t* rp, int lmin, int32_t* flags, int32_t* pos, long long* scan_tmp,
                            long long* total, int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_long_flags, dim3(nblocks(n, kBlk)), dim3(kBlk), 0, s, n, rp, lmin, flags);
    hipError_t e = launch_scan(flags, pos, n, scan_tmp, total, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_long_fill, dim3(nblocks(n, kBlk)), dim3(kBlk), 0, s, n, (const int32_t*)flags,
                       (const int32_t*)pos, (const long long*)total, out);
    return hipGetLastError();
}

hipError_t launch_partition(int n, int64_t nnz, const int32_t* rp, int nb, int32_t* part,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_partition, dim3(nblocks((int64_t)nb + 1, kBlk)), dim3(kBlk), 0, s, n, nnz, rp,
                       nb, part);
    return hipGetLastError();
}

hipError_t launch_hash_probe(uint64_t seed, int level, int count, unsigned long long* out,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_hash_probe, dim3(nblocks(count, kBlk)), dim3(kBlk), 0, s, seed, level, count, out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, unsigned v, int64_t m, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(nblocks(m, kBlk)), dim3(kBlk), 0, s, p, v, m);
    return hipGetLastError();
}

}  // namespace cmg
