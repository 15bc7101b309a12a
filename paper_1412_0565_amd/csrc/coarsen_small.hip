// Setup of the small levels in one workgroup: for a chain of levels of at
// most kChainMaxN vertices, the row pass (Gershgorin shift, heaviest
// neighbours), HEC (Algorithm 2, in the round-synchronous form of the grid
// kernels in setup.hip) and the Galerkin coarse graph (Section 2, the
// Proposition on restriction) run level after level inside one launch,
// separated only by workgroup barriers.  The grid kernels need about 40
// launches and 7 host synchronisations per level; on small levels those
// gaps, not the work, set the setup time.
//
// The Galerkin product is formed per coarse row: the members of aggregate
// a are visited in increasing index and their entries in CSR order, so the
// contributions to each coarse entry (a, b) are added in fine CSR order,
// the order the grid path's stable sort produces.  Results are bit-exact
// with the grid path and the oracle (integer and real weights alike).
#include "cmg_internal.h"

namespace cmg {

namespace {

constexpr uint8_t kSeedC = 1;
constexpr uint8_t kPartnerC = 2;
constexpr unsigned long long kNoKeyC = 0xFFFFFFFFFFFFFFFFull;

__device__ __forceinline__ unsigned long long ld_slot(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_slot(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inclusive scan over a wavefront.
__device__ __forceinline__ long long wave_scan_incl(long long v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of in[0..m) into out[0..m) by the whole workgroup (each
// thread a contiguous chunk); returns the total.  `in` is read before any
// out[] element is written, so in == out is allowed.  `sh` holds 17 longs.
__device__ long long chain_scan(const int32_t* in, int32_t* out, int m, long long* sh) {
    const int T = blockDim.x, tid = threadIdx.x;
    const int per = (m + T - 1) / T;
    const int lo = min(m, tid * per), hi = min(m, lo + per);
    long long s = 0;
    for (int i = lo; i < hi; ++i) s += in[i];
    const long long inc = wave_scan_incl(s);
    const int wv = tid >> 6, nw = T >> 6;
    if ((tid & 63) == 63) sh[wv] = inc;
    __syncthreads();
    long long off = 0, all = 0;
    for (int q = 0; q < nw; ++q) {
        if (q < wv) off += sh[q];
        all += sh[q];
    }
    long long run = off + inc - s;
    for (int i = lo; i < hi; ++i) {
        const int x = in[i];
        out[i] = (int32_t)run;
        run += x;
    }
    __syncthreads();
    return all;
}

// max over the workgroup of 4 doubles (exact, order independent)
__device__ void block_max4(double (&m)[4], double* sm) {
    for (int o = 32; o > 0; o >>= 1)
        for (int q = 0; q < 4; ++q) m[q] = fmax(m[q], __shfl_xor(m[q], o, kWave));
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 4; ++q) sm[q * 16 + wv] = m[q];
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
        double r = 0.0;
        for (int w = 0; w < nw; ++w) r = fmax(r, sm[q * 16 + w]);
        m[q] = r;
    }
    __syncthreads();
}

// Columns a thread keeps in registers while it forms a coarse row.
constexpr int kChainSlots = 12;
// Longest fine row of a level this kernel coarsens (measured on MI355X:
// 3D-grid levels with 27-47 entries per row took 0.27-1.9 ms here against
// a few hundred microseconds on the grid kernels).
constexpr int kChainLongRow = 24;
constexpr size_t kChainLds = sizeof(int32_t) * 2 * (kChainMaxN / 2 + 1);

__global__ void __launch_bounds__(kChainThreads) k_coarsen_chain(ChainJob J) {
    extern __shared__ int32_t lds_cnt[];  // acnt, afill
    int32_t* acnt = lds_cnt;
    int32_t* afill = lds_cnt + (kChainMaxN / 2 + 1);
    __shared__ long long sh[17];
    __shared__ double sm[4 * 16];
    __shared__ int s_bad;
    __shared__ int s_iso;
    const int tid = threadIdx.x, T = blockDim.x;
    if (tid == 0) s_iso = 0;
    __syncthreads();
    int n = J.n0;
    int64_t nnz = J.nnz0;
    const int32_t* rp = J.rp0;
    const int32_t* col = J.col0;
    const double* w = J.w0;
    int64_t i32_used = 0, cw_used = 0;
    int64_t cur_rp_off = -1, cur_cw_off = -1;
    int K = 0, collapsed = 0, stop_reason = 0;
    for (int k = 0;; ++k) {
        const int level = J.level0 + k;
        // ---- row pass: h, g = 2 max d, largest weight, FP32 rounding, longest row
        double m4[4] = {0.0, 0.0, 0.0, 0.0};
        for (int v = tid; v < n; v += T) {
            const int a = rp[v], b = rp[v + 1];
            m4[3] = fmax(m4[3], (double)(b - a));
            double bw = -1.0, d = 0.0;
            int bc = 0x7fffffff;
            for (int e = a; e < b; ++e) {
                const double x = w[e];
                const int c = col[e];
                d += x;
                m4[2] = fmax(m4[2], fabs(x - (double)(float)x));
                if (x > bw || (x == bw && c < bc)) {
                    bw = x;
                    bc = c;
                }
            }
            // a vertex with no neighbour (a component that became one
            // aggregate) names itself and stops the chain below
            if (b == a) {
                bc = v;
                s_iso = 1;
            }
            J.h[v] = bc;
            m4[0] = fmax(m4[0], 2.0 * d);
            m4[1] = fmax(m4[1], bw);
        }
        block_max4(m4, sm);
        ChainHdr hd{};
        hd.n = n;
        hd.nnz = nnz;
        hd.g = m4[0];
        hd.wmax = m4[1];
        hd.w32err = m4[2];
        hd.maxlen = m4[3];
        hd.rp_off = cur_rp_off;
        hd.cw_off = cur_cw_off;
        hd.agg_off = -1;
        hd.rounds = 0;
        K = k + 1;
        if (n <= J.coarsest_n || k + 1 >= J.max_levels) {
            stop_reason = (n <= J.coarsest_n) ? 1 : 5;
            if (tid == 0) J.hdr[k] = hd;
            break;
        }
        if (s_iso) {
            // HEC needs every vertex to have a neighbour (CMG_E_ISOLATED)
            stop_reason = 6;
            if (tid == 0) J.hdr[k] = hd;
            break;
        }
        if (hd.maxlen > kChainLongRow) {
            // rows this long make coarse rows that outgrow the register
            // slots, and one thread per row then works in global scratch,
            // slower than the grid kernels' sort: leave the level to them
            stop_reason = 4;
            if (tid == 0) J.hdr[k] = hd;
            break;
        }
        // ---- HEC: candidates, greedy rounds
        for (int v = tid; v < n; v += T) {
            J.pairseed[v] = v;
            J.live[v] = (hec_key(J.seed, level, v) < hec_key(J.seed, level, J.h[v])) ? 1 : 0;
            J.state[v] = 0;
            st_slot(&J.slot[v], kNoKeyC);
        }
        __syncthreads();
        int rounds = 0;
        while (true) {
            for (int v = tid; v < n; v += T) {
                if (!J.live[v]) continue;
                const unsigned long long kv = hec_key(J.seed, level, v);
                atomicMin(&J.slot[v], kv);
                atomicMin(&J.slot[J.h[v]], kv);
            }
            __syncthreads();
            for (int v = tid; v < n; v += T) {
                if (!J.live[v]) continue;
                const unsigned long long kv = hec_key(J.seed, level, v);
                const int m = J.h[v];
                if (ld_slot(&J.slot[v]) == kv && ld_slot(&J.slot[m]) == kv) {
                    J.state[v] = kSeedC;
                    J.state[m] = kPartnerC;
                    J.pairseed[v] = v;
                    J.pairseed[m] = v;
                    J.live[v] = 0;
                }
            }
            __syncthreads();
            int alive = 0;
            for (int v = tid; v < n; v += T) {
                if (!J.live[v]) continue;
                const int m = J.h[v];
                if (J.state[v] != 0 || J.state[m] != 0) {
                    J.live[v] = 0;
                } else {
                    st_slot(&J.slot[v], kNoKeyC);
                    st_slot(&J.slot[m], kNoKeyC);
                    alive = 1;
                }
            }
            ++rounds;
            if (!__syncthreads_or(alive)) break;
        }
        hd.rounds = rounds;
        // ---- attach: follow h to a matched vertex; seeds flagged
        for (int v = tid; v < n; v += T) {
            int r = v;
            for (int guard = 0; guard < n && J.state[r] == 0; ++guard) r = J.h[r];
            J.rootseed[v] = J.pairseed[r];
            J.rank[v] = (J.state[v] == kSeedC) ? 1 : 0;
        }
        __syncthreads();
        const int nc = (int)chain_scan(J.rank, J.rank, n, sh);
        if (nc < 2) {
            collapsed = 1;
            stop_reason = 2;
            if (tid == 0) J.hdr[k] = hd;
            break;
        }
        // room for agg[n], rp[nc+1] in the int arena and the coarse entries
        // (at most nnz: every coarse entry comes from a fine one; at most
        // nc (nc - 1): no diagonal)
        const int64_t nnz_bound = min(nnz, (int64_t)nc * (int64_t)(nc - 1));
        if (i32_used + n + nc + 1 > J.ai32_cap || cw_used + nnz_bound > J.acw_cap) {
            stop_reason = 3;
            if (tid == 0) J.hdr[k] = hd;
            break;
        }
        int32_t* agg = J.ai32 + i32_used;
        hd.agg_off = i32_used;
        for (int v = tid; v < n; v += T) agg[v] = J.rank[J.rootseed[v]];
        for (int a = tid; a < nc; a += T) {
            acnt[a] = 0;
            afill[a] = 0;
        }
        if (tid == 0) s_bad = 0;
        __syncthreads();
        // ---- members of each aggregate, in increasing vertex index
        for (int v = tid; v < n; v += T) atomicAdd(&acnt[agg[v]], 1);
        __syncthreads();
        for (int a = tid; a < nc; a += T) J.astart[a] = acnt[a];
        __syncthreads();
        chain_scan(J.astart, J.astart, nc, sh);
        for (int v = tid; v < n; v += T) {
            const int a = agg[v];
            J.members[J.astart[a] + atomicAdd(&afill[a], 1)] = v;
        }
        __syncthreads();
        for (int a = tid; a < nc; a += T) {
            int32_t* ms = J.members + J.astart[a];
            const int cnt = acnt[a];
            for (int i = 1; i < cnt; ++i) {
                const int x = ms[i];
                int j = i - 1;
                while (j >= 0 && ms[j] > x) {
                    ms[j + 1] = ms[j];
                    --j;
                }
                ms[j + 1] = x;
            }
            int64_t deg = 0;
            for (int i = 0; i < cnt; ++i) deg += rp[ms[i] + 1] - rp[ms[i]];
            if (deg > kChainMaxRow) s_bad = 1;
            J.soff[a] = (int32_t)deg;
        }
        __syncthreads();
        if (s_bad) {
            // a coarse row too long for one thread's accumulation: leave this
            // level to the grid kernels (its aggregates are discarded)
            stop_reason = 4;
            hd.agg_off = -1;
            if (tid == 0) J.hdr[k] = hd;
            break;
        }
        chain_scan(J.soff, J.soff, nc, sh);
        // aggregate of every entry's column, all threads over all entries:
        // the row loop below then reads its entries without a dependent load
        for (int64_t e = tid; e < nnz; e += T) J.bcol[e] = agg[col[e]];
        __syncthreads();
        // ---- Galerkin: one thread per coarse row, contributions added in
        // fine CSR order, row sorted by coarse column.  The row is formed in
        // the thread's register slots; a row with more distinct columns
        // moves to its global scratch and goes on there.
        for (int a = tid; a < nc; a += T) {
            const int32_t* ms = J.members + J.astart[a];
            const int cnt = acnt[a];
            int32_t* mb = J.mb + J.soff[a];
            double* mw = J.mw + J.soff[a];
            // the row in registers: columns rb[0..len) (unused: INT_MAX) and
            // their sums; every slot operation is unrolled and branch-free
            int rb[kChainSlots];
            double rw[kChainSlots];
#pragma unroll
            for (int q = 0; q < kChainSlots; ++q) {
                rb[q] = 0x7fffffff;
                rw[q] = 0.0;
            }
            int len = 0;
            bool in_regs = true;
            for (int i = 0; i < cnt; ++i) {
                const int m = ms[i];
                const int e0 = rp[m], e1 = rp[m + 1];
                if (e0 >= e1) continue;
                // one entry ahead: the next entry's coarse column and weight
                // are loaded before this one is added
                int bn = J.bcol[e0];
                double xn = w[e0];
                for (int e = e0; e < e1; ++e) {
                    const int b = bn;
                    const double x = xn;
                    if (e + 1 < e1) {
                        xn = w[e + 1];
                        bn = J.bcol[e + 1];
                    }
                    if (b == a) continue;
                    if (in_regs) {
                        bool found = false;
#pragma unroll
                        for (int q = 0; q < kChainSlots; ++q) {
                            if (rb[q] == b) {
                                rw[q] += x;
                                found = true;
                            }
                        }
                        if (found) continue;
                        if (len < kChainSlots) {
#pragma unroll
                            for (int q = 0; q < kChainSlots; ++q) {
                                if (q == len) {
                                    rb[q] = b;
                                    rw[q] = x;
                                }
                            }
                            ++len;
                            continue;
                        }
                        // more columns than slots: the row goes on in global scratch
#pragma unroll
                        for (int q = 0; q < kChainSlots; ++q) {
                            mb[q] = rb[q];
                            mw[q] = rw[q];
                        }
                        in_regs = false;
                    }
                    int q = 0;
                    while (q < len && mb[q] != b) ++q;
                    if (q == len) {
                        mb[len] = b;
                        mw[len] = x;
                        ++len;
                    } else {
                        mw[q] += x;
                    }
                }
            }
            if (in_regs) {
                // odd-even transposition sort by column (unused slots last)
#pragma unroll
                for (int pass = 0; pass < kChainSlots; ++pass) {
#pragma unroll
                    for (int q = pass & 1; q + 1 < kChainSlots; q += 2) {
                        if (rb[q] > rb[q + 1]) {
                            const int tb = rb[q];
                            rb[q] = rb[q + 1];
                            rb[q + 1] = tb;
                            const double tw = rw[q];
                            rw[q] = rw[q + 1];
                            rw[q + 1] = tw;
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < kChainSlots; ++q) {
                    if (q < len) {
                        mb[q] = rb[q];
                        mw[q] = rw[q];
                    }
                }
                J.rcount[a] = len;
                continue;
            }
            for (int i = 1; i < len; ++i) {
                const int b = mb[i];
                const double x = mw[i];
                int j = i - 1;
                while (j >= 0 && mb[j] > b) {
                    mb[j + 1] = mb[j];
                    mw[j + 1] = mw[j];
                    --j;
                }
                mb[j + 1] = b;
                mw[j + 1] = x;
            }
            J.rcount[a] = len;
        }
        __syncthreads();
        int32_t* rpc = J.ai32 + i32_used + n;
        const int64_t nnzc = chain_scan(J.rcount, rpc, nc, sh);
        if (tid == 0) rpc[nc] = (int32_t)nnzc;
        int32_t* colc = J.acol + cw_used;
        double* wc = J.aw + cw_used;
        for (int a = tid; a < nc; a += T) {
            const int32_t* mb = J.mb + J.soff[a];
            const double* mw = J.mw + J.soff[a];
            const int base = rpc[a], len = J.rcount[a];
            for (int q = 0; q < len; ++q) {
                colc[base + q] = mb[q];
                wc[base + q] = mw[q];
            }
        }
        if (tid == 0) J.hdr[k] = hd;
        cur_rp_off = i32_used + n;
        cur_cw_off = cw_used;
        i32_used += n + nc + 1;
        cw_used += nnzc;
        __syncthreads();
        n = nc;
        nnz = nnzc;
        rp = rpc;
        col = colc;
        w = wc;
    }
    if (tid == 0) {
        J.out[0] = K;
        J.out[1] = collapsed;
        J.out[2] = stop_reason;
    }
}

}  // namespace

hipError_t launch_coarsen_chain(const ChainJob& job, hipStream_t s) {
    hipLaunchKernelGGL(k_coarsen_chain, dim3(1), dim3(kChainThreads), kChainLds, s, job);
    return hipGetLastError();
}

}  // namespace cmg
