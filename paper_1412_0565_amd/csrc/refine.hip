// Coarsest solve and cascadic refinement kernels (Algorithm 1, Steps 2-3;
// power iteration, Algorithm 3).
//
// Power iteration on B_g = gI - L with the constant vector deflated.  The
// kernels never normalise a vector in place: a level keeps an unnormalised
// vector w plus scalars (mu, s) with the current iterate
// v = (w - mu) * s, deflated and of unit norm.  One step computes
//   y_i = ((gI - L) v)_i = s * ( g (w_i - mu) + sum_k a_ik (w_k - w_i) )
// (mu cancels in the Laplacian part because L 1 = 0) and, in the same pass,
// the FP64 sums  Sy = sum y, Syy = sum y^2, Syx = sum y v, Sx = sum v.
// From them:  mu' = Sy/n,  ||y - mu'||^2 = Syy - Sy mu',  s' = 1/||.||,
// and the stopping quantity (u, v) = s' (Syx - mu' Sx) for u = (y-mu')s'.
// Every reduction has a fixed order, so results are reproducible bitwise.
#include <algorithm>
#include <mutex>

#include "cmg_internal.h"

namespace cmg {

namespace {

__device__ __forceinline__ double ld_any(const void* p, int fp32, int64_t i) {
    return fp32 ? (double)gld((const float*)p, i) : gld((const double*)p, i);
}

__device__ __forceinline__ double ld_agent(const double* p) {
    unsigned long long b =
        __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)b);
}

__device__ __forceinline__ void st_agent(double* p, double v) {
    __hip_atomic_store((unsigned long long*)p, (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup b runs on XCD b % 8; give each XCD a contiguous range of row
// blocks so neighbouring rows (and their x gathers) share one L2.  XCD x
// runs the blocks x, x + 8, ... of [0, nb): nb / 8 of them, one more for the
// first nb % 8 XCDs.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// ~2 s at the 100 MHz constant clock: a safety bound, never reached when
// the grid is co-resident (launches are sized to the measured residency).
constexpr long long kSpinTicks = 200000000LL;

// Grids up to this many workgroups use the all-read form below (measured
// on MI355X: 88 and 112 workgroups 7% and 3% faster per level than with
// the broadcast, 184 workgroups 17% slower).
constexpr int kAllReadMax = 128;

// Spin until *p == e.  The abort flag and the time bound are checked only
// every 64 polls: the flag shares one line that every waiter would hit.
// Returns false (after raising the abort flag, recording the first
// timeout) if the wait was given up.
__device__ __forceinline__ bool spin_until(const unsigned long long* p, unsigned long long e,
                                           GridSync* gs, int nb, int tag) {
    const long long t0 = wall_clock64();
    unsigned polls = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != e) {
        __builtin_amdgcn_s_sleep(1);
        if ((++polls & 63u) == 0u &&
            (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
             wall_clock64() - t0 > kSpinTicks)) {
            if (atomicOr(&gs->abort, 1u) == 0u) {
                gs->where = (unsigned)nb | ((unsigned)(tag + 2) << 16);
                gs->abort_epoch = e;
            }
            return false;
        }
    }
    return true;
}

__device__ __forceinline__ GridSlot* bcast_line(GridSlot* bcast, int q) {
    return (GridSlot*)((char*)bcast + (size_t)q * kBcastStride);
}

// Grid-wide sum of NV (<= 7) doubles with a barrier, free of contended
// atomics: every workgroup writes its block sums and the barrier epoch into
// its own 64-byte slot (release); slots alternate between two banks by
// epoch parity, so a slot is rewritten only after every workgroup has
// passed the barrier in between.
//  * Small grids (nb <= kAllReadMax): every workgroup polls all slots and
//    adds them itself (one memory round trip less).
//  * Larger grids: workgroup 0 polls all slots, adds them and publishes
//    the totals with the epoch on kBcastLines lines that sit on different
//    memory channels (release); workgroup b waits on line b % kBcastLines,
//    so no line has more than nb / kBcastLines pollers.
// Either way the totals are the slot values added in slot order by the
// same fixed tree, so they do not depend on which workgroup adds them or
// on arrival order.  Returns false if the barrier timed out or was aborted;
// then every workgroup leaves.
template <int NV>
__device__ bool grid_allreduce_impl(double (&v)[NV], GridSync* gs, GridSlot* slots, GridSlot* bcast,
                                    unsigned long long& epoch, int vb, int lb, int nb, double* red,
                                    int tag) {
    __shared__ double s_tot[NV];
    __shared__ int s_ok;
    const unsigned long long e = ++epoch;
    GridSlot* bank = slots + (e & 1ull) * (unsigned long long)nb;
    const bool master = vb == 0;
    block_sum<NV>(v, red);
    if (threadIdx.x == 0) {
        GridSlot* my = bank + lb;
#pragma unroll
        for (int q = 0; q < NV; ++q) my->v[q] = v[q];
        __hip_atomic_store(&my->epoch, e, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        s_ok = 1;
    }
    __syncthreads();
    const bool allread = nb <= kAllReadMax;
    if (allread || master) {
        double acc[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            if (!spin_until(&bank[b].epoch, e, gs, nb, tag)) {
                s_ok = 0;
                break;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
            for (int q = 0; q < NV; ++q) acc[q] += ld_agent(&bank[b].v[q]);
        }
        block_sum<NV>(acc, red);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int q = 0; q < NV; ++q) s_tot[q] = acc[q];
        }
        if (master && s_ok) {
            if (allread) {
                if (threadIdx.x == 0)
                    __hip_atomic_store(&gs->epoch, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else if (threadIdx.x < kBcastLines) {
                GridSlot* line = bcast_line(bcast, threadIdx.x);
#pragma unroll
                for (int q = 0; q < NV; ++q) st_agent(&line->v[q], acc[q]);
                __hip_atomic_store(&line->epoch, e, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                if (threadIdx.x == 0)
                    __hip_atomic_store(&gs->epoch, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    } else if (threadIdx.x == 0) {
        GridSlot* line = bcast_line(bcast, vb % kBcastLines);
        if (!spin_until(&line->epoch, e, gs, nb, tag)) s_ok = 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
        for (int q = 0; q < NV; ++q) s_tot[q] = ld_agent(&line->v[q]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = s_tot[q];
    const bool ok = s_ok != 0;
    __syncthreads();
    return ok;
}

__device__ __forceinline__ unsigned long long start_epoch(GridSync* gs) {
    return __hip_atomic_load(&gs->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One power-iteration step on rows [r0, r1) with G lanes per row.  Lane 0
// of each group owns the row: writes y and adds {y, y^2, y v, v} to acc.
template <int G, typename T>
__device__ __forceinline__ void pi_rows(const LevelDev& L, const T* __restrict__ win,
                                        T* __restrict__ wout, double mu, double s, int r0, int r1,
                                        double (&acc)[4]) {
    const int lane = threadIdx.x & (G - 1);
    const int ngroups = blockDim.x / G;
    const T* __restrict__ wv = (const T*)(sizeof(T) == 4 ? (const void*)L.w32 : (const void*)L.w64);
    const int32_t* __restrict__ rp = L.rp;
    const int32_t* __restrict__ col = L.col;
    const double g = L.g;
    for (int i = r0 + (int)(threadIdx.x / G); i < r1; i += ngroups) {
        const int a = rp[i], b = rp[i + 1];
        const double wi = (double)win[i];
        double t = 0.0;
        for (int e = a + lane; e < b; e += G) t += (double)wv[e] * ((double)win[col[e]] - wi);
        t = group_sum_t<G>(t);
        if (lane == 0) {
            const double x = (wi - mu) * s;
            const T ys = (T)(s * (g * (wi - mu) + t));
            wout[i] = ys;
            const double yd = (double)ys;
            acc[0] += yd;
            acc[1] += yd * yd;
            acc[2] += yd * x;
            acc[3] += x;
        }
    }
}

template <typename T>
__device__ __forceinline__ void pi_rows_dispatch(int G, const LevelDev& L, const T* win, T* wout,
                                                 double mu, double s, int r0, int r1,
                                                 double (&acc)[4]) {
    switch (G) {
        case 1: pi_rows<1, T>(L, win, wout, mu, s, r0, r1, acc); break;
        case 2: pi_rows<2, T>(L, win, wout, mu, s, r0, r1, acc); break;
        case 4: pi_rows<4, T>(L, win, wout, mu, s, r0, r1, acc); break;
        case 8: pi_rows<8, T>(L, win, wout, mu, s, r0, r1, acc); break;
        case 16: pi_rows<16, T>(L, win, wout, mu, s, r0, r1, acc); break;
        case 32: pi_rows<32, T>(L, win, wout, mu, s, r0, r1, acc); break;
        default: pi_rows<64, T>(L, win, wout, mu, s, r0, r1, acc); break;
    }
}

// ---------------------------------------------------------- coarsest

// coarsest levels up to this size keep A and V in LDS (2 n^2 doubles)
constexpr int kDenseLds = 48;

// Dense coarsest solve in one workgroup: L^J assembled densely, Jacobi
// eigenvalue iteration with the parallel round-robin ("tournament") order
// (n/2 disjoint plane rotations per step, n-1 steps per sweep; disjoint
// rotations commute, so a step equals applying them one after another),
// until the off-diagonal norm is <= 1e-14 ||A||_F.  The vector is the
// normalised projection of the ramp z_i = i - (n-1)/2 onto the eigenspace
// of all eigenvalues (above the smallest) within 1e-10 ||A||_F of
// lambda_2; a hashed uniform vector replaces z if that projection is tiny.
__global__ void __launch_bounds__(256) k_coarse_jobs(const CoarseJob* __restrict__ jobs) {
    extern __shared__ double dyn[];
    const CoarseJob& Jb = jobs[blockIdx.x];
    const LevelDev L = Jb.L;
    LevelState* st = Jb.st;
    double* Ag = Jb.A;
    double* Vg = Jb.V;
    double* ev = Jb.ev;
    int32_t* idx = Jb.idx;
    const uint64_t seed = Jb.seed;
    FinishOut* fo = Jb.fo;
    __shared__ double red[16 * 2 + 8];
    __shared__ double cs_c[128], cs_s[128];
    __shared__ int pr_p[128], pr_q[128];
    const int n = L.n;
    const int tid = threadIdx.x, nt = blockDim.x;
    double* A = (n <= kDenseLds) ? dyn : Ag;
    double* V = (n <= kDenseLds) ? dyn + n * n : Vg;
    for (int t = tid; t < n * n; t += nt) {
        A[t] = 0.0;
        V[t] = ((t / n) == (t % n)) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int i = tid; i < n; i += nt) {
        double d = 0.0;
        for (int e = L.rp[i]; e < L.rp[i + 1]; ++e) {
            A[i * n + L.col[e]] = -L.w64[e];
            d += L.w64[e];
        }
        A[i * n + i] = d;
    }
    __syncthreads();
    double f[1] = {0.0};
    for (int t = tid; t < n * n; t += nt) f[0] += A[t] * A[t];
    block_sum<1>(f, red);
    const double fro = sqrt(f[0]);
    const int m = n + (n & 1);  // players in the tournament (dummy index n if odd)
    const int npair = m / 2;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double o[1] = {0.0};
        for (int t = tid; t < n * n; t += nt)
            if (t / n != t % n) o[0] += A[t] * A[t];
        block_sum<1>(o, red);
        if (sqrt(o[0]) <= 1e-14 * fro) break;
        for (int step = 0; step < m - 1; ++step) {
            // pairs of this step and their rotations (from the current A)
            for (int i = tid; i < npair; i += nt) {
                int a, b;
                if (i == 0) {
                    a = 0;
                    b = (step % (m - 1)) + 1;
                } else {
                    a = ((step + i) % (m - 1)) + 1;
                    b = ((step - i + (m - 1)) % (m - 1)) + 1;
                }
                int p = min(a, b), q = max(a, b);
                double c = 1.0, s = 0.0;
                if (q < n) {
                    double apq = A[p * n + q];
                    if (apq != 0.0) {
                        double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                        double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                }
                pr_p[i] = p;
                pr_q[i] = (q < n) ? q : -1;
                cs_c[i] = c;
                cs_s[i] = s;
            }
            __syncthreads();
            // rows p, q: A <- J^T A
            for (int t = tid; t < npair * n; t += nt) {
                int i = t / n, k = t % n;
                int p = pr_p[i], q = pr_q[i];
                if (q < 0 || cs_s[i] == 0.0) continue;
                double c = cs_c[i], s = cs_s[i];
                double x = A[p * n + k], y = A[q * n + k];
                A[p * n + k] = c * x - s * y;
                A[q * n + k] = s * x + c * y;
            }
            __syncthreads();
            // columns p, q: A <- A J ; V <- V J
            for (int t = tid; t < npair * n; t += nt) {
                int i = t / n, k = t % n;
                int p = pr_p[i], q = pr_q[i];
                if (q < 0 || cs_s[i] == 0.0) continue;
                double c = cs_c[i], s = cs_s[i];
                double x = A[k * n + p], y = A[k * n + q];
                A[k * n + p] = c * x - s * y;
                A[k * n + q] = s * x + c * y;
                x = V[k * n + p];
                y = V[k * n + q];
                V[k * n + p] = c * x - s * y;
                V[k * n + q] = s * x + c * y;
            }
            __syncthreads();
        }
    }
    for (int k = tid; k < n; k += nt) ev[k] = A[k * n + k];
    __syncthreads();
    if (tid == 0) {
        for (int i = 0; i < n; ++i) idx[i] = i;
        for (int i = 1; i < n; ++i) {
            int t = idx[i];
            int k = i - 1;
            while (k >= 0 && ev[idx[k]] > ev[t]) {
                idx[k + 1] = idx[k];
                --k;
            }
            idx[k + 1] = t;
        }
    }
    __syncthreads();
    const double l2 = ev[idx[1]];
    double* y = (double*)L.buf0;
    double* dots = ev + n;  // scratch: n entries after the eigenvalues
    for (int attempt = 0; attempt < 2; ++attempt) {
        // dots over the cluster
        for (int r = tid; r < n; r += nt) {
            int k = idx[r];
            double d = 0.0;
            if (r >= 1 && fabs(ev[k] - l2) <= 1e-10 * fro) {
                for (int i = 0; i < n; ++i) {
                    double z = attempt == 0 ? (double)i - 0.5 * (double)(n - 1)
                                            : hashed_uniform(seed, i) - 0.5;
                    d += V[i * n + k] * z;
                }
            }
            dots[r] = d;
        }
        __syncthreads();
        double acc[2] = {0.0, 0.0};
        for (int i = tid; i < n; i += nt) {
            double yi = 0.0;
            for (int r = 1; r < n; ++r) yi += dots[r] * V[i * n + idx[r]];
            y[i] = yi;
            acc[0] += yi * yi;
            double z = attempt == 0 ? (double)i - 0.5 * (double)(n - 1) : hashed_uniform(seed, i) - 0.5;
            acc[1] += z * z;
        }
        block_sum<2>(acc, red);
        if (sqrt(acc[0]) >= 1e-8 * sqrt(acc[1]) || attempt == 1) {
            double inv = 1.0 / sqrt(acc[0]);
            for (int i = tid; i < n; i += nt) y[i] *= inv;
            break;
        }
        __syncthreads();
    }
    // eigenvectors kept in LDS are left in Vg too (several-eigenpair starts read them)
    if (n <= kDenseLds)
        for (int t = tid; t < n * n; t += nt) Vg[t] = V[t];
    if (tid == 0) {
        int mult = 0;
        for (int r = 1; r < n; ++r)
            if (fabs(ev[idx[r]] - l2) <= 1e-10 * fro) ++mult;
        LevelState s0;
        s0.mu = 0.0;
        s0.s = 1.0;
        s0.mu_prev = 0.0;
        s0.s_prev = 1.0;
        s0.utv = 1.0;
        s0.margin = 0.0;
        s0.fin = 0;
        s0.k = -1;
        s0.maxit = 0;
        s0.err = 0;
        s0.ticks = 0;
        *st = s0;
        fo->coarse_lambda2 = l2;
        fo->coarse_mult = mult;
    }
}

// ------------------------------------------------ single-workgroup levels

__device__ __forceinline__ size_t align8(size_t b) { return (b + 7) & ~(size_t)7; }

// a load or store through the LDS view (LDS) or the global view
template <bool LDS, typename T>
__device__ __forceinline__ T ldx(const T* p, int i) {
    if constexpr (LDS) return sld(p, i);
    else return gld(p, i);
}
template <bool LDS, typename T>
__device__ __forceinline__ void stx(T* p, int i, T v) {
    if constexpr (LDS) sst(p, i, v);
    else gst(p, i, v);
}

// Bytes of the LDS image of a level: two vectors, weights (FP32 when that
// is exact), row pointers, columns (uint16 when n <= 65536).
__device__ __forceinline__ size_t staged_bytes(const LevelDev& L, int w32, int col16) {
    size_t b = align8(16 * (size_t)L.n);
    b += align8((size_t)L.nnz * (w32 ? 4 : 8));
    b += align8(4 * ((size_t)L.n + 1));
    b += align8((size_t)L.nnz * (col16 ? 2 : 4));
    return b;
}

// Levels up to this size run on one wavefront with no workgroup barrier.
constexpr int kWaveRows = 256;

// Sum of NV (<= 4) doubles over the active threads, identical in every
// thread.  Wave mode: wave sum.  Workgroup mode: waves post their sums
// (one barrier, alternating slots); each wave reads the posts with one LDS
// access per lane, adds them within rows of 16 lanes and reads row q.
template <int NV, bool WAVE>
__device__ __forceinline__ void small_sum(double (&v)[NV], double* red, int& parity) {
    const int lane = threadIdx.x & 63;
    if constexpr (WAVE) {
        // LDS writes of this step become visible to the other lanes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = group_sum_t<64>(v[q]);
    } else {
        const int wv = threadIdx.x >> 6;
        const int nw = blockDim.x >> 6;
        double* slot = red + parity * 64;
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = group_sum_t<64>(v[q]);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < NV; ++q) slot[q * 16 + wv] = v[q];
        }
        __syncthreads();
        double t = (lane < NV * 16 && (lane & 15) < nw) ? slot[lane] : 0.0;
        t = group_sum_t<16>(t);
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = read_lane(t, q * 16);
        parity ^= 1;
    }
}

// The four sums of a PI step over one wavefront, identical in every lane.
// Lanes trade halves of their partials so that each exchange adds one
// value per lane: after the two quad exchanges lane p of a quad holds the
// quad sum of value 2 (p & 1) + (p >> 1); rotations of each row by 4 and 8
// lanes, then the row and half swaps, complete the sums.
__device__ __forceinline__ void wave_sum4(double (&v)[4]) {
    const int lane = threadIdx.x & 63;
    const bool odd = (lane & 1) != 0;
    double k0 = odd ? v[2] : v[0];
    double k1 = odd ? v[3] : v[1];
    const double s0 = odd ? v[0] : v[2];
    const double s1 = odd ? v[1] : v[3];
    k0 += dpp_move<0xB1>(s0);
    k1 += dpp_move<0xB1>(s1);
    const bool hi = (lane & 2) != 0;
    double k = hi ? k1 : k0;
    k += dpp_move<0x4E>(hi ? k0 : k1);
    k += dpp_move<0x124>(k);
    k += dpp_move<0x128>(k);
    k = pair_sum_rows<16>(k);
    k = pair_sum_rows<32>(k);
    v[0] = read_lane(k, 0);
    v[2] = read_lane(k, 1);
    v[1] = read_lane(k, 2);
    v[3] = read_lane(k, 3);
}

// Sums of a PI step over the `nw` wavefronts that run the steps (the first
// nw of the workgroup), identical in each of their lanes.  nw == 1: no
// workgroup barrier.  Otherwise every such wave posts its four sums (one
// barrier, alternating slots) and adds the posts within rows of 16 lanes.
template <bool WAVE>
__device__ __forceinline__ void step_sum4(double (&v)[4], double* red, int& parity, int nw) {
    if constexpr (WAVE) {
        // LDS writes of this step become visible to the other lanes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        wave_sum4(v);
    } else {
        const int lane = threadIdx.x & 63;
        const int wv = threadIdx.x >> 6;
        double* slot = red + parity * 64;
        wave_sum4(v);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) slot[q * 16 + wv] = v[q];
        }
        __syncthreads();
        double t = ((lane & 15) < nw) ? slot[lane] : 0.0;
        t = group_sum_t<16>(t);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = read_lane(t, q * 16);
        parity ^= 1;
    }
}

// One PI step of a small level, rows shared by `nthr` threads in G-lane
// groups.  Pointers are either all LDS (staged modes) or all global.
template <int G, bool W32, bool C16, bool LDS>
__device__ __forceinline__ void pi_small(int n, int nthr, const int32_t* rp, const void* colp,
                                         const void* wp, double g, const double* win, double* wout,
                                         double mu, double s, double (&acc)[4]) {
    const int lane = threadIdx.x & (G - 1);
    const int ngroups = nthr / G;
    for (int i = (int)(threadIdx.x / G); i < n; i += ngroups) {
        const int a = ldx<LDS>(rp, i), b = ldx<LDS>(rp, i + 1);
        const double wi = ldx<LDS>(win, i);
        double t = 0.0;
        int e = a + lane;
        // four entries per trip: their column and value loads, then their
        // gathers, are in flight together; the sum keeps the entry order
        for (; e + 3 * G < b; e += 4 * G) {
            int c[4];
            double wt[4], x[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int f = e + q * G;
                if constexpr (C16) c[q] = (int)ldx<LDS>((const uint16_t*)colp, f);
                else c[q] = ldx<LDS>((const int32_t*)colp, f);
                if constexpr (W32) wt[q] = (double)ldx<LDS>((const float*)wp, f);
                else wt[q] = ldx<LDS>((const double*)wp, f);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) x[q] = ldx<LDS>(win, c[q]);
#pragma unroll
            for (int q = 0; q < 4; ++q) t += wt[q] * (x[q] - wi);
        }
        for (; e < b; e += G) {
            int c;
            double wt;
            if constexpr (C16) c = (int)ldx<LDS>((const uint16_t*)colp, e);
            else c = ldx<LDS>((const int32_t*)colp, e);
            if constexpr (W32) wt = (double)ldx<LDS>((const float*)wp, e);
            else wt = ldx<LDS>((const double*)wp, e);
            t += wt * (ldx<LDS>(win, c) - wi);
        }
        t = group_sum_t<G>(t);
        if (lane == 0) {
            const double x = (wi - mu) * s;
            const double y = s * (g * (wi - mu) + t);
            stx<LDS>(wout, i, y);
            acc[0] += y;
            acc[1] += y * y;
            acc[2] += y * x;
            acc[3] += x;
        }
    }
}

struct SmallIn {
    const void* cbuf;  // final vector of the coarser level
    int cfp32;
    int uniform;
    double cm, cs;     // its transform (v - cm) * cs
    uint64_t seed;
    double tol;
    int maxit;
};

// Rows of a small level read from its CSR arrays every step (an LDS image
// or global memory), in G-lane groups with G = L.lanes.
// Rows of a small level held in registers for all its steps: each G-lane
// group owns rows grp + r * ngroups (r < R) and each lane E entries of
// every such row (entry a + lane + m G in slot m; columns as uint16 pairs,
// weights as FP32, which the level's weights equal exactly), so a step is
// one round of independent gathers from the LDS vector.  Unused slots point
// at the row's own vertex with weight 0 and add an exact zero, which keeps
// the sums bit for bit those of the CSR traversal with the same G.
// A row longer than G E keeps its further entries (column, FP32 weight)
// in an LDS list; the lanes take them as slots E, E + 1, ... of the same
// stride, so each lane still sums its entries in CSR order.
template <int G, int R, int E>
struct RegRows {
    uint32_t c2[R][E / 2];
    float w[R][E];
    int row[R];
    int ooff[R], ocnt[R];  // the row's entries beyond G E: LDS list offset and count
    const uint64_t* ovl;
    int n;
    double g;

    // ov: LDS list of ovcap entries, filled from *ofill (zero before the
    // first call of the level); a list that would overflow sets *bad
    __device__ __forceinline__ void load(const LevelDev& L, int nact, int* bad, uint64_t* ov, int ovcap, int* ofill) {
        n = L.n;
        g = L.g;
        ovl = ov;
        const int lane = (int)threadIdx.x & (G - 1);
        const int lead = ((int)threadIdx.x & (kWave - 1)) & ~(G - 1);
        const int ngroups = nact / G;
        const int grp = (int)threadIdx.x / G;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = grp + r * ngroups;
            row[r] = i < n ? i : -1;
            int a = 0, b = 0;
            if (i < n) {
                a = gld(L.rp, i);
                b = gld(L.rp, i + 1);
            }
            // the same count in every lane of the group; its first lane
            // takes the list space for all of them
            int extra = max(b - a - G * E, 0);
            int off = 0;
            if (extra > 0 && lane == 0) off = atomicAdd(ofill, extra);
            off = __shfl(off, lead, kWave);
            if (extra > 0 && (off < 0 || off > ovcap - extra)) {
                if (lane == 0) *bad = 1;
                extra = 0;
            }
            ooff[r] = off;
            ocnt[r] = extra;
            for (int q = lane; q < extra; q += G) {
                const int e = a + G * E + q;
                const uint64_t wb = __float_as_uint((float)gld(L.w64, e));
                sst(ov, off + q, (uint64_t)(uint32_t)gld(L.col, e) | (wb << 32));
            }
            const uint32_t self = i < n ? (uint32_t)i : 0u;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int e = a + lane + m * G;
                uint32_t cv = self;
                float wv = 0.0f;
                if (e < b) {
                    cv = (uint32_t)gld(L.col, e);
                    wv = (float)gld(L.w64, e);
                }
                if (m & 1) c2[r][m >> 1] |= cv << 16;
                else c2[r][m >> 1] = cv;
                w[r][m] = wv;
            }
        }
        // the list entries are read back by the lanes of the group that
        // wrote them, in the same wavefront
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    __device__ __forceinline__ void step(const double* win, double* wout, double mu, double s, double (&acc)[4]) {
        const int lane = (int)threadIdx.x & (G - 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = row[r];
            const double wi = sld(win, i < 0 ? 0 : i);
            if constexpr (R * E > 32) {
                // decode the columns and widen the weights every step:
                // hoisted out of the step loop they would not fit
#pragma unroll
                for (int q = 0; q < E / 2; ++q) asm volatile("" : "+v"(c2[r][q]));
#pragma unroll
                for (int q = 0; q < E; ++q) asm volatile("" : "+v"(w[r][q]));
            }
            double x[E];
#pragma unroll
            for (int m = 0; m < E; ++m) x[m] = sld(win, (int)((m & 1) ? (c2[r][m >> 1] >> 16) : (c2[r][m >> 1] & 0xffffu)));
            double t = 0.0;
#pragma unroll
            for (int m = 0; m < E; ++m) t += (double)w[r][m] * (x[m] - wi);
            // entries beyond G E, two per trip; the second of a trip past
            // the row's end is its own vertex with weight 0 (an exact zero)
            for (int q = lane; q < ocnt[r]; q += 2 * G) {
                const uint64_t p0 = sld(ovl, ooff[r] + q);
                const uint64_t p1 = q + G < ocnt[r] ? sld(ovl, ooff[r] + q + G) : (uint64_t)(uint32_t)i;
                const double x0 = sld(win, (int)(uint32_t)p0), x1 = sld(win, (int)(uint32_t)p1);
                t += (double)__uint_as_float((uint32_t)(p0 >> 32)) * (x0 - wi);
                t += (double)__uint_as_float((uint32_t)(p1 >> 32)) * (x1 - wi);
            }
            t = group_sum_t<G>(t);
            if (lane == 0 && i >= 0) {
                const double xv = (wi - mu) * s;
                const double y = s * (g * (wi - mu) + t);
                sst(wout, i, y);
                acc[0] += y;
                acc[1] += y * y;
                acc[2] += y * xv;
                acc[3] += xv;
            }
        }
    }
};

// Prolongation, deflation, normalisation and PI steps of one small level
// read from its CSR arrays.  MODE 0: LDS image, one wavefront; 1: LDS
// image, whole workgroup; 2: global memory, whole workgroup.
template <int MODE, bool W32, bool C16>
__device__ void small_level(const LevelDev& L, const SmallIn& in, double* lds, double* red, int& parity,
                            int* stop_flag, int nw_run, LevelState& out) {
    constexpr bool WAVE = (MODE == 0);
    constexpr bool LDS = (MODE != 2);
    const int n = L.n;
    const int nthr = WAVE ? 64 : (int)blockDim.x;
    double* b0;
    double* b1;
    const int32_t* rp;
    const void* colp;
    const void* wp;
    if constexpr (MODE != 2) {
        char* p = (char*)lds;
        b0 = (double*)p;
        b1 = b0 + n;
        p += align8(16 * (size_t)n);
        wp = p;
        p += align8((size_t)L.nnz * (W32 ? 4 : 8));
        rp = (const int32_t*)p;
        p += align8(4 * ((size_t)n + 1));
        colp = p;
    } else {
        b0 = (double*)L.buf0;
        b1 = (double*)L.buf1;
        rp = L.rp;
        colp = L.col;
        wp = L.w64;
    }
    double sum[1] = {0.0};
    if (in.uniform) {
        for (int i = threadIdx.x; i < n; i += nthr) {
            const double v = hashed_uniform(in.seed, i) - 0.5;
            stx<LDS>(b0, i, v);
            sum[0] += v;
        }
    } else {
        for (int i = threadIdx.x; i < n; i += nthr) {
            const double v = (ld_any(in.cbuf, in.cfp32, gld(L.agg, i)) - in.cm) * in.cs;
            stx<LDS>(b0, i, v);
            sum[0] += v;
        }
    }
    small_sum<1, WAVE>(sum, red, parity);
    double mu = sum[0] / (double)n;
    double ss[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += nthr) {
        const double d = ldx<LDS>(b0, i) - mu;
        ss[0] += d * d;
    }
    small_sum<1, WAVE>(ss, red, parity);
    double s = 1.0 / sqrt(ss[0]);
    int cur = 0, k = 0, hit = 0;
    double utv = 0.0, pmu = mu, ps = s;
    // The PI steps run on the first `nw` wavefronts; the others only keep
    // the barrier count: after each barrier they read the stop decision of
    // the step before it, and the running waves end with one more barrier.
    const int nw = WAVE ? 1 : nw_run;
    const int nact = 64 * nw;
    // wave-uniform test, taken as a scalar branch
    if (WAVE || __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) < nw) {
        while (true) {
            const double* win = cur ? b1 : b0;
            double* wout = cur ? b0 : b1;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            switch (L.lanes) {
                case 1: pi_small<1, W32, C16, LDS>(n, nact, rp, colp, wp, L.g, win, wout, mu, s, acc); break;
                case 2: pi_small<2, W32, C16, LDS>(n, nact, rp, colp, wp, L.g, win, wout, mu, s, acc); break;
                case 4: pi_small<4, W32, C16, LDS>(n, nact, rp, colp, wp, L.g, win, wout, mu, s, acc); break;
                case 8: pi_small<8, W32, C16, LDS>(n, nact, rp, colp, wp, L.g, win, wout, mu, s, acc); break;
                case 16: pi_small<16, W32, C16, LDS>(n, nact, rp, colp, wp, L.g, win, wout, mu, s, acc); break;
                case 32: pi_small<32, W32, C16, LDS>(n, nact, rp, colp, wp, L.g, win, wout, mu, s, acc); break;
                default: pi_small<64, W32, C16, LDS>(n, nact, rp, colp, wp, L.g, win, wout, mu, s, acc); break;
            }
            step_sum4<WAVE>(acc, red, parity, nw);
            const double mu2 = acc[0] / (double)n;
            const double s2 = 1.0 / sqrt(acc[1] - acc[0] * mu2);
            utv = s2 * (acc[2] - mu2 * acc[3]);
            ++k;
            cur ^= 1;
            pmu = mu;
            ps = s;
            mu = mu2;
            s = s2;
            bool stop = !(utv < 1.0 - in.tol);
            if (!stop && k >= in.maxit) {
                hit = 1;
                stop = true;
            }
            if (!WAVE && threadIdx.x == 0) stop_flag[k & 1] = stop ? 1 : 0;
            if (stop) break;
        }
        if constexpr (!WAVE) __syncthreads();
    } else {
        // barrier q closes step q unless step q - 1 was the last one; the
        // slot parity follows the steps, as in the running waves
        for (int q = 1;; ++q) {
            __syncthreads();
            if (q > 1 && stop_flag[(q - 1) & 1]) break;
            parity ^= 1;
        }
        return;  // the state is kept by thread 0
    }
    int fin = cur;
    if constexpr (MODE != 2) {
        // the LDS vectors are discarded: final vector to buf0, previous to buf1
        const double* src = cur ? b1 : b0;
        const double* prv = cur ? b0 : b1;
        double* g0 = (double*)L.buf0;
        double* g1 = (double*)L.buf1;
        for (int i = threadIdx.x; i < n; i += nact) {
            gst(g0, i, sld(src, i));
            gst(g1, i, sld(prv, i));
        }
        fin = 0;
    }
    out.mu = mu;
    out.s = s;
    out.mu_prev = pmu;
    out.s_prev = ps;
    out.utv = utv;
    out.margin = utv - (1.0 - in.tol);
    out.fin = fin;
    out.k = k;
    out.maxit = hit;
    out.err = 0;
    out.ticks = 0;
}

// Levels jhi down to jlo (all FP64, small) refined inside one workgroup:
// prolongation, deflation, normalisation and every PI step separated only
// by workgroup (or wavefront) barriers, so thousands of steps cost no
// launches.  A level whose CSR and two vectors fit in `lds_budget` bytes
// is first copied to LDS (columns as uint16 when n <= 65536, weights as
// FP32 when that is exact) and its steps touch no global memory; levels of
// at most kWaveRows vertices then run on a single wavefront, larger ones on
// LevelDev::bwaves wavefronts (0: all).  Larger levels stream from global
// memory (L2).  The final vector of each level goes to buf0 (its
// predecessor to buf1).
__global__ void __launch_bounds__(kBlockKernelThreads)
    k_block_jobs(const BlockJob* __restrict__ jobs, int lds_budget) {
    extern __shared__ double lds[];
    __shared__ double red[2 * 64];
    __shared__ double s_cm, s_cs;
    __shared__ int s_cfin;
    __shared__ int s_stop[2];
    const BlockJob Jb = jobs[blockIdx.x];
    const LevelDev* __restrict__ lv = Jb.lv;
    int parity = 0;
    if (threadIdx.x == 0 && !Jb.uniform) {
        LevelState c = Jb.st[Jb.jhi + 1];
        s_cm = c.mu;
        s_cs = c.s;
        s_cfin = c.fin;
    }
    __syncthreads();
    for (int j = Jb.jhi; j >= Jb.jlo; --j) {
        const long long t_start = wall_clock64();
        const LevelDev L = lv[j];
        const int n = L.n;
        const int nwmax = (int)(blockDim.x >> 6);
        const int nw = L.bwaves > 0 ? min(L.bwaves, nwmax) : (n <= kWaveRows ? 1 : nwmax);
        const int c16 = (n <= 65536) ? 1 : 0;
        int w32 = 0;
        size_t need = staged_bytes(L, 0, c16);
        if (need > (size_t)lds_budget && L.w32exact) {
            w32 = 1;
            need = staged_bytes(L, 1, c16);
        }
        const bool staged = need <= (size_t)lds_budget;
        const int mode = staged ? (nw == 1 ? 0 : 1) : 2;
        if (staged) {
            char* p = (char*)lds + align8(16 * (size_t)n);
            void* wdst = p;
            p += align8((size_t)L.nnz * (w32 ? 4 : 8));
            int32_t* rdst = (int32_t*)p;
            p += align8(4 * ((size_t)n + 1));
            void* cdst = p;
            for (int i = threadIdx.x; i <= n; i += blockDim.x) sst(rdst, i, gld(L.rp, i));
            for (int e = threadIdx.x; e < (int)L.nnz; e += blockDim.x) {
                const int cv = gld(L.col, e);
                const double wv = gld(L.w64, e);
                if (c16) sst((uint16_t*)cdst, e, (uint16_t)cv);
                else sst((int32_t*)cdst, e, (int32_t)cv);
                if (w32) sst((float*)wdst, e, (float)wv);
                else sst((double*)wdst, e, wv);
            }
            __syncthreads();
        }
        SmallIn in;
        in.uniform = (Jb.uniform && j == Jb.jhi) ? 1 : 0;
        if (!in.uniform) {
            const LevelDev C = lv[j + 1];
            in.cbuf = s_cfin ? C.buf1 : C.buf0;
            in.cfp32 = C.fp32;
        } else {
            in.cbuf = nullptr;
            in.cfp32 = 0;
        }
        in.cm = s_cm;
        in.cs = s_cs;
        in.seed = Jb.seed;
        in.tol = L.kfix > 0 ? -1.0 : Jb.tol;  // a fixed schedule never passes the test
        in.maxit = L.kfix > 0 ? L.kfix : Jb.maxit;
        LevelState o;
        if (mode == 0) {
            if (threadIdx.x < 64) {
                if (w32) {
                    if (c16) small_level<0, true, true>(L, in, lds, red, parity, s_stop, 1, o);
                    else small_level<0, true, false>(L, in, lds, red, parity, s_stop, 1, o);
                } else {
                    if (c16) small_level<0, false, true>(L, in, lds, red, parity, s_stop, 1, o);
                    else small_level<0, false, false>(L, in, lds, red, parity, s_stop, 1, o);
                }
            }
        } else if (mode == 1) {
            if (w32) {
                if (c16) small_level<1, true, true>(L, in, lds, red, parity, s_stop, nw, o);
                else small_level<1, true, false>(L, in, lds, red, parity, s_stop, nw, o);
            } else {
                if (c16) small_level<1, false, true>(L, in, lds, red, parity, s_stop, nw, o);
                else small_level<1, false, false>(L, in, lds, red, parity, s_stop, nw, o);
            }
        } else {
            small_level<2, false, false>(L, in, lds, red, parity, s_stop, nw, o);
        }
        if (threadIdx.x == 0) {
            o.ticks = wall_clock64() - t_start;
            Jb.st[j] = o;
            s_cm = o.mu;
            s_cs = o.s;
            s_cfin = o.fin;
        }
        __syncthreads();
    }
}

// One level on register rows with both vectors in LDS (and the entries of
// rows longer than the layout in the LDS list ov of ovcap entries, filled
// from *ofill).  nw == 1: on wavefront 0 alone with no workgroup barrier
// (the caller keeps the other waves out); else the first nw waves run the
// steps and the others keep the barrier count as in the CSR traversal.
template <int G, int R, int E>
__device__ void reg_level(const LevelDev& L, const SmallIn& in, double* b0, double* b1, uint64_t* ov, int ovcap,
                          int* ofill, double* red, int& parity, int* stop_flag, int* bad, int nw, LevelState& out) {
    const bool wave = (nw == 1);
    const int n = L.n;
    const int nthr = wave ? 64 : (int)blockDim.x;
    double sum[1] = {0.0};
    if (in.uniform) {
        for (int i = threadIdx.x; i < n; i += nthr) {
            const double v = hashed_uniform(in.seed, i) - 0.5;
            sst(b0, i, v);
            sum[0] += v;
        }
    } else {
        for (int i = threadIdx.x; i < n; i += nthr) {
            const double v = (ld_any(in.cbuf, in.cfp32, gld(L.agg, i)) - in.cm) * in.cs;
            sst(b0, i, v);
            sum[0] += v;
        }
    }
    if (wave) small_sum<1, true>(sum, red, parity);
    else small_sum<1, false>(sum, red, parity);
    double mu = sum[0] / (double)n;
    double ss[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += nthr) {
        const double d = sld(b0, i) - mu;
        ss[0] += d * d;
    }
    if (wave) small_sum<1, true>(ss, red, parity);
    else small_sum<1, false>(ss, red, parity);
    double s = 1.0 / sqrt(ss[0]);
    int cur = 0, k = 0, hit = 0;
    double utv = 0.0, pmu = mu, ps = s;
    const int nact = 64 * nw;
    if (!(wave || __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) < nw)) {
        // barrier q closes step q unless step q - 1 was the last one
        for (int q = 1;; ++q) {
            __syncthreads();
            if (q > 1 && stop_flag[(q - 1) & 1]) break;
            parity ^= 1;
        }
        return;  // the state is kept by thread 0
    }
    RegRows<G, R, E> rows;
    rows.load(L, nact, bad, ov, ovcap, ofill);
    while (true) {
        const double* win = cur ? b1 : b0;
        double* wout = cur ? b0 : b1;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        rows.step(win, wout, mu, s, acc);
        if (wave) step_sum4<true>(acc, red, parity, 1);
        else step_sum4<false>(acc, red, parity, nw);
        const double mu2 = acc[0] / (double)n;
        const double s2 = 1.0 / sqrt(acc[1] - acc[0] * mu2);
        utv = s2 * (acc[2] - mu2 * acc[3]);
        ++k;
        cur ^= 1;
        pmu = mu;
        ps = s;
        mu = mu2;
        s = s2;
        bool stop = !(utv < 1.0 - in.tol);
        if (!stop && k >= in.maxit) {
            hit = 1;
            stop = true;
        }
        if (!wave && threadIdx.x == 0) stop_flag[k & 1] = stop ? 1 : 0;
        if (stop) break;
    }
    if (!wave) __syncthreads();
    // the LDS vectors are discarded: final vector to buf0, previous to buf1
    const double* src = cur ? b1 : b0;
    const double* prv = cur ? b0 : b1;
    double* g0 = (double*)L.buf0;
    double* g1 = (double*)L.buf1;
    for (int i = threadIdx.x; i < n; i += nact) {
        gst(g0, i, sld(src, i));
        gst(g1, i, sld(prv, i));
    }
    if (wave) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    out.mu = mu;
    out.s = s;
    out.mu_prev = pmu;
    out.s_prev = ps;
    out.utv = utv;
    out.margin = utv - (1.0 - in.tol);
    out.fin = 0;
    out.k = k;
    out.maxit = hit;
    out.err = *bad;
    out.ticks = 0;
}

// Levels jhi down to jlo refined inside one workgroup on register rows of
// G lanes per row, R rows per lane group and E slots per lane and row
// (every level of the job has that layout and LevelDev::bwaves waves;
// FP32-exact weights; rows longer than G E keep the rest in the LDS left
// after the two vectors).  A level whose layout does not fit is skipped
// with err = 2 in its state; err = 1 if the entries beyond the layout do
// not fit the LDS left.
template <int G, int R, int E>
__global__ void __launch_bounds__(kBlockRegsThreads)
    k_block_regs(const BlockJob* __restrict__ jobs, int lds_budget) {
    extern __shared__ double lds[];
    __shared__ double red[2 * 64];
    __shared__ double s_cm, s_cs;
    __shared__ int s_cfin;
    __shared__ int s_stop[2];
    __shared__ int s_bad;
    __shared__ int s_ofill;
    const BlockJob Jb = jobs[blockIdx.x];
    const LevelDev* __restrict__ lv = Jb.lv;
    int parity = 0;
    if (threadIdx.x == 0 && !Jb.uniform) {
        LevelState c = Jb.st[Jb.jhi + 1];
        s_cm = c.mu;
        s_cs = c.s;
        s_cfin = c.fin;
    }
    __syncthreads();
    for (int j = Jb.jhi; j >= Jb.jlo; --j) {
        const long long t_start = wall_clock64();
        const LevelDev L = lv[j];
        const int n = L.n;
        const int nw = max(1, min(L.bwaves, (int)(blockDim.x >> 6)));
        const bool fits = L.lanes == G && L.bregs == R && L.bslots == E && L.w32exact && n >= 1 && n <= 65536 &&
                          16 * (size_t)n <= (size_t)lds_budget && n <= R * (64 * nw / G) &&
                          (nw > 1 || (G == 1 && R == 1));
        if (threadIdx.x == 0) {
            s_bad = 0;
            s_ofill = 0;
        }
        // list of the entries beyond the layout: the LDS left after the vectors
        uint64_t* ov = (uint64_t*)(lds + 2 * (size_t)n);
        const int ovcap = fits ? (int)(((size_t)lds_budget - 16 * (size_t)n) / 8) : 0;
        SmallIn in;
        in.uniform = (Jb.uniform && j == Jb.jhi) ? 1 : 0;
        if (!in.uniform) {
            const LevelDev C = lv[j + 1];
            in.cbuf = s_cfin ? C.buf1 : C.buf0;
            in.cfp32 = C.fp32;
        } else {
            in.cbuf = nullptr;
            in.cfp32 = 0;
        }
        in.cm = s_cm;
        in.cs = s_cs;
        in.seed = Jb.seed;
        in.tol = L.kfix > 0 ? -1.0 : Jb.tol;  // a fixed schedule never passes the test
        in.maxit = L.kfix > 0 ? L.kfix : Jb.maxit;
        LevelState o{};
        if (!fits) {
            o.err = 2;
        } else if (nw == 1) {
            if (threadIdx.x < 64)
                reg_level<G, R, E>(L, in, lds, lds + n, ov, ovcap, &s_ofill, red, parity, s_stop, &s_bad, 1, o);
        } else {
            reg_level<G, R, E>(L, in, lds, lds + n, ov, ovcap, &s_ofill, red, parity, s_stop, &s_bad, nw, o);
        }
        if (threadIdx.x == 0) {
            o.ticks = wall_clock64() - t_start;
            Jb.st[j] = o;
            s_cm = o.mu;
            s_cs = o.s;
            s_cfin = o.fin;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- grid levels

// A job's view of the launch: jobs of a packed launch own disjoint ranges
// of workgroups; a single-graph launch is one job.  Every job has its own
// barrier state, so graphs refined together never wait for each other.
struct GridCtx {
    GridSync* gs;
    GridSlot* slots;
    GridSlot* bcast;
    unsigned long long epoch;
    int nb;  // workgroups of the job
    int vb;  // this workgroup within the job
    int lb;  // row block of this workgroup
    int tag;
};

template <int NV>
__device__ __forceinline__ bool job_allreduce(double (&v)[NV], GridCtx& c, double* red) {
    return grid_allreduce_impl<NV>(v, c.gs, c.slots, c.bcast, c.epoch, c.vb, c.lb, c.nb, red, c.tag);
}

// ---- per-row operations fed by the two traversal drivers
//
// Edge weights are read through WRead<W>: W = double or float (an FP32
// copy, used only where every weight of the level is exact in FP32),
// uint8_t or uint16_t (a copy where every weight is an integer in 1..255
// or 1..65535), or
// WUnit where every weight is 1 and nothing is read.  The value is the
// same double in all of them, so results do not depend on the storage.
struct WUnit {};
template <typename W, bool LDS = false>
struct WRead {
    const W* __restrict__ p;
    __device__ __forceinline__ double operator[](int e) const {
        if constexpr (LDS) return (double)sld(p, e);
        else return (double)gld(p, e);
    }
};
template <bool LDS>
struct WRead<WUnit, LDS> {
    const void* p;
    __device__ __forceinline__ double operator[](int) const { return 1.0; }
};
// storage type of kind WK for iterates of type T
template <typename T, int WK>
struct WStore {
    using type = T;
};
template <typename T>
struct WStore<T, kWF32> {
    using type = float;
};
template <typename T>
struct WStore<T, kWUnit> {
    using type = WUnit;
};
template <typename T>
struct WStore<T, kWU8> {
    using type = uint8_t;
};
template <typename T>
struct WStore<T, kWU16> {
    using type = uint16_t;
};
// the level's weights of kind WK for iterates of type T
template <typename T, int WK>
__device__ __forceinline__ WRead<typename WStore<T, WK>::type> weights_of(const LevelDev& L) {
    WRead<typename WStore<T, WK>::type> r;
    if constexpr (WK == kWUnit) r.p = nullptr;
    else if constexpr (WK == kWU8) r.p = L.w8;
    else if constexpr (WK == kWU16) r.p = L.w16;
    else if constexpr (WK == kWF32 || sizeof(T) == 4) r.p = L.w32;
    else r.p = L.w64;
    return r;
}
// the finishing pass reads FP64 weights, or the exact FP32 copy, or none
template <int WK>
using FinW = WRead<typename WStore<double, WK>::type>;
template <int WK>
__device__ __forceinline__ FinW<WK> fin_weights(const LevelDev& L) {
    return weights_of<double, WK>(L);
}

// One PI step: y_i = s (g (w_i - mu) + sum_k a_ik (w_k - w_i)), stored as
// T; acc += {y, y^2, y v, v} with v = (w_i - mu) s.
// Rows and entries are numbered from the arrays the traversal reads (the
// level's, or with STG a workgroup's LDS stage); vector index = row + roff.
template <typename T, int WK, bool STG = false>
struct PiOp {
    const int32_t* __restrict__ col;
    WRead<typename WStore<T, WK>::type, STG> wv;
    const T* __restrict__ win;
    T* __restrict__ wout;
    int roff;
    double mu, s, g;
    double acc[4];
    __device__ __forceinline__ double xi(int i) const { return (double)gld(win, roff + i); }
    __device__ __forceinline__ int vidx(int i) const { return roff + i; }
    // an entry's term split into its loads (column and weight, then the
    // gathered vector value) and its arithmetic, so a traversal can issue
    // the loads of several entries before it adds their terms in order
    __device__ __forceinline__ int colof(int e) const {
        if constexpr (STG) return sld(col, e);
        else return gld(col, e);
    }
    __device__ __forceinline__ double wof(int e) const { return wv[e]; }
    __device__ __forceinline__ double xk(int c) const { return (double)gld(win, c); }
    __device__ __forceinline__ double term(double xc, double wt, double x) const { return wt * (xc - x); }
    __device__ __forceinline__ double entry(int e, double x) const { return term(xk(colof(e)), wof(e), x); }
    __device__ __forceinline__ double entry_cw(int c, double wt, double x) const { return term(xk(c), wt, x); }
    __device__ __forceinline__ void row(int i, double x, double t) {
        const double v = (x - mu) * s;
        const T ys = (T)(s * (g * (x - mu) + t));
        gst(wout, roff + i, ys);
        const double yd = (double)ys;
        acc[0] += yd;
        acc[1] += yd * yd;
        acc[2] += yd * v;
        acc[3] += v;
    }
};

// FP64 recomputation of a step from a (possibly FP32) iterate.
template <int WK>
struct RedoOp {
    const int32_t* __restrict__ col;
    FinW<WK> w;
    const void* src;
    int f32;
    double* __restrict__ dst;
    double mu, s, g;
    double acc[2];
    __device__ __forceinline__ double xi(int i) const { return ld_any(src, f32, i); }
    __device__ __forceinline__ int vidx(int i) const { return i; }
    __device__ __forceinline__ int colof(int e) const { return gld(col, e); }
    __device__ __forceinline__ double wof(int e) const { return w[e]; }
    __device__ __forceinline__ double xk(int c) const { return ld_any(src, f32, c); }
    __device__ __forceinline__ double term(double xc, double wt, double x) const { return wt * (xc - x); }
    __device__ __forceinline__ double entry(int e, double x) const { return term(xk(colof(e)), wof(e), x); }
    __device__ __forceinline__ double entry_cw(int c, double wt, double x) const { return term(xk(c), wt, x); }
    __device__ __forceinline__ void row(int i, double x, double t) {
        const double y = s * (g * (x - mu) + t);
        gst(dst, i, y);
        acc[0] += y;
        acc[1] += y * y;
    }
};

// Sums of u = (src - mu) s and the edge form sum_k a_ik ((src_k - src_i) s)^2.
template <int WK>
struct EdgeOp {
    const int32_t* __restrict__ col;
    FinW<WK> w;
    const void* src;
    int f32;
    double mu, s;
    double acc[3];
    __device__ __forceinline__ double xi(int i) const { return ld_any(src, f32, i); }
    __device__ __forceinline__ int vidx(int i) const { return i; }
    __device__ __forceinline__ int colof(int e) const { return gld(col, e); }
    __device__ __forceinline__ double wof(int e) const { return w[e]; }
    __device__ __forceinline__ double xk(int c) const { return ld_any(src, f32, c); }
    __device__ __forceinline__ double term(double xc, double wt, double x) const {
        const double d = (xc - x) * s;
        return wt * d * d;
    }
    __device__ __forceinline__ double entry(int e, double x) const { return term(xk(colof(e)), wof(e), x); }
    __device__ __forceinline__ double entry_cw(int c, double wt, double x) const { return term(xk(c), wt, x); }
    __device__ __forceinline__ void row(int i, double x, double t) {
        const double u = (x - mu) * s;
        acc[0] += u;
        acc[1] += u * u;
        acc[2] += t;
    }
};

// Output y = (u - mean)/nrm and residual terms (L y - lambda y)_i.
template <int WK>
struct ResidualOp {
    const int32_t* __restrict__ col;
    FinW<WK> w;
    const void* src;
    int f32;
    double mu, s, mean_u, nrm, lam;
    double* __restrict__ yout;
    double acc[1];
    __device__ __forceinline__ double xi(int i) const { return ld_any(src, f32, i); }
    __device__ __forceinline__ int vidx(int i) const { return i; }
    __device__ __forceinline__ int colof(int e) const { return gld(col, e); }
    __device__ __forceinline__ double wof(int e) const { return w[e]; }
    __device__ __forceinline__ double xk(int c) const { return ld_any(src, f32, c); }
    __device__ __forceinline__ double term(double xc, double wt, double x) const { return wt * (x - xc); }
    __device__ __forceinline__ double entry(int e, double x) const { return term(xk(colof(e)), wof(e), x); }
    __device__ __forceinline__ double entry_cw(int c, double wt, double x) const { return term(xk(c), wt, x); }
    __device__ __forceinline__ void row(int i, double x, double t) {
        const double yi = ((x - mu) * s - mean_u) / nrm;
        const double r = t * s / nrm - lam * yi;
        acc[0] += r * r;
        gst(yout, i, yi);
    }
};

// ---- traversal driver 1: G lanes per row (G = 64: a wavefront per row)
//
// Each lane group takes two rows at a time (rows i and i + ngroups) so the
// loads of both are in flight together; the rows are still emitted in the
// order i, i + ngroups, i + 2 ngroups, ... of a one-row loop.
//
// Rows with more than lmin entries (the hubs of a skewed degree
// distribution; lrows lists them in ascending order after their count) are
// left out of the groups' loop and summed afterwards by the whole
// workgroup, one after the other in ascending order, so a hub row no longer
// holds one lane group while the others idle.  `red` is block_sum scratch;
// rows r of the traversal are rows r + loff of the list (an LDS stage).

__device__ __forceinline__ int lower_bound_i32(const int32_t* __restrict__ a, int n, int v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (gld(a, mid) < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// The first kRowBatch entries of each lane in a row are loaded before any
// of them is added: all column and weight loads of both rows are issued,
// then all their vector gathers, then the terms are added in entry order
// (so the sums are those of the plain loop), and a row with more entries
// finishes in the loop.  Without the batch a lane waits for a column and
// then its gather once per entry.  The loads are unconditional, so no
// loaded value passes through a branch (which would make the compiler wait
// for it early): a slot past the row's end reads the entry before the row
// end (a valid index whenever the level has entries; the term is then
// dropped) and gathers the row's own vector value.
constexpr int kRowBatch = 2;

template <int U, int G, class Op>
__device__ __forceinline__ void rows_batch(const Op& op, int lane, int self1, int a1, int b1, double x1, double& t1,
                                           int self2, int a2, int b2, double x2, double& t2) {
    int c1[U], c2[U];
    double w1[U], w2[U], y1[U], y2[U];
    const int z1 = max(b1 - 1, 0), z2 = max(b2 - 1, 0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e1 = a1 + lane + u * G, e2 = a2 + lane + u * G;
        const int q1 = e1 < b1 ? e1 : z1, q2 = e2 < b2 ? e2 : z2;
        c1[u] = op.colof(q1);
        w1[u] = op.wof(q1);
        c2[u] = op.colof(q2);
        w2[u] = op.wof(q2);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        y1[u] = op.xk(a1 + lane + u * G < b1 ? c1[u] : self1);
        y2[u] = op.xk(a2 + lane + u * G < b2 ? c2[u] : self2);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const double v1 = op.term(y1[u], w1[u], x1);
        const double v2 = op.term(y2[u], w2[u], x2);
        t1 = a1 + lane + u * G < b1 ? t1 + v1 : t1;
        t2 = a2 + lane + u * G < b2 ? t2 + v2 : t2;
    }
}

// SRP: the row pointers are an LDS stage (else global memory).
template <bool SRP>
__device__ __forceinline__ int ld_rp(const int32_t* rp, int i) {
    if constexpr (SRP) return sld(rp, i);
    else return gld(rp, i);
}

// A lane's entries e, e + G, ... of a row up to b, four per trip, while
// four remain: e is left at the first entry not taken.
template <int G, typename Op>
__device__ __forceinline__ void row_rest4(const Op& op, int& e, int b, double x, double& t) {
    for (; e + 3 * G < b; e += 4 * G) {
        int c[4];
        double w[4], v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c[q] = op.colof(e + q * G);
            w[q] = op.wof(e + q * G);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = op.xk(c[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q) t += op.term(v[q], w[q], x);
    }
}

// the long rows of [r0, r1) (listed in lrows), each summed by the whole
// workgroup
template <bool SRP = false, bool HUB4 = false, typename Op>
__device__ __forceinline__ void drive_long_rows(const int32_t* __restrict__ rp, int r0, int r1, Op& op,
                                                const int32_t* __restrict__ lrows, double* red, int loff = 0) {
    const int cnt = gld(lrows, 0);
    const int32_t* lr = lrows + 1;
    const int q1 = lower_bound_i32(lr, cnt, r1 + loff);
    for (int q = lower_bound_i32(lr, cnt, r0 + loff); q < q1; ++q) {
        const int r = gld(lr, q) - loff;
        const int a = ld_rp<SRP>(rp, r), b = ld_rp<SRP>(rp, r + 1);
        const double x = op.xi(r);
        double t[1] = {0.0};
        // HUB4: each thread's entries four per trip, their loads in flight
        // together (a hub row holds one workgroup while the grid waits)
        const int bd = (int)blockDim.x;
        int e = a + (int)threadIdx.x;
        for (; HUB4 && e + 3 * bd < b; e += 4 * bd) {
            int c[4];
            double w[4], v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                c[q] = op.colof(e + q * bd);
                w[q] = op.wof(e + q * bd);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = op.xk(c[q]);
#pragma unroll
            for (int q = 0; q < 4; ++q) t[0] += op.term(v[q], w[q], x);
        }
        for (; e < b; e += bd) t[0] += op.entry(e, x);
        block_sum<1>(t, red);
        if (threadIdx.x == 0) op.row(r, x, t[0]);
    }
}

template <int G, bool SRP = false, bool REST4 = false, class Op>
__device__ __forceinline__ void drive_rows(const int32_t* __restrict__ rp, int r0, int r1, Op& op,
                                           const int32_t* __restrict__ lrows = nullptr, int lmin = 0x7fffffff,
                                           double* red = nullptr, int loff = 0) {
    const int lane = threadIdx.x & (G - 1);
    const int ngroups = blockDim.x / G;
    int i = r0 + (int)(threadIdx.x / G);
    for (; i + ngroups < r1; i += 2 * ngroups) {
        const int i2 = i + ngroups;
        const int a1 = ld_rp<SRP>(rp, i), a2 = ld_rp<SRP>(rp, i2);
        int b1 = ld_rp<SRP>(rp, i + 1), b2 = ld_rp<SRP>(rp, i2 + 1);
        const bool l1 = b1 - a1 > lmin, l2 = b2 - a2 > lmin;
        if (l1) b1 = a1;
        if (l2) b2 = a2;
        const double x1 = op.xi(i), x2 = op.xi(i2);
        double t1 = 0.0, t2 = 0.0;
        rows_batch<kRowBatch, G>(op, lane, op.vidx(i), a1, b1, x1, t1, op.vidx(i2), a2, b2, x2, t2);
        int e1 = a1 + lane + kRowBatch * G, e2 = a2 + lane + kRowBatch * G;
        if constexpr (REST4) {
            // rows of hundreds of entries: each lane's rest in trips of
            // four, their columns and weights, then their gathers, in
            // flight together (the sum keeps the entry order); only where
            // the registers allow it (the step kernels: the persistent
            // kernels' cap would spill)
            row_rest4<G>(op, e1, b1, x1, t1);
            row_rest4<G>(op, e2, b2, x2, t2);
        }
        while (e1 < b1 || e2 < b2) {
            if (e1 < b1) {
                t1 += op.entry(e1, x1);
                e1 += G;
            }
            if (e2 < b2) {
                t2 += op.entry(e2, x2);
                e2 += G;
            }
        }
        t1 = group_sum_t<G>(t1);
        t2 = group_sum_t<G>(t2);
        if (lane == 0) {
            if (!l1) op.row(i, x1, t1);
            if (!l2) op.row(i2, x2, t2);
        }
    }
    if (i < r1) {
        const int a = ld_rp<SRP>(rp, i), b = ld_rp<SRP>(rp, i + 1);
        if (b - a <= lmin) {
            const double x = op.xi(i);
            double t = 0.0;
            for (int e = a + lane; e < b; e += G) t += op.entry(e, x);
            t = group_sum_t<G>(t);
            if (lane == 0) op.row(i, x, t);
        }
    }
    // levels of 32 or 64 lanes per row (skewed degrees, hub rows) batch the
    // hub rows' loads; on the others the extra registers would spill
    if (lrows != nullptr) drive_long_rows<SRP, (G >= 32)>(rp, r0, r1, op, lrows, red, loff);
}

// ---- traversal driver 2: merge path
//
// The block's rows [r0, r1) and entries are merged into one sequence
// (the entries of a row followed by its row end) that is cut into equal
// pieces of kMergeIPT items per thread, so a row of any length is shared
// by many threads and a chunk of short rows by few (Merrill & Garland,
// "Merge-based parallel sparse matrix-vector multiplication", SC 2016).
// Per chunk the row ends and the chunk's entries (columns and weights, a
// contiguous range starting where the previous chunk's ended) are copied to
// LDS with coalesced loads, every thread finds its start by binary search
// on its diagonal and walks its items from there, and the partial sums of
// rows split across threads are combined by a segmented scan in thread
// order (deterministic), then added by the thread that completes the row.
// The entry arithmetic is the operation's own, so staging changes no
// result.
constexpr int kMergeIPT = 8;
constexpr int kMergeChunk = kGridBlock * kMergeIPT;

struct MergeShared {
    int win[kMergeChunk + 2];  // row starts/ends of rows ia .. ia + W (relative to the block's first entry)
    int scol[kMergeChunk];     // entries js .. js + kMergeChunk (relative to the block's first entry)
    double sw[kMergeChunk];
    int crow[kGridBlock];
    double cval[kGridBlock];
    int wrow[16];
    int wfirst[16];
    double wtail[16];
    int inrow[17];
    double inval[17];
    int s_ia, s_js;
};

template <class Op>
__device__ __forceinline__ void drive_merge(const int32_t* __restrict__ rp, int r0, int r1, Op& op,
                                            MergeShared& sh) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
    const int e0 = gld(rp, r0);
    const int nrows = r1 - r0;
    const int nent = gld(rp, r1) - e0;
    const int total = nrows + nent;
    int carry_row = -1;
    double carry_val = 0.0;
    int ia = 0, js = 0;
    for (int d0 = 0; d0 < total; d0 += kMergeChunk) {
        const int dl_end = min(kMergeChunk, total - d0);
        const int W = min(kMergeChunk + 1, nrows - ia);  // rows whose ends can lie in this chunk
        for (int q = tid; q <= W; q += blockDim.x) sh.win[q] = gld(rp, r0 + ia + q) - e0;
        // the chunk's entries start where the previous chunk's ended and
        // are at most kMergeChunk (those past its end serve the next one)
        const int ns = min(kMergeChunk, nent - js);
        for (int q = tid; q < ns; q += blockDim.x) {
            sh.scol[q] = op.colof(e0 + js + q);
            sh.sw[q] = op.wof(e0 + js + q);
        }
        __syncthreads();
        // start coordinate (i, j) on my diagonal: i rows completed, j entries consumed
        const int dl = min(tid * kMergeIPT, dl_end);
        const int diag = d0 + dl;
        int lo = max(ia, diag - nent), hi = min(ia + W, diag);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sh.win[mid - ia + 1] <= diag - mid - 1) lo = mid + 1;
            else hi = mid;
        }
        int i = lo, j = diag - lo;
        const int steps = min(dl + kMergeIPT, dl_end) - dl;
        double x = (i < nrows) ? op.xi(r0 + i) : 0.0;
        double part = 0.0;
        int frow = -1;
        double fx = 0.0, fpart = 0.0;
        for (int q = 0; q < steps; ++q) {
            if (i < nrows && j < sh.win[i - ia + 1]) {
                part += op.entry_cw(sh.scol[j - js], sh.sw[j - js], x);
                ++j;
            } else {
                if (frow < 0) {
                    frow = i;
                    fx = x;
                    fpart = part;
                } else {
                    op.row(r0 + i, x, part);
                }
                part = 0.0;
                ++i;
                x = (i < nrows) ? op.xi(r0 + i) : 0.0;
            }
        }
        if (tid * kMergeIPT < dl_end && min(tid * kMergeIPT + kMergeIPT, dl_end) == dl_end) {
            sh.s_ia = i;
            sh.s_js = j;
        }
        // inclusive segmented scan of the carries (rows are non-decreasing in tid)
        int myrow = i;
        double v = part;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int ro = __shfl_up(myrow, o, 64);
            const double vo = __shfl_up(v, o, 64);
            if (lane >= o && ro == myrow) v += vo;
        }
        const int first_in_wave = __shfl(myrow, 0, 64);
        if (lane == 63) {
            sh.wrow[wv] = myrow;
            sh.wtail[wv] = v;
            sh.wfirst[wv] = first_in_wave;
        }
        __syncthreads();
        if (tid == 0) {
            int r = carry_row;
            double cv = carry_val;
            for (int w = 0; w < nw; ++w) {
                sh.inrow[w] = r;
                sh.inval[w] = cv;
                const bool whole = sh.wfirst[w] == sh.wrow[w];
                const double tail = sh.wtail[w] + ((whole && r == sh.wrow[w]) ? cv : 0.0);
                r = sh.wrow[w];
                cv = tail;
            }
            sh.inrow[nw] = r;
            sh.inval[nw] = cv;
        }
        __syncthreads();
        if (myrow == first_in_wave && myrow == sh.inrow[wv]) v += sh.inval[wv];
        sh.crow[tid] = myrow;
        sh.cval[tid] = v;
        __syncthreads();
        if (frow >= 0) {
            double cin = 0.0;
            if (tid == 0) {
                if (carry_row == frow) cin = carry_val;
            } else if (sh.crow[tid - 1] == frow) {
                cin = sh.cval[tid - 1];
            }
            op.row(r0 + frow, fx, fpart + cin);
        }
        carry_row = sh.inrow[nw];
        carry_val = sh.inval[nw];
        ia = sh.s_ia;
        js = sh.s_js;
        __syncthreads();
    }
}

// TRAV = 0: merge path; TRAV = G > 0: G lanes per row.
template <int TRAV, class Op>
__device__ __forceinline__ void drive(const LevelDev& L, int r0, int r1, Op& op, MergeShared* sh, double* red) {
    if constexpr (TRAV == 0) {
        drive_merge(L.rp, r0, r1, op, *sh);
    } else {
        drive_rows<TRAV>(L.rp, r0, r1, op, L.lrows, L.lmin, red);
    }
}

// ---- a workgroup's rows staged in LDS
//
// A grid barrier's acquire invalidates the L2, so on a level whose
// workgroup shares are small every step would fetch the row pointers,
// columns and weights again before it can gather.  When a workgroup's rows
// and entries fit the LDS stage (FP64 levels, G lanes per row) they are
// copied there once per level and the steps read them from LDS through the
// same traversal; only the vector gathers go to memory.  Rows and entries
// are visited in the same order, so the sums are bit for bit those of the
// global traversal.
constexpr int kStageRows = kGridStageRows;
constexpr int kStageEnts = 3840;
struct StageLds {
    int32_t rp[kStageRows + 1];  // row pointers relative to the first entry
    int32_t col[kStageEnts];
    double w[kStageEnts];
};

// ---- refinement of one level by a job's workgroups

template <typename T, int TRAV, int WK>
__device__ void refine_level(const GridJob& J, GridCtx& c, double* red, MergeShared* sh, StageLds* stg) {
    const LevelDev& L = J.L;
    const double tol = J.tol;
    const int maxit = J.maxit;
    const uint64_t seed = J.seed;
    const int r0 = L.part[c.lb], r1 = L.part[c.lb + 1];
    T* b0 = (T*)L.buf0;
    T* b1 = (T*)L.buf1;
    const double n = (double)L.n;
    // traversal arrays of the PI steps: the level's, or the LDS stage
    // (weights staged in their storage type; none where all are 1)
    using WT = typename WStore<T, WK>::type;
    PiOp<T, WK> op;
    op.col = L.col;
    op.wv = weights_of<T, WK>(L);
    op.roff = 0;
    op.g = L.g;
    PiOp<T, WK, true> ops;
    bool staged = false;
    if constexpr (TRAV > 0 && sizeof(T) == 8) {
        const int a0 = gld(L.rp, r0), a1 = gld(L.rp, r1);
        // the same in every thread of the workgroup
        if (stg != nullptr && L.stage && !L.ileave && r1 - r0 <= kStageRows && a1 - a0 <= kStageEnts) {
            for (int i = threadIdx.x; i <= r1 - r0; i += blockDim.x) stg->rp[i] = gld(L.rp, r0 + i) - a0;
            for (int e = threadIdx.x; e < a1 - a0; e += blockDim.x) {
                stg->col[e] = gld(L.col, a0 + e);
                if constexpr (WK != kWUnit) ((WT*)stg->w)[e] = gld(op.wv.p, a0 + e);
            }
            __syncthreads();
            ops.col = stg->col;
            if constexpr (WK != kWUnit) ops.wv.p = (const WT*)stg->w;
            ops.roff = r0;
            ops.g = L.g;
            staged = true;
        }
    }
    // interleaved steps: this workgroup's XCD holds parts xl0 .. xl0 + np - 1
    // (the grouping of xcd_remap); their rows [x0, x1) go in chunks of four
    // passes, chunk q to the workgroup at position q mod np
    int x0 = r0, x1 = r1, xp = 0, np = 1;
    if (TRAV > 0 && L.ileave) {
        const int q = c.nb >> 3, rr = c.nb & 7, x = c.vb & 7;
        const int xl0 = x * q + min(x, rr);
        np = q + (x < rr ? 1 : 0);
        xp = c.vb >> 3;
        x0 = gld(L.part, xl0);
        x1 = gld(L.part, xl0 + np);
    }
    // prolongation from level j+1 (or the hashed uniform start)
    double sum[1] = {0.0};
    if (J.uniform) {
        for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            const T v = (T)(hashed_uniform(seed, i) - 0.5);
            gst(b0, i, v);
            sum[0] += (double)v;
        }
    } else {
        const LevelState cst = *J.stc;
        const void* cb = cst.fin ? J.C.buf1 : J.C.buf0;
        for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            const T v = (T)((ld_any(cb, J.C.fp32, gld(L.agg, i)) - cst.mu) * cst.s);
            gst(b0, i, v);
            sum[0] += (double)v;
        }
    }
    if (!job_allreduce<1>(sum, c, red)) return;
    double mu = sum[0] / n;
    double ss[1] = {0.0};
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        const double d = (double)gld(b0, i) - mu;
        ss[0] += d * d;
    }
    if (!job_allreduce<1>(ss, c, red)) return;
    double s = 1.0 / sqrt(ss[0]);
    int cur = 0, k = 0, hit = 0;
    double utv = 0.0, pmu = mu, ps = s;
    while (true) {
        double acc[4];
        if (TRAV > 0 && staged) {
            ops.win = cur ? b1 : b0;
            ops.wout = cur ? b0 : b1;
            ops.mu = mu;
            ops.s = s;
            ops.acc[0] = ops.acc[1] = ops.acc[2] = ops.acc[3] = 0.0;
            if constexpr (TRAV > 0 && sizeof(T) == 8)
                drive_rows<TRAV, true>(stg->rp, 0, r1 - r0, ops, L.lrows, L.lmin, red, r0);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = ops.acc[q];
        } else {
            op.win = cur ? b1 : b0;
            op.wout = cur ? b0 : b1;
            op.mu = mu;
            op.s = s;
            op.acc[0] = op.acc[1] = op.acc[2] = op.acc[3] = 0.0;
            if constexpr (TRAV == 0) {
                drive_merge(L.rp, r0, r1, op, *sh);
            } else if (L.ileave) {
                const int cw = 4 * ((int)blockDim.x / TRAV);
                for (int a = x0 + xp * cw; a < x1; a += np * cw)
                    drive_rows<TRAV>(L.rp, a, min(a + cw, x1), op, nullptr, L.lmin, red);
                if (L.lrows != nullptr) drive_long_rows<false, (TRAV >= 32)>(L.rp, r0, r1, op, L.lrows, red);
            } else {
                drive_rows<TRAV>(L.rp, r0, r1, op, L.lrows, L.lmin, red);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = op.acc[q];
        }
        if (!job_allreduce<4>(acc, c, red)) return;
        const double mu2 = acc[0] / n;
        const double s2 = 1.0 / sqrt(acc[1] - acc[0] * mu2);
        utv = s2 * (acc[2] - mu2 * acc[3]);
        ++k;
        cur ^= 1;
        pmu = mu;
        ps = s;
        mu = mu2;
        s = s2;
        if (!(utv < 1.0 - tol)) break;
        if (k >= maxit) {
            hit = 1;
            break;
        }
    }
    if (c.vb == 0 && threadIdx.x == 0) {
        LevelState o;
        o.mu = mu;
        o.s = s;
        o.mu_prev = pmu;
        o.s_prev = ps;
        o.utv = utv;
        o.margin = utv - (1.0 - tol);
        o.fin = cur;
        o.k = k;
        o.maxit = hit;
        o.err = 0;
        o.ticks = 0;
        *J.st = o;
    }
}

// ---- finishing pass on the finest level
//
// With `redo` = 1 (mixed precision) the last power-iteration step is
// recomputed in FP64 from the FP32 iterate before it, so the step count
// equals the FP64 path and only that earlier iterate carries FP32
// rounding.  Then the output y = deflated, normalised iterate, the
// edge-form Rayleigh quotient r = sum_edges w (y_i - y_k)^2 and the
// residual ||L y - r y||, all in FP64.
template <int TRAV, int WK>
__device__ void finish_level(const GridJob& J, GridCtx& c, double* red, MergeShared* sh) {
    const LevelDev& L = J.L;
    const int r0 = L.part[c.lb], r1 = L.part[c.lb + 1];
    const double n = (double)L.n;
    const LevelState st = *J.stc;
    const void* src = st.fin ? L.buf1 : L.buf0;
    int f32 = L.fp32;
    double mu = st.mu, s = st.s;
    if (J.redo && st.k > 0) {
        RedoOp<WK> op;
        op.col = L.col;
        op.w = fin_weights<WK>(L);
        op.src = st.fin ? L.buf0 : L.buf1;
        op.f32 = f32;
        op.dst = J.fa;
        op.mu = st.mu_prev;
        op.s = st.s_prev;
        op.g = L.g;
        op.acc[0] = op.acc[1] = 0.0;
        drive<TRAV>(L, r0, r1, op, sh, red);
        if (!job_allreduce<2>(op.acc, c, red)) return;
        mu = op.acc[0] / n;
        s = 1.0 / sqrt(op.acc[1] - op.acc[0] * mu);
        src = J.fa;
        f32 = 0;
    }
    EdgeOp<WK> eo;
    eo.col = L.col;
    eo.w = fin_weights<WK>(L);
    eo.src = src;
    eo.f32 = f32;
    eo.mu = mu;
    eo.s = s;
    eo.acc[0] = eo.acc[1] = eo.acc[2] = 0.0;
    drive<TRAV>(L, r0, r1, eo, sh, red);
    if (!job_allreduce<3>(eo.acc, c, red)) return;
    const double mean_u = eo.acc[0] / n;
    const double nrm2 = eo.acc[1] - eo.acc[0] * mean_u;
    const double nrm = sqrt(nrm2);
    const double lam = 0.5 * eo.acc[2] / nrm2;
    ResidualOp<WK> ro;
    ro.col = L.col;
    ro.w = fin_weights<WK>(L);
    ro.src = src;
    ro.f32 = f32;
    ro.mu = mu;
    ro.s = s;
    ro.mean_u = mean_u;
    ro.nrm = nrm;
    ro.lam = lam;
    ro.yout = J.yout;
    ro.acc[0] = 0.0;
    drive<TRAV>(L, r0, r1, ro, sh, red);
    if (!job_allreduce<1>(ro.acc, c, red)) return;
    if (c.vb == 0 && threadIdx.x == 0) {
        J.fo->lambda = lam;
        J.fo->residual = sqrt(ro.acc[0]);
        J.fo->sum_u = eo.acc[0];
        J.fo->sum_uu = eo.acc[1];
        J.fo->edge = eo.acc[2];
    }
}

// Which job owns this workgroup (jobs sorted by first workgroup).
__device__ __forceinline__ int find_job(const GridJob* jobs, int njobs) {
    int lo = 0, hi = njobs - 1;
    const int b = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].b0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ GridCtx make_ctx(const GridJob& J) {
    GridCtx c;
    c.gs = J.gs;
    c.slots = J.slots;
    c.bcast = J.bcast;
    c.nb = J.L.grid;
    c.vb = (int)blockIdx.x - J.b0;
    c.lb = xcd_remap(c.vb, c.nb);
    c.epoch = start_epoch(J.gs);
    c.tag = J.tag;
    return c;
}

// nslots: the slot array holds two banks of nslots
__global__ void k_raise_abort(GridSync* gs) {
    if (threadIdx.x == 0) atomicOr(&gs->abort, 1u);
}

__global__ void k_reset_sync(GridSync* gs, GridSlot* slots, int nslots, GridSlot* bcast) {
    nslots *= 2;
    for (int b = threadIdx.x; b < nslots; b += blockDim.x) {
        for (int q = 0; q < 7; ++q) slots[b].v[q] = 0.0;
        slots[b].epoch = 0ull;
    }
    if (threadIdx.x < kBcastLines) {
        GridSlot* line = bcast_line(bcast, threadIdx.x);
        for (int q = 0; q < 7; ++q) line->v[q] = 0.0;
        line->epoch = 0ull;
    }
    if (threadIdx.x == 0) {
        gs->epoch = 0ull;
        gs->abort = 0u;
        gs->where = 0u;
        gs->abort_epoch = 0ull;
    }
}

// Residency count: each workgroup counts itself in, raises the recorded
// peak, stays `hold` ticks and counts itself out.  The peak is how many
// workgroups of this kernel the device keeps resident at once.
__device__ void residency_count(const GridJob& J) {
    if (threadIdx.x == 0) {
        const unsigned now = atomicAdd(J.count, 1u) + 1u;
        atomicMax(J.count + 1, now);
    }
    __syncthreads();
    const long long t0 = wall_clock64();
    while (wall_clock64() - t0 < J.hold) __builtin_amdgcn_s_sleep(2);
    __syncthreads();
    if (threadIdx.x == 0) atomicSub(J.count, 1u);
}

// One launch refines one level of each job (one graph per job).  Kernels
// are specialised by traversal (merge path, or G lanes per row) and
// storage precision to keep registers low; a packed launch holds one kind.
template <int TRAV, typename T, int WK>
__device__ __forceinline__ void refine_entry(const GridJob* __restrict__ jobs, int njobs, double* red,
                                             MergeShared* sh, StageLds* stg) {
    const GridJob J = jobs[find_job(jobs, njobs)];
    if (J.tag == kResidencyTag) {
        residency_count(J);
        return;
    }
    GridCtx c = make_ctx(J);
    if (c.vb < 0 || c.vb >= c.nb) return;
    refine_level<T, TRAV, WK>(J, c, red, sh, stg);
}

// At most 128 VGPRs: two workgroups of 512 threads per CU.
template <typename T, int WK>
__global__ void __launch_bounds__(kGridBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_refine_merge(const GridJob* __restrict__ jobs, int njobs) {
    __shared__ double red[16 * 5 + 8];
    __shared__ MergeShared msh;
    refine_entry<0, T, WK>(jobs, njobs, red, &msh, nullptr);
}

// G lanes per row.  Held to 6 waves per SIMD (at most 80 VGPRs): grids
// run at most 3 workgroups of 512 threads per CU.
template <int G, typename T, int WK>
__global__ void __launch_bounds__(kGridBlock) __attribute__((amdgpu_waves_per_eu(6, 6)))
k_refine_rows(const GridJob* __restrict__ jobs, int njobs) {
    __shared__ double red[16 * 5 + 8];
    StageLds* stg = nullptr;
    if constexpr (sizeof(T) == 8) {
        __shared__ StageLds st;
        stg = &st;
    }
    refine_entry<G, T, WK>(jobs, njobs, red, nullptr, stg);
}

// One launch finishes the finest level of each job.
template <int TRAV, int WK>
__global__ void __launch_bounds__(kGridBlock) k_finish_jobs(const GridJob* __restrict__ jobs, int njobs) {
    __shared__ double red[16 * 5 + 8];
    MergeShared* sh = nullptr;
    if constexpr (TRAV == 0) {
        __shared__ MergeShared msh;
        sh = &msh;
    }
    const GridJob J = jobs[find_job(jobs, njobs)];
    if (J.tag == kResidencyTag) {
        residency_count(J);
        return;
    }
    GridCtx c = make_ctx(J);
    if (c.vb < 0 || c.vb >= c.nb) return;
    finish_level<TRAV, WK>(J, c, red, sh);
}

// ------------------------------------------ large levels: a launch per step
//
// The same arithmetic as refine_level, with the grid-wide sums formed by a
// one-workgroup kernel after each launch instead of a grid barrier inside
// it: each workgroup posts its block sums, the check kernel adds the posts
// in workgroup order, applies the stopping test and leaves (mu, s) for the
// next step.  A step launched after the test passed returns at once.

constexpr int kCheckThreads = 1024;

template <int NV>
__device__ __forceinline__ void post_part(double (&v)[NV], double* red, double* part, int slot) {
    block_sum<NV>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) part[4 * (size_t)slot + q] = v[q];
    }
}

// fixed-order total of the posts of nb workgroups, in every thread
template <int NV>
__device__ __forceinline__ void sum_parts(const double* part, int nb, double (&v)[NV], double* red) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] += part[4 * (size_t)b + q];
    }
    block_sum<NV>(v, red);
}

// prolongation (or the hashed uniform start) into buf0; posts its sum
template <typename T>
__global__ void __launch_bounds__(kStepBlock) k_step_prolong(const StepJob* __restrict__ jp) {
    __shared__ double red[16 * 5 + 8];
    const StepJob J = *jp;
    const LevelDev& L = J.L;
    const int lb = xcd_remap((int)blockIdx.x, (int)gridDim.x);  // row block, posted in row order
    const int r0 = L.part[lb], r1 = L.part[lb + 1];
    T* b0 = (T*)L.buf0;
    double sum[1] = {0.0};
    if (J.uniform) {
        for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            const T v = (T)(hashed_uniform(J.seed, i) - 0.5);
            gst(b0, i, v);
            sum[0] += (double)v;
        }
    } else {
        const LevelState cst = *J.stc;
        const void* cb = cst.fin ? J.C.buf1 : J.C.buf0;
        for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            const T v = (T)((ld_any(cb, J.C.fp32, gld(L.agg, i)) - cst.mu) * cst.s);
            gst(b0, i, v);
            sum[0] += (double)v;
        }
    }
    post_part<1>(sum, red, J.part, lb);
}

// mean of the start vector
__global__ void __launch_bounds__(kCheckThreads) k_step_mean(const StepJob* __restrict__ jp, int nb) {
    __shared__ double red[16 * 5 + 8];
    const StepJob J = *jp;
    double v[1];
    sum_parts<1>(J.part, nb, v, red);
    if (threadIdx.x == 0) J.ctl->mu = v[0] / (double)J.L.n;
}

// squared distance of the start vector from its mean
template <typename T>
__global__ void __launch_bounds__(kStepBlock) k_step_sumsq(const StepJob* __restrict__ jp) {
    __shared__ double red[16 * 5 + 8];
    const StepJob J = *jp;
    const LevelDev& L = J.L;
    const int lb = xcd_remap((int)blockIdx.x, (int)gridDim.x);  // row block, posted in row order
    const int r0 = L.part[lb], r1 = L.part[lb + 1];
    const T* b0 = (const T*)L.buf0;
    const double mu = J.ctl->mu;
    double ss[1] = {0.0};
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        const double d = (double)gld(b0, i) - mu;
        ss[0] += d * d;
    }
    post_part<1>(ss, red, J.part, lb);
}

// normalisation of the start vector; arms the step loop
__global__ void __launch_bounds__(kCheckThreads) k_step_norm(const StepJob* __restrict__ jp, int nb) {
    __shared__ double red[16 * 5 + 8];
    const StepJob J = *jp;
    double v[1];
    sum_parts<1>(J.part, nb, v, red);
    if (threadIdx.x == 0) {
        StepCtl* c = J.ctl;
        const double mu = c->mu;
        const double s = 1.0 / sqrt(v[0]);
        c->s = s;
        c->pmu = mu;
        c->ps = s;
        c->utv = 0.0;
        c->k = 0;
        c->cur = 0;
        c->done = 0;
        c->hit = 0;
    }
}

// one power-iteration step: buf[cur] -> buf[cur ^ 1], posts {y, y^2, y v, v}
template <int G, typename T, int WK>
__global__ void __launch_bounds__(kStepBlock) k_step_spmv(const StepJob* __restrict__ jp) {
    __shared__ double red[16 * 5 + 8];
    const StepJob J = *jp;
    const StepCtl c = *J.ctl;
    if (c.done) return;
    const LevelDev& L = J.L;
    const int lb = xcd_remap((int)blockIdx.x, (int)gridDim.x);  // row block, posted in row order
    const int r0 = L.part[lb], r1 = L.part[lb + 1];
    PiOp<T, WK> op;
    op.col = L.col;
    op.wv = weights_of<T, WK>(L);
    op.roff = 0;
    op.g = L.g;
    op.win = (const T*)(c.cur ? L.buf1 : L.buf0);
    op.wout = (T*)(c.cur ? L.buf0 : L.buf1);
    op.mu = c.mu;
    op.s = c.s;
    op.acc[0] = op.acc[1] = op.acc[2] = op.acc[3] = 0.0;
    drive_rows<G, false, (G >= 32)>(L.rp, r0, r1, op, L.lrows, L.lmin, red);
    post_part<4>(op.acc, red, J.part, lb);
}

// sums of the step, stopping test, state for the next step; writes the
// level state when the level is done
__global__ void __launch_bounds__(kCheckThreads) k_step_check(const StepJob* __restrict__ jp, int nb) {
    __shared__ double red[16 * 5 + 8];
    const StepJob J = *jp;
    if (J.ctl->done) return;
    double acc[4];
    sum_parts<4>(J.part, nb, acc, red);
    if (threadIdx.x == 0) {
        StepCtl c = *J.ctl;
        const double n = (double)J.L.n;
        const double mu2 = acc[0] / n;
        const double s2 = 1.0 / sqrt(acc[1] - acc[0] * mu2);
        c.utv = s2 * (acc[2] - mu2 * acc[3]);
        ++c.k;
        c.cur ^= 1;
        c.pmu = c.mu;
        c.ps = c.s;
        c.mu = mu2;
        c.s = s2;
        if (!(c.utv < 1.0 - J.tol)) {
            c.done = 1;
        } else if (c.k >= J.maxit) {
            c.done = 1;
            c.hit = 1;
        }
        *J.ctl = c;
        if (c.done) {
            LevelState o;
            o.mu = c.mu;
            o.s = c.s;
            o.mu_prev = c.pmu;
            o.s_prev = c.ps;
            o.utv = c.utv;
            o.margin = c.utv - (1.0 - J.tol);
            o.fin = c.cur;
            o.k = c.k;
            o.maxit = c.hit;
            o.err = 0;
            o.ticks = 0;
            *J.st = o;
        }
    }
}

}  // namespace

// ================================================================ launchers

hipError_t launch_coarse_jobs(const CoarseJob* jobs, int njobs, hipStream_t s) {
    const size_t shmem = sizeof(double) * 2 * kDenseLds * kDenseLds;
    hipLaunchKernelGGL(k_coarse_jobs, dim3(njobs), dim3(256), shmem, s, jobs);
    return hipGetLastError();
}

namespace {
template <int G, int E>
const void* block_regs_kernel(int ri) {
    return ri == 0 ? (const void*)k_block_regs<G, 1, E> : ri == 1 ? (const void*)k_block_regs<G, 2, E>
                                                                 : (const void*)k_block_regs<G, 4, E>;
}
// kind 0: CSR traversal; 1 + 3 l + log2(R): register rows of layout l
const void* block_kernel(int kind) {
    if (kind <= 0) return (const void*)k_block_jobs;
    const int l = (kind - 1) / 3, ri = (kind - 1) % 3;
    switch (l) {
        case 0: return block_regs_kernel<1, 8>(ri);
        case 1: return block_regs_kernel<2, 8>(ri);
        case 2: return block_regs_kernel<4, 8>(ri);
        case 3: return block_regs_kernel<8, 8>(ri);
        case 4: return block_regs_kernel<1, 16>(ri);
        case 5: return block_regs_kernel<2, 16>(ri);
        default: return block_regs_kernel<4, 16>(ri);
    }
}
}  // namespace

int refine_block_lds_budget() {
    static int budget = -1;
    if (budget < 0) {
        int dev = 0, maxsh = 65536;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        size_t stat = 0;
        for (int r = 0; r < kBlockKinds; ++r) {
            hipFuncAttributes fa;
            if (hipFuncGetAttributes(&fa, block_kernel(r)) == hipSuccess) stat = std::max(stat, fa.sharedSizeBytes);
        }
        long b = std::min<long>(kBlockLdsMax, (long)maxsh - (long)stat - 256);
        b = std::max<long>(b, 0);
        for (int r = 0; r < kBlockKinds; ++r) {
            if (b > 65536 - (long)stat - 256 &&
                hipFuncSetAttribute(block_kernel(r), hipFuncAttributeMaxDynamicSharedMemorySize, (int)b) != hipSuccess) {
                (void)hipGetLastError();
                b = std::max<long>(0, 65536 - (long)stat - 256);
            }
        }
        budget = (int)(b & ~7L);
    }
    return budget;
}

hipError_t launch_block_jobs(const BlockJob* jobs, int njobs, int kind, hipStream_t s) {
    if (kind < 0 || kind >= kBlockKinds) return hipErrorInvalidValue;
    const int budget = refine_block_lds_budget();
    void* args[] = {(void*)&jobs, (void*)&budget};
    return hipLaunchKernel(block_kernel(kind), dim3(njobs), dim3(kind ? kBlockRegsThreads : kBlockKernelThreads), args,
                           (size_t)budget, s);
}

namespace {
// kind = 16 wk + 2 t + fp32 with t = 0 (merge path) or 1 + log2(G) and wk
// the weight storage (FP32 iterates have no kWF32 form: FP32 is their own)
template <int TRAV, int WK>
const void* refine_kernel_w(int fp32) {
    if constexpr (TRAV == 0) {
        if constexpr (WK == kWF32) return (const void*)k_refine_merge<double, kWF32>;
        else return fp32 ? (const void*)k_refine_merge<float, WK> : (const void*)k_refine_merge<double, WK>;
    } else if constexpr (WK == kWF32) {
        return (const void*)k_refine_rows<TRAV, double, kWF32>;
    } else {
        return fp32 ? (const void*)k_refine_rows<TRAV, float, WK> : (const void*)k_refine_rows<TRAV, double, WK>;
    }
}
template <int TRAV>
const void* refine_kernel_t(int fp32, int wk) {
    return wk == kWUnit ? refine_kernel_w<TRAV, kWUnit>(fp32)
           : wk == kWF32 ? refine_kernel_w<TRAV, kWF32>(fp32)
           : wk == kWU8  ? refine_kernel_w<TRAV, kWU8>(fp32)
           : wk == kWU16 ? refine_kernel_w<TRAV, kWU16>(fp32)
                         : refine_kernel_w<TRAV, kWNative>(fp32);
}
const void* refine_kernel(int kind) {
    const int fp32 = kind & 1, wk = kind >> 4;
    switch ((kind >> 1) & 7) {
        case 0: return refine_kernel_t<0>(fp32, wk);
        case 1: return refine_kernel_t<1>(fp32, wk);
        case 2: return refine_kernel_t<2>(fp32, wk);
        case 3: return refine_kernel_t<4>(fp32, wk);
        case 4: return refine_kernel_t<8>(fp32, wk);
        case 5: return refine_kernel_t<16>(fp32, wk);
        case 6: return refine_kernel_t<32>(fp32, wk);
        default: return refine_kernel_t<64>(fp32, wk);
    }
}
template <int TRAV>
const void* finish_kernel_t(int wk) {
    return wk == kWUnit ? (const void*)k_finish_jobs<TRAV, kWUnit>
           : wk == kWF32 ? (const void*)k_finish_jobs<TRAV, kWF32>
           : wk == kWU8  ? (const void*)k_finish_jobs<TRAV, kWU8>
           : wk == kWU16 ? (const void*)k_finish_jobs<TRAV, kWU16>
                         : (const void*)k_finish_jobs<TRAV, kWNative>;
}
const void* finish_kernel(int kind) {
    const int wk = kind >> 4;
    switch ((kind >> 1) & 7) {
        case 0: return finish_kernel_t<0>(wk);
        case 1: return finish_kernel_t<1>(wk);
        case 2: return finish_kernel_t<2>(wk);
        case 3: return finish_kernel_t<4>(wk);
        case 4: return finish_kernel_t<8>(wk);
        case 5: return finish_kernel_t<16>(wk);
        case 6: return finish_kernel_t<32>(wk);
        default: return finish_kernel_t<64>(wk);
    }
}
// Workgroups of kernel `k` that can be resident at once.  The occupancy
// query alone can promise more than the device delivers (for kernels at
// 64 VGPRs and about 90 SGPRs it reports 4 workgroups of 512 threads per CU
// where 3 are resident), and a grid barrier over workgroups that are not
// all resident never completes.  So the kernel itself is launched once in
// residency-count mode at the queried size and the observed peak is used,
// rounded down to a multiple of 8.  Returns 0 on any error.
thread_local MeasureBuffers t_meas{nullptr, nullptr, nullptr};

int max_blocks_ptr(const void* k) {
    int dev = 0, ncu = 0, occ = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, kGridBlock, 0) != hipSuccess) return 0;
    const int want = occ * ncu;
    if (want <= 0) return 0;
    unsigned* cnt = nullptr;
    GridJob* dj = nullptr;
    hipStream_t s = nullptr;
    unsigned peak[2] = {0u, 0u};
    const bool own = t_meas.cnt == nullptr;  // else buffers and stream given by the caller
    // the count needs an idle device: work already queued (a coarsest solve
    // launched during setup, another thread's solve) finishes first
    bool ok = hipDeviceSynchronize() == hipSuccess;
    if (ok && own) {
        ok = hipMalloc((void**)&cnt, 2 * sizeof(unsigned)) == hipSuccess &&
             hipMalloc((void**)&dj, sizeof(GridJob)) == hipSuccess &&
             hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    } else if (ok) {
        cnt = t_meas.cnt;
        dj = t_meas.job;
        s = t_meas.stream;
    }
    if (ok) {
        GridJob j{};
        j.tag = kResidencyTag;
        j.count = cnt;
        j.hold = (long long)khz;  // 1 ms: dispatch of the grid takes microseconds
        j.b0 = 0;
        int njobs = 1;
        void* args[] = {(void*)&dj, &njobs};
        ok = hipMemsetAsync(cnt, 0, 2 * sizeof(unsigned), s) == hipSuccess &&
             hipMemcpyAsync(dj, &j, sizeof(GridJob), hipMemcpyHostToDevice, s) == hipSuccess &&
             hipLaunchKernel(k, dim3(want), dim3(kGridBlock), args, 0, s) == hipSuccess &&
             hipMemcpyAsync(peak, cnt, 2 * sizeof(unsigned), hipMemcpyDeviceToHost, s) == hipSuccess &&
             hipStreamSynchronize(s) == hipSuccess;
    }
    if (own) {
        if (s) (void)hipStreamDestroy(s);
        if (dj) (void)hipFree(dj);
        if (cnt) (void)hipFree(cnt);
    }
    if (!ok) {
        (void)hipGetLastError();
        return 0;
    }
    const int got = std::min<int>(want, (int)peak[1]);
    return got >= 8 ? (got / 8) * 8 : got;
}
}  // namespace

void set_measure_buffers(const MeasureBuffers* b) { t_meas = b ? *b : MeasureBuffers{nullptr, nullptr, nullptr}; }

int job_kind(int variant, int lanes, int fp32, int wk) {
    int t = 0;
    if (variant != 2) {
        t = 1;
        for (int g = lanes; g > 1 && t < 7; g >>= 1) ++t;
    }
    // FP32 iterates read FP32 weights (their native storage)
    if (fp32 && wk == kWF32) wk = kWNative;
    return 16 * wk + 2 * t + (fp32 ? 1 : 0);
}

namespace {
std::mutex g_cap_mutex;
int g_refine_cap[kJobKinds];
int g_finish_cap[kJobKinds];
bool g_caps_init = false;
}  // namespace

// Measured once per kernel and process (the first call launches it).
void caps_init() {
    if (g_caps_init) return;
    for (int k = 0; k < kJobKinds; ++k) g_refine_cap[k] = g_finish_cap[k] = -1;
    g_caps_init = true;
}

int refine_jobs_max_blocks(int kind) {
    std::lock_guard<std::mutex> lock(g_cap_mutex);
    caps_init();
    if (g_refine_cap[kind] < 0) g_refine_cap[kind] = max_blocks_ptr(refine_kernel(kind));
    return g_refine_cap[kind];
}

int finish_jobs_max_blocks(int kind) {
    std::lock_guard<std::mutex> lock(g_cap_mutex);
    caps_init();
    if (g_finish_cap[kind] < 0) g_finish_cap[kind] = max_blocks_ptr(finish_kernel(kind));
    return g_finish_cap[kind];
}

// Grid launches are plain launches of at most the measured co-resident
// workgroup count: on an otherwise idle device every workgroup is resident
// at once, which is all the grid barrier needs.  (A cooperative launch
// costs about 17 us more per launch on MI355X and gave no protection from
// kernels on other streams either; the barrier's bounded wait turns such
// a case into CMG_E_DEVICE.)
hipError_t launch_refine_jobs(const GridJob* jobs, int njobs, int nblocks, int kind, hipStream_t s) {
    void* args[] = {(void*)&jobs, &njobs};
    return hipLaunchKernel(refine_kernel(kind), dim3(nblocks), dim3(kGridBlock), args, 0, s);
}

hipError_t launch_finish_jobs(const GridJob* jobs, int njobs, int nblocks, int kind, hipStream_t s) {
    void* args[] = {(void*)&jobs, &njobs};
    return hipLaunchKernel(finish_kernel(kind), dim3(nblocks), dim3(kGridBlock), args, 0, s);
}

hipError_t launch_step_begin(const StepJob* job, int nblocks, int kind, hipStream_t s) {
    if (kind & 1) {
        hipLaunchKernelGGL(k_step_prolong<float>, dim3(nblocks), dim3(kStepBlock), 0, s, job);
        hipLaunchKernelGGL(k_step_mean, dim3(1), dim3(kCheckThreads), 0, s, job, nblocks);
        hipLaunchKernelGGL(k_step_sumsq<float>, dim3(nblocks), dim3(kStepBlock), 0, s, job);
    } else {
        hipLaunchKernelGGL(k_step_prolong<double>, dim3(nblocks), dim3(kStepBlock), 0, s, job);
        hipLaunchKernelGGL(k_step_mean, dim3(1), dim3(kCheckThreads), 0, s, job, nblocks);
        hipLaunchKernelGGL(k_step_sumsq<double>, dim3(nblocks), dim3(kStepBlock), 0, s, job);
    }
    hipLaunchKernelGGL(k_step_norm, dim3(1), dim3(kCheckThreads), 0, s, job, nblocks);
    return hipGetLastError();
}

namespace {
template <int G, int WK>
void step_spmv_w(const StepJob* job, int nblocks, int fp32, hipStream_t s) {
    if constexpr (WK == kWF32) {
        hipLaunchKernelGGL((k_step_spmv<G, double, WK>), dim3(nblocks), dim3(kStepBlock), 0, s, job);
    } else {
        if (fp32) hipLaunchKernelGGL((k_step_spmv<G, float, WK>), dim3(nblocks), dim3(kStepBlock), 0, s, job);
        else hipLaunchKernelGGL((k_step_spmv<G, double, WK>), dim3(nblocks), dim3(kStepBlock), 0, s, job);
    }
}
template <int G>
void step_spmv_g(const StepJob* job, int nblocks, int fp32, int wk, hipStream_t s) {
    if (wk == kWUnit) step_spmv_w<G, kWUnit>(job, nblocks, fp32, s);
    else if (wk == kWF32) step_spmv_w<G, kWF32>(job, nblocks, fp32, s);
    else if (wk == kWU8) step_spmv_w<G, kWU8>(job, nblocks, fp32, s);
    else if (wk == kWU16) step_spmv_w<G, kWU16>(job, nblocks, fp32, s);
    else step_spmv_w<G, kWNative>(job, nblocks, fp32, s);
}
}  // namespace

hipError_t launch_step_pi(const StepJob* job, int nblocks, int kind, hipStream_t s) {
    const int fp32 = kind & 1, wk = kind >> 4;
    switch ((kind >> 1) & 7) {
        case 1: step_spmv_g<1>(job, nblocks, fp32, wk, s); break;
        case 2: step_spmv_g<2>(job, nblocks, fp32, wk, s); break;
        case 3: step_spmv_g<4>(job, nblocks, fp32, wk, s); break;
        case 4: step_spmv_g<8>(job, nblocks, fp32, wk, s); break;
        case 5: step_spmv_g<16>(job, nblocks, fp32, wk, s); break;
        case 6: step_spmv_g<32>(job, nblocks, fp32, wk, s); break;
        case 7: step_spmv_g<64>(job, nblocks, fp32, wk, s); break;
        default: return hipErrorInvalidValue;  // the merge path has no step form
    }
    hipLaunchKernelGGL(k_step_check, dim3(1), dim3(kCheckThreads), 0, s, job, nblocks);
    return hipGetLastError();
}

hipError_t launch_reset_sync(GridSync* gs, GridSlot* slots, int nslots, GridSlot* bcast, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_sync, dim3(1), dim3(256), 0, s, gs, slots, nslots, bcast);
    return hipGetLastError();
}

hipError_t launch_raise_abort(GridSync* gs, hipStream_t s) {
    hipLaunchKernelGGL(k_raise_abort, dim3(1), dim3(64), 0, s, gs);
    return hipGetLastError();
}

}  // namespace cmg
