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

#include "cmg_internal.h"

namespace cmg {

namespace {

__device__ __forceinline__ double ld_any(const void* p, int fp32, int64_t i) {
    return fp32 ? (double)((const float*)p)[i] : ((const double*)p)[i];
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
// blocks so neighbouring rows (and their x gathers) share one L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    if (nb % 8) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

// ~4 s at the 100 MHz constant clock: a safety bound, never reached when
// the grid is co-resident (cooperative launch).
constexpr long long kSpinTicks = 400000000LL;

// Grid-wide sum of NV doubles with a barrier.  Every workgroup posts its
// block sum; the last to arrive adds all posts in workgroup order (fixed
// tree, independent of arrival order), publishes the totals and releases
// the others.  Returns false if the barrier timed out or another
// workgroup aborted.
template <int NV>
__device__ bool grid_allreduce(double (&v)[NV], GridSync* gs, double* partials, double* bcast,
                               int lb, double* red) {
    __shared__ unsigned s_gen;
    __shared__ int s_last;
    __shared__ double s_tot[NV];
    __shared__ int s_ok;
    const int nb = gridDim.x;
    block_sum<NV>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) partials[lb * NV + q] = v[q];
        s_gen = __hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        unsigned prev = atomicAdd(&gs->count, 1u);
        s_last = (prev == (unsigned)nb - 1);
        s_ok = 1;
    }
    __syncthreads();
    if (s_last) {
        __threadfence();
        double acc[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
            for (int q = 0; q < NV; ++q) acc[q] += ld_agent(partials + b * NV + q);
        }
        block_sum<NV>(acc, red);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                st_agent(bcast + q, acc[q]);
                s_tot[q] = acc[q];
            }
            __hip_atomic_store(&gs->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            __hip_atomic_store(&gs->gen, s_gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (threadIdx.x == 0) {
        long long t0 = wall_clock64();
        while (__hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == s_gen) {
            __builtin_amdgcn_s_sleep(2);
            if (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                s_ok = 0;
                break;
            }
            if (wall_clock64() - t0 > kSpinTicks) {
                atomicOr(&gs->abort, 1u);
                s_ok = 0;
                break;
            }
        }
        __threadfence();
        if (s_ok) {
#pragma unroll
            for (int q = 0; q < NV; ++q) s_tot[q] = ld_agent(bcast + q);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = s_tot[q];
    bool ok = s_ok != 0;
    __syncthreads();
    return ok;
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
__global__ void __launch_bounds__(256) k_coarse_dense(LevelDev L, LevelState* st, double* Ag,
                                                     double* Vg, double* ev, int32_t* idx,
                                                     uint64_t seed, FinishOut* fo) {
    extern __shared__ double dyn[];
    __shared__ double red[16 * 2 + 8];
    __shared__ double cs_c[128], cs_s[128];
    __shared__ int pr_p[128], pr_q[128];
    __shared__ double s_fro, s_norm;
    __shared__ int s_m;
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
        s_fro = fro;
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
        *st = s0;
        fo->coarse_lambda2 = l2;
        fo->coarse_mult = mult;
    }
}

// ------------------------------------------------ single-workgroup levels

// LDS image of one small level: vectors first (8-byte aligned), then
// weights, row pointers and columns.
struct StagedLevel {
    double* x0;
    double* x1;
    const void* w;  // float if w32, else double
    const int32_t* rp;
    const void* col;  // uint16 if col16, else int32
};

__device__ __forceinline__ size_t align8(size_t b) { return (b + 7) & ~(size_t)7; }

// bytes of the LDS image; 0 if it does not fit in `budget`
__device__ __forceinline__ size_t staged_bytes(const LevelDev& L, int w32, int col16) {
    size_t b = align8(16 * (size_t)L.n);
    b += align8((size_t)L.nnz * (w32 ? 4 : 8));
    b += align8(4 * ((size_t)L.n + 1));
    b += align8((size_t)L.nnz * (col16 ? 2 : 4));
    return b;
}

// One PI step reading the LDS image; lane 0 of each G-lane group owns a row.
template <int G, bool W32, bool C16>
__device__ __forceinline__ void pi_rows_lds(const StagedLevel& S, int n, double g, const double* win,
                                            double* wout, double mu, double s, double (&acc)[4]) {
    const int lane = threadIdx.x & (G - 1);
    const int ngroups = blockDim.x / G;
    for (int i = (int)(threadIdx.x / G); i < n; i += ngroups) {
        const int a = S.rp[i], b = S.rp[i + 1];
        const double wi = win[i];
        double t = 0.0;
        for (int e = a + lane; e < b; e += G) {
            const int c = C16 ? (int)((const uint16_t*)S.col)[e] : ((const int32_t*)S.col)[e];
            const double wt = W32 ? (double)((const float*)S.w)[e] : ((const double*)S.w)[e];
            t += wt * (win[c] - wi);
        }
        t = group_sum_t<G>(t);
        if (lane == 0) {
            const double x = (wi - mu) * s;
            const double y = s * (g * (wi - mu) + t);
            wout[i] = y;
            acc[0] += y;
            acc[1] += y * y;
            acc[2] += y * x;
            acc[3] += x;
        }
    }
}

template <bool W32, bool C16>
__device__ __forceinline__ void pi_rows_lds_dispatch(int G, const StagedLevel& S, int n, double g,
                                                     const double* win, double* wout, double mu, double s,
                                                     double (&acc)[4]) {
    switch (G) {
        case 1: pi_rows_lds<1, W32, C16>(S, n, g, win, wout, mu, s, acc); break;
        case 2: pi_rows_lds<2, W32, C16>(S, n, g, win, wout, mu, s, acc); break;
        case 4: pi_rows_lds<4, W32, C16>(S, n, g, win, wout, mu, s, acc); break;
        case 8: pi_rows_lds<8, W32, C16>(S, n, g, win, wout, mu, s, acc); break;
        case 16: pi_rows_lds<16, W32, C16>(S, n, g, win, wout, mu, s, acc); break;
        case 32: pi_rows_lds<32, W32, C16>(S, n, g, win, wout, mu, s, acc); break;
        default: pi_rows_lds<64, W32, C16>(S, n, g, win, wout, mu, s, acc); break;
    }
}

// Levels jhi down to jlo (all FP64, small) refined inside one workgroup:
// prolongation, deflation, normalisation and every PI step separated only
// by workgroup barriers, so thousands of steps cost no launches.  A level
// whose CSR and two vectors fit in `lds_budget` bytes is first copied to
// LDS (columns as uint16 when n <= 65536, weights as FP32 when that is
// exact), so its steps touch no global memory; larger levels stream from
// global memory (L2).  The final vector of each level goes to buf0.
__global__ void __launch_bounds__(kBlockKernelThreads)
    k_refine_block(const LevelDev* __restrict__ lv, LevelState* st, int jhi, int jlo,
                   int uniform_start, double tol, int maxit, uint64_t seed, int lds_budget) {
    extern __shared__ double lds[];
    __shared__ double red[2 * 4 * 16];
    __shared__ double s_cm, s_cs;
    __shared__ int s_cfin;
    int parity = 0;
    if (threadIdx.x == 0 && !uniform_start) {
        LevelState c = st[jhi + 1];
        s_cm = c.mu;
        s_cs = c.s;
        s_cfin = c.fin;
    }
    __syncthreads();
    for (int j = jhi; j >= jlo; --j) {
        const LevelDev L = lv[j];
        const int n = L.n;
        // ---- choose where the level lives
        const int c16 = (n <= 65536) ? 1 : 0;
        int w32 = 0;
        size_t need = staged_bytes(L, 0, c16);
        if (need > (size_t)lds_budget && L.w32exact) {
            w32 = 1;
            need = staged_bytes(L, 1, c16);
        }
        const bool staged = need <= (size_t)lds_budget;
        StagedLevel S;
        double* b0;
        double* b1;
        if (staged) {
            char* p = (char*)lds;
            S.x0 = (double*)p;
            S.x1 = S.x0 + n;
            p += align8(16 * (size_t)n);
            S.w = p;
            p += align8((size_t)L.nnz * (w32 ? 4 : 8));
            S.rp = (const int32_t*)p;
            p += align8(4 * ((size_t)n + 1));
            S.col = p;
            for (int i = threadIdx.x; i <= n; i += blockDim.x) ((int32_t*)S.rp)[i] = L.rp[i];
            for (int e = threadIdx.x; e < (int)L.nnz; e += blockDim.x) {
                if (c16) ((uint16_t*)S.col)[e] = (uint16_t)L.col[e];
                else ((int32_t*)S.col)[e] = L.col[e];
                if (w32) ((float*)S.w)[e] = (float)L.w64[e];
                else ((double*)S.w)[e] = L.w64[e];
            }
            b0 = S.x0;
            b1 = S.x1;
        } else {
            b0 = (double*)L.buf0;
            b1 = (double*)L.buf1;
        }
        // ---- prolongation (or hashed uniform start), deflation, norm
        double sum[1] = {0.0};
        if (uniform_start && j == jhi) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                double v = hashed_uniform(seed, i) - 0.5;
                b0[i] = v;
                sum[0] += v;
            }
        } else {
            const LevelDev C = lv[j + 1];
            const void* cb = s_cfin ? C.buf1 : C.buf0;
            const double cm = s_cm, cs = s_cs;
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                double v = (ld_any(cb, C.fp32, L.agg[i]) - cm) * cs;
                b0[i] = v;
                sum[0] += v;
            }
        }
        block_sum1<1>(sum, red, parity);
        double mu = sum[0] / (double)n;
        double ss[1] = {0.0};
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            double d = b0[i] - mu;
            ss[0] += d * d;
        }
        block_sum1<1>(ss, red, parity);
        double s = 1.0 / sqrt(ss[0]);
        int cur = 0, k = 0, hit = 0;
        double utv = 0.0, pmu = mu, ps = s;
        while (true) {
            const double* win = cur ? b1 : b0;
            double* wout = cur ? b0 : b1;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            if (staged) {
                if (w32) {
                    if (c16) pi_rows_lds_dispatch<true, true>(L.lanes, S, n, L.g, win, wout, mu, s, acc);
                    else pi_rows_lds_dispatch<true, false>(L.lanes, S, n, L.g, win, wout, mu, s, acc);
                } else {
                    if (c16) pi_rows_lds_dispatch<false, true>(L.lanes, S, n, L.g, win, wout, mu, s, acc);
                    else pi_rows_lds_dispatch<false, false>(L.lanes, S, n, L.g, win, wout, mu, s, acc);
                }
            } else {
                pi_rows_dispatch<double>(L.lanes, L, win, wout, mu, s, 0, n, acc);
            }
            block_sum1<4>(acc, red, parity);
            const double mu2 = acc[0] / (double)n;
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
        // final vector to global buf0 (staged levels live in LDS until here)
        int fin = cur;
        if (staged) {
            const double* src = cur ? b1 : b0;
            const double* prv = cur ? b0 : b1;
            double* g0 = (double*)L.buf0;
            double* g1 = (double*)L.buf1;
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                g0[i] = src[i];
                g1[i] = prv[i];
            }
            fin = 0;
        }
        if (threadIdx.x == 0) {
            LevelState o;
            o.mu = mu;
            o.s = s;
            o.mu_prev = pmu;
            o.s_prev = ps;
            o.utv = utv;
            o.margin = utv - (1.0 - tol);
            o.fin = fin;
            o.k = k;
            o.maxit = hit;
            o.err = 0;
            st[j] = o;
            s_cm = mu;
            s_cs = s;
            s_cfin = fin;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- grid levels

template <typename T, int G>
__global__ void __launch_bounds__(kGridBlock)
    k_refine_grid(LevelDev L, LevelDev C, LevelState* st_j, const LevelState* st_c, int uniform_start,
                  GridSync* gs, double* partials, double* bcast, double tol, int maxit,
                  uint64_t seed) {
    __shared__ double red[16 * 5 + 8];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int r0 = L.part[lb], r1 = L.part[lb + 1];
    T* b0 = (T*)L.buf0;
    T* b1 = (T*)L.buf1;
    const double n = (double)L.n;
    // prolongation from level j+1 (or the hashed uniform start)
    double sum[1] = {0.0};
    if (uniform_start) {
        for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            T v = (T)(hashed_uniform(seed, i) - 0.5);
            b0[i] = v;
            sum[0] += (double)v;
        }
    } else {
        const LevelState c = *st_c;
        const void* cb = c.fin ? C.buf1 : C.buf0;
        for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            T v = (T)((ld_any(cb, C.fp32, L.agg[i]) - c.mu) * c.s);
            b0[i] = v;
            sum[0] += (double)v;
        }
    }
    if (!grid_allreduce<1>(sum, gs, partials, bcast, lb, red)) return;
    double mu = sum[0] / n;
    double ss[1] = {0.0};
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        double d = (double)b0[i] - mu;
        ss[0] += d * d;
    }
    if (!grid_allreduce<1>(ss, gs, partials, bcast, lb, red)) return;
    double s = 1.0 / sqrt(ss[0]);
    int cur = 0, k = 0, hit = 0;
    double utv = 0.0, pmu = mu, ps = s;
    while (true) {
        const T* win = cur ? b1 : b0;
        T* wout = cur ? b0 : b1;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        pi_rows<G, T>(L, win, wout, mu, s, r0, r1, acc);
        if (!grid_allreduce<4>(acc, gs, partials, bcast, lb, red)) return;
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
    if (blockIdx.x == 0 && threadIdx.x == 0) {
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
        *st_j = o;
    }
}

// ----------------------------------------------------------- finishing

// Finest level.  With `redo` = 1 (mixed precision) the last power-iteration
// step is recomputed in FP64 from the FP32 iterate before it, so the step
// count equals the FP64 path and only that earlier iterate carries FP32
// rounding.  Then the output y = deflated, normalised iterate, the
// edge-form Rayleigh quotient r = sum_edges w (y_i - y_k)^2 and the
// residual ||L y - r y||, all in FP64.
template <typename T, int G>
__global__ void __launch_bounds__(kGridBlock)
    k_finish(LevelDev L, const LevelState* st0, int redo, double* fa, double* fb, double* yout,
             GridSync* gs, double* partials, double* bcast, FinishOut* fo) {
    __shared__ double red[16 * 5 + 8];
    (void)fb;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int r0 = L.part[lb], r1 = L.part[lb + 1];
    const int lane = threadIdx.x & (G - 1);
    const int ngroups = blockDim.x / G;
    const double n = (double)L.n;
    const int32_t* __restrict__ rp = L.rp;
    const int32_t* __restrict__ col = L.col;
    const double* __restrict__ w = L.w64;
    const LevelState st = *st0;
    const void* src = st.fin ? L.buf1 : L.buf0;
    int src_f32 = (sizeof(T) == 4);
    double mu = st.mu, s = st.s;
    if (redo && st.k > 0) {
        const void* prev = st.fin ? L.buf0 : L.buf1;
        const double pmu = st.mu_prev, ps = st.s_prev;
        double acc[2] = {0.0, 0.0};
        for (int i = r0 + (int)(threadIdx.x / G); i < r1; i += ngroups) {
            const double wi = ld_any(prev, src_f32, i);
            double t = 0.0;
            for (int e = rp[i] + lane; e < rp[i + 1]; e += G) t += w[e] * (ld_any(prev, src_f32, col[e]) - wi);
            t = group_sum_t<G>(t);
            if (lane == 0) {
                double y = ps * (L.g * (wi - pmu) + t);
                fa[i] = y;
                acc[0] += y;
                acc[1] += y * y;
            }
        }
        if (!grid_allreduce<2>(acc, gs, partials, bcast, lb, red)) return;
        mu = acc[0] / n;
        s = 1.0 / sqrt(acc[1] - acc[0] * mu);
        src = fa;
        src_f32 = 0;
    }
    // pass 1: sums of u = (src - mu) s and the edge form
    double a3[3] = {0.0, 0.0, 0.0};
    for (int i = r0 + (int)(threadIdx.x / G); i < r1; i += ngroups) {
        const double si = ld_any(src, src_f32, i);
        double e2 = 0.0;
        for (int e = rp[i] + lane; e < rp[i + 1]; e += G) {
            double d = (ld_any(src, src_f32, col[e]) - si) * s;
            e2 += w[e] * d * d;
        }
        e2 = group_sum_t<G>(e2);
        if (lane == 0) {
            double u = (si - mu) * s;
            a3[0] += u;
            a3[1] += u * u;
            a3[2] += e2;
        }
    }
    if (!grid_allreduce<3>(a3, gs, partials, bcast, lb, red)) return;
    const double mean_u = a3[0] / n;
    const double nrm2 = a3[1] - a3[0] * mean_u;
    const double nrm = sqrt(nrm2);
    const double lam = 0.5 * a3[2] / nrm2;
    // pass 2: output and residual
    double r1s[1] = {0.0};
    for (int i = r0 + (int)(threadIdx.x / G); i < r1; i += ngroups) {
        const double si = ld_any(src, src_f32, i);
        double t = 0.0;
        for (int e = rp[i] + lane; e < rp[i + 1]; e += G) t += w[e] * (si - ld_any(src, src_f32, col[e]));
        t = group_sum_t<G>(t);
        if (lane == 0) {
            const double yi = ((si - mu) * s - mean_u) / nrm;
            const double ly = t * s / nrm;
            const double r = ly - lam * yi;
            r1s[0] += r * r;
            yout[i] = yi;
        }
    }
    if (!grid_allreduce<1>(r1s, gs, partials, bcast, lb, red)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        fo->lambda = lam;
        fo->residual = sqrt(r1s[0]);
        fo->sum_u = a3[0];
        fo->sum_uu = a3[1];
        fo->edge = a3[2];
    }
}

__global__ void k_reset_sync(GridSync* gs) {
    gs->count = 0;
    gs->gen = 0;
    gs->abort = 0;
    gs->pad = 0;
}

template <typename K>
int max_blocks_of(K kern, int threads) {
    int dev = 0, ncu = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, threads, 0) != hipSuccess) return 0;
    return occ * ncu;
}

}  // namespace

// ================================================================ launchers

hipError_t launch_coarse_dense(LevelDev L, LevelState* st, double* A, double* V, double* ev,
                               int32_t* idx, uint64_t seed, FinishOut* fo, hipStream_t s) {
    size_t shmem = (L.n <= kDenseLds) ? sizeof(double) * 2 * L.n * L.n : 0;
    int threads = (L.n <= kDenseLds) ? 64 : 256;
    hipLaunchKernelGGL(k_coarse_dense, dim3(1), dim3(threads), shmem, s, L, st, A, V, ev, idx, seed, fo);
    return hipGetLastError();
}

int refine_block_lds_budget() {
    static int budget = -1;
    if (budget < 0) {
        int dev = 0, maxsh = 65536;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        hipFuncAttributes fa;
        size_t stat = 0;
        if (hipFuncGetAttributes(&fa, (const void*)k_refine_block) == hipSuccess) stat = fa.sharedSizeBytes;
        long b = std::min<long>(kBlockLdsMax, (long)maxsh - (long)stat - 256);
        b = std::max<long>(b, 0);
        if (b > 65536 - (long)stat - 256 &&
            hipFuncSetAttribute((const void*)k_refine_block, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)b) != hipSuccess) {
            (void)hipGetLastError();
            b = std::max<long>(0, 65536 - (long)stat - 256);
        }
        budget = (int)(b & ~7L);
    }
    return budget;
}

hipError_t launch_refine_block(const LevelDev* lv, LevelState* st, int jhi, int jlo, int uniform_start,
                               double tol, int maxit, uint64_t seed, hipStream_t s) {
    const int budget = refine_block_lds_budget();
    hipLaunchKernelGGL(k_refine_block, dim3(1), dim3(kBlockKernelThreads), (size_t)budget, s, lv, st, jhi,
                       jlo, uniform_start, tol, maxit, seed, budget);
    return hipGetLastError();
}

#define CMG_GRID_SWITCH(MACRO, T)                                                                  \
    switch (lanes) {                                                                               \
        case 1: MACRO(T, 1); break;                                                                \
        case 2: MACRO(T, 2); break;                                                                \
        case 4: MACRO(T, 4); break;                                                                \
        case 8: MACRO(T, 8); break;                                                                \
        case 16: MACRO(T, 16); break;                                                              \
        case 32: MACRO(T, 32); break;                                                              \
        default: MACRO(T, 64); break;                                                              \
    }

int refine_grid_max_blocks(int fp32, int lanes, int variant) {
    (void)variant;
    int r = 0;
#define CMG_MB(T, G) r = max_blocks_of(k_refine_grid<T, G>, kGridBlock)
    if (fp32) {
        CMG_GRID_SWITCH(CMG_MB, float)
    } else {
        CMG_GRID_SWITCH(CMG_MB, double)
    }
#undef CMG_MB
    return r;
}

int finish_max_blocks(int fp32, int lanes, int variant) {
    (void)variant;
    int r = 0;
#define CMG_MB(T, G) r = max_blocks_of(k_finish<T, G>, kGridBlock)
    if (fp32) {
        CMG_GRID_SWITCH(CMG_MB, float)
    } else {
        CMG_GRID_SWITCH(CMG_MB, double)
    }
#undef CMG_MB
    return r;
}

hipError_t launch_refine_grid(const LevelDev& L, const LevelDev& C, LevelState* st_j,
                              const LevelState* st_c, int uniform_start, GridSync* gs,
                              double* partials, double* bcast, double tol, int maxit, uint64_t seed,
                              hipStream_t s) {
    LevelDev Lc = L, Cc = C;
    void* args[] = {&Lc, &Cc, &st_j, &st_c, &uniform_start, &gs, &partials, &bcast, &tol, &maxit, &seed};
    const int lanes = L.lanes;
    hipError_t e = hipSuccess;
#define CMG_LG(T, G)                                                                               \
    e = hipLaunchCooperativeKernel((const void*)k_refine_grid<T, G>, dim3(L.grid), dim3(kGridBlock), \
                                   args, 0, s)
    if (L.fp32) {
        CMG_GRID_SWITCH(CMG_LG, float)
    } else {
        CMG_GRID_SWITCH(CMG_LG, double)
    }
#undef CMG_LG
    return e;
}

hipError_t launch_finish(const LevelDev& L0, const LevelState* st0, int redo, double* f64a,
                         double* f64b, double* yout, GridSync* gs, double* partials, double* bcast,
                         FinishOut* fo, hipStream_t s) {
    LevelDev Lc = L0;
    void* args[] = {&Lc, &st0, &redo, &f64a, &f64b, &yout, &gs, &partials, &bcast, &fo};
    const int lanes = L0.lanes;
    hipError_t e = hipSuccess;
#define CMG_LF(T, G)                                                                               \
    e = hipLaunchCooperativeKernel((const void*)k_finish<T, G>, dim3(L0.grid), dim3(kGridBlock), args, \
                                   0, s)
    if (L0.fp32) {
        CMG_GRID_SWITCH(CMG_LF, float)
    } else {
        CMG_GRID_SWITCH(CMG_LF, double)
    }
#undef CMG_LF
    return e;
}

hipError_t launch_reset_sync(GridSync* gs, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_sync, dim3(1), dim3(1), 0, s, gs);
    return hipGetLastError();
}

}  // namespace cmg
