// Several eigenpairs at once (the Remark after Algorithm 4: start from p
// approximate eigenpairs of the coarsest level, smooth every vector on each
// level, orthogonalise them and take Rayleigh quotients).
//
// A level keeps an n x P row-major block W plus a column mean mu and an
// upper-triangular R^{-1}; the current orthonormal block is
// V = (W - 1 mu^T) R^{-1}.  One step computes, row by row,
//   Z_i = ( g (W_i - mu) + sum_k a_ik (W_k - W_i) ) R^{-1}  (= (B_g V)_i,
// since L 1 = 0) and, in the same pass, the FP64 sums 1^T Z, Z^T Z, Z^T V
// and 1^T V.  From them the next mean, the Gram matrix of the deflated Z,
// its Cholesky factor R' (Cholesky QR: the same orthonormal block as
// Gram-Schmidt in column order, exactly so in exact arithmetic) and the
// stopping quantities (u_c, v_c) = (R'^{-T} (Z^T V - mu' 1^T V))_cc.  All
// sums have a fixed order, so results are reproducible bitwise.  One
// launch per step plus a one-workgroup check, as in the step mode of the
// single-vector path.
#include "cmg_internal.h"

namespace cmg {

namespace {

constexpr int kBlkThreads = 256;
constexpr int kBlkCheck = 1024;

template <int P>
struct BlkN {
    static constexpr int kTri = P * (P + 1) / 2;
    static constexpr int kStep = P + kTri + P * P + P;  // 1^T Z, Z^T Z (upper), Z^T V, 1^T V
    static constexpr int kProl = P + kTri;              // 1^T W, W^T W (upper)
    static constexpr int kOut = 2 * P;                  // edge-form numerators, squared norms
};

// v = (w - mu) R^{-1} for one row (R^{-1} upper triangular, row-major)
template <int P>
__device__ __forceinline__ void to_v(const double* __restrict__ w, const double* mu, const double* rinv,
                                     double (&v)[P]) {
    double d[P];
#pragma unroll
    for (int r = 0; r < P; ++r) d[r] = w[r] - mu[r];
#pragma unroll
    for (int c = 0; c < P; ++c) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r <= c; ++r) s += d[r] * rinv[r * P + c];
        v[c] = s;
    }
}

// Totals of the per-workgroup partial sums, in workgroup order, in every thread.
template <int NV>
__device__ __forceinline__ void blk_totals(const double* part, int nb, double (&v)[NV], double* red) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] += part[(size_t)NV * b + q];
    }
    block_sum<NV>(v, red);
}

template <int NV>
__device__ __forceinline__ void blk_post(double (&v)[NV], double* red, double* part) {
    block_sum<NV>(v, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) part[(size_t)NV * blockIdx.x + q] = v[q];
    }
}

// From the sums of a block Z (n rows): mu = 1^T Z / n, the Gram matrix of
// Z - 1 mu^T, its Cholesky factor R (upper, R^T R = G) and R^{-1}.
// Returns false if G is not positive definite.
template <int P>
__device__ bool chol_inv(const double* colsum, const double* tri, double n, double* mu, double* R, double* rinv) {
    double G[P][P];
#pragma unroll
    for (int r = 0; r < P; ++r) mu[r] = colsum[r] / n;
    int t = 0;
    for (int r = 0; r < P; ++r)
        for (int c = r; c < P; ++c, ++t) {
            G[r][c] = tri[t] - n * mu[r] * mu[c];
            G[c][r] = G[r][c];
        }
    for (int r = 0; r < P; ++r)
        for (int c = 0; c < P; ++c) R[r * P + c] = 0.0;
    for (int c = 0; c < P; ++c) {
        double s = G[c][c];
        for (int k = 0; k < c; ++k) s -= R[k * P + c] * R[k * P + c];
        if (!(s > 0.0)) return false;
        const double d = sqrt(s);
        R[c * P + c] = d;
        for (int j = c + 1; j < P; ++j) {
            double u = G[c][j];
            for (int k = 0; k < c; ++k) u -= R[k * P + c] * R[k * P + j];
            R[c * P + j] = u / d;
        }
    }
    // R^{-1} by back substitution, column by column
    for (int r = 0; r < P; ++r)
        for (int c = 0; c < P; ++c) rinv[r * P + c] = 0.0;
    for (int c = 0; c < P; ++c) {
        rinv[c * P + c] = 1.0 / R[c * P + c];
        for (int r = c - 1; r >= 0; --r) {
            double s = 0.0;
            for (int k = r + 1; k <= c; ++k) s += R[r * P + k] * rinv[k * P + c];
            rinv[r * P + c] = -s / R[r * P + r];
        }
    }
    return true;
}

// ---- coarsest level: p vectors from the dense eigensolve
//
// E = the eigenvectors above the smallest eigenvalue whose eigenvalue is at
// most lambda_{P+1} + 1e-10 ||L||_F (whole clusters: independent of the
// eigensolver's basis).  Start c = U(seed ^ (c+1) 0xD1B54A32D192ED03, i) - 1/2
// is projected onto E; the P projections are orthonormalised in column order
// (mean removed, modified Gram-Schmidt, normalised).
template <int P>
__global__ void __launch_bounds__(kBlkThreads) k_blk_coarse(BlkJob J, const double* __restrict__ V,
                                                            const double* __restrict__ ev,
                                                            const int32_t* __restrict__ idx) {
    __shared__ double y[P][128];
    __shared__ double red[16 * 2 + 8];
    const int n = J.n;
    // ||L^J||_F from the coarsest CSR: degrees on the diagonal, weights off it
    double f[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double d = 0.0, o = 0.0;
        for (int e = J.rp[i]; e < J.rp[i + 1]; ++e) {
            d += J.w[e];
            o += J.w[e] * J.w[e];
        }
        f[0] += d * d + o;
    }
    block_sum<1>(f, red);
    const double fro = sqrt(f[0]);
    const double top = ev[idx[P]];
    // projections: y_c = sum_{r in E} (q_r . z_c) q_r
    for (int c = 0; c < P; ++c) {
        const uint64_t sc = J.seed ^ ((uint64_t)(c + 1) * 0xD1B54A32D192ED03ull);
        for (int i = threadIdx.x; i < n; i += blockDim.x) y[c][i] = 0.0;
        __syncthreads();
        for (int r = 1; r < n; ++r) {
            const int k = idx[r];
            if (ev[k] > top + 1e-10 * fro) continue;
            double d[1] = {0.0};
            for (int i = threadIdx.x; i < n; i += blockDim.x) d[0] += V[i * n + k] * (hashed_uniform(sc, i) - 0.5);
            block_sum<1>(d, red);
            for (int i = threadIdx.x; i < n; i += blockDim.x) y[c][i] += d[0] * V[i * n + k];
            __syncthreads();
        }
    }
    // orthonormalise in column order
    for (int c = 0; c < P; ++c) {
        double m[1] = {0.0};
        for (int i = threadIdx.x; i < n; i += blockDim.x) m[0] += y[c][i];
        block_sum<1>(m, red);
        const double mean = m[0] / (double)n;
        for (int i = threadIdx.x; i < n; i += blockDim.x) y[c][i] -= mean;
        __syncthreads();
        for (int d = 0; d < c; ++d) {
            double t[1] = {0.0};
            for (int i = threadIdx.x; i < n; i += blockDim.x) t[0] += y[d][i] * y[c][i];
            block_sum<1>(t, red);
            for (int i = threadIdx.x; i < n; i += blockDim.x) y[c][i] -= t[0] * y[d][i];
            __syncthreads();
        }
        double q[1] = {0.0};
        for (int i = threadIdx.x; i < n; i += blockDim.x) q[0] += y[c][i] * y[c][i];
        block_sum<1>(q, red);
        const double nr = sqrt(q[0]);
        for (int i = threadIdx.x; i < n; i += blockDim.x) y[c][i] /= nr;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        for (int c = 0; c < P; ++c) J.W0[(size_t)i * P + c] = y[c][i];
    if (threadIdx.x == 0) {
        BlkCtl s{};
        for (int r = 0; r < P * P; ++r) s.rinv[r] = (r / P == r % P) ? 1.0 : 0.0;
        s.k = -1;
        s.cur = 0;
        s.done = 1;
        *J.ctl = s;
        for (int c = 0; c < P; ++c) J.out->coarse[c] = ev[idx[c + 1]];
    }
}

// ---- prolongation: W_i = V_{j+1}[agg(i)], posts 1^T W and W^T W
template <int P>
__global__ void __launch_bounds__(kBlkThreads) k_blk_prolong(const BlkJob* __restrict__ jp) {
    __shared__ double red[16 * BlkN<P>::kProl + BlkN<P>::kProl + 8];
    const BlkJob J = *jp;
    const BlkCtl cc = *J.cctl;
    const double* cw = cc.cur ? J.cW1 : J.cW0;
    const int r0 = J.rpart[blockIdx.x], r1 = J.rpart[blockIdx.x + 1];
    double acc[BlkN<P>::kProl];
#pragma unroll
    for (int q = 0; q < BlkN<P>::kProl; ++q) acc[q] = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        double v[P];
        to_v<P>(cw + (size_t)J.agg[i] * P, cc.mu, cc.rinv, v);
        int t = P;
#pragma unroll
        for (int r = 0; r < P; ++r) {
            J.W0[(size_t)i * P + r] = v[r];
            acc[r] += v[r];
#pragma unroll
            for (int c = r; c < P; ++c) acc[t++] += v[r] * v[c];
        }
    }
    blk_post<BlkN<P>::kProl>(acc, red, J.part);
}

// mean, Cholesky factor and R^{-1} of the prolongated block; arms the steps
template <int P>
__global__ void __launch_bounds__(kBlkCheck) k_blk_norm(const BlkJob* __restrict__ jp) {
    __shared__ double red[16 * BlkN<P>::kProl + BlkN<P>::kProl + 8];
    const BlkJob J = *jp;
    double v[BlkN<P>::kProl];
    blk_totals<BlkN<P>::kProl>(J.part, J.nb, v, red);
    if (threadIdx.x == 0) {
        BlkCtl s{};
        double R[P * P];
        if (!chol_inv<P>(v, v + P, (double)J.n, s.mu, R, s.rinv)) s.hit = 2;
        s.k = 0;
        s.cur = 0;
        s.done = s.hit == 2 ? 1 : 0;
        s.minutv = 0.0;
        *J.ctl = s;
    }
}

// one step of orthogonal iteration: W[cur] -> W[cur ^ 1]
template <int P>
__global__ void __launch_bounds__(kBlkThreads) k_blk_step(const BlkJob* __restrict__ jp) {
    __shared__ double red[16 * BlkN<P>::kStep + BlkN<P>::kStep + 8];
    const BlkJob J = *jp;
    const BlkCtl c = *J.ctl;
    if (c.done) return;
    const double* win = c.cur ? J.W1 : J.W0;
    double* wout = c.cur ? J.W0 : J.W1;
    const int r0 = J.rpart[blockIdx.x], r1 = J.rpart[blockIdx.x + 1];
    constexpr int T = BlkN<P>::kTri;
    double acc[BlkN<P>::kStep];
#pragma unroll
    for (int q = 0; q < BlkN<P>::kStep; ++q) acc[q] = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        double wi[P], y[P];
#pragma unroll
        for (int r = 0; r < P; ++r) {
            wi[r] = win[(size_t)i * P + r];
            y[r] = J.g * (wi[r] - c.mu[r]);
        }
        for (int e = J.rp[i]; e < J.rp[i + 1]; ++e) {
            const double a = J.w[e];
            const double* wk = win + (size_t)J.col[e] * P;
#pragma unroll
            for (int r = 0; r < P; ++r) y[r] += a * (wk[r] - wi[r]);
        }
        double z[P], v[P];
#pragma unroll
        for (int cc = 0; cc < P; ++cc) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r <= cc; ++r) s += y[r] * c.rinv[r * P + cc];
            z[cc] = s;
        }
        to_v<P>(wi, c.mu, c.rinv, v);
        int t = P;
#pragma unroll
        for (int r = 0; r < P; ++r) {
            wout[(size_t)i * P + r] = z[r];
            acc[r] += z[r];
#pragma unroll
            for (int cc = r; cc < P; ++cc) acc[t++] += z[r] * z[cc];
        }
#pragma unroll
        for (int r = 0; r < P; ++r)
#pragma unroll
            for (int cc = 0; cc < P; ++cc) acc[P + T + r * P + cc] += z[r] * v[cc];
#pragma unroll
        for (int r = 0; r < P; ++r) acc[P + T + P * P + r] += v[r];
    }
    blk_post<BlkN<P>::kStep>(acc, red, J.part);
}

// sums of the step, the new (mu, R^{-1}), the stopping test of every column
template <int P>
__global__ void __launch_bounds__(kBlkCheck) k_blk_check(const BlkJob* __restrict__ jp) {
    __shared__ double red[16 * BlkN<P>::kStep + BlkN<P>::kStep + 8];
    const BlkJob J = *jp;
    if (J.ctl->done) return;
    constexpr int T = BlkN<P>::kTri;
    double v[BlkN<P>::kStep];
    blk_totals<BlkN<P>::kStep>(J.part, J.nb, v, red);
    if (threadIdx.x == 0) {
        BlkCtl s = *J.ctl;
        double mu[P], R[P * P], rinv[P * P];
        const bool ok = chol_inv<P>(v, v + P, (double)J.n, mu, R, rinv);
        // (u_c, v_c) = (R^{-T} (Z^T V - mu 1^T V))_cc
        double minu = 2.0;
        for (int cc = 0; cc < P; ++cc) {
            double d = 0.0;
            for (int r = 0; r <= cc; ++r) {
                const double m = v[P + T + r * P + cc] - mu[r] * v[P + T + P * P + cc];
                d += rinv[r * P + cc] * m;
            }
            minu = d < minu ? d : minu;
        }
        ++s.k;
        s.cur ^= 1;
        for (int r = 0; r < P; ++r) s.mu[r] = mu[r];
        for (int r = 0; r < P * P; ++r) s.rinv[r] = rinv[r];
        s.minutv = minu;
        if (!ok) {
            s.done = 1;
            s.hit = 2;
        } else if (J.kfix > 0) {
            if (s.k >= J.kfix) s.done = 1;
        } else if (!(minu < 1.0 - J.tol)) {
            s.done = 1;
        } else if (s.k >= J.maxit) {
            s.done = 1;
            s.hit = 1;
        }
        *J.ctl = s;
    }
}

// ---- level 0: the output block (column-major) and the edge-form Rayleigh
// quotient numerators and norms of every column
template <int P>
__global__ void __launch_bounds__(kBlkThreads) k_blk_out(const BlkJob* __restrict__ jp, double* __restrict__ X) {
    __shared__ double red[16 * BlkN<P>::kOut + BlkN<P>::kOut + 8];
    const BlkJob J = *jp;
    const BlkCtl c = *J.ctl;
    const double* W = c.cur ? J.W1 : J.W0;
    const int r0 = J.rpart[blockIdx.x], r1 = J.rpart[blockIdx.x + 1];
    double acc[BlkN<P>::kOut];
#pragma unroll
    for (int q = 0; q < BlkN<P>::kOut; ++q) acc[q] = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        double vi[P];
        to_v<P>(W + (size_t)i * P, c.mu, c.rinv, vi);
        for (int e = J.rp[i]; e < J.rp[i + 1]; ++e) {
            double vk[P];
            to_v<P>(W + (size_t)J.col[e] * P, c.mu, c.rinv, vk);
#pragma unroll
            for (int r = 0; r < P; ++r) {
                const double d = vi[r] - vk[r];
                acc[r] += 0.5 * J.w[e] * d * d;
            }
        }
#pragma unroll
        for (int r = 0; r < P; ++r) {
            X[(size_t)r * J.n + i] = vi[r];
            acc[P + r] += vi[r] * vi[r];
        }
    }
    blk_post<BlkN<P>::kOut>(acc, red, J.part);
}

template <int P>
__global__ void __launch_bounds__(kBlkCheck) k_blk_rq(const BlkJob* __restrict__ jp) {
    __shared__ double red[16 * BlkN<P>::kOut + BlkN<P>::kOut + 8];
    const BlkJob J = *jp;
    double v[BlkN<P>::kOut];
    blk_totals<BlkN<P>::kOut>(J.part, J.nb, v, red);
    if (threadIdx.x == 0)
        for (int r = 0; r < P; ++r) {
            J.out->lambda[r] = v[r] / v[P + r];
            J.out->norm2[r] = v[P + r];
        }
}

// residual terms ((L x)_i - lambda x_i)^2 of every column
template <int P>
__global__ void __launch_bounds__(kBlkThreads) k_blk_res(const BlkJob* __restrict__ jp, const double* __restrict__ X) {
    __shared__ double red[16 * P + P + 8];
    const BlkJob J = *jp;
    double lam[P];
#pragma unroll
    for (int r = 0; r < P; ++r) lam[r] = J.out->lambda[r];
    const int r0 = J.rpart[blockIdx.x], r1 = J.rpart[blockIdx.x + 1];
    double acc[P];
#pragma unroll
    for (int r = 0; r < P; ++r) acc[r] = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const double* x = X + (size_t)r * J.n;
            const double xi = x[i];
            double t = 0.0;
            for (int e = J.rp[i]; e < J.rp[i + 1]; ++e) t += J.w[e] * (xi - x[J.col[e]]);
            const double d = t - lam[r] * xi;
            acc[r] += d * d;
        }
    }
    blk_post<P>(acc, red, J.part);
}

template <int P>
__global__ void __launch_bounds__(kBlkCheck) k_blk_fin(const BlkJob* __restrict__ jp) {
    __shared__ double red[16 * P + P + 8];
    const BlkJob J = *jp;
    double v[P];
    blk_totals<P>(J.part, J.nb, v, red);
    if (threadIdx.x == 0)
        for (int r = 0; r < P; ++r) J.out->residual[r] = sqrt(v[r] / J.out->norm2[r]);
}

template <int P>
hipError_t blk_launch(int what, const BlkJob* dj, const BlkJob& hj, double* X, const double* V, const double* ev,
                      const int32_t* idx, hipStream_t s) {
    const dim3 g(hj.nb), b(kBlkThreads), one(1), chk(kBlkCheck);
    switch (what) {
        case kBlkCoarse: hipLaunchKernelGGL(k_blk_coarse<P>, one, b, 0, s, hj, V, ev, idx); break;
        case kBlkProlong:
            hipLaunchKernelGGL(k_blk_prolong<P>, g, b, 0, s, dj);
            hipLaunchKernelGGL(k_blk_norm<P>, one, chk, 0, s, dj);
            break;
        case kBlkStep:
            hipLaunchKernelGGL(k_blk_step<P>, g, b, 0, s, dj);
            hipLaunchKernelGGL(k_blk_check<P>, one, chk, 0, s, dj);
            break;
        case kBlkOut:
            hipLaunchKernelGGL(k_blk_out<P>, g, b, 0, s, dj, X);
            hipLaunchKernelGGL(k_blk_rq<P>, one, chk, 0, s, dj);
            hipLaunchKernelGGL(k_blk_res<P>, g, b, 0, s, dj, (const double*)X);
            hipLaunchKernelGGL(k_blk_fin<P>, one, chk, 0, s, dj);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

int blk_parts(int p) {
    const int tri = p * (p + 1) / 2;
    return p + tri + p * p + p;
}

hipError_t launch_blk(int what, int p, const BlkJob* dj, const BlkJob& hj, double* X, const double* V,
                      const double* ev, const int32_t* idx, hipStream_t s) {
    switch (p) {
        case 1: return blk_launch<1>(what, dj, hj, X, V, ev, idx, s);
        case 2: return blk_launch<2>(what, dj, hj, X, V, ev, idx, s);
        case 3: return blk_launch<3>(what, dj, hj, X, V, ev, idx, s);
        case 4: return blk_launch<4>(what, dj, hj, X, V, ev, idx, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cmg
