// Recursive spectral bisection: the graph-partitioning use of the Fiedler
// vector (Section 1), with the repeated solves the remark on the coarsest
// level anticipates.  Per depth, all current parts are handled together:
// their induced subgraphs are compacted into one block-diagonal CSR (parts
// contiguous, vertices in ascending index within a part, columns local to
// the part), connected components are labelled by hooking and pointer
// jumping, the Fiedler vectors of the connected parts come from one
// batched solve, and each part is split at the median of its sort key
// (the Fiedler value, or the component's smallest vertex for a
// disconnected part; ties by index) with two stable radix sorts.
#include "cmg_internal.h"

namespace cmg {

namespace {

constexpr int kRsbBlk = 256;

unsigned nblk(int64_t m) { return (unsigned)((m + kRsbBlk - 1) / kRsbBlk); }

// keys (part << 32 | v) of every vertex, for the stable sort by part
__global__ void k_rsb_keys(int n, const int32_t* __restrict__ part, unsigned long long* __restrict__ keys) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) keys[v] = ((unsigned long long)(uint32_t)part[v] << 32) | (uint32_t)v;
}

// perm[t] = vertex at position t; pos[v] = t; first position of each
// part; every position its own component to start with
__global__ void k_rsb_perm(int n, const unsigned long long* __restrict__ keys, int32_t* __restrict__ perm,
                           int32_t* __restrict__ pos, int32_t* __restrict__ first, int32_t* __restrict__ comp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int v = (int)(keys[t] & 0xffffffffull);
    const int p = (int)(keys[t] >> 32);
    perm[t] = v;
    pos[v] = t;
    comp[t] = t;
    if (t == 0 || (int)(keys[t - 1] >> 32) != p) first[p] = t;
}

// entries of each vertex's row that stay inside its part, in position order
__global__ void k_rsb_deg(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const int32_t* __restrict__ part, const int32_t* __restrict__ perm,
                          int32_t* __restrict__ deg) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int v = perm[t];
    const int p = part[v];
    int d = 0;
    for (int e = rp[v]; e < rp[v + 1]; ++e) d += part[col[e]] == p ? 1 : 0;
    deg[t] = d;
}

// block-diagonal CSR: columns local to the part (position - first position
// of the part), weights as FP64; each part's row pointers start at 0 in
// rpl[first[p] + p ..]
__global__ void k_rsb_fill(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const double* __restrict__ w, const int32_t* __restrict__ part,
                           const int32_t* __restrict__ perm, const int32_t* __restrict__ pos,
                           const int32_t* __restrict__ first, const int32_t* __restrict__ eoff,
                           int32_t* __restrict__ rpl, int32_t* __restrict__ colk, double* __restrict__ wk,
                           int32_t* __restrict__ cnt, int32_t* __restrict__ pnnz, int32_t* __restrict__ pbase) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int v = perm[t];
    const int p = part[v];
    const int f = first[p];
    const int base = eoff[f];
    int o = eoff[t];
    rpl[f + p + (t - f)] = o - base;
    for (int e = rp[v]; e < rp[v + 1]; ++e) {
        const int u = col[e];
        if (part[u] != p) continue;
        colk[o] = pos[u] - f;
        wk[o] = w[e];
        ++o;
    }
    if (t == n - 1 || part[perm[t + 1]] != p) {  // last row of the part
        rpl[f + p + (t - f) + 1] = o - base;
        cnt[p] = t - f + 1;
        pnnz[p] = o - base;
        pbase[p] = base;
    }
}

// connected components on the block-diagonal CSR (global positions):
// every edge hooks the larger of its endpoints' roots under the smaller
__device__ __forceinline__ int cc_find(const int32_t* comp, int x) {
    int y = comp[x];
    while (y != x) {
        x = y;
        y = comp[x];
    }
    return x;
}

__global__ void k_rsb_hook(int n, const int32_t* __restrict__ rpl, const int32_t* __restrict__ colk,
                           const int32_t* __restrict__ part, const int32_t* __restrict__ perm,
                           const int32_t* __restrict__ first, const int32_t* __restrict__ eoff, int32_t* comp,
                           int* changed) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int p = part[perm[t]];
    const int f = first[p];
    const int32_t* r = rpl + f + p;   // the part's row pointers start at 0 ...
    const int32_t* cp = colk + eoff[f];  // ... at the part's first entry
    const int i = t - f;
    for (int e = r[i]; e < r[i + 1]; ++e) {
        const int a = cc_find(comp, t), b = cc_find(comp, f + cp[e]);
        if (a != b) {
            atomicMin(&comp[a > b ? a : b], a < b ? a : b);
            *changed = 1;
        }
    }
}

__global__ void k_rsb_jump(int n, int32_t* comp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) comp[t] = cc_find(comp, t);
}

// component roots per part
__global__ void k_rsb_roots(int n, const int32_t* __restrict__ comp, const int32_t* __restrict__ part,
                            const int32_t* __restrict__ perm, int32_t* __restrict__ ncomp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && comp[t] == t) atomicAdd(&ncomp[part[perm[t]]], 1);
}

// sort key of every position: the Fiedler value (order-preserving bits,
// -0 as +0) in a connected part, the component's smallest position in a
// disconnected one, 0 in a part that is not split; value = position
__global__ void k_rsb_split_keys(int n, const double* __restrict__ x, const int32_t* __restrict__ comp,
                                 const int32_t* __restrict__ part, const int32_t* __restrict__ perm,
                                 const int32_t* __restrict__ mode, unsigned long long* __restrict__ keys,
                                 double* __restrict__ vals) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int md = mode[part[perm[t]]];  // 0 leaf, 1 Fiedler, 2 components
    unsigned long long k = 0;
    if (md == 1) {
        double xv = x[t];
        if (xv == 0.0) xv = 0.0;
        const unsigned long long b = (unsigned long long)__double_as_longlong(xv);
        k = (b >> 63) ? ~b : (b | 0x8000000000000000ull);
    } else if (md == 2) {
        k = (unsigned long long)(uint32_t)comp[t];
    }
    keys[t] = k;
    vals[t] = __longlong_as_double((long long)t);
}

// keys (part << 32) for the second stable sort, from the position values
__global__ void k_rsb_part_keys(int n, const double* __restrict__ vals, const int32_t* __restrict__ part,
                                const int32_t* __restrict__ perm, unsigned long long* __restrict__ keys) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int t = (int)__double_as_longlong(vals[q]);
    keys[q] = (unsigned long long)(uint32_t)part[perm[t]] << 32;
}

// q-th item of its part's segment: first half -> 2p, second -> 2p + 1
__global__ void k_rsb_assign(int n, const double* __restrict__ vals, const int32_t* __restrict__ part,
                             const int32_t* __restrict__ perm, const int32_t* __restrict__ first,
                             const int32_t* __restrict__ cnt, const int32_t* __restrict__ mode,
                             int32_t* __restrict__ next) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int t = (int)__double_as_longlong(vals[q]);
    const int v = perm[t];
    const int p = part[v];
    const int r = q - first[p];
    next[v] = mode[p] == 0 ? 2 * p : 2 * p + (r < cnt[p] / 2 ? 0 : 1);
}

// sum of w over edges whose ends lie in different parts (each counted from
// both ends, halved by the caller); per-block sums, added on the host
__global__ void k_rsb_cut(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const double* __restrict__ w, const int32_t* __restrict__ part, double* __restrict__ bsum) {
    __shared__ double red[kRsbBlk / 64];
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (v < n)
        for (int e = rp[v]; e < rp[v + 1]; ++e)
            if (part[col[e]] != part[v]) s += w[e];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kRsbBlk / 64; ++q) t += red[q];
        bsum[blockIdx.x] = t;
    }
}

}  // namespace

#define RSB_LAUNCH(k, m, ...)                                                      \
    do {                                                                           \
        if ((m) > 0) hipLaunchKernelGGL(k, dim3(nblk(m)), dim3(kRsbBlk), 0, s, __VA_ARGS__); \
    } while (0)

hipError_t launch_rsb_keys(int n, const int32_t* part, unsigned long long* keys, hipStream_t s) {
    RSB_LAUNCH(k_rsb_keys, n, n, part, keys);
    return hipGetLastError();
}
hipError_t launch_rsb_perm(int n, const unsigned long long* keys, int32_t* perm, int32_t* pos, int32_t* first,
                           int32_t* comp, hipStream_t s) {
    RSB_LAUNCH(k_rsb_perm, n, n, keys, perm, pos, first, comp);
    return hipGetLastError();
}
hipError_t launch_rsb_deg(int n, const int32_t* rp, const int32_t* col, const int32_t* part, const int32_t* perm,
                          int32_t* deg, hipStream_t s) {
    RSB_LAUNCH(k_rsb_deg, n, n, rp, col, part, perm, deg);
    return hipGetLastError();
}
hipError_t launch_rsb_fill(int n, const int32_t* rp, const int32_t* col, const double* w, const int32_t* part,
                           const int32_t* perm, const int32_t* pos, const int32_t* first, const int32_t* eoff,
                           int32_t* rpl, int32_t* colk, double* wk, int32_t* cnt, int32_t* pnnz, int32_t* pbase,
                           hipStream_t s) {
    RSB_LAUNCH(k_rsb_fill, n, n, rp, col, w, part, perm, pos, first, eoff, rpl, colk, wk, cnt, pnnz, pbase);
    return hipGetLastError();
}
hipError_t launch_rsb_components(int n, const int32_t* rpl, const int32_t* colk, const int32_t* part,
                                 const int32_t* perm, const int32_t* first, const int32_t* eoff, int32_t* comp,
                                 int* changed, int* h_changed, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int it = 0; it < 64; ++it) {
        *h_changed = 0;
        e = hipMemcpyAsync(changed, h_changed, sizeof(int), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        RSB_LAUNCH(k_rsb_hook, n, n, rpl, colk, part, perm, first, eoff, comp, changed);
        RSB_LAUNCH(k_rsb_jump, n, n, comp);
        e = hipMemcpyAsync(h_changed, changed, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess || *h_changed == 0) return e;
    }
    return hipErrorUnknown;  // did not settle (a hook round never stalls on a finite graph)
}
hipError_t launch_rsb_roots(int n, const int32_t* comp, const int32_t* part, const int32_t* perm, int32_t* ncomp,
                            hipStream_t s) {
    RSB_LAUNCH(k_rsb_roots, n, n, comp, part, perm, ncomp);
    return hipGetLastError();
}
hipError_t launch_rsb_split_keys(int n, const double* x, const int32_t* comp, const int32_t* part,
                                 const int32_t* perm, const int32_t* mode, unsigned long long* keys, double* vals,
                                 hipStream_t s) {
    RSB_LAUNCH(k_rsb_split_keys, n, n, x, comp, part, perm, mode, keys, vals);
    return hipGetLastError();
}
hipError_t launch_rsb_part_keys(int n, const double* vals, const int32_t* part, const int32_t* perm,
                                unsigned long long* keys, hipStream_t s) {
    RSB_LAUNCH(k_rsb_part_keys, n, n, vals, part, perm, keys);
    return hipGetLastError();
}
hipError_t launch_rsb_assign(int n, const double* vals, const int32_t* part, const int32_t* perm,
                             const int32_t* first, const int32_t* cnt, const int32_t* mode, int32_t* next,
                             hipStream_t s) {
    RSB_LAUNCH(k_rsb_assign, n, n, vals, part, perm, first, cnt, mode, next);
    return hipGetLastError();
}
hipError_t launch_rsb_cut(int n, const int32_t* rp, const int32_t* col, const double* w, const int32_t* part,
                          double* bsum, hipStream_t s) {
    RSB_LAUNCH(k_rsb_cut, n, n, rp, col, w, part, bsum);
    return hipGetLastError();
}
int rsb_cut_blocks(int n) { return (int)nblk(n); }

}  // namespace cmg
