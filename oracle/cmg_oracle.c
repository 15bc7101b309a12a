/*
 * CPU oracle for the cascadic multigrid (CMG) Fiedler-vector method of
 * Urschel, Hu, Xu & Zikatanov, "A Cascadic Multigrid Algorithm for Computing
 * the Fiedler Vector of Graph Laplacians" (arXiv 1412.0565).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It is plain, single-threaded C in IEEE FP64
 * (built with -ffp-contract=off so no FMA contraction happens), written to
 * be checked against the paper by eye, and shares no code, header or table
 * with the GPU path.
 *
 * Every function cites the passage of the paper it follows.  Readings of
 * passages that are silent, ambiguous or garbled are marked READING.
 *
 * Random draws.  The paper draws a random permutation in HEC (Algorithm 2,
 * randperm) and a Gaussian start for the coarsest power iteration
 * (Algorithm 1, Step 2).  Both are replaced by counter-based SplitMix64
 * values (Steele, Lea & Flood, OOPSLA 2014), implemented here from the
 * published definition and pinned to its published test vector.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG 1
#define ORC_E_GRAPH 2
#define ORC_E_ISOLATED 3
#define ORC_E_OOM 4
#define ORC_W_MAXIT 6
#define ORC_MAXP 8

/* ------------------------------------------------------------------ hash */

/* SplitMix64 output function (the "mix" applied to the state). */
uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* SplitMix64 generator: state += golden gamma, output mix(state). */
void orc_splitmix64_sequence(uint64_t seed, int32_t count, uint64_t* out)
{
    uint64_t s = seed;
    for (int32_t i = 0; i < count; ++i) {
        s += 0x9E3779B97F4A7C15ull;
        out[i] = orc_mix64(s);
    }
}

/* Priority key of vertex v at level j; replaces randperm (Algorithm 2).
 * READING: visiting vertices in ascending key order is a uniformly random
 * order for a random seed; the seed is exposed so runs are reproducible. */
uint64_t orc_hec_key(uint64_t seed, int32_t level, int32_t v)
{
    return orc_mix64(seed ^ ((uint64_t)(uint32_t)level << 40) ^ (uint64_t)(uint32_t)v);
}

/* Uniform start value in [0,1) used only where the coarsest level is too
 * large for the dense solve (power iteration on a random vector,
 * Section 2, Remark on the coarsest level). */
double orc_uniform(uint64_t seed, int32_t i)
{
    uint64_t h = orc_mix64(seed ^ 0x9E3779B97F4A7C15ull ^ (uint64_t)(uint32_t)i);
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------- Laplacian */

/* Weighted degree d_i = sum_k w_ik (Section 2, definition of L: rows of L
 * sum to zero, so the diagonal is the weighted degree). */
static double orc_degree(const int32_t* rp, const double* w, int32_t i)
{
    double d = 0.0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) d += w[e];
    return d;
}

/* y = L x with L = D - W (Section 2, definition of the graph Laplacian). */
void orc_laplacian_apply(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                         const double* x, double* y)
{
    for (int32_t i = 0; i < n; ++i) {
        double d = orc_degree(rp, w, i);
        double s = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) s += w[e] * x[col[e]];
        y[i] = d * x[i] - s;
    }
}

/* Gershgorin bound g = max_i sum_j |l_ij| = max_i 2 d_i
 * (Section 2.2 and Algorithm 3, first line). */
double orc_gershgorin(int32_t n, const int32_t* rp, const double* w)
{
    double g = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double r = 2.0 * orc_degree(rp, w, i);
        if (r > g) g = r;
    }
    return g;
}

/* ------------------------------------------------------------- validation */

int orc_validate(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col, const double* w)
{
    if (n < 2 || nnz < 0) return ORC_E_ARG;
    if (rp[0] != 0 || (int64_t)rp[n] != nnz) return ORC_E_GRAPH;
    for (int32_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return ORC_E_GRAPH;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n || col[e] == i) return ORC_E_GRAPH;
            if (e > rp[i] && col[e] <= col[e - 1]) return ORC_E_GRAPH;
            if (!(w[e] > 0.0) || !isfinite(w[e])) return ORC_E_GRAPH;
        }
    }
    for (int32_t i = 0; i < n; ++i)
        if (rp[i + 1] == rp[i]) return ORC_E_ISOLATED;
    return ORC_OK;
}

/* ------------------------------------------------------------------ HEC */

/* Heaviest neighbour: m = argmin of column v of L (Algorithm 2).  The
 * off-diagonal entries of L are -w, so this is the neighbour with the
 * largest weight.  READING: ties go to the lowest index (the first minimum,
 * as MATLAB's argmin returns).  The diagonal is positive and never chosen. */
int orc_heaviest(int32_t n, const int32_t* rp, const int32_t* col, const double* w, int32_t* h)
{
    for (int32_t v = 0; v < n; ++v) {
        if (rp[v + 1] == rp[v]) return ORC_E_ISOLATED;
        int32_t best = col[rp[v]];
        double bw = w[rp[v]];
        for (int32_t e = rp[v] + 1; e < rp[v + 1]; ++e) {
            if (w[e] > bw || (w[e] == bw && col[e] < best)) {
                bw = w[e];
                best = col[e];
            }
        }
        h[v] = best;
    }
    return ORC_OK;
}

typedef struct {
    uint64_t key;
    int32_t v;
} orc_keyv;

static int orc_cmp_keyv(const void* a, const void* b)
{
    const orc_keyv* x = (const orc_keyv*)a;
    const orc_keyv* y = (const orc_keyv*)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->v > y->v) - (x->v < y->v);
}

/* Heavy edge coarsening with an explicit visit order (Algorithm 2 and the
 * text of Section 2.1).  Definition: the vertices are taken in the given
 * order; one that belongs to no aggregate yet looks at its heaviest
 * neighbour m.  If m belongs to no aggregate either, the two form a new
 * aggregate, which the visited vertex opens (its "seed"); otherwise the
 * visited vertex joins the aggregate m belongs to.
 *
 * Here each vertex records the seed of its aggregate (owner[], -1 while it
 * has none), so an aggregate is named by its seed throughout.
 *
 * READING: the paper numbers aggregates in visit order; here they are
 * renumbered by ascending index of their seed vertex (a permutation of the
 * coarse vertices, which changes nothing else).
 *
 * agg[n] receives coarse ids, is_seed[n] marks seeds; returns the number of
 * aggregates, or -1 on an isolated vertex / allocation failure. */
int32_t orc_hec_order(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                      const int32_t* order, int32_t* agg, uint8_t* is_seed)
{
    int32_t* h = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!h || !owner || !rank) {
        free(h); free(owner); free(rank);
        return -1;
    }
    if (orc_heaviest(n, rp, col, w, h) != ORC_OK) {
        free(h); free(owner); free(rank);
        return -1;
    }
    for (int32_t v = 0; v < n; ++v) owner[v] = -1;
    for (int32_t t = 0; t < n; ++t) {
        const int32_t v = order[t];
        if (owner[v] >= 0) continue;             /* already in an aggregate */
        const int32_t m = h[v];
        /* m's aggregate if it has one, else a new one seeded at v */
        const int32_t sd = owner[m] >= 0 ? owner[m] : v;
        owner[v] = sd;
        owner[m] = sd;
    }
    int32_t count = 0;
    for (int32_t v = 0; v < n; ++v) {
        is_seed[v] = (uint8_t)(owner[v] == v);
        rank[v] = count;
        count += is_seed[v];
    }
    for (int32_t v = 0; v < n; ++v) agg[v] = rank[owner[v]];
    free(h); free(owner); free(rank);
    return count;
}

/* HEC with the seeded visit order of level j: ascending orc_hec_key. */
int32_t orc_hec(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                uint64_t seed, int32_t level, int32_t* agg, uint8_t* is_seed)
{
    orc_keyv* kv = (orc_keyv*)malloc(sizeof(orc_keyv) * (size_t)n);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!kv || !order) {
        free(kv); free(order);
        return -1;
    }
    for (int32_t v = 0; v < n; ++v) {
        kv[v].key = orc_hec_key(seed, level, v);
        kv[v].v = v;
    }
    qsort(kv, (size_t)n, sizeof(orc_keyv), orc_cmp_keyv);
    for (int32_t t = 0; t < n; ++t) order[t] = kv[t].v;
    int32_t c = orc_hec_order(n, rp, col, w, order, agg, is_seed);
    free(kv); free(order);
    return c;
}

/* Heavy edge matching (HEM; the matching the paper contrasts HEC with in
 * Section 2.1, after Karypis and Kumar), with an explicit visit order.
 * Definition: the vertices are taken in the given order; one that is not
 * matched yet is matched to its heaviest neighbour among those not matched
 * yet (lowest index on ties), if it has any, else it stays alone.  Every
 * aggregate is a matched pair or a single vertex, so n_{j+1} >= n_j / 2
 * (the lemma on coarsening rates: k_M >= 1/2).
 *
 * READING (as for HEC): aggregates are numbered by ascending index of the
 * vertex that opened them (the one visited first; a single vertex opens
 * its own).  Ties between equal weights go to the lowest neighbour index.
 *
 * agg[n] receives coarse ids, is_seed[n] marks opening vertices; returns
 * the number of aggregates, or -1 on an isolated vertex / allocation
 * failure. */
int32_t orc_hem_order(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                      const int32_t* order, int32_t* agg, uint8_t* is_seed)
{
    int32_t* opener = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!opener || !rank) {
        free(opener); free(rank);
        return -1;
    }
    for (int32_t v = 0; v < n; ++v) {
        if (rp[v + 1] == rp[v]) { free(opener); free(rank); return -1; }
        opener[v] = -1;
    }
    for (int32_t t = 0; t < n; ++t) {
        const int32_t v = order[t];
        if (opener[v] >= 0) continue;            /* matched earlier */
        int32_t best = -1;
        double bw = 0.0;
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int32_t u = col[e];
            if (opener[u] >= 0) continue;        /* only unmatched partners */
            if (best < 0 || w[e] > bw || (w[e] == bw && u < best)) {
                best = u;
                bw = w[e];
            }
        }
        opener[v] = v;
        if (best >= 0) opener[best] = v;
    }
    int32_t count = 0;
    for (int32_t v = 0; v < n; ++v) {
        is_seed[v] = (uint8_t)(opener[v] == v);
        rank[v] = count;
        count += is_seed[v];
    }
    for (int32_t v = 0; v < n; ++v) agg[v] = rank[opener[v]];
    free(opener); free(rank);
    return count;
}

/* HEM with the seeded visit order of level j (the HEC keys). */
int32_t orc_hem(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                uint64_t seed, int32_t level, int32_t* agg, uint8_t* is_seed)
{
    orc_keyv* kv = (orc_keyv*)malloc(sizeof(orc_keyv) * (size_t)n);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!kv || !order) {
        free(kv); free(order);
        return -1;
    }
    for (int32_t v = 0; v < n; ++v) {
        kv[v].key = orc_hec_key(seed, level, v);
        kv[v].v = v;
    }
    qsort(kv, (size_t)n, sizeof(orc_keyv), orc_cmp_keyv);
    for (int32_t t = 0; t < n; ++t) order[t] = kv[t].v;
    int32_t c = orc_hem_order(n, rp, col, w, order, agg, is_seed);
    free(kv); free(order);
    return c;
}

/* -------------------------------------------------------------- Galerkin */

typedef struct {
    int32_t b;
    int64_t seq;
    double w;
} orc_entry;

static int orc_cmp_entry(const void* a, const void* b)
{
    const orc_entry* x = (const orc_entry*)a;
    const orc_entry* y = (const orc_entry*)b;
    if (x->b != y->b) return (x->b > y->b) - (x->b < y->b);
    return (x->seq > y->seq) - (x->seq < y->seq);
}

/* Galerkin coarse graph L^{i+1} = I L^i I^T (Section 2, Step 1, and the
 * Proposition on restriction): the coarse weight between aggregates a != b
 * is the sum of the fine weights of edges joining them; edges inside one
 * aggregate vanish from the adjacency (they only enter the implicit
 * diagonal, which stays equal to the row sum).  Sums are taken in fine CSR
 * order (exact for integer weights).  Output CSR has ascending columns and
 * no diagonal; arrays are malloc'd and owned by the caller.
 * Returns the coarse nnz, or -1 on allocation failure. */
int64_t orc_galerkin(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                     const int32_t* agg, int32_t nc,
                     int32_t** rp_out, int32_t** col_out, double** w_out)
{
    /* members of each aggregate, ascending vertex index */
    int32_t* mptr = (int32_t*)calloc((size_t)nc + 1, sizeof(int32_t));
    int32_t* mem = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)nc);
    if (!mptr || !mem || !fill) { free(mptr); free(mem); free(fill); return -1; }
    for (int32_t v = 0; v < n; ++v) mptr[agg[v] + 1]++;
    for (int32_t a = 0; a < nc; ++a) mptr[a + 1] += mptr[a];
    for (int32_t a = 0; a < nc; ++a) fill[a] = mptr[a];
    for (int32_t v = 0; v < n; ++v) mem[fill[agg[v]]++] = v;
    free(fill);

    int64_t cap = 1024, nz = 0;
    int32_t* crp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nc + 1));
    int32_t* ccol = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    double* cw = (double*)malloc(sizeof(double) * (size_t)cap);
    int64_t bufcap = 1024;
    orc_entry* buf = (orc_entry*)malloc(sizeof(orc_entry) * (size_t)bufcap);
    if (!crp || !ccol || !cw || !buf) goto oom;
    crp[0] = 0;
    for (int32_t a = 0; a < nc; ++a) {
        int64_t cnt = 0;
        for (int32_t t = mptr[a]; t < mptr[a + 1]; ++t) {
            int32_t i = mem[t];
            for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
                int32_t b = agg[col[e]];
                if (b == a) continue;
                if (cnt == bufcap) {
                    bufcap *= 2;
                    orc_entry* nb = (orc_entry*)realloc(buf, sizeof(orc_entry) * (size_t)bufcap);
                    if (!nb) goto oom;
                    buf = nb;
                }
                buf[cnt].b = b;
                buf[cnt].seq = e; /* fine CSR position: members ascend, so this is CSR order */
                buf[cnt].w = w[e];
                ++cnt;
            }
        }
        qsort(buf, (size_t)cnt, sizeof(orc_entry), orc_cmp_entry);
        for (int64_t t = 0; t < cnt;) {
            int32_t b = buf[t].b;
            double s = 0.0;
            while (t < cnt && buf[t].b == b) { s += buf[t].w; ++t; }
            if (nz == cap) {
                cap *= 2;
                int32_t* nc2 = (int32_t*)realloc(ccol, sizeof(int32_t) * (size_t)cap);
                if (!nc2) goto oom;
                ccol = nc2;
                double* nw2 = (double*)realloc(cw, sizeof(double) * (size_t)cap);
                if (!nw2) goto oom;
                cw = nw2;
            }
            ccol[nz] = b;
            cw[nz] = s;
            ++nz;
        }
        if (nz >= 2147483647LL) goto oom;
        crp[a + 1] = (int32_t)nz;
    }
    free(buf); free(mptr); free(mem);
    *rp_out = crp; *col_out = ccol; *w_out = cw;
    return nz;
oom:
    free(buf); free(mptr); free(mem); free(crp); free(ccol); free(cw);
    return -1;
}

/* ----------------------------------------------------------- dense solve */

/* Cyclic-by-row Jacobi eigenvalue method for a symmetric matrix (Golub &
 * Van Loan, Matrix Computations, Section 8.5): sweep over all pairs p < q
 * in row order; each plane rotation J(p,q,theta) is chosen so that the
 * (p,q) entry of J^T A J vanishes.  Stops when the off-diagonal Frobenius
 * norm is at most 1e-14 * ||A||_F, or after 50 sweeps.
 * A (n*n, row major) is overwritten; V (n*n) gets eigenvectors in columns;
 * evals[k] = A[k][k] at exit (unsorted).  Returns the sweeps used. */
int orc_jacobi(int32_t n, double* A, double* V, double* evals)
{
    double fro = 0.0;
    for (int64_t t = 0; t < (int64_t)n * n; ++t) fro += A[t] * A[t];
    fro = sqrt(fro);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < n; ++k) V[(int64_t)i * n + k] = (i == k) ? 1.0 : 0.0;
    int sweep = 0;
    for (; sweep < 50; ++sweep) {
        double off = 0.0;
        for (int32_t i = 0; i < n; ++i)
            for (int32_t k = 0; k < n; ++k)
                if (i != k) off += A[(int64_t)i * n + k] * A[(int64_t)i * n + k];
        if (sqrt(off) <= 1e-14 * fro) break;
        for (int32_t p = 0; p < n - 1; ++p) {
            for (int32_t q = p + 1; q < n; ++q) {
                double apq = A[(int64_t)p * n + q];
                if (apq == 0.0) continue;
                double app = A[(int64_t)p * n + p];
                double aqq = A[(int64_t)q * n + q];
                /* symmetric 2x2 Schur decomposition */
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                /* rows p, q:  A <- J^T A */
                for (int32_t k = 0; k < n; ++k) {
                    double x = A[(int64_t)p * n + k];
                    double y = A[(int64_t)q * n + k];
                    A[(int64_t)p * n + k] = c * x - s * y;
                    A[(int64_t)q * n + k] = s * x + c * y;
                }
                /* columns p, q:  A <- A J */
                for (int32_t k = 0; k < n; ++k) {
                    double x = A[(int64_t)k * n + p];
                    double y = A[(int64_t)k * n + q];
                    A[(int64_t)k * n + p] = c * x - s * y;
                    A[(int64_t)k * n + q] = s * x + c * y;
                }
                /* eigenvector accumulation V <- V J */
                for (int32_t k = 0; k < n; ++k) {
                    double x = V[(int64_t)k * n + p];
                    double y = V[(int64_t)k * n + q];
                    V[(int64_t)k * n + p] = c * x - s * y;
                    V[(int64_t)k * n + q] = s * x + c * y;
                }
            }
        }
    }
    for (int32_t k = 0; k < n; ++k) evals[k] = A[(int64_t)k * n + k];
    return sweep;
}

/* Coarsest-level eigenvector (Algorithm 1, Step 2; the geometric variant,
 * Algorithm 4, solves the coarsest problem exactly).
 * READING: dense L^J, Jacobi, then the vector is the normalised projection
 * of the fixed ramp z_i = i - (n-1)/2 onto the eigenspace E of every
 * eigenvalue (other than the smallest) within 1e-10 ||L||_F of lambda_2.
 * This is basis independent when lambda_2 is repeated and fixes the sign.
 * If the projection is below 1e-8 ||z||, the hashed uniform start
 * (orc_uniform - 1/2) is projected instead.
 * y[n] receives the unit vector; *lam2 the second smallest eigenvalue;
 * *mult the size of E. */
int orc_coarsest_dense(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                       uint64_t seed, double* y, double* lam2, int32_t* mult)
{
    double* A = (double*)calloc((size_t)n * n, sizeof(double));
    double* V = (double*)malloc(sizeof(double) * (size_t)n * n);
    double* ev = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    double* z = (double*)malloc(sizeof(double) * (size_t)n);
    if (!A || !V || !ev || !idx || !z) {
        free(A); free(V); free(ev); free(idx); free(z);
        return ORC_E_OOM;
    }
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            A[(int64_t)i * n + col[e]] = -w[e];
            d += w[e];
        }
        A[(int64_t)i * n + i] = d;
    }
    double fro = 0.0;
    for (int64_t t = 0; t < (int64_t)n * n; ++t) fro += A[t] * A[t];
    fro = sqrt(fro);
    orc_jacobi(n, A, V, ev);
    /* ascending order of eigenvalues (insertion sort, stable) */
    for (int32_t i = 0; i < n; ++i) idx[i] = i;
    for (int32_t i = 1; i < n; ++i) {
        int32_t t = idx[i];
        int32_t k = i - 1;
        while (k >= 0 && ev[idx[k]] > ev[t]) { idx[k + 1] = idx[k]; --k; }
        idx[k + 1] = t;
    }
    double l2 = ev[idx[1]];
    for (int attempt = 0; attempt < 2; ++attempt) {
        double zn = 0.0;
        if (attempt == 0) {
            for (int32_t i = 0; i < n; ++i) z[i] = (double)i - 0.5 * (double)(n - 1);
        } else {
            for (int32_t i = 0; i < n; ++i) z[i] = orc_uniform(seed, i) - 0.5;
        }
        for (int32_t i = 0; i < n; ++i) zn += z[i] * z[i];
        zn = sqrt(zn);
        for (int32_t i = 0; i < n; ++i) y[i] = 0.0;
        int32_t m = 0;
        for (int32_t r = 1; r < n; ++r) {
            int32_t k = idx[r];
            if (fabs(ev[k] - l2) > 1e-10 * fro) continue;
            ++m;
            double dot = 0.0;
            for (int32_t i = 0; i < n; ++i) dot += V[(int64_t)i * n + k] * z[i];
            for (int32_t i = 0; i < n; ++i) y[i] += dot * V[(int64_t)i * n + k];
        }
        double pn = 0.0;
        for (int32_t i = 0; i < n; ++i) pn += y[i] * y[i];
        pn = sqrt(pn);
        *mult = m;
        if (pn >= 1e-8 * zn || attempt == 1) {
            for (int32_t i = 0; i < n; ++i) y[i] /= pn;
            break;
        }
    }
    *lam2 = l2;
    free(A); free(V); free(ev); free(idx); free(z);
    return ORC_OK;
}

/* --------------------------------------------------------- power iteration */

static double orc_dot(int32_t n, const double* a, const double* b)
{
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static void orc_deflate_normalise(int32_t n, double* u)
{
    double mean = 0.0;
    for (int32_t i = 0; i < n; ++i) mean += u[i];
    mean /= (double)n;
    for (int32_t i = 0; i < n; ++i) u[i] -= mean;
    double nr = sqrt(orc_dot(n, u, u));
    for (int32_t i = 0; i < n; ++i) u[i] /= nr;
}

/* Power iteration on B_g = g I - L (Algorithm 3; convergence test of
 * Section 2.2: stop once (u^k, u^{k-1}) >= 1 - tol).
 * READING: the start is deflated by subtracting its mean, i.e. one
 * Gram-Schmidt step against the constant vector (Section 2.2); the printed
 * formula multiplies the mean by the start vector itself, which would leave
 * the constant component in place.  Deflation is repeated after every
 * product (exactly a no-op in exact arithmetic, since 1-perp is invariant
 * under B_g).  Norms are Euclidean.  k counts executed loop bodies.
 * Returns k; *margin = u^T v - (1 - tol) at exit. */
int32_t orc_pi(int32_t n, const int32_t* rp, const int32_t* col, const double* w, double g,
               const double* y0, double tol, int32_t maxit, double* y, double* margin)
{
    double* v = (double*)calloc((size_t)n, sizeof(double));
    double* t = (double*)malloc(sizeof(double) * (size_t)n);
    if (!v || !t) { free(v); free(t); return -1; }
    memcpy(y, y0, sizeof(double) * (size_t)n);
    orc_deflate_normalise(n, y); /* u */
    int32_t k = 0;
    while (orc_dot(n, y, v) < 1.0 - tol && k < maxit) {
        memcpy(v, y, sizeof(double) * (size_t)n);        /* v <- u */
        orc_laplacian_apply(n, rp, col, w, v, t);        /* t = L v */
        for (int32_t i = 0; i < n; ++i) y[i] = g * v[i] - t[i]; /* u = B_g v */
        orc_deflate_normalise(n, y);                     /* u <- u/||u|| */
        ++k;
    }
    *margin = orc_dot(n, y, v) - (1.0 - tol);
    free(v); free(t);
    return k;
}

/* Number of smoothing steps on level j of the fixed schedule of the
 * geometric cascadic method (Algorithm 4 and the main theorem of Section 3:
 * k_j = beta^j k_0).  READING: a step count is an integer; k_j is the
 * smallest integer >= k_0 beta^j, with beta^j formed by j multiplications
 * in FP64 (exact for the integers and halves used in the tests), capped at
 * max_iters. */
int32_t orc_fixed_steps(int32_t k0, double beta, int32_t j, int32_t max_iters)
{
    double p = (double)k0;
    for (int32_t t = 0; t < j; ++t) p *= beta;
    double c = ceil(p);
    if (c > (double)max_iters) return max_iters;
    return (int32_t)c;
}

/* Fixed-schedule smoothing on one level (Algorithm 4, line "u_j = (I -
 * omega_j A_j)^{k_j} u_{j+1}" with omega_j = 1 / ||A_j||_inf): exactly
 * `steps` applications of B_g = g I - L, g = ||L||_inf (the Gershgorin
 * bound), each followed by deflation and normalisation as in Algorithm 3.
 * (I - L/g)^k u = g^{-k} (g I - L)^k u, so the direction is the same; no
 * stopping test is applied.  *utv receives the last (u^k, u^{k-1}). */
void orc_pi_fixed(int32_t n, const int32_t* rp, const int32_t* col, const double* w, double g,
                  const double* y0, int32_t steps, double* y, double* utv)
{
    double* v = (double*)calloc((size_t)n, sizeof(double));
    double* t = (double*)malloc(sizeof(double) * (size_t)n);
    if (!v || !t) { free(v); free(t); *utv = NAN; return; }
    memcpy(y, y0, sizeof(double) * (size_t)n);
    orc_deflate_normalise(n, y);
    for (int32_t k = 0; k < steps; ++k) {
        memcpy(v, y, sizeof(double) * (size_t)n);
        orc_laplacian_apply(n, rp, col, w, v, t);
        for (int32_t i = 0; i < n; ++i) y[i] = g * v[i] - t[i];
        orc_deflate_normalise(n, y);
    }
    *utv = orc_dot(n, y, v);
    free(v); free(t);
}

/* Rayleigh quotient in edge form r = sum_{edges} w_ik (y_i - y_k)^2 / ||y||^2
 * (equal to y^T L y / y^T y, the eigenvalue estimate of Section 4), and the
 * residual ||L y - r y|| / ||y|| reported as the error in Table 2. */
void orc_rq_residual(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                     const double* y, double* rq, double* res)
{
    double num = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
            if (col[e] > i) {
                double d = y[i] - y[col[e]];
                num += w[e] * d * d;
            }
    double yy = orc_dot(n, y, y);
    double r = num / yy;
    double* t = (double*)malloc(sizeof(double) * (size_t)n);
    double s = 0.0;
    if (t) {
        orc_laplacian_apply(n, rp, col, w, y, t);
        for (int32_t i = 0; i < n; ++i) {
            double d = t[i] - r * y[i];
            s += d * d;
        }
        free(t);
    }
    *rq = r;
    *res = sqrt(s / yy);
}

/* ------------------------------------------------------------------ driver */

typedef struct {
    int32_t n;
    int64_t nnz;
    int32_t* rp;
    int32_t* col;
    double* w;
    int32_t* agg;      /* to the next level (NULL on the coarsest) */
    double g;
    int32_t k;         /* power-iteration steps on this level (-1: coarsest dense) */
    double margin;
} orc_level;

typedef struct {
    int32_t status;
    int32_t nlevels;   /* J + 1 */
    orc_level lv[64];
    double lambda;     /* r~ */
    double residual;
    double coarse_lambda2;
    int32_t coarse_mult;
    int32_t collapsed; /* 1 if the level loop stopped on a collapse */
    double* y;         /* n0 */
} orc_result;

void orc_free(orc_result* r)
{
    if (!r) return;
    for (int32_t j = 0; j < r->nlevels; ++j) {
        if (j > 0) {
            free(r->lv[j].rp);
            free(r->lv[j].col);
            free(r->lv[j].w);
        }
        free(r->lv[j].agg);
    }
    free(r->y);
    free(r);
}

/* Multilevel cascadic eigensolver (Algorithm 1).
 *  Step 1: while n_i > coarsest_n: HEC, Galerkin coarse graph.
 *          READING: if HEC would produce fewer than 2 aggregates (complete
 *          graphs, stars, dense power-law levels) the level is discarded and
 *          the loop stops there.
 *  Step 2: coarsest solve (dense if n_J <= dense_max, else power iteration
 *          from the hashed uniform start).
 *  Step 3: for j = J-1 .. 0: prolongate (y_hat_v = y[agg_j(v)]; the
 *          printed index i inside the loop is read as j) and refine by PI.
 * The returned vector is deflated and normalised once more; lambda is the
 * edge-form Rayleigh quotient and residual ||L y - lambda y||.
 * The level-0 arrays are borrowed from the caller (not copied). */
orc_result* orc_cmg_ex(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                       const double* w, double tol, int32_t coarsest_n, int32_t dense_max,
                       uint64_t seed, int32_t max_iters, int32_t fixed_k0, double fixed_beta,
                       int32_t coarsen);

orc_result* orc_cmg(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                    const double* w, double tol, int32_t coarsest_n, int32_t dense_max,
                    uint64_t seed, int32_t max_iters)
{
    return orc_cmg_ex(n, nnz, rp, col, w, tol, coarsest_n, dense_max, seed, max_iters, 0, 0.0, 0);
}

/* The same driver with two variations:
 *  fixed_k0 > 0: every refined level j runs exactly
 *      k_j = orc_fixed_steps(fixed_k0, fixed_beta, j, max_iters) smoothing
 *      steps (Algorithm 4's schedule) instead of Algorithm 3's stopping
 *      test; the coarsest level, when it is refined by power iteration
 *      (after a collapse), follows the same schedule.
 *  coarsen = 1: heavy edge matching (orc_hem) instead of HEC in Step 1. */
/* Step 1 of Algorithm 1 into r->lv (level 0 borrows the caller's arrays):
 * while n_j > coarsest_n, coarsen (HEC, or HEM with coarsen = 1) and form
 * the Galerkin coarse graph; a coarsening to fewer than 2 aggregates is
 * discarded and ends the loop.  Leaves r->status set. */
static void orc_build_hierarchy(orc_result* r, int32_t n, int64_t nnz, const int32_t* rp,
                                const int32_t* col, const double* w, int32_t coarsest_n,
                                uint64_t seed, int32_t coarsen)
{
    r->status = orc_validate(n, nnz, rp, col, w);
    if (r->status != ORC_OK) return;
    r->lv[0].n = n;
    r->lv[0].nnz = nnz;
    r->lv[0].rp = (int32_t*)rp;
    r->lv[0].col = (int32_t*)col;
    r->lv[0].w = (double*)w;
    r->nlevels = 1;
    int32_t j = 0;
    while (r->lv[j].n > coarsest_n && j < 63) {
        orc_level* L = &r->lv[j];
        int32_t* agg = (int32_t*)malloc(sizeof(int32_t) * (size_t)L->n);
        uint8_t* sd = (uint8_t*)malloc((size_t)L->n);
        if (!agg || !sd) { free(agg); free(sd); r->status = ORC_E_OOM; return; }
        int32_t nc = coarsen == 1 ? orc_hem(L->n, L->rp, L->col, L->w, seed, j, agg, sd)
                                  : orc_hec(L->n, L->rp, L->col, L->w, seed, j, agg, sd);
        free(sd);
        if (nc < 0) { free(agg); r->status = ORC_E_ISOLATED; return; }
        if (nc < 2) { free(agg); r->collapsed = 1; break; }
        orc_level* C = &r->lv[j + 1];
        int64_t cnz = orc_galerkin(L->n, L->rp, L->col, L->w, agg, nc, &C->rp, &C->col, &C->w);
        if (cnz < 0) { free(agg); r->status = ORC_E_OOM; return; }
        L->agg = agg;
        C->n = nc;
        C->nnz = cnz;
        r->nlevels = j + 2;
        ++j;
    }
    for (int32_t t = 0; t < r->nlevels; ++t)
        r->lv[t].g = orc_gershgorin(r->lv[t].n, r->lv[t].rp, r->lv[t].w);
}

orc_result* orc_cmg_ex(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                       const double* w, double tol, int32_t coarsest_n, int32_t dense_max,
                       uint64_t seed, int32_t max_iters, int32_t fixed_k0, double fixed_beta,
                       int32_t coarsen)
{
    orc_result* r = (orc_result*)calloc(1, sizeof(orc_result));
    if (!r) return NULL;
    orc_build_hierarchy(r, n, nnz, rp, col, w, coarsest_n, seed, coarsen);
    if (r->status != ORC_OK) return r;
    int32_t J = r->nlevels - 1;
    for (int32_t t = 0; t <= J; ++t) {
        r->lv[t].k = 0;
        r->lv[t].margin = 0.0;
    }
    double* ycur = (double*)malloc(sizeof(double) * (size_t)r->lv[J].n);
    if (!ycur) { r->status = ORC_E_OOM; return r; }
    orc_level* CJ = &r->lv[J];
    if (CJ->n <= dense_max) {
        orc_coarsest_dense(CJ->n, CJ->rp, CJ->col, CJ->w, seed, ycur, &r->coarse_lambda2,
                           &r->coarse_mult);
        CJ->k = -1;
    } else {
        double* st = (double*)malloc(sizeof(double) * (size_t)CJ->n);
        if (!st) { free(ycur); r->status = ORC_E_OOM; return r; }
        for (int32_t i = 0; i < CJ->n; ++i) st[i] = orc_uniform(seed, i) - 0.5;
        if (fixed_k0 > 0) {
            CJ->k = orc_fixed_steps(fixed_k0, fixed_beta, J, max_iters);
            orc_pi_fixed(CJ->n, CJ->rp, CJ->col, CJ->w, CJ->g, st, CJ->k, ycur, &CJ->margin);
            CJ->margin -= 1.0;
        } else {
            CJ->k = orc_pi(CJ->n, CJ->rp, CJ->col, CJ->w, CJ->g, st, tol, max_iters, ycur, &CJ->margin);
            if (CJ->k >= max_iters) r->status = ORC_W_MAXIT;
        }
        free(st);
    }
    for (int32_t t = J - 1; t >= 0; --t) {
        orc_level* F = &r->lv[t];
        double* yh = (double*)malloc(sizeof(double) * (size_t)F->n);
        double* yn = (double*)malloc(sizeof(double) * (size_t)F->n);
        if (!yh || !yn) { free(yh); free(yn); free(ycur); r->status = ORC_E_OOM; return r; }
        for (int32_t v = 0; v < F->n; ++v) yh[v] = ycur[F->agg[v]];
        if (fixed_k0 > 0) {
            F->k = orc_fixed_steps(fixed_k0, fixed_beta, t, max_iters);
            orc_pi_fixed(F->n, F->rp, F->col, F->w, F->g, yh, F->k, yn, &F->margin);
            F->margin -= 1.0;   /* (u^k, u^{k-1}) - 1: no tolerance applies */
        } else {
            F->k = orc_pi(F->n, F->rp, F->col, F->w, F->g, yh, tol, max_iters, yn, &F->margin);
            if (F->k >= max_iters) r->status = ORC_W_MAXIT;
        }
        free(yh);
        free(ycur);
        ycur = yn;
    }
    orc_deflate_normalise(n, ycur);
    r->y = ycur;
    orc_rq_residual(n, rp, col, w, ycur, &r->lambda, &r->residual);
    return r;
}

/* ------------------------------------------- several eigenpairs (block) */

/* Start vector c of the block variant: U(seed ^ (c + 1) * 0xD1B54A32D192ED03, i) - 1/2
 * (hashed uniforms of a stream of their own per column). */
static double orc_block_start(uint64_t seed, int32_t c, int32_t i)
{
    return orc_uniform(seed ^ ((uint64_t)(c + 1) * 0xD1B54A32D192ED03ull), i) - 0.5;
}

/* Orthonormalise the p columns of V (n x p, column c at V + c n) in column
 * order: remove the column's mean (deflation against the constant vector),
 * then its components along the earlier columns (modified Gram-Schmidt),
 * then normalise. */
static void orc_orthonormalise(int32_t n, int32_t p, double* V)
{
    for (int32_t c = 0; c < p; ++c) {
        double* v = V + (size_t)c * n;
        double mean = 0.0;
        for (int32_t i = 0; i < n; ++i) mean += v[i];
        mean /= (double)n;
        for (int32_t i = 0; i < n; ++i) v[i] -= mean;
        for (int32_t d = 0; d < c; ++d) {
            const double* u = V + (size_t)d * n;
            double dot = orc_dot(n, u, v);
            for (int32_t i = 0; i < n; ++i) v[i] -= dot * u[i];
        }
        double nr = sqrt(orc_dot(n, v, v));
        for (int32_t i = 0; i < n; ++i) v[i] /= nr;
    }
}

/* Several approximate eigenpairs at the coarsest level (Remark after
 * Algorithm 4: start from p approximate eigenpairs of the coarsest level).
 * READING: dense L^J and Jacobi as in orc_coarsest_dense; E = the
 * eigenvectors above the smallest eigenvalue whose eigenvalue is at most
 * lambda_{p+1} + 1e-10 ||L||_F (whole clusters, so E does not depend on the
 * eigensolver's basis); the p start vectors orc_block_start are projected
 * onto E and orthonormalised in column order.  V: n x p; lams[c] receives
 * the (c+2)-th smallest eigenvalue.  Needs p <= n - 1. */
int orc_coarsest_block(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                       uint64_t seed, int32_t p, double* V, double* lams)
{
    if (p < 1 || p > n - 1) return ORC_E_ARG;
    double* A = (double*)calloc((size_t)n * n, sizeof(double));
    double* Q = (double*)malloc(sizeof(double) * (size_t)n * n);
    double* ev = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!A || !Q || !ev || !idx) {
        free(A); free(Q); free(ev); free(idx);
        return ORC_E_OOM;
    }
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            A[(int64_t)i * n + col[e]] = -w[e];
            d += w[e];
        }
        A[(int64_t)i * n + i] = d;
    }
    double fro = 0.0;
    for (int64_t t = 0; t < (int64_t)n * n; ++t) fro += A[t] * A[t];
    fro = sqrt(fro);
    orc_jacobi(n, A, Q, ev);
    for (int32_t i = 0; i < n; ++i) idx[i] = i;
    for (int32_t i = 1; i < n; ++i) {
        int32_t t = idx[i];
        int32_t k = i - 1;
        while (k >= 0 && ev[idx[k]] > ev[t]) { idx[k + 1] = idx[k]; --k; }
        idx[k + 1] = t;
    }
    const double top = ev[idx[p]];
    for (int32_t c = 0; c < p; ++c) {
        double* v = V + (size_t)c * n;
        for (int32_t i = 0; i < n; ++i) v[i] = 0.0;
        for (int32_t r = 1; r < n; ++r) {
            int32_t k = idx[r];
            if (ev[k] > top + 1e-10 * fro) continue;
            double dot = 0.0;
            for (int32_t i = 0; i < n; ++i) dot += Q[(int64_t)i * n + k] * orc_block_start(seed, c, i);
            for (int32_t i = 0; i < n; ++i) v[i] += dot * Q[(int64_t)i * n + k];
        }
        lams[c] = ev[idx[c + 1]];
    }
    orc_orthonormalise(n, p, V);
    free(A); free(Q); free(ev); free(idx);
    return ORC_OK;
}

/* Block power iteration on one level (Remark after Algorithm 4: smooth
 * each approximate eigenfunction, orthogonalise them, take Rayleigh
 * quotients).  READING: each step applies B_g = gI - L to every column and
 * orthonormalises the result (orc_orthonormalise), i.e. orthogonal
 * iteration; Algorithm 3's stopping test is applied to every column (stop
 * once (u_c, v_c) >= 1 - tol for all c, the first step always runs), or,
 * with steps > 0, exactly `steps` steps run (Algorithm 4's schedule).
 * V0, V: n x p.  Returns the number of steps; *minutv the smallest
 * (u_c, v_c) of the last step. */
int32_t orc_block_pi(int32_t n, const int32_t* rp, const int32_t* col, const double* w, double g,
                     int32_t p, const double* V0, double tol, int32_t maxit, int32_t steps,
                     double* V, double* minutv)
{
    const size_t np = (size_t)n * (size_t)p;
    double* Vold = (double*)calloc(np, sizeof(double));
    double* t = (double*)malloc(sizeof(double) * (size_t)n);
    if (!Vold || !t) { free(Vold); free(t); return -1; }
    memcpy(V, V0, sizeof(double) * np);
    orc_orthonormalise(n, p, V);
    int32_t k = 0;
    double mu = 0.0;  /* min_c (u_c, v_c); 0 before the first step */
    while (steps > 0 ? k < steps : (mu < 1.0 - tol && k < maxit)) {
        memcpy(Vold, V, sizeof(double) * np);
        for (int32_t c = 0; c < p; ++c) {
            const double* v = Vold + (size_t)c * n;
            double* u = V + (size_t)c * n;
            orc_laplacian_apply(n, rp, col, w, v, t);
            for (int32_t i = 0; i < n; ++i) u[i] = g * v[i] - t[i];
        }
        orc_orthonormalise(n, p, V);
        ++k;
        mu = 2.0;
        for (int32_t c = 0; c < p; ++c) {
            double d = orc_dot(n, V + (size_t)c * n, Vold + (size_t)c * n);
            if (d < mu) mu = d;
        }
    }
    *minutv = mu;
    free(Vold); free(t);
    return k;
}

typedef struct {
    int32_t status;
    int32_t nlevels;
    int32_t p;
    int32_t k[64];
    double lambdas[ORC_MAXP];    /* Rayleigh quotients of the output columns */
    double residuals[ORC_MAXP];  /* ||L x_c - lambda_c x_c|| */
    double coarse[ORC_MAXP];     /* lambda_2 .. lambda_{p+1} of the coarsest level */
    double* X;                   /* n0 x p, column-major */
} orc_block_result;

/* Several eigenpairs (Remark after Algorithm 4) on the hierarchy of
 * Algorithm 1, Step 1: the coarsest block (orc_coarsest_block; the
 * coarsest level must be dense, n_J <= dense_max, with p < n_J), then for
 * j = J-1 .. 0 the columns are prolongated (x_v = x[agg_j(v)]) and refined
 * by orc_block_pi, with the fixed schedule when fixed_k0 > 0.  The output
 * columns are orthonormalised once more; lambdas are edge-form Rayleigh
 * quotients and residuals ||L x - lambda x|| per column. */
orc_block_result* orc_cmg_block(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                                const double* w, double tol, int32_t coarsest_n, int32_t dense_max,
                                uint64_t seed, int32_t max_iters, int32_t fixed_k0,
                                double fixed_beta, int32_t p)
{
    orc_block_result* out = (orc_block_result*)calloc(1, sizeof(orc_block_result));
    orc_result* r = (orc_result*)calloc(1, sizeof(orc_result));
    if (!out || !r) { free(out); free(r); return NULL; }
    out->p = p;
    if (p < 1 || p > ORC_MAXP) { out->status = ORC_E_ARG; free(r); return out; }
    orc_build_hierarchy(r, n, nnz, rp, col, w, coarsest_n, seed, 0);
    out->status = r->status;
    out->nlevels = r->nlevels;
    int32_t J = r->nlevels - 1;
    if (out->status == ORC_OK && (r->lv[J].n > dense_max || p > r->lv[J].n - 1)) out->status = ORC_E_ARG;
    double* cur = NULL;
    if (out->status == ORC_OK) {
        cur = (double*)malloc(sizeof(double) * (size_t)r->lv[J].n * p);
        if (!cur || orc_coarsest_block(r->lv[J].n, r->lv[J].rp, r->lv[J].col, r->lv[J].w, seed, p, cur,
                                       out->coarse) != ORC_OK)
            out->status = ORC_E_OOM;
        out->k[J] = -1;
    }
    for (int32_t t = J - 1; t >= 0 && out->status == ORC_OK; --t) {
        orc_level* F = &r->lv[t];
        const int32_t nc = r->lv[t + 1].n;
        double* start = (double*)malloc(sizeof(double) * (size_t)F->n * p);
        double* next = (double*)malloc(sizeof(double) * (size_t)F->n * p);
        if (!start || !next) { free(start); free(next); out->status = ORC_E_OOM; break; }
        for (int32_t c = 0; c < p; ++c)
            for (int32_t v = 0; v < F->n; ++v)
                start[(size_t)c * F->n + v] = cur[(size_t)c * nc + F->agg[v]];
        const int32_t steps = fixed_k0 > 0 ? orc_fixed_steps(fixed_k0, fixed_beta, t, max_iters) : 0;
        double mu;
        out->k[t] = orc_block_pi(F->n, F->rp, F->col, F->w, F->g, p, start, tol, max_iters, steps, next, &mu);
        if (fixed_k0 == 0 && out->k[t] >= max_iters) out->status = ORC_W_MAXIT;
        free(start);
        free(cur);
        cur = next;
    }
    if (cur && (out->status == ORC_OK || out->status == ORC_W_MAXIT)) {
        orc_orthonormalise(n, p, cur);
        for (int32_t c = 0; c < p; ++c)
            orc_rq_residual(n, rp, col, w, cur + (size_t)c * n, &out->lambdas[c], &out->residuals[c]);
        out->X = cur;
        cur = NULL;
    }
    free(cur);
    orc_free(r);
    return out;
}

void orc_block_free(orc_block_result* b)
{
    if (!b) return;
    free(b->X);
    free(b);
}

int32_t orc_block_status(const orc_block_result* b) { return b->status; }
int32_t orc_block_nlevels(const orc_block_result* b) { return b->nlevels; }
int32_t orc_block_k(const orc_block_result* b, int32_t j) { return b->k[j]; }
double orc_block_lambda(const orc_block_result* b, int32_t c) { return b->lambdas[c]; }
double orc_block_residual(const orc_block_result* b, int32_t c) { return b->residuals[c]; }
double orc_block_coarse(const orc_block_result* b, int32_t c) { return b->coarse[c]; }
void orc_block_copy_x(const orc_block_result* b, int32_t n, double* X)
{
    if (b->X) memcpy(X, b->X, sizeof(double) * (size_t)n * b->p);
}

/* ------------------------------------------- recursive spectral bisection */

/* Induced subgraph of the vertices with sel[v] == 1: vertices relabelled
 * 0..m-1 in ascending original index (glob[] maps back), edges to
 * unselected vertices dropped, CSR order kept.  Returns m (-1 on
 * allocation failure); the caller frees *prp, *pcol, *pw, *pglob. */
int32_t orc_induced(int32_t n, const int32_t* rp, const int32_t* col, const double* w,
                           const uint8_t* sel, int32_t** prp, int32_t** pcol, double** pw,
                           int32_t** pglob)
{
    int32_t* loc = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!loc) return -1;
    int32_t m = 0;
    int64_t z = 0;
    for (int32_t v = 0; v < n; ++v) {
        loc[v] = sel[v] ? m++ : -1;
        if (sel[v])
            for (int32_t e = rp[v]; e < rp[v + 1]; ++e) z += sel[col[e]] ? 1 : 0;
    }
    int32_t* srp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)m + 1));
    int32_t* scol = (int32_t*)malloc(sizeof(int32_t) * (size_t)(z > 0 ? z : 1));
    double* sw = (double*)malloc(sizeof(double) * (size_t)(z > 0 ? z : 1));
    int32_t* glob = (int32_t*)malloc(sizeof(int32_t) * ((size_t)m + 1));
    if (!srp || !scol || !sw || !glob) {
        free(loc); free(srp); free(scol); free(sw); free(glob);
        return -1;
    }
    int64_t t = 0;
    srp[0] = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (!sel[v]) continue;
        glob[loc[v]] = v;
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e)
            if (sel[col[e]]) {
                scol[t] = loc[col[e]];
                sw[t] = w[e];
                ++t;
            }
        srp[loc[v] + 1] = (int32_t)t;
    }
    free(loc);
    *prp = srp; *pcol = scol; *pw = sw; *pglob = glob;
    return m;
}

/* Connected components: comp[v] = smallest vertex of v's component
 * (breadth-first search from each unlabelled vertex in index order).
 * Returns the number of components. */
int32_t orc_components(int32_t n, const int32_t* rp, const int32_t* col, int32_t* comp)
{
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    if (!queue) return -1;
    for (int32_t v = 0; v < n; ++v) comp[v] = -1;
    int32_t count = 0;
    for (int32_t s = 0; s < n; ++s) {
        if (comp[s] >= 0) continue;
        ++count;
        int32_t head = 0, tail = 0;
        queue[tail++] = s;
        comp[s] = s;
        while (head < tail) {
            int32_t v = queue[head++];
            for (int32_t e = rp[v]; e < rp[v + 1]; ++e)
                if (comp[col[e]] < 0) {
                    comp[col[e]] = s;
                    queue[tail++] = col[e];
                }
        }
    }
    free(queue);
    return count;
}

typedef struct {
    double key;
    int32_t v;
} orc_split_item;

static int orc_cmp_split(const void* a, const void* b)
{
    const orc_split_item* x = (const orc_split_item*)a;
    const orc_split_item* y = (const orc_split_item*)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->v > y->v) - (x->v < y->v);
}

/* Recursive spectral bisection (the graph-partitioning use of the Fiedler
 * vector named in Section 1, with the repeated coarse solves the remark on
 * the coarsest level anticipates): every part is split in two, `depth`
 * times, giving part ids 0 .. 2^depth - 1 (part p splits into 2p, 2p + 1).
 * READING (the paper gives no bisection rule): a part of fewer than 2
 * vertices is not split (its children are 2p alone); a connected part is
 * split at the median of its Fiedler vector (orc_cmg on the induced
 * subgraph, default options): its vertices ordered by (x_i, index), the
 * first floor(m/2) go to 2p; a disconnected part is ordered by (smallest
 * vertex of the component, index) instead, so whole components stay
 * together except the one the median falls in.  part[n] receives the ids;
 * returns ORC_OK or the first failing status. */
int orc_rsb(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col, const double* w,
            int32_t depth, int32_t* part)
{
    int st = orc_validate(n, nnz, rp, col, w);
    if (st != ORC_OK) return st;
    uint8_t* sel = (uint8_t*)malloc((size_t)n);
    int32_t* next = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!sel || !next) { free(sel); free(next); return ORC_E_OOM; }
    for (int32_t v = 0; v < n; ++v) part[v] = 0;
    for (int32_t d = 0; d < depth && st == ORC_OK; ++d) {
        const int32_t nparts = 1 << d;
        for (int32_t p = 0; p < nparts && st == ORC_OK; ++p) {
            for (int32_t v = 0; v < n; ++v) sel[v] = (uint8_t)(part[v] == p);
            int32_t *srp = NULL, *scol = NULL, *glob = NULL;
            double* sw = NULL;
            int32_t m = orc_induced(n, rp, col, w, sel, &srp, &scol, &sw, &glob);
            if (m < 0) { st = ORC_E_OOM; break; }
            orc_split_item* it = (orc_split_item*)malloc(sizeof(orc_split_item) * ((size_t)m + 1));
            int32_t* comp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)m + 1));
            if (!it || !comp) { st = ORC_E_OOM; }
            if (st == ORC_OK && m >= 2) {
                int32_t nc = orc_components(m, srp, scol, comp);
                if (nc == 1) {
                    orc_result* r = orc_cmg(m, srp[m], srp, scol, sw, 1e-8, 25, 128, 14120565ull, 100000);
                    if (!r) st = ORC_E_OOM;
                    else if (r->status != ORC_OK && r->status != ORC_W_MAXIT) st = r->status;
                    else
                        for (int32_t i = 0; i < m; ++i) { it[i].key = r->y[i]; it[i].v = i; }
                    orc_free(r);
                } else {
                    for (int32_t i = 0; i < m; ++i) { it[i].key = (double)comp[i]; it[i].v = i; }
                }
                if (st == ORC_OK) {
                    qsort(it, (size_t)m, sizeof(orc_split_item), orc_cmp_split);
                    for (int32_t t = 0; t < m; ++t) next[glob[it[t].v]] = 2 * p + (t < m / 2 ? 0 : 1);
                }
            } else if (st == ORC_OK) {
                for (int32_t i = 0; i < m; ++i) next[glob[i]] = 2 * p;
            }
            free(it); free(comp); free(srp); free(scol); free(sw); free(glob);
        }
        memcpy(part, next, sizeof(int32_t) * (size_t)n);
    }
    free(sel);
    free(next);
    return st;
}

/* ----------------------------------------------------- result accessors */

int32_t orc_res_status(const orc_result* r) { return r->status; }
int32_t orc_res_nlevels(const orc_result* r) { return r->nlevels; }
int32_t orc_res_level_n(const orc_result* r, int32_t j) { return r->lv[j].n; }
int64_t orc_res_level_nnz(const orc_result* r, int32_t j) { return r->lv[j].nnz; }
double orc_res_level_g(const orc_result* r, int32_t j) { return r->lv[j].g; }
int32_t orc_res_level_k(const orc_result* r, int32_t j) { return r->lv[j].k; }
double orc_res_level_margin(const orc_result* r, int32_t j) { return r->lv[j].margin; }
double orc_res_lambda(const orc_result* r) { return r->lambda; }
double orc_res_residual(const orc_result* r) { return r->residual; }
double orc_res_coarse_lambda2(const orc_result* r) { return r->coarse_lambda2; }
int32_t orc_res_coarse_mult(const orc_result* r) { return r->coarse_mult; }
int32_t orc_res_collapsed(const orc_result* r) { return r->collapsed; }

void orc_res_copy_level(const orc_result* r, int32_t j, int32_t* rp, int32_t* col, double* w,
                        int32_t* agg)
{
    const orc_level* L = &r->lv[j];
    if (rp) memcpy(rp, L->rp, sizeof(int32_t) * ((size_t)L->n + 1));
    if (col) memcpy(col, L->col, sizeof(int32_t) * (size_t)L->nnz);
    if (w) memcpy(w, L->w, sizeof(double) * (size_t)L->nnz);
    if (agg && L->agg) memcpy(agg, L->agg, sizeof(int32_t) * (size_t)L->n);
}

void orc_res_copy_y(const orc_result* r, double* y)
{
    if (r->y) memcpy(y, r->y, sizeof(double) * (size_t)r->lv[0].n);
}
