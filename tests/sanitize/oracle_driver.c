/* Runs the C oracle's entry points on small graphs built here, for an
 * AddressSanitizer / UndefinedBehaviorSanitizer build (tests/test_sanitize.py).
 * Exit status 0 if every call returns a status it should. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_result orc_result;
typedef struct orc_block_result orc_block_result;
orc_result* orc_cmg_ex(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col, const double* w,
                       double tol, int32_t coarsest_n, int32_t dense_max, uint64_t seed, int32_t max_iters,
                       int32_t fixed_k0, double fixed_beta, int32_t coarsen);
int32_t orc_res_status(const orc_result* r);
void orc_free(orc_result* r);
orc_block_result* orc_cmg_block(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col, const double* w,
                                double tol, int32_t coarsest_n, int32_t dense_max, uint64_t seed,
                                int32_t max_iters, int32_t fixed_k0, double fixed_beta, int32_t p);
int32_t orc_block_status(const orc_block_result* b);
void orc_block_free(orc_block_result* b);
int orc_rsb(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col, const double* w, int32_t depth,
            int32_t* part);

typedef struct {
    int32_t n;
    int64_t nnz;
    int32_t* rp;
    int32_t* col;
    double* w;
} csr;

/* symmetric CSR from an adjacency matrix given as a predicate */
static csr build(int32_t n, int (*adj)(int32_t, int32_t, int32_t), double (*wt)(int32_t, int32_t)) {
    csr g;
    g.n = n;
    g.rp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    g.nnz = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j) g.nnz += (i != j && adj(n, i, j)) ? 1 : 0;
    g.col = (int32_t*)malloc(sizeof(int32_t) * (size_t)g.nnz);
    g.w = (double*)malloc(sizeof(double) * (size_t)g.nnz);
    int64_t t = 0;
    for (int32_t i = 0; i < n; ++i) {
        g.rp[i] = (int32_t)t;
        for (int32_t j = 0; j < n; ++j)
            if (i != j && adj(n, i, j)) {
                g.col[t] = j;
                g.w[t] = wt(i, j);
                ++t;
            }
    }
    g.rp[n] = (int32_t)t;
    return g;
}

static int side;
static int path(int32_t n, int32_t i, int32_t j) { (void)n; return abs(i - j) == 1; }
static int cycle(int32_t n, int32_t i, int32_t j) { return abs(i - j) == 1 || abs(i - j) == n - 1; }
static int complete(int32_t n, int32_t i, int32_t j) { (void)n; (void)i; (void)j; return 1; }
static int star(int32_t n, int32_t i, int32_t j) { (void)n; return (i == 0) != (j == 0); }
static int grid(int32_t n, int32_t i, int32_t j) {
    (void)n;
    int ri = i / side, ci = i % side, rj = j / side, cj = j % side;
    return abs(ri - rj) + abs(ci - cj) == 1;
}
static int sparse(int32_t n, int32_t i, int32_t j) {  /* a ring plus hashed chords */
    if (abs(i - j) == 1 || abs(i - j) == n - 1) return 1;
    uint32_t a = (uint32_t)(i < j ? i : j), b = (uint32_t)(i < j ? j : i);
    uint32_t h = (a * 2654435761u) ^ (b * 40503u + 17u);
    return (h % 97u) == 0u;
}
static double unit(int32_t i, int32_t j) { (void)i; (void)j; return 1.0; }
static double varied(int32_t i, int32_t j) { return 1.0 + (double)((i + j) % 5) * 0.25; }

int main(void) {
    int bad = 0;
    side = 12;
    csr gs[] = {build(40, path, unit), build(33, cycle, unit), build(30, complete, unit), build(60, star, unit),
                build(144, grid, varied), build(300, sparse, varied)};
    const int ng = (int)(sizeof(gs) / sizeof(gs[0]));
    for (int k = 0; k < ng; ++k) {
        csr* g = &gs[k];
        for (int mode = 0; mode < 3; ++mode) {
            orc_result* r = orc_cmg_ex(g->n, g->nnz, g->rp, g->col, g->w, 1e-8, 25, 128, 14120565ull, 100000,
                                       mode == 1 ? 3 : 0, 1.6, mode == 2 ? 1 : 0);
            const int st = r ? orc_res_status(r) : -1;
            if (st != 0 && st != 6) { printf("cmg graph %d mode %d: status %d\n", k, mode, st); bad = 1; }
            if (getenv("ORC_VERBOSE")) printf("cmg %d mode %d st %d\n", k, mode, st);
            orc_free(r);
        }
        orc_block_result* b = orc_cmg_block(g->n, g->nnz, g->rp, g->col, g->w, 1e-8, 25, 128, 14120565ull, 100000,
                                            0, 2.0, 2);
        const int bs = b ? orc_block_status(b) : -1;
        if (bs != 0 && bs != 1 && bs != 6) { printf("block graph %d: status %d\n", k, bs); bad = 1; }
        orc_block_free(b);
        int32_t* part = (int32_t*)malloc(sizeof(int32_t) * (size_t)g->n);
        const int rs = orc_rsb(g->n, g->nnz, g->rp, g->col, g->w, 3, part);
        if (rs != 0) { printf("rsb graph %d: status %d\n", k, rs); bad = 1; }
        free(part);
        free(g->rp); free(g->col); free(g->w);
    }
    /* rejected inputs: an isolated vertex, an unsorted row, a non-positive weight, n = 1 */
    {
        int32_t rp_iso[4] = {0, 1, 2, 2}, col_iso[2] = {1, 0};
        double w2[2] = {1.0, 1.0};
        orc_result* r = orc_cmg_ex(3, 2, rp_iso, col_iso, w2, 1e-8, 25, 128, 1ull, 1000, 0, 2.0, 0);
        if (!r || orc_res_status(r) != 3) { printf("isolated vertex not rejected\n"); bad = 1; }
        orc_free(r);
        int32_t rp_uns[4] = {0, 2, 3, 4}, col_uns[4] = {2, 1, 0, 0};
        double w4[4] = {1.0, 1.0, 1.0, 1.0};
        r = orc_cmg_ex(3, 4, rp_uns, col_uns, w4, 1e-8, 25, 128, 1ull, 1000, 0, 2.0, 0);
        if (!r || orc_res_status(r) != 2) { printf("unsorted row not rejected\n"); bad = 1; }
        orc_free(r);
        int32_t rp_p[3] = {0, 1, 2}, col_p[2] = {1, 0};
        double wneg[2] = {-1.0, -1.0};
        r = orc_cmg_ex(2, 2, rp_p, col_p, wneg, 1e-8, 25, 128, 1ull, 1000, 0, 2.0, 0);
        if (!r || orc_res_status(r) != 2) { printf("negative weight not rejected\n"); bad = 1; }
        orc_free(r);
        int32_t rp_1[2] = {0, 0};
        r = orc_cmg_ex(1, 0, rp_1, col_p, w2, 1e-8, 25, 128, 1ull, 1000, 0, 2.0, 0);
        if (!r || orc_res_status(r) != 1) { printf("n = 1 not rejected\n"); bad = 1; }
        orc_free(r);
    }
    printf(bad ? "FAIL\n" : "OK\n");
    return bad;
}
