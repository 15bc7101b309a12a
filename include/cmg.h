/*
 * cmg.h - C ABI of libcmg, an MI355X (gfx950) implementation of the
 * cascadic multigrid (CMG) Fiedler-vector method of Urschel, Hu, Xu and
 * Zikatanov, "A Cascadic Multigrid Algorithm for Computing the Fiedler
 * Vector of Graph Laplacians" (arXiv 1412.0565).
 *
 * Problem (Section 2, definitions of the graph Laplacian and of the
 * algebraic connectivity): given a connected, weighted, undirected,
 * loop-free graph G with Laplacian L = D - W, approximate the eigenpair
 * (lambda_2, phi_2) of L: the second smallest eigenvalue and its
 * eigenvector, the Fiedler vector.  Method (Algorithm 1): heavy edge
 * coarsening (Algorithm 2) builds aggregates and Galerkin coarse Laplacians
 * L^{i+1} = I L^i I^T until at most `coarsest_n` vertices remain; the
 * coarsest problem is solved directly; then, level by level, the vector is
 * prolongated and refined by power iteration on gI - L with the constant
 * vector deflated (Algorithm 3).  The returned eigenvalue estimate is the
 * Rayleigh quotient r = y^T L y (Section 4), with the residual
 * ||L y - r y|| (Table 2's error measure).
 *
 * Every step after argument checking runs in HIP kernels on the GPU; the
 * host only sequences launches and reads back sizes.
 *
 * Conventions
 *  - Input graph: symmetric adjacency CSR.  Both directions stored, no
 *    diagonal, columns strictly increasing within a row, weights finite
 *    and > 0, n >= 2, nnz < 2^31, every vertex has a neighbour.  Parallel
 *    edges must be merged by the caller.  The Laplacian is implicit.
 *  - Ownership: the caller owns all arrays it passes.  cmg_setup copies the
 *    graph into memory owned by the handle and keeps no caller pointer.
 *    Output buffers (x, stats, level arrays) are caller allocated.
 *  - Memory: CMG_MEM_HOST pointers are host memory; CMG_MEM_DEVICE pointers
 *    are device memory on the current HIP device.  The library allocates
 *    its own device memory through `allocator` (hipMalloc if NULL) and
 *    issues all work on `stream` (the null stream if NULL).
 *  - Errors: only status codes cross the ABI.  On failure of cmg_setup,
 *    *out is set to NULL and everything allocated is released.
 *    CMG_W_MAXIT is a warning: the result is still written.
 *  - Synchronisation: every call returns after its work has completed,
 *    also with device arrays (the step counts, statistics and the barrier
 *    fallback decision are read on the host before returning).  To queue
 *    several solves, pass them to cmg_fiedler_batch, which shares launches.
 *  - Threads: one handle is used by one thread at a time; distinct handles
 *    are independent.  Calls on one device share no mutable state except
 *    the allocator the caller supplies.
 */
#ifndef CMG_H
#define CMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cmg_ctx* cmg_handle;

typedef enum {
    CMG_OK = 0,
    CMG_E_ARG = 1,      /* bad argument (NULL pointer, n < 2, sizes out of range, bad option) */
    CMG_E_GRAPH = 2,    /* bad index, unsorted/duplicate column, self-loop, w <= 0 or non-finite,
                           asymmetric (only detected with validate_full) */
    CMG_E_ISOLATED = 3, /* a vertex without neighbours: in the input, or on a level HEC
                           coarsens (a component of a disconnected graph that became one
                           aggregate; Algorithm 2 needs a heaviest neighbour) */
    CMG_E_OOM = 4,      /* an allocation failed */
    CMG_E_DEVICE = 5,   /* a HIP runtime error or a device-side failure */
    CMG_W_MAXIT = 6     /* warning: a level hit max_iters_per_level; result still valid */
} cmg_status;

typedef enum {
    CMG_FP64 = 0,  /* every level in FP64 */
    CMG_MIXED = 1  /* large levels: FP32 values and vectors, FP64 arithmetic and reductions */
} cmg_precision;

typedef enum { CMG_MEM_HOST = 0, CMG_MEM_DEVICE = 1 } cmg_memspace;

typedef enum { CMG_VAL_F64 = 0, CMG_VAL_F32 = 1 } cmg_valtype;

/* Device-memory allocator.  alloc returns NULL on failure; free accepts
 * what alloc returned.  `stream` is the hipStream_t the library works on. */
typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* user);
    void (*free)(void* p, void* stream, void* user);
    void* user;
} cmg_allocator;

typedef struct {
    uint32_t struct_size;        /* sizeof(cmg_options) */
    double tol;                  /* PI stops once (u^k, u^{k-1}) >= 1 - tol (Section 4: 1e-8) */
    int32_t coarsest_n;          /* coarsen while n > coarsest_n (Algorithm 1: 25) */
    int32_t dense_max;           /* coarsest level solved densely if n <= dense_max (128) */
    uint64_t seed;               /* seeds the HEC visit order (replaces randperm) */
    int32_t precision;           /* cmg_precision */
    int32_t fp64_final_sweeps;   /* MIXED only, 0 or 1 (default 1): the last level-0 PI step is
                                    recomputed in FP64 from the FP32 iterate before it, so the
                                    step count equals the FP64 path */
    int32_t max_iters_per_level; /* PI cap per level (100000), then CMG_W_MAXIT */
    int32_t validate_full;       /* 1: also check symmetry of the input (O(nnz log deg)) */
    void* stream;                /* hipStream_t; NULL = null stream */
    const cmg_allocator* allocator; /* NULL = hipMalloc/hipFree */
    int32_t block_rows;          /* > 0: levels with n <= block_rows are refined inside one
                                    workgroup; 0 = library default (n <= 4096 and the
                                    level's CSR fits LDS or has <= 8192 entries) */
    int64_t mixed_min_nnz;       /* MIXED: levels with nnz >= this run FP32 (0 = default) */
    int32_t spmv_variant;        /* 0 = auto, 1 = rows per lane group, 2 = merge path */
    int32_t autotune;            /* 1: cmg_setup times candidate lanes-per-row and workgroup
                                    counts of every grid-refined level with a few power-
                                    iteration steps of the real kernel and keeps the fastest;
                                    choices are cached per process by level shape, so results
                                    are reproducible within a process but may differ (within
                                    rounding) between processes.  0 (default): fixed rules. */
    int32_t block_regs;          /* levels refined inside one workgroup: 0 (default) holds each
                                    level's rows in registers for all its PI steps where a
                                    layout fits (rows of at most 128 entries, those beyond
                                    the layout's slots in an LDS list); -1 always reads the
                                    CSR arrays.  Both give the same lambda to rounding. */
    int32_t grid_stage;          /* FP64 levels refined by the whole grid with lanes per row:
                                    1 (default) copies each workgroup's rows, columns and
                                    weights to LDS once per level when they fit (at most 1024
                                    rows and 3840 entries) and runs the PI steps from there;
                                    0 always reads them from global memory.  Results are
                                    bitwise equal. */
    int32_t step_mode;           /* grid levels traversed by rows: 0 (default) refines the levels
                                    below the finest whose PI step streams >= 16 MB (counted in
                                    FP64) with one launch
                                    per step (no grid barrier), the others with one persistent
                                    launch; 1 uses one launch per step on every such level; -1 on
                                    none.  The same arithmetic in the same order either way:
                                    results are equal to rounding of the sums' tree. */
    int32_t fixed_k0;            /* > 0: fixed smoothing schedule of the geometric cascadic method
                                    (Algorithm 4; Section 3, main theorem): level j runs exactly
                                    k_j = ceil(fixed_k0 * fixed_beta^j) power-iteration steps
                                    (capped at max_iters_per_level) and no stopping test; the
                                    launch sequence of a solve is then fixed.  0 (default): the
                                    stopping test of Algorithm 3 with `tol`. */
    double fixed_beta;           /* beta >= 1 of the fixed schedule (default 2) */
    int32_t graph;               /* 1: the first cmg_fiedler on the handle captures its launch
                                    sequence in a HIP graph and later solves replay it (only
                                    when the sequence is fixed: a fixed schedule, or no level
                                    refined one launch per step); per-level device times
                                    (pi_ms) are then not measured.  0 (default): launches. */
    int32_t coarsen;             /* 0 (default): heavy edge coarsening (Algorithm 2).  1: heavy
                                    edge matching, the coarsening Section 2.1 contrasts HEC with
                                    (each unmatched vertex, in the same visit order, is matched to
                                    its heaviest unmatched neighbour or stays alone; aggregates of
                                    one or two vertices, so n_{j+1} >= n_j / 2), for comparison. */
    int32_t galerkin;            /* Galerkin product of the large levels: 0 (default) forms each
                                    coarse row from its aggregate's member rows where no aggregate
                                    has more than 1024 entries (in registers, or by a wavefront's
                                    sort in LDS for rows with many distinct columns), else sorts
                                    (key, weight) pairs over the level; 1 always sorts; 2 forms
                                    every row by the wavefront's sort (to test that former).  All
                                    sum in fine CSR order: coarse graphs are bitwise equal. */
    int32_t test_abort_level;    /* tests of the barrier fallback only (default -1): the first
                                    attempt of every solve raises the grid barrier's abort flag
                                    before refining this level, as if its bounded wait had been
                                    given up; every kernel then exits and the solve is re-run
                                    with the persistent levels one launch per step. */
    int32_t weight_storage;      /* 0 (default): the grid and step kernels read no weights on a
                                    level whose weights are all 1; an 8-bit (16-bit) copy when
                                    every input weight is an integer and the level's largest is
                                    at most 255 (65535); else on an FP64 level an FP32 copy when
                                    its weights are all exact in FP32 (the same values: results
                                    are bitwise those of FP64 storage); 1: always the iterates'
                                    precision. */
} cmg_options;

/* Per-level information (available after cmg_setup; PI fields after
 * cmg_fiedler). */
typedef struct {
    int32_t n;           /* vertices */
    int64_t nnz;         /* stored directed off-diagonal entries */
    double g;            /* Gershgorin shift g = max_i sum_j |l_ij| (Algorithm 3) */
    double wmax;         /* largest edge weight */
    int32_t k;           /* PI steps executed (-1: dense coarsest solve, 0: not run) */
    double margin;       /* (u^k,u^{k-1}) - (1 - tol) at exit */
    int32_t fp32;        /* 1 if this level ran FP32 storage */
    int32_t in_block;    /* 1 if refined inside one workgroup, 0 if by the whole grid */
    int32_t variant;     /* SpMV variant used (1 rows, 2 merge path) */
    int32_t lanes;       /* lanes per row (variant 1) */
    int32_t grid;        /* workgroups of the grid kernel */
    double pi_ms;        /* device time of this level's refinement launch (grid levels) */
    double bytes_per_iter; /* algorithmic bytes of one PI step: 4(n+1)+nnz(4+s_v)+2 s_x n */
    int32_t block_waves;   /* in_block: wavefronts running the PI steps (0: all) */
    int32_t block_regs;    /* in_block: rows per lane group held in registers (0: CSR reads) */
    int32_t step;          /* 1 if refined with one launch per PI step (no grid barrier) */
    int32_t weights;       /* edge weights as the level's PI steps read them: 0 FP64, 1 FP32
                              (mixed-precision level, or an exact FP32 copy beside FP64
                              iterates), 2 none (every weight is 1), 3 an 8-bit copy (every
                              weight an integer in 1..255), 4 a 16-bit copy (every weight an
                              integer in 1..65535) */
    int32_t block_slots;   /* in_block with register rows: entry slots per lane and row; the
                              entries of rows longer than lanes x block_slots (at most twice
                              that) are read from a list in LDS */
} cmg_level_stats;

typedef struct {
    uint32_t struct_size;
    int32_t nlevels;        /* J + 1 */
    int32_t collapsed;      /* 1 if coarsening stopped because HEC gave < 2 aggregates */
    int32_t hec_rounds;     /* total greedy rounds over all levels */
    double lambda;          /* r = y^T L y */
    double residual;        /* ||L y - r y|| */
    double coarse_lambda2;  /* lambda_2 of the coarsest level (dense solve) */
    int32_t coarse_mult;    /* size of the coarsest lambda_2 cluster */
    double setup_ms;        /* wall time of cmg_setup */
    double fiedler_ms;      /* wall time of the last cmg_fiedler */
    double finest_pi_ms;    /* device time of the level-0 refinement launch */
    int32_t finest_k;       /* PI steps on level 0 */
    double finest_bytes;    /* algorithmic bytes of level-0 PI: k_0 * bytes_per_iter(0) */
    int32_t status;         /* status of the last call */
    int32_t fallback;       /* 1 if a grid barrier's wait was given up and the refinement was
                               re-run with the persistent levels one launch per step */
} cmg_stats;

/* Fill `o` with defaults: tol 1e-8, coarsest_n 25, dense_max 128,
 * seed 14120565, FP64, 1 final sweep, 100000 iterations, no full
 * validation, null stream, hipMalloc allocator, library tuning. */
void cmg_options_default(cmg_options* o);

/* Setup phase (Algorithm 1, Step 1): validate and copy the graph, then
 * coarsen with HEC (Algorithm 2) and form Galerkin coarse graphs until
 * n <= coarsest_n or HEC collapses to one aggregate.
 *   n, nnz         vertex count and stored entries (row_ptr[n] == nnz)
 *   row_ptr[n+1]   int32 offsets; col[nnz] int32 neighbours
 *   w[nnz]         weights, double (CMG_VAL_F64) or float (CMG_VAL_F32)
 *   where          memory space of row_ptr/col/w
 *   opt            options (NULL = defaults)
 *   out            receives the handle (NULL on failure) */
cmg_status cmg_setup(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                     const void* w, cmg_valtype wtype, cmg_memspace where,
                     const cmg_options* opt, cmg_handle* out);

/* Coarsest solve and cascadic refinement (Algorithm 1, Steps 2-3).
 *   lambda   receives r = y^T L y (host pointer, may be NULL)
 *   x        receives the unit-norm Fiedler approximation (n doubles, in
 *            memory space `where`; may be NULL)
 *   stats    optional (host pointer)
 * Returns CMG_OK or CMG_W_MAXIT on success.
 * Large levels run as persistent launches whose workgroups meet at grid
 * barriers, so all of them must be resident together (the library sizes
 * each launch to the co-resident count it measured on the idle device).  Kernels that other
 * streams keep launching on the same device can hold compute units long
 * enough that a barrier's bounded wait (2 s) ends: every kernel of the
 * solve then exits and the refinement is re-run with the persistent
 * levels that traverse rows one launch per step, which needs no waits
 * between workgroups (stats->fallback = 1; the result matches the
 * oracle to the same tolerances).  Levels on the merge path and the
 * finishing pass have no such form: if their wait is given up, the call
 * returns CMG_E_DEVICE (cmg_last_error() names the level) and the handle
 * stays usable.  Callers that overlap work should keep other kernels off
 * the device while a solve runs, e.g. by issuing both on one stream. */
cmg_status cmg_fiedler(cmg_handle h, double* lambda, void* x, cmg_memspace where,
                       cmg_stats* stats);

/* Refine several hierarchies together: the coarse levels of all handles
 * run in one launch (one workgroup per graph), larger levels in packed
 * grid launches.  All handles must share one device and stream.
 * lambdas[count], xs[count] (each n_i doubles in `where`), stats[count]
 * are optional.  Results equal those of cmg_fiedler on each handle. */
cmg_status cmg_fiedler_batch(cmg_handle* hs, int32_t count, double* lambdas, void** xs,
                             cmg_memspace where, cmg_stats* stats);

/* Several eigenpairs at once (the Remark after Algorithm 4): the p
 * eigenvectors of the coarsest level above the constant one (the dense
 * solve's lowest eigenspaces, whole clusters, onto which p hashed-uniform
 * starts are projected and orthonormalised) are prolongated level by level;
 * on each level every vector is smoothed with B_g = gI - L and the block
 * is orthonormalised after each step (orthogonal iteration), until every
 * column passes Algorithm 3's test (or the fixed schedule's count, with
 * fixed_k0 > 0).  The hierarchy is the handle's (cmg_setup).
 *   p            1..4, and below the coarsest level's vertex count, which
 *                must be solved densely (n_J <= dense_max); else CMG_E_ARG
 *   lambdas[p]   edge-form Rayleigh quotients of the output columns (host)
 *   X            n x p doubles, column-major (column c at X + c n), unit
 *                columns orthogonal to each other and to the constant
 *                vector, in memory space `where` (may be NULL)
 *   residuals[p] ||L x_c - lambda_c x_c|| (host, may be NULL)
 *   level_steps  steps per level, J + 1 entries (-1 on the coarsest; host,
 *                may be NULL)
 * FP64 throughout.  Returns CMG_OK, CMG_W_MAXIT (a level hit the cap), or
 * CMG_E_DEVICE if the block lost rank. */
cmg_status cmg_fiedler_block(cmg_handle h, int32_t p, double* lambdas, void* X, cmg_memspace where,
                             double* residuals, int32_t* level_steps);

/* Recursive spectral bisection (the graph-partitioning use of the Fiedler
 * vector, Section 1; repeated solves as the remark on the coarsest level
 * anticipates): every part is split in two, `depth` times, giving part ids
 * 0 .. 2^depth - 1 (part p splits into 2p and 2p + 1).  Per depth all
 * parts are handled at once: their induced subgraphs are compacted on the
 * device, connected components labelled, and the connected parts of two
 * vertices or more solved in one cmg_fiedler_batch (options `opt` apply to
 * every solve); a connected part is split at the median of its Fiedler
 * vector (ordered by (x_i, index); the first floor(m/2) go to 2p), a
 * disconnected part by (smallest vertex of the component, index), a part
 * of one vertex is not split.
 *   n, nnz, row_ptr, col, w, wtype, where, opt   as cmg_setup
 *   depth    0..16
 *   part[n]  receives the part ids (int32, in `where`)
 *   cut      receives the total weight of edges between parts (host, may
 *            be NULL)
 * Returns CMG_OK or the first failing status. */
cmg_status cmg_bisect(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, const void* w,
                      cmg_valtype wtype, cmg_memspace where, const cmg_options* opt, int32_t depth,
                      int32_t* part, double* cut);

/* Copy per-level information into out[0..cap-1]; *nlevels gets J+1. */
cmg_status cmg_level_info(cmg_handle h, cmg_level_stats* out, int32_t cap, int32_t* nlevels);

/* Copy level `level` of the hierarchy to host arrays (each may be NULL):
 * row_ptr[n+1], col[nnz], w[nnz] (double), agg[n] (aggregate of each
 * vertex in level+1; not available on the coarsest level). */
cmg_status cmg_level_copy(cmg_handle h, int32_t level, int32_t* row_ptr, int32_t* col, double* w,
                          int32_t* agg);

/* Make later calls on `h` issue their work on `stream` (a hipStream_t;
 * NULL = null stream), e.g. to solve on another stream than the one the
 * hierarchy was built on.  The caller orders any pending work itself. */
cmg_status cmg_set_stream(cmg_handle h, void* stream);

/* Device bytes held by the handle (hierarchy plus refinement buffers). */
cmg_status cmg_footprint(cmg_handle h, size_t* bytes);

/* Release everything owned by the handle.  NULL is a no-op. */
void cmg_free(cmg_handle h);

/* Static string for a status code. */
const char* cmg_status_string(cmg_status s);

/* Description of the last failure reported by a call on this thread
 * (which step failed and the HIP error, or a grid-barrier timeout); ""
 * if the last call succeeded.  Valid until the next call. */
const char* cmg_last_error(void);

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc; code under HIP graph capture is not
 * supported, since the call synchronises): cmg_setup, cmg_fiedler and
 * cmg_free of one graph in a single call that allocates nothing.  Every
 * device buffer is carved from a static scratch array of 64 MiB that each
 * device the library runs on holds until the process ends; the call makes
 * no hipMalloc, hipFree, host-pinned, event or stream allocation (the
 * allocator in `opt` is ignored).
 *   Arguments as cmg_setup (n, nnz, row_ptr, col, w, wtype, where, opt)
 *   followed by cmg_fiedler's outputs (lambda, x of n doubles in `where`,
 *   stats).  The solve is the same as cmg_setup + cmg_fiedler with the same
 *   options except that no level is refined one launch per step (step_mode
 *   -1), autotune and graph are off, and per-level device times are not
 *   measured.
 *   Size limit: 64 nnz + 128 n + 4 MiB <= 64 MiB - 4 KiB (about 100k
 *   vertices with 600k entries); a larger graph returns CMG_E_ARG with the
 *   bound in cmg_last_error().  Running out of scratch returns CMG_E_OOM.
 *   Calls on one device share its scratch: the library serialises the
 *   calls of one process, and a caller must not read the scratch's
 *   contents from one call in another (each call initialises what it
 *   uses).  Work another thread queues on the same device while a call
 *   runs can race with it through the grid barriers (see cmg_fiedler). */
cmg_status cmg_fiedler_noalloc(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                               const void* w, cmg_valtype wtype, cmg_memspace where,
                               const cmg_options* opt, double* lambda, void* x, cmg_stats* stats);

/* Diagnostics: evaluate on the GPU the counter-based hash the library uses
 * for HEC priorities, key(v) = mix64(seed ^ (level << 40) ^ v) with mix64
 * the SplitMix64 output function, for v = 0..count-1 into host out[].
 * With level = -1 it instead writes the SplitMix64 sequence seeded with
 * `seed` (state += 0x9E3779B97F4A7C15, output mix64(state)). */
cmg_status cmg_hash_probe(uint64_t seed, int32_t level, int32_t count, uint64_t* out);

#ifdef __cplusplus
}
#endif

#endif /* CMG_H */
