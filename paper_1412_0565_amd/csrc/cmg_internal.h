// Host-side declarations shared by the libcmg translation units: kernel
// launchers implemented next to their kernels, called by the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cmg_dev.h"

namespace cmg {

// validation flag bits
constexpr unsigned kBadGraph = 1u;
constexpr unsigned kIsolated = 2u;
constexpr unsigned kAsym = 4u;
// Not an error: some weight is not an integer below 2^20.  Without it every
// sum of weights of the hierarchy is an integer below 2^51, exact in any order.
constexpr unsigned kWideWeight = 8u;
// Not an error: some weight is not 1.
constexpr unsigned kNonUnit = 16u;

// ---- coarsen_small.hip: the setup of small levels in one workgroup
constexpr int kChainThreads = 1024;
constexpr int kChainMaxN = 8192;         // levels with at most this many vertices
constexpr int64_t kChainMaxNnz = 262144; // ... and at most this many entries
constexpr int kChainMaxRow = 1024;       // longest coarse row (member entries) one thread forms

// One level visited by the chain: its row information, and where its
// arrays were written (offsets into the arenas; -1 for the first level,
// whose arrays are the input, and agg_off = -1 if it was not coarsened).
struct ChainHdr {
    int32_t n;
    int32_t rounds;   // HEC rounds of this level's coarsening
    int64_t nnz;
    double g, wmax, w32err, maxlen;
    int64_t rp_off, cw_off, agg_off;
};

struct ChainJob {
    int32_t n0;
    int32_t level0;
    int64_t nnz0;
    const int32_t* rp0;
    const int32_t* col0;
    const double* w0;
    uint64_t seed;
    int32_t coarsest_n;
    int32_t max_levels;  // levels that may be visited, the first included
    // scratch (sized for level 0 of the graph)
    int32_t *h, *pairseed, *rootseed, *rank, *members, *astart, *soff, *rcount, *mb;
    int32_t* bcol;  // aggregate of each entry's column (nnz0 ints)
    unsigned long long* slot;
    uint8_t *live, *state;
    double* mw;
    // arenas for the levels produced: agg and row pointers (ai32), columns
    // and weights (acol, aw)
    int32_t* ai32;
    int64_t ai32_cap;
    int32_t* acol;
    double* aw;
    int64_t acw_cap;
    ChainHdr* hdr;  // [max_levels]
    int32_t* out;   // [0] levels visited, [1] collapsed, [2] stop reason
                    // (1 size, 2 collapse, 3 arena, 4 long coarse row, 5 level cap)
};
hipError_t launch_coarsen_chain(const ChainJob& job, hipStream_t s);

// ---- setup.hip
// flags[0]: kBadGraph | kIsolated | kAsym | kWideWeight | kNonUnit; flags[1]: longest
// row if it exceeds 64 entries, else left as it was (both zeroed by the caller)
hipError_t launch_validate(int n, int64_t nnz, const int32_t* rp, const int32_t* col, const void* w,
                           int wf32, int full, unsigned* flags, hipStream_t s);
hipError_t launch_convert_w(int64_t nnz, const void* w, int wf32, double* w64, hipStream_t s);
hipError_t launch_to_f32(int64_t nnz, const double* w64, float* w32, hipStream_t s);
// weights known to be integers in 1..255 (1..65535) to an 8-bit (16-bit) copy
hipError_t launch_to_u8(int64_t nnz, const double* w64, uint8_t* w8, hipStream_t s);
hipError_t launch_to_u16(int64_t nnz, const double* w64, uint16_t* w16, hipStream_t s);
// h[v] = heaviest neighbour (lowest index on ties); out[0] = bits of the
// Gershgorin shift 2 max_v d_v, out[1] = bits of the largest weight,
// out[2] = bits of the largest FP32 rounding error of a weight, out[3] =
// bits of the longest row length (as a double).
// bmax: scratch of 4 * kRowinfoMaxBlocks doubles.
constexpr int kRowinfoMaxBlocks = 1024;
// (unit: every weight is 1; w is then not read)
// *iso is raised if some vertex of the level has no neighbour (it is then
// its own h)
hipError_t launch_rowinfo(int n, int lanes, const int32_t* rp, const int32_t* col, const double* w, int unit,
                          int32_t* h, double* bmax, unsigned long long* out, unsigned* iso, hipStream_t s);
// flags: two words; after round r, flags[r & 1] is 1 if a candidate edge
// survived it, else 0 (a round after one that left none does nothing)
hipError_t launch_hec_init(int n, const int32_t* h, uint64_t seed, int level, uint8_t* live,
                           uint8_t* state, int32_t* pairseed, unsigned long long* slot,
                           unsigned long long* flags, hipStream_t s);
// greedy round `round` (0, 1, ... in launch order)
hipError_t launch_hec_round(int n, const int32_t* h, uint64_t seed, int level, uint8_t* live,
                            uint8_t* state, int32_t* pairseed, unsigned long long* slot,
                            unsigned long long* flags, int round, hipStream_t s);
hipError_t launch_hec_attach(int n, const int32_t* h, const uint8_t* state, const int32_t* pairseed,
                             int32_t* rootseed, int32_t* flags, hipStream_t s);
hipError_t launch_hec_label(int n, const int32_t* rootseed, const int32_t* rank, int32_t* agg,
                            hipStream_t s);
// Galerkin product by aggregates (levels whose aggregates have at most
// kGalWaveCap entries in their member rows): members sorted by aggregate
// (ascending vertex inside one), their row lengths and each aggregate's
// first member (mstart[nc] = n); moff = exclusive scan of mdeg; *emax
// (zeroed by the caller) the most entries of one aggregate, for the
// aggregate count *ncp (at most ncmax) read on the device; gather writes each
// coarse row at moff[mstart[a]] of tcol/tw and its length; compact moves the
// rows to the coarse CSR given its row pointers crp[nc + 1].
constexpr int kGalWaveCap = 1024;       // entries per aggregate; above this the level sorts
constexpr int kGalLaneMinRows = 65536;  // fewer coarse rows: all formed by wavefronts
hipError_t launch_gal_members(int n, const int32_t* agg, const int32_t* rp, unsigned long long* k0,
                              unsigned long long* k1, int aggbits, int32_t* sort_counts, long long* sort_scan,
                              int32_t* members, int32_t* mdeg, int32_t* mstart, hipStream_t s);
// the same lists in any order within an aggregate (integer weights below
// 2^20 only); cnt: ncmax + 1 ints of scratch; mstart: ncmax + 1 entries
hipError_t launch_gal_members_count(int n, int ncmax, const int32_t* agg, const int32_t* rp, int32_t* cnt,
                                    long long* scan_tmp, long long* total, int32_t* members, int32_t* mdeg,
                                    int32_t* mstart, hipStream_t s);
hipError_t launch_gal_agg_len(int ncmax, const long long* ncp, int n, int64_t nnz, const int32_t* mstart,
                              const int32_t* moff, unsigned long long* emax, hipStream_t s);
// (slots: 16 or 32 distinct columns a lane keeps in registers, 0 for none;
// int32sum: all weights are integers summing below 2^32, kept as 32-bit
// integer sums; big: nc ints listing the aggregates with more, nbig their count)
hipError_t launch_gal_gather(int nc, int n, int64_t nnz, int slots, int unit, int int32sum, const int32_t* members,
                             const int32_t* mstart, const int32_t* moff, const int32_t* rp, const int32_t* col,
                             const double* w, const int32_t* agg, int32_t* tcol, double* tw, int32_t* rowlen,
                             int32_t* big, unsigned* nbig, hipStream_t s);
// Up to kPackWordsMax device words (4 or 8 bytes each) gathered into
// dst[0 ..) as 64-bit values by one launch, for one host read.
constexpr int kPackWordsMax = 8;
struct PackWords {
    const void* src[kPackWordsMax];
    int32_t bytes[kPackWordsMax];
    int32_t n;
};
hipError_t launch_pack_words(const PackWords& p, unsigned long long* dst, hipStream_t s);
hipError_t launch_gal_compact(int nc, const int32_t* mstart, const int32_t* moff, const int32_t* crp,
                              const int32_t* tcol, const double* tw, const int32_t* big, const unsigned* nbig,
                              int32_t* col_out, double* w_out, hipStream_t s);
// One round of heavy edge matching (two passes; opener[v] = -1 while v is
// unmatched, else the vertex that opened its aggregate); alive[round] is
// raised if any vertex was unmatched when the round began.
hipError_t launch_hem_round(int n, const int32_t* rp, const int32_t* col, const double* w, uint64_t seed, int level,
                            int32_t* opener, uint8_t* live, unsigned long long* mkey, unsigned* alive, int round,
                            hipStream_t s);
// flags[v] = 1 where v opened its aggregate
hipError_t launch_hem_flags(int n, const int32_t* opener, int32_t* flags, hipStream_t s);
constexpr int kHemMaxRounds = 4096;
// exclusive scan of int32 -> int32; *total (device int64) gets the sum.
// tmp must hold scan_tmp_elems(m) int64 values.
int64_t scan_tmp_elems(int64_t m);
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t m, long long* tmp, long long* total,
                       hipStream_t s);
// Galerkin keys: a * mult + b (mult >= coarse vertex count), or `sent`
// (all ones in the sorted bits) for entries inside an aggregate, which
// sort last.  With vals == nullptr the keys are packed as
// key << pshift | fine position.
constexpr unsigned long long kGalSentinel = 0xFFFFFFFFFFFFFFFFull;
hipError_t launch_gal_emit(int n, int lanes, const int32_t* rp, const int32_t* col, const double* w,
                           const int32_t* agg, int64_t mult, int pshift, unsigned long long sent,
                           unsigned long long* keys, double* vals, hipStream_t s);
// The same keys, entries spread evenly over the lanes (levels with very long rows).
hipError_t launch_gal_emit_entries(int n, int64_t nnz, const int32_t* rp, const int32_t* col,
                                   const double* w, const int32_t* agg, int64_t mult, int pshift,
                                   unsigned long long sent, unsigned long long* keys, double* vals,
                                   hipStream_t s);
// *out = number of keys[0..m) below `sent` (keys sorted ascending)
hipError_t launch_count_below(const unsigned long long* keys, int64_t m, unsigned long long sent,
                              unsigned long long* out, hipStream_t s);
// stable LSD radix sort of keys (with values unless v0 == nullptr) on
// bits [shift0, shift0 + bits); the result ends in (k0, v0) or (k1, v1):
// returns which through *in_second.
int64_t sort_tmp_elems(int64_t m);
hipError_t launch_sort(unsigned long long* k0, double* v0, unsigned long long* k1, double* v1,
                       int64_t m, int shift0, int bits, int32_t* tmp_counts, long long* tmp_scan,
                       int* in_second, hipStream_t s);
// heads[t] = 1 where a run of equal keys starts among the first *nvalid
// keys (read on the device), 0 elsewhere in [0, m)
hipError_t launch_gal_heads(int64_t m, const unsigned long long* nvalid, const unsigned long long* keys,
                            int kshift, int32_t* heads, hipStream_t s);
// part: nullptr sums every run in key order (fine CSR order, bit-exact for
// any weights); else a scratch of gal_part_elems(m) doubles, and runs that
// cross workgroups are summed in pieces (exact only for integer weights
// whose sums stay below 2^53).
hipError_t launch_gal_reduce(int64_t m, const unsigned long long* keys, const double* vals,
                             const double* wfine, int kshift, const int32_t* heads, const int32_t* idx,
                             int64_t mult, int nc, int64_t zc, int32_t* rp_out, int32_t* col_out,
                             double* w_out, double* part, hipStream_t s);
int64_t gal_part_elems(int64_t m);
hipError_t launch_partition(int n, int64_t nnz, const int32_t* rp, int nb, int32_t* part,
                            hipStream_t s);
// Rows with more than lmin entries: out[0] = count, out[1..] = the rows in
// ascending order (out holds 1 + nnz / (lmin + 1) ints; flags, pos: n ints;
// scan_tmp: scan_tmp_elems(n) + 4; total: one long long).
hipError_t launch_long_rows(int n, const int32_t* rp, int lmin, int32_t* flags, int32_t* pos, long long* scan_tmp,
                            long long* total, int32_t* out, hipStream_t s);
hipError_t launch_hash_probe(uint64_t seed, int level, int count, unsigned long long* out,
                             hipStream_t s);
hipError_t launch_fill_u32(unsigned* p, unsigned v, int64_t m, hipStream_t s);

// ---- refine.hip
// dense coarsest solves, one workgroup per job
hipError_t launch_coarse_jobs(const CoarseJob* jobs, int njobs, hipStream_t s);
// coarse levels of each job inside one workgroup (FP64 levels only)
// Register-row layouts of single-workgroup levels: G lanes per row and E
// entry slots per lane and row (rows of up to G E entries).
constexpr int kRegLayouts = 7;
constexpr int kRegLayoutG[kRegLayouts] = {1, 2, 4, 8, 1, 2, 4};
constexpr int kRegLayoutE[kRegLayouts] = {8, 8, 8, 8, 16, 16, 16};
// kind 0: CSR traversal on kBlockKernelThreads threads; 1 + 3 l + log2(R)
// (layout l, R = 1, 2 or 4 rows per lane group): register rows on
// kBlockRegsThreads threads.
constexpr int kBlockKinds = 1 + 3 * kRegLayouts;
hipError_t launch_block_jobs(const BlockJob* jobs, int njobs, int kind, hipStream_t s);
// Job kernels are specialised by traversal (merge path or G lanes per
// row) and precision: kind = 2 * t + fp32, t = 0 for the merge path, else
// 1 + log2(G); finishing kernels depend on the traversal only.
constexpr int kJobKinds = 80;
// 16 wk + 2 t + fp32: traversal t (0 merge path, else 1 + log2(lanes)),
// FP32 iterates, weight storage wk
int job_kind(int variant, int lanes, int fp32, int wk);
// co-resident workgroups of a job kernel kind (measured once per process)
int refine_jobs_max_blocks(int kind);
int finish_jobs_max_blocks(int kind);
// one level of each job (all of one kind); nblocks = sum of the jobs' grids
hipError_t launch_refine_jobs(const GridJob* jobs, int njobs, int nblocks, int kind, hipStream_t s);
hipError_t launch_finish_jobs(const GridJob* jobs, int njobs, int nblocks, int kind, hipStream_t s);
// Device buffers a residency count may use instead of allocating its own,
// and the stream it then runs on (set per thread by the entry point that
// allocates nothing; nullptr clears).  cnt: 2 unsigned; job: one GridJob.
struct MeasureBuffers {
    unsigned* cnt;
    GridJob* job;
    hipStream_t stream;
};
void set_measure_buffers(const MeasureBuffers* b);
// ---- block.hip: several eigenpairs (Remark after Algorithm 4), P <= kBlkMaxP
constexpr int kBlkMaxP = 4;
// Block state of one level (device written): V = (W[cur] - 1 mu^T) rinv.
struct BlkCtl {
    double mu[kBlkMaxP];
    double rinv[kBlkMaxP * kBlkMaxP];  // R^{-1}, upper triangular, row-major P x P
    double minutv;                     // smallest (u_c, v_c) of the last step
    int32_t k, cur, done, hit;         // hit: 1 step cap, 2 Gram matrix not positive definite
};
struct BlkOut {
    double lambda[kBlkMaxP], residual[kBlkMaxP], norm2[kBlkMaxP], coarse[kBlkMaxP];
};
// One level of the block refinement (P columns, n x P row-major blocks).
struct BlkJob {
    int32_t n;
    int32_t nb;              // workgroups; rows rpart[b] .. rpart[b+1] for workgroup b
    const int32_t* rp;
    const int32_t* col;
    const double* w;
    double g;
    const int32_t* agg;      // prolongation: vertex -> aggregate of the coarser level
    const double* cW0;       // coarser level's blocks and state
    const double* cW1;
    const BlkCtl* cctl;
    double* W0;
    double* W1;
    BlkCtl* ctl;
    double* part;            // blk_parts(P) partial sums per workgroup
    const int32_t* rpart;
    BlkOut* out;
    double tol;
    uint64_t seed;
    int32_t maxit, kfix;
};
constexpr int kBlkCoarse = 0, kBlkProlong = 1, kBlkStep = 2, kBlkOut = 3;
int blk_parts(int p);
// what: kBlkCoarse (one workgroup; V (n x n, eigenvector k in column k),
// ev and the ascending order idx from the dense coarsest solve; hj by
// value), kBlkProlong (prolongation + normalisation), kBlkStep (one step +
// its check; does nothing once the level is done), kBlkOut (level 0: X
// (n x P column-major), Rayleigh quotients and residuals).
hipError_t launch_blk(int what, int p, const BlkJob* dj, const BlkJob& hj, double* X, const double* V,
                      const double* ev, const int32_t* idx, hipStream_t s);
// ---- bisect.hip: recursive spectral bisection (one depth of all parts at once)
hipError_t launch_rsb_keys(int n, const int32_t* part, unsigned long long* keys, hipStream_t s);
hipError_t launch_rsb_perm(int n, const unsigned long long* keys, int32_t* perm, int32_t* pos, int32_t* first,
                           int32_t* comp, hipStream_t s);
hipError_t launch_rsb_deg(int n, const int32_t* rp, const int32_t* col, const int32_t* part, const int32_t* perm,
                          int32_t* deg, hipStream_t s);
hipError_t launch_rsb_fill(int n, const int32_t* rp, const int32_t* col, const double* w, const int32_t* part,
                           const int32_t* perm, const int32_t* pos, const int32_t* first, const int32_t* eoff,
                           int32_t* rpl, int32_t* colk, double* wk, int32_t* cnt, int32_t* pnnz, int32_t* pbase,
                           hipStream_t s);
// hook and jump until nothing changes (host-checked; changed/h_changed: one int each)
hipError_t launch_rsb_components(int n, const int32_t* rpl, const int32_t* colk, const int32_t* part,
                                 const int32_t* perm, const int32_t* first, const int32_t* eoff, int32_t* comp,
                                 int* changed, int* h_changed, hipStream_t s);
hipError_t launch_rsb_roots(int n, const int32_t* comp, const int32_t* part, const int32_t* perm, int32_t* ncomp,
                            hipStream_t s);
hipError_t launch_rsb_split_keys(int n, const double* x, const int32_t* comp, const int32_t* part,
                                 const int32_t* perm, const int32_t* mode, unsigned long long* keys, double* vals,
                                 hipStream_t s);
hipError_t launch_rsb_part_keys(int n, const double* vals, const int32_t* part, const int32_t* perm,
                                unsigned long long* keys, hipStream_t s);
hipError_t launch_rsb_assign(int n, const double* vals, const int32_t* part, const int32_t* perm,
                             const int32_t* first, const int32_t* cnt, const int32_t* mode, int32_t* next,
                             hipStream_t s);
hipError_t launch_rsb_cut(int n, const int32_t* rp, const int32_t* col, const double* w, const int32_t* part,
                          double* bsum, hipStream_t s);
int rsb_cut_blocks(int n);
// raise the abort flag of a graph's barrier state (tests of the fallback)
hipError_t launch_raise_abort(GridSync* gs, hipStream_t s);
// zero the barrier state and the slots (2 * nslots; at setup, and after an abort)
hipError_t launch_reset_sync(GridSync* gs, GridSlot* slots, int nslots, GridSlot* bcast, hipStream_t s);

// Large levels, one launch per step (rows traversal; kind as job_kind).
// Sequence: step_begin (prolongation, mean and norm), then step_pi per
// power-iteration step; a step launched after the stopping test passed
// does nothing.  job points to device memory.
hipError_t launch_step_begin(const StepJob* job, int nblocks, int kind, hipStream_t s);
hipError_t launch_step_pi(const StepJob* job, int nblocks, int kind, hipStream_t s);
constexpr int kStepBlock = 512;

constexpr int kGridBlock = 512;
constexpr int kBlockKernelThreads = 1024;
constexpr int kBlockRegsThreads = 512;   // 256 VGPRs per lane for register rows
constexpr int kBlockLdsMax = 144 * 1024;  // LDS image budget of the single-workgroup kernel
constexpr int kGridStageRows = 1024;       // most rows of a grid workgroup's LDS stage
int refine_block_lds_budget();

}  // namespace cmg
