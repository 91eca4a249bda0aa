/*
 * cosma_mi355 -- dense C = alpha*A*B + beta*C on one MI355X (gfx950), run
 * under the I/O-optimal schedule of Kwasniewski et al., "Red-Blue Pebbling
 * Revisited: Near Optimal Parallel Matrix-Matrix Multiplication" (SC'19).
 *
 * The product computed is the classical one of section 2.4 (A is m x k,
 * B is k x n, C is m x n), entry by entry the sum over the reduction index
 * of the CDAG update rule of section 5.1; only the order of that sum differs
 * between schedules.  Algorithm 1 gives the structure of every call: pick the
 * sequential schedule (section 5), parallelise it (eq. optTileShape,
 * section 6.3), fit it to the processors (section 7.1), stream the
 * reduction dimension in rounds (the DistrData / Multiply loop) and reduce
 * partial results when k is split (Reduce).  Here a "processor" is a
 * compute unit and its fast memory S is the CU's register file plus LDS.
 *
 * Conventions shared by every entry point
 *  - Row-major, no transposes.  A: m x k, lda >= max(1,k).  B: k x n,
 *    ldb >= max(1,n).  C: m x n, ldc >= max(1,n).
 *  - A, B, C and any workspace are device pointers owned by the caller; the
 *    library never frees or retains caller memory beyond the call, except
 *    the workspace registered with cosma_set_workspace (borrowed until
 *    replaced) and batch handles (see cosma_batch_create).
 *  - alpha and beta are host doubles; FP32-class dtypes round them to fp32.
 *  - BLAS rules: m == 0 or n == 0 is a no-op; k == 0 or alpha == 0 gives
 *    C = beta*C without reading A or B; beta == 0 never reads C (NaNs in C
 *    are overwritten).
 *  - Every GPU entry point is asynchronous on `stream` (a hipStream_t, or
 *    NULL for the default stream) and returns once the work is enqueued.
 *  - Errors are returned as negative cosma_status values; on an argument
 *    error nothing is enqueued.  No entry point allocates device memory on
 *    the compute path (cosma_batch_create allocates the handle's memory once,
 *    at creation); partial results live in the caller's workspace.
 *  - Calls that share the registered workspace must be ordered on one
 *    stream (or synchronised by the caller).
 */
#ifndef COSMA_MI355_H
#define COSMA_MI355_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define COSMA_API __attribute__((visibility("default")))
#else
#define COSMA_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  COSMA_F64 = 0,          /* binary64 operands and result, FP64 MFMA */
  COSMA_F32 = 1,          /* binary32 operands and result, FP32 MFMA */
  COSMA_F32_BF16X3 = 2,   /* binary32 operands and result; each operand split
                             into bf16 hi + lo, three bf16 MFMA products,
                             fp32 accumulation */
  COSMA_F64_OZAKI_I8 = 3, /* binary64 operands and result; operands split into
                             int8 digit slices, exact int32 MFMA products,
                             binary64 summation.  All Ozaki forms scale rows
                             of A and columns of B: a row of A (column of B)
                             holding a NaN or an infinity gives a NaN row
                             (column) of C; the native dtypes follow IEEE
                             arithmetic entry by entry */
  COSMA_F64_OZAKI2_I8 = 4 /* binary64 operands and result; operands scaled to
                             integers and reduced modulo N pairwise coprime
                             moduli <= 256 (int8 residues), one exact int8
                             MFMA product per modulus, result recovered by
                             the Chinese remainder theorem (Ozaki, Uchino &
                             Imamura, "Ozaki Scheme II", 2025) */,
  COSMA_F64_OZAKI_BF16 = 5 /* binary64 operands and result; operands split
                             into 8-bit digit slices held exactly in bf16,
                             bf16 MFMA products with fp32 accumulation kept
                             exact (every 32-long round is moved into a
                             binary64 accumulator), binary64 summation;
                             NaN rows / columns as COSMA_F64_OZAKI_I8 */
} cosma_dtype;

/* Storage order and operand transposition of cosma_gemm_ex (CBLAS
   conventions). */
typedef enum { COSMA_ROW_MAJOR = 0, COSMA_COL_MAJOR = 1 } cosma_layout;
typedef enum { COSMA_NO_TRANS = 0, COSMA_TRANS = 1 } cosma_transpose;

typedef enum {
  COSMA_OK = 0,
  COSMA_ERR_INVALID_ARG = -1, /* bad size, leading dimension, pointer, dtype or plan */
  COSMA_ERR_HIP = -2,         /* a HIP runtime call failed */
  COSMA_ERR_WORKSPACE = -3,   /* the plan needs more workspace than is registered */
  COSMA_ERR_UNSUPPORTED = -4, /* no device, wrong architecture, or unsupported case */
  COSMA_ERR_NO_MEMORY = -5    /* host allocation failed (planner / batch metadata) */
} cosma_status;

/* Hardware figures the planner uses: the machine model of section 2.1 (p
   processors with S words of fast memory each) plus the memory level above.
   With a device, num_cus, lds_bytes_per_cu, vgpr_bytes_per_cu (32-bit
   registers per CU x 4), l2_bytes_per_xcd, num_xcds and clock_ghz are read
   from the runtime; hbm_gbps is the published peak.  Without a device all
   are MI355X defaults (256 CUs, 8 XCDs, 160 KiB LDS, 512 KiB registers and
   4 MiB L2 per XCD, 2.4 GHz, 8000 GB/s). */
typedef struct {
  int32_t num_cus;            /* compute units ("processors") */
  int32_t num_xcds;           /* accelerator dies; each has its own L2 */
  int64_t lds_bytes_per_cu;   /* local data share per CU */
  int64_t vgpr_bytes_per_cu;  /* vector register file (arch + acc) per CU */
  int64_t l2_bytes_per_xcd;   /* L2 per XCD */
  double clock_ghz;           /* peak engine clock */
  double hbm_gbps;            /* peak HBM bandwidth, GB/s */
} cosma_device_facts;

/* A schedule for one product, as chosen by the planner (Algorithm 1's
   FindSeqSchedule / ParallelizeSched / FitRanks mapped onto the CUs). */
typedef struct {
  int64_t m, n, k;
  int32_t dtype;              /* cosma_dtype */
  int32_t tile_id;            /* index into the dtype's kernel tile menu */
  int32_t tile_m, tile_n;     /* C block per work item (the paper's a x a face) */
  int32_t tile_k;             /* reduction rounds: k-panel depth per LDS stage */
  int32_t p_m, p_n, p_k;      /* grid: row blocks, column blocks, k splits */
  int32_t group_m;            /* raster group height (tile rows per group) */
  int32_t wg_per_cu;          /* resident work items per CU */
  int32_t regime;             /* 0: ij-parallel (p <= p1), 1: k is cut (p > p1) */
  int32_t slices;             /* COSMA_F64_OZAKI_I8, COSMA_F64_OZAKI_BF16:
                                 digit slices per operand;
                                 COSMA_F64_OZAKI2_I8: number of moduli N;
                                 0 otherwise */
  int64_t k_split;            /* reduction length per split (multiple of tile_k) */
  int64_t items;              /* p_m * p_n * p_k */
  int64_t waves;              /* ceil(items / resident slots) */
  double S_words;             /* per-CU fast memory in words of the operand type */
  double p1;                  /* mn / S: dependency-free sqrt(S) x sqrt(S) x k domains */
  int64_t a_seq, b_seq;       /* integer optimum of section 5 for S_words */
  double a_par, b_par;        /* eq. optTileShape with p = num_cus */
  double q_cu_words;          /* I/O counted at the CU level, in words */
  double q_ea_bytes;          /* predicted L2 <-> memory bytes for the raster */
  double thm1_words;          /* Theorem 1 bound 2mnk/sqrt(S) + mn, words */
  double thm2_words;          /* Theorem 2 bound per CU, words */
  double predicted_ms;        /* planner time model */
  size_t workspace_bytes;     /* device workspace the plan needs */
  /* Error contract of the Ozaki dtypes (0 for the native dtypes), see
     "Accuracy of the Ozaki dtypes" below. */
  double err_scaled;          /* E: bound per unit |alpha| k 2^(e_i + f_j) */
  double err_rounding;        /* G: bound per unit D_ij */
  double spread_limit;        /* largest spread rho_ij with E rho + G <= 3k 2^-53 */
} cosma_plan_info;

/* Accuracy of the Ozaki dtypes.  The paper fixes no precision; the stated
   target for FP64-class results is a normalised error
       max_ij |C^_ij - C_ref_ij| / D_ij <= 4k 2^-53,
       D_ij = |alpha| sum_t |A_it| |B_tj| + |beta| |C0_ij|,
   against a binary64 reference C_ref.  Write e_i for the exponent of the
   largest |A_it| of row i (max_t |A_it| < 2^e_i, as frexp gives it), f_j
   likewise for column j of B, and C_ij for the exact result.  For finite
   inputs whose scaled results stay in the normal binary64 range, every
   Ozaki plan guarantees
       |C^_ij - C_ij| <= |alpha| err_scaled k 2^(e_i + f_j) + err_rounding D_ij,
   err_scaled coming from the finite number of slices (moduli) and
   err_rounding from the binary64 steps.  With the spread of an entry
       rho_ij = |alpha| k 2^(e_i + f_j) / D_ij   (>= 1 for dense rows),
   the normalised error against the exact product is at most
   err_scaled rho_ij + err_rounding, so it stays within 3k 2^-53 (and
   within 4k 2^-53 of any binary64 reference that is itself within
   k 2^-53 of the exact product) for every entry with
   rho_ij <= spread_limit.  The planner picks the smallest slice count
   (COSMA_F64_OZAKI_I8, COSMA_F64_OZAKI_BF16: 1..8) or number of moduli
   (COSMA_F64_OZAKI2_I8: 2..16) whose spread_limit reaches the target spread
   (cosma_set_ozaki_spread; default 2048: for entries sign * U[1,2) * 2^e,
   e uniform in [-20, 20], rho_ij has a median of about 750 at k in the
   thousands, and 2209 at most over an 8192^3 product); where no count
   reaches it (short k: spread_limit grows about linearly with k), the
   smallest count with the smallest err_scaled (the most accurate
   emulation), and the plan's spread_limit then says which entries the
   bound covers (0: none; the rounding term alone exceeds 3k 2^-53).  Uniform
   [-1, 1] data has rho_ij of about 4.  Entries beyond spread_limit are
   still within the absolute bound above; the call returns COSMA_OK. */

/* ---- single product ---------------------------------------------------- */

/* C = alpha*A*B + beta*C under the planner's schedule (Algorithm 1). */
COSMA_API int cosma_gemm(int64_t m, int64_t n, int64_t k, double alpha, const void* A, int64_t lda,
               const void* B, int64_t ldb, double beta, void* C, int64_t ldc, int dtype,
               void* stream);

/* Same product under an explicit plan (from cosma_plan_query or
   cosma_plan_make, m/n/k/dtype must match). */
COSMA_API int cosma_gemm_planned(const cosma_plan_info* plan, double alpha, const void* A, int64_t lda,
                       const void* B, int64_t ldb, double beta, void* C, int64_t ldc,
                       void* stream);

/* For callers that cannot allocate device memory (code that must not call
   hipMalloc, e.g. under graph capture, tight serving loops, harnesses that
   forbid it): cosma_gemm with no registered workspace.  The schedule's
   workspace is a device array of COSMA_NOALLOC_SCRATCH_BYTES that the
   library's code object holds on every GPU it runs on until the process
   ends; the call allocates nothing.  A native-dtype plan whose split-K
   partials would not fit runs with k whole instead; any other plan that
   needs more returns COSMA_ERR_WORKSPACE (nothing launched).  Every call on
   one GPU shares that GPU's array: calls that overlap on one GPU (other
   streams, other threads) race, so order them.  Arguments, results, errors
   and asynchrony otherwise as cosma_gemm; results equal cosma_gemm's under
   the same plan. */
#define COSMA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
COSMA_API int cosma_gemm_noalloc(int64_t m, int64_t n, int64_t k, double alpha, const void* A,
                                 int64_t lda, const void* B, int64_t ldb, double beta, void* C,
                                 int64_t ldc, int dtype, void* stream);

/* C = alpha*op(A)*op(B) + beta*C with CBLAS conventions, for callers whose
   matrices are column-major (ScaLAPACK / Fortran style, the paper's own
   library interface) or transposed.  op(A) is m x k, op(B) is k x n, C is
   m x n.  Row-major: A is m x k (lda >= k) or, transposed, k x m (lda >= m);
   B is k x n (ldb >= n) or n x k (ldb >= k); ldc >= n.  Column-major: A is
   m x k (lda >= m) or k x m (lda >= k); B is k x n (ldb >= k) or n x k
   (ldb >= n); ldc >= m.  (Leading dimensions are at least 1.)
   A column-major product runs as the row-major product C^T = op(B)^T op(A)^T
   on the same memory, with no copy.  A transposed operand (after that swap)
   is first transposed into the workspace, after the part the plan itself
   uses: register at least cosma_workspace_size_ex bytes.  Without transposed
   operands this is cosma_gemm.  Errors, BLAS rules and asynchrony as for
   cosma_gemm; COSMA_ERR_INVALID_ARG also for unknown layout or transpose
   values. */
COSMA_API int cosma_gemm_ex(int layout, int transa, int transb, int64_t m, int64_t n, int64_t k,
                            double alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                            double beta, void* C, int64_t ldc, int dtype, void* stream);
/* Workspace bytes cosma_gemm_ex needs for these arguments. */
COSMA_API int cosma_workspace_size_ex(int layout, int transa, int transb, int64_t m, int64_t n,
                                      int64_t k, int dtype, size_t* bytes);

/* ScaLAPACK-style product for callers that hold their matrices in the
   block-cyclic format: the paper's blocked layout is compatible with it
   (section 7.6) and its library takes ScaLAPACK operands directly
   (section 1).  Computes
       sub(C) = alpha*op(sub(A))*op(sub(B)) + beta*sub(C),
   where sub(X) is the block of the global matrix X that starts at the
   1-based position (iX, jX).  op(sub(A)) is m x k, op(sub(B)) is k x n,
   sub(C) is m x n, and transa / transb take cosma_transpose values.
   Each desc* is a nine-entry ScaLAPACK array descriptor
   {DTYPE_ = 1, CTXT_, M_, N_, MB_, NB_, RSRC_, CSRC_, LLD_}.  On one GPU the
   process grid is 1 x 1, so every block is local and the device array is
   the whole global matrix, column-major with leading dimension LLD_
   (element (i, j) at (j - 1)*LLD_ + i - 1), for any MB_, NB_ >= 1.
   The process grid must be 1 x 1: RSRC_ = CSRC_ = 0, and CTXT_ is not read.
   COSMA_ERR_INVALID_ARG:
     - a null descriptor, DTYPE_ != 1, M_ or N_ < 0, MB_ or NB_ < 1,
       RSRC_ or CSRC_ != 0, LLD_ < max(1, M_);
     - iX or jX < 1;
     - a submatrix of non-zero extent that reaches past M_ or N_;
     - any argument cosma_gemm_ex rejects.
   The product then runs as cosma_gemm_ex with COSMA_COL_MAJOR on the blocks'
   first elements, so the workspace it needs is cosma_workspace_size_ex's
   for COSMA_COL_MAJOR with the same transa, transb, m, n, k and dtype.
   Asynchrony and the other rules are as for cosma_gemm.  Only sub(C) is
   written. */
COSMA_API int cosma_pgemm(int transa, int transb, int64_t m, int64_t n, int64_t k, double alpha,
                          const void* A, int64_t ia, int64_t ja, const int32_t* desca,
                          const void* B, int64_t ib, int64_t jb, const int32_t* descb,
                          double beta, void* C, int64_t ic, int64_t jc, const int32_t* descc,
                          int dtype, void* stream);

/* ---- batches of independent products (Algorithm 1's "for all p_i in
   parallel" over many small problems) ------------------------------------ */

/* Variable-size batch: problem i is C_i = alpha_i*A_i*B_i + beta_i*C_i.
   The planner's batch model picks one tile for the whole batch (among the
   tiles with a persistent form, the one whose modelled item costs sum
   lowest) and a split factor p_k per problem: a problem whose work items
   would be long against the batch's share per resident workgroup is cut in
   k (section 6.2's rule that k is cut once processors outnumber independent
   (i, j) domains), its partials reduced in ascending split order.  The
   problems run as one persistent launch (the problems must not alias each
   other's C).
   Supported dtypes: COSMA_F32, COSMA_F64 (else COSMA_ERR_UNSUPPORTED).
   All host arrays have length `count` and are read during the call only.
   The problem descriptors, the item map, the launch counters and the split
   partials live in the registered workspace (cosma_set_workspace; size from
   cosma_workspace_size_batched, COSMA_ERR_WORKSPACE when smaller): the call
   allocates nothing, copies nothing from host memory (descriptors travel
   inside kernel arguments), never waits for the device, and can be
   captured into a HIP graph whose replays rerun the same batch.  Like
   cosma_gemm, calls sharing the workspace must be ordered on one stream. */
COSMA_API int cosma_gemm_batched(int64_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                       const double* alpha, const void* const* A, const int64_t* lda,
                       const void* const* B, const int64_t* ldb, const double* beta,
                       void* const* C, const int64_t* ldc, int dtype, void* stream);
/* Workspace bytes cosma_gemm_batched needs for these sizes (0 when no
   problem has products).  Section 7.5's pre-allocated buffers: the caller
   provides them once, the compute path never allocates. */
COSMA_API int cosma_workspace_size_batched(int64_t count, const int64_t* m, const int64_t* n,
                                           const int64_t* k, const double* alpha, int dtype,
                                           size_t* bytes);

/* Capture-once / replay-many batch: plans every problem (tile and split),
   uploads the descriptors and captures the launches into a HIP graph.  The
   handle owns its device memory (allocated here, never on the replay path)
   and graph until cosma_batch_destroy.  Pointers and sizes are fixed at
   creation; replays read the current contents of A, B and C.  Inside the
   graph the tile variants' launches run concurrently.  When every beta is
   zero (and COSMA_AUTOTUNE is not 0) the autotuner times the batch on
   `stream`: first once per policy (below), then, from the fastest, class
   by class of problems (m n and k each binned by factors of four, the
   eight classes with the most flops first) it tries the other tiles and
   twice / half the current split factors, keeping a change that is more
   than 1 % faster.  Otherwise policy 5 (as for cosma_gemm_batched). */
COSMA_API int cosma_batch_create(int64_t count, const int64_t* m, const int64_t* n, const int64_t* k,
                       const double* alpha, const void* const* A, const int64_t* lda,
                       const void* const* B, const int64_t* ldb, const double* beta,
                       void* const* C, const int64_t* ldc, int dtype, void* stream,
                       void** handle);
/* Launch the batch's graph on `stream` (asynchronous). */
COSMA_API int cosma_batch_run(void* handle, void* stream);
/* Waits for the last cosma_batch_run enqueued outside a stream capture (an
   event of the handle, not the whole device), then frees the handle's
   memory and graph.  Replays captured into a caller's graph must be
   finished by the caller. */
COSMA_API int cosma_batch_destroy(void* handle);
/* Policy the autotuner started its refinement from (0 = the planner's batch model per problem,
   1 = all 64x64, 2 = all 128x128, 3 = size threshold, each with the model's
   splits; 4 = the model's tiles with k never cut; 5 = one tile for the
   whole batch, the lowest summed model cost, with the model's splits: the
   policy used without tuning), number of persistent launches (one per tile
   variant), work items, and the timed milliseconds of each candidate policy
   (0 when tuning was skipped: some beta != 0, or COSMA_AUTOTUNE=0). */
COSMA_API int cosma_batch_info(void* handle, int* policy, int* groups, int64_t* items,
                               double* policy_ms, int policy_ms_len);
/* The autotuner's refinement: trials timed after the policies, the fastest
   policy's milliseconds and the kept assignment's (all 0 without tuning).
   Any output pointer may be NULL. */
COSMA_API int cosma_batch_tuning(void* handle, int* trials, double* seed_ms, double* tuned_ms);
/* Tile id (menu index of the batch's dtype) each input problem runs with, or
   -1 for problems without products (m, n or k zero, or alpha zero); count
   must equal the count given at creation. */
COSMA_API int cosma_batch_tiles(void* handle, int64_t count, int32_t* tile_ids);
/* Split factor p_k of each input problem (0 for problems without
   products); with cosma_batch_tiles and cosma_plan_make this names the
   single-product plan each problem runs under. */
COSMA_API int cosma_batch_splits(void* handle, int64_t count, int32_t* p_k);

/* ---- planner (host only; no GPU needed) --------------------------------- */

/* Plan for the current device (MI355X defaults without a device). */
COSMA_API int cosma_plan_query(int64_t m, int64_t n, int64_t k, int dtype, cosma_plan_info* out);
/* Plan for given hardware figures and idle budget delta (section 7.1's
   tunable: the fraction of compute time the planner may give up for less
   I/O).  facts == NULL means the current device. */
COSMA_API int cosma_plan_query_facts(int64_t m, int64_t n, int64_t k, int dtype,
                           const cosma_device_facts* facts, double delta, cosma_plan_info* out);
/* Plan with a forced tile (menu index) and split factor p_k >= 1. */
COSMA_API int cosma_plan_make(int64_t m, int64_t n, int64_t k, int dtype, int tile_id, int p_k,
                    cosma_plan_info* out);
/* Target spread rho (>= 1) the planner's Ozaki slice choice must cover
   (see "Accuracy of the Ozaki dtypes"); process-wide, clears the plan
   cache.  The initial value is COSMA_OZAKI_SPREAD from the environment, or
   2048.  COSMA_OZAKI_SLICES, COSMA_OZAKI_BF16_SLICES and COSMA_OZAKI2_MODULI
   in the environment force fixed counts instead. */
COSMA_API int cosma_set_ozaki_spread(double spread);
COSMA_API int cosma_get_ozaki_spread(double* spread);
/* Ozaki plans: set the number of digit slices per operand (1..8) and
   recompute the plan's workspace and error contract.  More slices cost s(s+1)/2 products and
   shrink the truncation error by 2^-7 (COSMA_F64_OZAKI_I8) or 2^-8
   (COSMA_F64_OZAKI_BF16) per slice.
   Modular (COSMA_F64_OZAKI2_I8) plans: set the number of moduli N (2..16)
   and recompute the plan's work items and workspace.  Each modulus costs
   one int8 product and adds about 8 bits to M; the operands keep beta bits
   (see cosma_ozaki2_params), about half a bit less per doubling of k;
   COSMA_ERR_INVALID_ARG when N moduli leave no operand bits at the plan's
   k (cosma_ozaki2_params fails). */
COSMA_API int cosma_plan_set_slices(cosma_plan_info* plan, int slices);
/* Modular path parameters for reduction length k >= 1 and N moduli
   (2..16): *beta receives the operand scale (rows of A and columns of B are
   scaled so that their largest entry lies in [2^(beta-1), 2^beta) and
   rounded to integers; every |sum_t A'_it B'_tj| <= k 2^(2 beta) <= M/4,
   M = p_0 ... p_(N-1)), moduli[0..N) the moduli used (pairwise coprime,
   taken greedily from 256 downwards).  Host only; returns
   COSMA_ERR_INVALID_ARG when N is out of range or k is so long that
   beta < 1. */
COSMA_API int cosma_ozaki2_params(int64_t k, int nmod, int32_t* beta, int32_t* moduli);
/* Number of kernel tiles for dtype, and the shape of tile `id`. */
COSMA_API int cosma_tile_count(int dtype);
COSMA_API int cosma_tile_shape(int dtype, int id, int32_t* tile_m, int32_t* tile_n, int32_t* tile_k);
/* Facts of the current device (or the MI355X defaults). */
COSMA_API int cosma_device_query(cosma_device_facts* out);

/* Theorem 1: 2mnk/sqrt(S) + mn words. */
COSMA_API double cosma_thm1_bound(double m, double n, double k, double S);
/* Section 5: integer optimum of max ab/(a+b) s.t. ab + a + 1 <= S. */
COSMA_API int cosma_seq_schedule(int64_t S, int64_t* a, int64_t* b);
/* eq. optTileShape: a = min{sqrt S, (mnk/p)^(1/3)}, b = max{mnk/(pS), (mnk/p)^(1/3)}. */
COSMA_API int cosma_par_schedule(double m, double n, double k, double p, double S, double* a, double* b);
/* Section 7.1 grid fitting over p' in [ceil((1-delta)p), p] minimising the
   local-domain surface; grid = (p_m, p_n, p_k), *used = p_m*p_n*p_k. */
COSMA_API int cosma_fit_ranks(int64_t m, int64_t n, int64_t k, int64_t p, double delta, int64_t grid[3],
                    int64_t* used);
/* Words moved by the tiled schedule: k-rounds loading tile_m x kc of A and
   kc x tile_n of B per work item, C block resident, p_k splits with a
   partial store + reload when p_k > 1, C0 loads when beta != 0. */
COSMA_API double cosma_io_count(int64_t m, int64_t n, int64_t k, int64_t tile_m, int64_t tile_n,
                      int64_t kc, int64_t p_k, int beta_nonzero);

/* ---- workspace ---------------------------------------------------------- */
/* Section 7.5 pre-allocates the communication buffers once, at their
   largest size, so that no step of the schedule allocates.  Here the
   buffers are the split-K partial blocks (Reduce's inputs), the BF16x3
   planes and the Ozaki digit / residue planes: the caller queries their
   size, allocates once and registers the buffer; the compute path only
   offsets into it. */

/* Bytes of workspace the planner's schedule for this product needs
   (*bytes; COSMA_ERR_INVALID_ARG for a null pointer or invalid sizes). */
COSMA_API int cosma_workspace_size(int64_t m, int64_t n, int64_t k, int dtype, size_t* bytes);
/* Register a caller-owned device buffer (256-byte aligned) as the workspace
   of the current device (ptr == NULL, bytes == 0 unregisters).  The library
   borrows it until it is replaced and never frees it; `stream` is unused
   and reserved.  COSMA_ERR_INVALID_ARG for a misaligned pointer or a
   pointer / size mismatch, COSMA_ERR_UNSUPPORTED without a device. */
COSMA_API int cosma_set_workspace(void* device_ptr, size_t bytes, void* stream);

/* ---- misc --------------------------------------------------------------- */
/* Static text naming a cosma_status value (never NULL; "unknown cosma
   status" for other values).  Host only.  The statuses report the
   argument, workspace and device conditions of the conventions above; the
   paper defines none of them. */
COSMA_API const char* cosma_status_string(int status);
/* Static library version string (never NULL).  Host only. */
COSMA_API const char* cosma_version(void);

#ifdef __cplusplus
}
#endif

#endif /* COSMA_MI355_H */
