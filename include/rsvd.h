/*
 * rsvd.h -- C ABI of the MI355X randomized-SVD library.
 *
 * Computes a rank-k approximate SVD  A ~ U diag(S) V^T  of an m x n matrix A
 * by the randomized SVD of Halko, Martinsson and Tropp as the paper states it
 * (Section 2.1, steps 1-7): a Gaussian test matrix O (n x l), the sketch
 * Y = A O, a thin QR of Y, the projection B = Q^T A, an SVD of the small B,
 * and U = Q U_B.  The sketch is taken of the power matrix (A A^T)^q A
 * (Section 2.2, Eq. (1)), evaluated right to left (Eq. (2)) and
 * re-orthonormalised after every product with A or A^T.  The sketch has
 * l = k + p columns (p = oversampling); the result keeps k.  Products with A
 * run block by block over the block-cyclic tiles of A (Section 2.3, Eq. (3);
 * Section 3.1); workspace is sized before anything runs (Section 3.4).
 *
 * Conventions
 *   - All integer sizes are int64_t and counted in elements.
 *   - A dense A is row-major: element (i, j) at data[i * ld + j], ld >= n.
 *   - U (m x k) and V (n x k) are column-major: U(i, j) at U[i + j * ldu],
 *     ldu >= m; V(i, j) at V[i + j * ldv], ldv >= n.  S holds k doubles,
 *     descending.  Signs: the largest-magnitude entry of every column of V
 *     (lowest row on ties) is positive.
 *   - Device pointers are HIP device (or managed) memory on the current
 *     device; "stream" arguments are hipStream_t handles passed as void*
 *     (NULL = the default stream).
 *   - The caller owns every buffer: A, U, S, V, gradients and workspaces.
 *     The library never allocates device memory in rsvd_factor or
 *     rsvd_backward; a plan owns only host metadata.
 *   - Every call returns an rsvd_status; nothing throws across the ABI.
 *     A text message for the last failure of a plan is available from
 *     rsvd_last_error(plan) (or rsvd_last_error(NULL) for plan-less calls).
 *   - Calls on one plan must not overlap; different plans are independent.
 */
#ifndef RSVD_H
#define RSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rsvd_status;
enum {
  RSVD_OK = 0,
  RSVD_W_RANK_DEFICIENT = 1, /* results valid; some sketch directions were dropped */
  RSVD_W_DEGENERATE = 2,     /* results valid; backward met equal singular values  */
  RSVD_STOPPED = 3,          /* stopped after the requested pass; see checkpoints  */
  RSVD_E_INVALID_ARG = -1,
  RSVD_E_BUDGET = -2,        /* workspace does not fit the HBM budget              */
  RSVD_E_HIP = -3,           /* a HIP runtime call failed                          */
  RSVD_E_UNSUPPORTED = -4,   /* legal but not implemented combination              */
  RSVD_E_NUMERIC = -5        /* NaN/Inf met on the device                          */
};

enum { RSVD_DENSE = 0, RSVD_CSR = 1, RSVD_COO = 2 };                /* formats   */
enum { RSVD_F64 = 0, RSVD_F32 = 1, RSVD_BF16 = 2, RSVD_FP8E4M3 = 3 }; /* dtypes    */
enum { RSVD_LOC_DEVICE = 0, RSVD_LOC_HOST_PINNED = 1 };              /* locations */
enum { RSVD_ORTHO_EACH = 0, RSVD_ORTHO_FINAL_ONLY = 2 };             /* schedules */
enum {
  RSVD_FLAG_NO_SIGN_FIX = 1,   /* skip the sign convention                          */
  RSVD_FLAG_CHOLQR1 = 2,       /* one CholeskyQR pass for intermediate bases        */
  RSVD_FLAG_BACKWARD = 4,      /* size the workspace for rsvd_backward too          */
  RSVD_FLAG_AUTO_Q = 8,        /* choose q <= prob.q automatically (q_tol)          */
  RSVD_FLAG_JACOBI_ONLY = 16   /* small SVD by Cholesky and one-sided Jacobi only,
                                  also at widths <= 128 (where the tridiagonal
                                  eigensolver runs first by default)              */
};

/* The problem: A is m x n, rank k, oversampling p, q power steps
 * (Section 2.1; Section 2.2, Eq. (1)), Gaussian test matrix from `seed`. */
typedef struct {
  int64_t m, n, k, p, q;
  int32_t format;   /* RSVD_DENSE, RSVD_CSR or RSVD_COO (rsvd_factor_coo) */
  int32_t dtype;    /* storage type of A: RSVD_F32 or RSVD_F64            */
  int32_t loc;      /* RSVD_LOC_DEVICE, or RSVD_LOC_HOST_PINNED (dense)   */
  int32_t reserved;
  uint64_t seed;
  int64_t nnz;      /* CSR and COO only                                   */
} rsvd_problem;

/* Options.  prec_* choose the operand type of the products with A in the
 * sketch, the power steps and the projection: RSVD_F32, RSVD_BF16 (A and the
 * panel rounded to nearest even once; Section 3.2 stores half precision and
 * computes in single) or RSVD_FP8E4M3 (OCP e4m3, A quantised once with one
 * power-of-two scale per 64 x 64 block, panels with one per column; tiles must
 * be multiples of 64).  All products accumulate in FP32; Gram, Cholesky and
 * the small SVD run in FP64.
 * tile_m/tile_n: block-cyclic tile size (0 = chosen by the plan);
 * grid_p/grid_q: process grid of the block-cyclic map (1 x 1 on one GPU).
 * hbm_budget_bytes: cap on the device workspace (0 = none). */
typedef struct {
  int32_t prec_sketch, prec_power, prec_project;
  int32_t ortho;
  int64_t tile_m, tile_n;
  int64_t grid_p, grid_q;
  uint64_t hbm_budget_bytes;
  int32_t flags;
  int32_t reserved;
  /* RSVD_FLAG_AUTO_Q (Section 2.2, automatic iteration parameter): after
   * each product A^T Q the singular values the factorisation would return
   * for the q reached so far are computed; the loop stops at the first q
   * whose leading k values moved by at most q_tol (relative) from those of
   * q - 1, or at prob.q.  0 means 1e-4.  Needs prec_power == prec_project;
   * each step then waits for the device once. */
  double q_tol;
  /* Per-operand device memory, the three limits of Section 3.5 (per matrix,
   * new matrices, global):
   *   a_budget_bytes    HBM that the tiles of A may occupy.  Host-resident
   *                     A gets floor(a_budget / tile slot) slots, at least
   *                     two, at most one per tile: with a slot for every
   *                     tile, A is copied once per call and stays resident
   *                     for the later passes (kept in-core).  A
   *                     device-resident dense or sparse A larger than the
   *                     limit is RSVD_E_BUDGET (plan it host-resident).
   *   new_budget_bytes  HBM for the matrices the plan builds (panels,
   *                     partial products, small factors, the CSC copy of a
   *                     sparse A): RSVD_E_BUDGET when they need more.
   *   hbm_budget_bytes  (above) the whole workspace.
   * A limit left at 0 takes the next one's value (a_budget from new_budget,
   * new_budget from hbm_budget_bytes); with only hbm_budget_bytes set, the
   * slots get what the plan's own matrices leave of it.  With none set, a
   * host-resident A streams through four slots. */
  uint64_t a_budget_bytes;
  uint64_t new_budget_bytes;
} rsvd_options;

/* Stage timers follow the paper's stage list (Section 4.1): 0 Gaussian O,
 * 1 sketch A O, 2 orthogonalisation of the sketch, 3 power steps (products
 * and their orthogonalisation), 4 projection A^T Q, 5 SVD0 preparation
 * (Gram of B), 6 SVD0, 7 post-processing.  gemm_*_ms sum the device time of
 * the product kernels alone (HIP events around each launch on the stream). */
typedef struct {
  double stage_ms[8];
  double total_ms;
  double flops_alg;        /* algorithmic flops of the passes over A        */
  double bytes_alg;        /* algorithmic HBM bytes of the passes over A    */
  double gemm_nn_ms;       /* summed time of the A X product kernels        */
  double gemm_tn_ms;       /* summed time of the A^T X product kernels      */
  int64_t ws_bytes;        /* device workspace used                         */
  int32_t gemm_nn_launches;
  int32_t gemm_tn_launches;
  int32_t dropped;         /* sketch directions dropped as dependent        */
  int32_t jacobi_sweeps;   /* one-sided Jacobi sweeps of the small SVD; 0
                              when the tridiagonal eigensolver's result
                              was kept (widths <= 128, checks held)        */
  int32_t nonfinite;       /* NaN/Inf seen on the device                    */
  int32_t slots;           /* host-resident A: HBM tile slots               */
  double h2d_bytes;        /* host-resident A: bytes copied host -> device  */
  int64_t tile_loads;      /* host-resident A: tiles copied                 */
  int32_t q_used;          /* power steps run (RSVD_FLAG_AUTO_Q: chosen)    */
  int32_t reserved2;
  double q_delta;          /* last relative change of the leading k values  */
  double sketch_ms;        /* device time of the first A X launch (the
                              sketch pass; in the BF16 form it also writes
                              the BF16 copy of an FP32 A)                  */
  int64_t peak_hbm;        /* device bytes the call touches: workspace
                              + device-resident A (m n elements; 0 for host
                              A) or the caller's CSR (8 nnz + 4 (m + 1))
                              or COO (nnz (2 index bytes + 4)) arrays
                              + U, V (4 (m + n) k) + S (8 k)               */
} rsvd_report;

typedef struct rsvd_plan_s* rsvd_plan_t;

/* Validate the problem and options, build the block-cyclic tile maps and size
 * the device workspace (Section 3.4: sizes are known before running).  Host
 * only: makes no HIP call.  On success *out holds a new plan and
 * *device_ws_bytes the workspace rsvd_factor needs (256-byte aligned).
 * Errors: RSVD_E_INVALID_ARG (k < 1, p < 0, q < 0, k + p > min(m, n),
 * bad enum, tile sizes), RSVD_E_UNSUPPORTED (format/dtype/location not
 * implemented, or k + p above 512), RSVD_E_BUDGET (workspace above hbm_budget_bytes; the message
 * states the bytes needed).  opt may be NULL (defaults: FP32 everywhere,
 * ortho EACH, automatic tiles, no budget). */
rsvd_status rsvd_plan(const rsvd_problem* prob, const rsvd_options* opt, rsvd_plan_t* out,
                      size_t* device_ws_bytes);

/* Run the randomized SVD (Section 2.1 steps 1-7 on the power matrix of
 * Section 2.2) on the device stream `stream`.
 *   A      device pointer, row-major m x n of the plan's dtype, leading
 *          dimension lda >= n (elements), naturally aligned.  Rows that are
 *          16-byte aligned (lda % 4 == 0 and A 16-byte aligned for FP32) take
 *          the vector-load path.
 *   ws     device workspace of at least device_ws_bytes, 256-byte aligned.
 *   U, S, V outputs (device): U m x k column-major (ldu >= m), S k doubles,
 *          V n x k column-major (ldv >= n).
 *   report optional (may be NULL).  If given, the call waits for the
 *          stream, fills the report and turns device-side outcomes into the
 *          status (RSVD_E_NUMERIC, RSVD_W_RANK_DEFICIENT); if NULL the call
 *          only enqueues work and returns RSVD_OK on successful launch. */
rsvd_status rsvd_factor(rsvd_plan_t plan, const void* A, int64_t lda, void* ws,
                        float* U, int64_t ldu, double* S, float* V, int64_t ldv,
                        void* stream, rsvd_report* report);

/* rsvd_factor for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation on a dense, device-resident A, with the workspace
 * taken from a static device array of RSVD_NOALLOC_WS_BYTES inside the
 * library (one per device, held until the process ends) instead of a caller
 * buffer.  The call allocates nothing: no device memory, no streams, no
 * events.  Both CholeskyQR passes of every basis run on `stream` (no side
 * stream), so results agree with rsvd_factor to rounding, not bit for bit.
 * No report: the call only enqueues work; device-side warnings (dropped
 * directions, non-finite values) are not returned.
 *   A, lda, U, ldu, S, V, ldv, stream   as for rsvd_factor.
 * Errors: RSVD_E_BUDGET when the plan's workspace exceeds
 * RSVD_NOALLOC_WS_BYTES (the message states both sizes); RSVD_E_UNSUPPORTED
 * for CSR/COO or host-resident plans; RSVD_E_INVALID_ARG as rsvd_factor.
 * All calls on one device share its array and it keeps the last call's
 * contents (every call initialises what it reads): calls that overlap on
 * one device, on any streams, race and must be serialised by the caller. */
#define RSVD_NOALLOC_WS_BYTES (64ull << 20)
rsvd_status rsvd_factor_noalloc(rsvd_plan_t plan, const void* A, int64_t lda, float* U,
                                int64_t ldu, double* S, float* V, int64_t ldv, void* stream);

/* Reverse-mode derivative (adjoint) of rsvd_factor.  The paper has no
 * derivative; this treats the l = k + p Ritz triplets (U_l, S_l, V_l) of the
 * randomized SVD as exact singular triplets of A and applies the real-SVD
 * adjoint: with cotangents gU (m x k), gS (k), gV (n x k) zero-padded to l
 * columns, F_ij = 1 / (s_j^2 - s_i^2) (i != j, FP64) and skew(X) = X - X^T,
 *   gA = U_l [(F o skew(U_l^T gU)) S_l + S_l (F o skew(V_l^T gV)) + diag(gS)] V_l^T
 *        + (I - U_l U_l^T) gU S_k^-1 V_k^T + U_k S_k^-1 gV^T (I - V_l V_l^T).
 * Ties |s_i^2 - s_j^2| <= 1e-12 s_1^2 set F_ij = 0 (status
 * RSVD_W_DEGENERATE); 1/s_i = 0 for s_i <= 1e-12 s_1.
 *   A       the same matrix passed to rsvd_factor (device, row-major, lda).
 *   gU, gV  device, column-major (ldgu >= m, ldgv >= n), FP32; NULL = zero.
 *   gS      device, k doubles; NULL = zero.
 *   gA      device output, row-major m x n FP32, ldga >= n.
 * The range basis is recomputed from the plan's seed (2q + 2 passes over A)
 * instead of being stored by the forward call.  The plan must have been made
 * with RSVD_FLAG_BACKWARD (else RSVD_E_INVALID_ARG).  `report` as in
 * rsvd_factor. */
rsvd_status rsvd_backward(rsvd_plan_t plan, const void* A, int64_t lda, const float* gU,
                          int64_t ldgu, const double* gS, const float* gV, int64_t ldgv,
                          float* gA, int64_t ldga, void* ws, void* stream, rsvd_report* report);

/* Accuracy pass: *out (device, one double) = ||A - U diag(S) V^T||_F for the
 * first k columns, computed directly tile by tile (U S V^T rebuilt on the
 * matrix cores, differences squared and summed in FP64; no ||A||^2 - sum s^2
 * cancellation).  One more pass over A.  Uses the plan's workspace. */
rsvd_status rsvd_residual(rsvd_plan_t plan, const void* A, int64_t lda, const float* U, int64_t ldu,
                          const double* S, const float* V, int64_t ldv, double* out, void* ws,
                          void* stream);

/* Streams the plan uses beside the caller's compute stream (Section 3.5
 * overlaps copies with computation): copy_stream carries the host-to-device
 * tile copies of a host-resident A, side_stream the second CholeskyQR pass
 * of each basis, which runs beside the next product.  NULL (the default)
 * lets the plan create its own non-blocking stream of default priority when
 * first needed.  Streams given here stay owned by the caller, who keeps them
 * alive until the plan is destroyed or the streams are replaced.  Call it
 * between calls on the plan, never while one is running on another host
 * thread (the plan is not thread-safe).  Host only; RSVD_E_INVALID_ARG for a
 * NULL plan. */
rsvd_status rsvd_plan_set_streams(rsvd_plan_t plan, void* copy_stream, void* side_stream);

/* Free a plan (NULL is ignored). */
void rsvd_plan_destroy(rsvd_plan_t plan);

/* Static text of a status code. */
const char* rsvd_status_str(rsvd_status s);

/* Message of the last failing call on `plan` (NULL: last plan-less call or
 * last rsvd_plan failure).  Valid until the next call on that plan. */
const char* rsvd_last_error(rsvd_plan_t plan);

/* Library version, e.g. "rsvd-mi355x 0.1". */
const char* rsvd_version(void);

/* ---- inspection hooks (used by the parity tests) ------------------------ */

/* Tile descriptors of the plan's block-cyclic map over A (Sections 2.3, 3.1),
 * 12 int64 per tile in I-major order:
 *   I, J, row0, rows, col0, cols, owner_p, owner_q, local_I, local_J,
 *   local_row0, local_col0.
 * Writes min(cap, 12 * tiles) values to out (host memory) and the full count
 * of values to *n_out.  Host only. */
rsvd_status rsvd_tile_map(rsvd_plan_t plan, int64_t* out, size_t cap, size_t* n_out);

/* Order in which pass `pass_index` (0 = sketch, then alternating A^T and A
 * products, 2q+1 = projection) visits the tiles, as linear indices
 * I * tiles_n + J: even passes row-major forward, odd passes column-major
 * backward (each pass starts on the tile the previous one ended on).
 * Host only; semantics of cap/n_out as in rsvd_tile_map. */
rsvd_status rsvd_visit_order(rsvd_plan_t plan, int64_t pass_index, int64_t* out, size_t cap,
                             size_t* n_out);

/* Raw Philox-4x32-10 words of the Gaussian test matrix (Section 2.1, step 1):
 * for rows j in [row0, row0 + rows) and column blocks b in [0, blocks) writes
 * the four 32-bit words of counter (b, j mod 2^32, j / 2^32, stream) under key
 * (seed mod 2^32, seed / 2^32) to out[((j - row0) * blocks + b) * 4 + w]
 * (device memory, rows * blocks * 4 uint32).  Asynchronous on `stream`. */
rsvd_status rsvd_philox_raw(uint64_t seed, uint32_t stream_id, int64_t row0, int64_t rows,
                            int64_t blocks, uint32_t* out, void* stream);

/* Gaussian test matrix O (n x l) rows [row0, row0 + rows), entry (j, c) from
 * Philox words -> uniforms (x + 1/2) 2^-32 -> Box-Muller in FP64, written as
 * FP64 (dtype RSVD_F64) or FP32 (RSVD_F32) into out[(j - row0) * ldo + c]
 * (device, row-major, ldo >= l).  Asynchronous on `stream`. */
rsvd_status rsvd_omega(uint64_t seed, int64_t n, int64_t l, int64_t row0, int64_t rows,
                       int32_t dtype, void* out, int64_t ldo, void* stream);


/* Sparse A (Section 2.1 on a sparse matrix; the paper's library takes sparse
 * input, Section 3.3): the plan's problem has format RSVD_CSR, dtype
 * RSVD_F32, loc RSVD_LOC_DEVICE, nnz set, and all products in FP32.
 *   rowptr  device int32[m + 1], rowptr[0] = 0, non-decreasing, rowptr[m] = nnz
 *   colind  device int32[nnz], column of each nonzero in [0, n) (any order
 *           within a row)
 *   values  device float[nnz]
 * A^T is applied through a CSC copy built in the workspace once per call by
 * a stable sort of the nonzeros by column, so results are bitwise
 * reproducible.  Malformed arrays are detected on the device: with a report
 * the call returns RSVD_E_INVALID_ARG (without one the outputs are undefined
 * but every kernel stays in bounds).  RSVD_E_BUDGET if the sort needs more
 * scratch than the plan reserved (the message states the bytes).  Other
 * arguments, outputs and the report are as for rsvd_factor. */
rsvd_status rsvd_factor_csr(rsvd_plan_t plan, const int32_t* rowptr, const int32_t* colind,
                            const float* values, void* ws, float* U, int64_t ldu, double* S,
                            float* V, int64_t ldv, void* stream, rsvd_report* report);

/* ---- per-pass persistence and resume (Section 3.8) ----------------------- */
/* The paper keeps every intermediate matrix with a header that places it in
 * the execution plan, so that an interrupted run recomputes only what was not
 * completed.  Here the state of a factorisation after each completed pass
 * over A is one FP32 panel plus a header:
 *   pass 1 (sketch A O, orthonormalised)           Q   m x lp   side 0
 *   pass 2t   (t = 1..q, A^T Q, orthonormalised)   Z   n x lp   side 1
 *   pass 2t+1 (t = 1..q, A Z, orthonormalised)     Q   m x lp   side 0
 *   pass 2q+2 (the projection B^T = A^T Q)   Q over B^T  (m + n) x lp  side 2
 * lp is the sketch width rounded up to 32 (columns l..lp-1 are zero).  Below
 * the state come lp more rows: the basis is kept as Q1 W (the second
 * CholeskyQR pass of a basis gives its right factor W while the next product
 * already runs on Q1), and these rows hold that factor (column c of the
 * lp x lp W under column c), zero unless `pending`.  The panel is
 * column-major with leading dimension `rows` (host memory, owned by the
 * caller).  All reductions of the library are deterministic, so a run
 * resumed from the checkpoint of pass t returns the same U, S and V, bit for
 * bit, as an uninterrupted run. */
#define RSVD_CKPT_MAGIC 0x31504B4344565352ull   /* "RSVDCKP1" little-endian */
typedef struct {
  uint64_t magic;          /* RSVD_CKPT_MAGIC                                 */
  int32_t version;         /* 1                                               */
  int32_t passes;          /* passes over A completed, 1 .. 2q + 2            */
  int64_t m, n, k, p, q;   /* the plan's problem                              */
  uint64_t seed;
  int32_t prec_sketch, prec_power, prec_project;
  int32_t flags;           /* the plan's RSVD_FLAG_CHOLQR1 bit                */
  int64_t rows, cols;      /* panel shape: rows x cols (cols = lp; rows
                              include the lp rows of the pending factor)    */
  int32_t side;            /* 0: m-side basis, 1: n-side panel                */
  int32_t dropped;         /* directions dropped so far                       */
  int32_t nonfinite;       /* non-finite values met so far                    */
  int32_t pending;         /* 1: the last lp rows hold a pending right factor */
  uint64_t panel_hash;     /* 64-bit hash of the panel bytes (see below)      */
} rsvd_checkpoint;

/* Bytes of the largest checkpoint panel of the plan: (m + n + lp) * lp * 4. */
rsvd_status rsvd_checkpoint_bytes(rsvd_plan_t plan, size_t* panel_bytes);

/* rsvd_factor (dense A, device- or host-resident) with persistence:
 *   resume, resume_panel  NULL: start from the beginning.  Otherwise a
 *          checkpoint of this plan (problem, seed, precisions and CHOLQR1 bit
 *          must match, the panel hash must match the bytes) and its panel
 *          (host): the run continues after pass resume->passes.
 *   ckpt, ckpt_panel      NULL: no saving.  Otherwise after every pass the
 *          call waits for the stream and copies the state into *ckpt and
 *          ckpt_panel (host, rsvd_checkpoint_bytes), so that they always hold
 *          the last completed pass.
 *   stop_after            0: run to the end.  1 .. 2q + 2: return
 *          RSVD_STOPPED once that many passes are complete (U, S, V are then
 *          not written); with ckpt the state of that pass is saved.
 * The panel hash is 64-bit FNV-1a over the panel's 32-bit words taken as
 * units (offset basis 0xcbf29ce484222325, prime 0x100000001b3).
 * RSVD_E_INVALID_ARG for a checkpoint of another problem, a pass out of
 * range, a shape that does not match its pass, or a hash mismatch (nothing
 * runs).  RSVD_E_UNSUPPORTED for RSVD_FLAG_AUTO_Q plans and CSR plans.
 * `report` as in rsvd_factor (not filled by a call that stops): stage times
 * of a resumed call cover only the passes it ran.  A call that resumes after
 * the projection runs no pass and leaves *ckpt untouched. */
rsvd_status rsvd_factor_resumable(rsvd_plan_t plan, const void* A, int64_t lda, void* ws,
                                  float* U, int64_t ldu, double* S, float* V, int64_t ldv,
                                  void* stream, rsvd_report* report,
                                  const rsvd_checkpoint* resume, const float* resume_panel,
                                  int32_t stop_after, rsvd_checkpoint* ckpt, float* ckpt_panel);

/* ---- single-step hooks: one step of rsvd_factor in isolation ------------- */
/* They run the same kernels as rsvd_factor on caller panels, using the plan's
 * workspace `ws` for staging.  Panels are column-major FP32 (element (i, c) at
 * P[i + c * ld]) with l = k + p columns.  Asynchronous on `stream`. */

/* Randomized SVD of a sparse A in coordinate (COO) form (Section 3.3: the
 * paper's sparse format, with 32- or 64-bit indices).  The plan's problem has
 * format RSVD_COO, dtype RSVD_F32, nnz entries, device location, FP32
 * products (as for CSR).
 *   rowind, colind  device arrays of nnz indices, int32 (index_bits 32) or
 *                   int64 (index_bits 64); any order; repeated (row, col)
 *                   pairs add up.
 *   values          device, nnz FP32.
 * The entries are ordered by row with a stable radix sort into CSR arrays in
 * the workspace (within a row they keep their input order, so a row-sorted
 * input gives exactly the CSR path's result), and the call continues as
 * rsvd_factor_csr.  An index outside [0, m) x [0, n) returns
 * RSVD_E_INVALID_ARG once `report` is given (every kernel stays in bounds).
 * Other arguments and statuses as rsvd_factor_csr. */
rsvd_status rsvd_factor_coo(rsvd_plan_t plan, const void* rowind, const void* colind,
                            int32_t index_bits, const float* values, void* ws, float* U,
                            int64_t ldu, double* S, float* V, int64_t ldv, void* stream,
                            rsvd_report* report);

/* Sparse product with the plan's CSR matrix (arrays as in rsvd_factor_csr):
 * op 0: out (m x l) = A X with X n x l; op 1: out (n x l) = A^T X with X
 * m x l.  Panels column-major FP32.  Synchronises `stream`; returns
 * RSVD_E_INVALID_ARG for malformed CSR arrays. */
rsvd_status rsvd_step_spmm(rsvd_plan_t plan, int32_t op, const int32_t* rowptr,
                           const int32_t* colind, const float* values, const float* X,
                           int64_t ldx, float* out, int64_t ldo, void* ws, void* stream);

/* Block-wise product with A over the plan's tiles (Section 2.3, Eq. (3)):
 * op 0: out (m x l, ldo >= m) = A X with X n x l (ldx >= n);
 * op 1: out (n x l, ldo >= n) = A^T X with X m x l (ldx >= m).
 * A as in rsvd_factor (dtype of the plan; FP64 is cast to FP32 first). */
rsvd_status rsvd_step_product(rsvd_plan_t plan, int32_t op, const void* A, int64_t lda,
                              const float* X, int64_t ldx, float* out, int64_t ldo, void* ws,
                              void* stream);

/* Orthonormal basis of the columns of Y (Section 2.1, steps 3-4) by
 * CholeskyQR twice (FP64 Gram and Cholesky), dependent directions dropped as
 * zero columns.  side 0: Y has m rows, side 1: n rows.  Q may alias Y. */
rsvd_status rsvd_step_orth(rsvd_plan_t plan, int32_t side, const float* Y, int64_t ldy, float* Q,
                           int64_t ldq, void* ws, void* stream);

/* Gram matrix G = Y^T Y (l x l, FP64, row-major at G[a * l + c]) of a panel
 * with m rows (side 0) or n rows (side 1): FP64 products of the FP32
 * entries summed in FP64 (the CholeskyQR and SVD0-preparation step). */
rsvd_status rsvd_step_gram(rsvd_plan_t plan, int32_t side, const float* Y, int64_t ldy, double* G,
                           void* ws, void* stream);

/* SVD of the small B = Bt^T (Section 2.1, step 6) from Bt (n x l, ldb >= n):
 * C = B B^T in FP64, cyclic Jacobi eigensolver, sorted descending.  Writes
 * the l singular values to sig (device, FP64) and U_B (l x l, FP64,
 * row-major: U_B(a, c) at ub[a * l + c], column c belongs to sig[c]). */
rsvd_status rsvd_step_small_svd(rsvd_plan_t plan, const float* Bt, int64_t ldb, double* sig,
                                double* ub, void* ws, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RSVD_H */
