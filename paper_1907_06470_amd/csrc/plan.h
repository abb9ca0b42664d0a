// Host-only planner of the randomized SVD: argument validation, block-cyclic
// tile maps, kernel splits and the device workspace layout.  No HIP calls:
// everything here is decided before any device work starts (Section 3.4 of
// the paper: memory needs of dense products are known exactly beforehand).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/rsvd.h"

namespace rsvd {

constexpr int64_t kPanelAlign = 256;   // panel leading dimensions (elements)
constexpr int64_t kColAlign = 32;      // sketch width is padded to this
constexpr int64_t kWideMax = 512;      // largest padded sketch width
constexpr int64_t kSliceMax = 192;     // widest panel slice of one product launch
// Column slices of a panel of width lp for kernels that take at most
// kSliceMax columns: as few as possible, of equal width (a multiple of 32);
// slice_width() is the width of all but possibly the last.
inline int64_t slice_count(int64_t lp) { return (lp + kSliceMax - 1) / kSliceMax; }
inline int64_t slice_width(int64_t lp) {
  const int64_t ns = slice_count(lp);
  return ((lp + ns - 1) / ns + 31) / 32 * 32;
}
constexpr int kGramBlock = 64;         // Gram output block edge
constexpr int kJacobiMaxSweeps = 40;
constexpr int kBjMaxSweeps = 20;     // sweeps enqueued by the block Jacobi of wide sketches
constexpr int64_t kPanelFp8Chunks = 32;   // row chunks per column of the panel FP8 conversion
constexpr int kStatusWords = 64;
constexpr int64_t kSpmmChunk = 2048;   // nonzeros per wave in the sparse products

// Device status word indices (int32 array in the workspace).
enum StatusWord {
  kStDropped = 0,      // directions dropped by the Cholesky step (sum over calls)
  kStNonFinite = 1,    // NaN/Inf pivots met
  kStSweeps = 2,       // Jacobi sweeps of the small eigensolver
  kStRounds = 3,       // Jacobi rotation rounds logged
  kStRankSmall = 4,    // zero singular values in the small SVD
  kStTies = 5,         // equal singular-value pairs met by the adjoint
  kStBadSparse = 6,    // malformed CSR input (pointers or column indices)
  kStTriOk = 7,        // 1 when the tridiagonal eigensolver's small SVD passed its checks
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

struct Workspace {
  // byte offsets into the device workspace
  size_t Xop, Mop;        // operand panels (n x lp, m x lp)
  size_t M0, M1;          // FP32 m-side panels (column-major, ld = ldm)
  size_t N0, N1;          // FP32 n-side panels (ld = ldn)
  size_t part;            // split-K partial products
  size_t gpart;           // Gram partial blocks (FP64)
  size_t G;               // lp x lp FP64 Gram
  size_t L;               // lp x lp FP64 Cholesky factor
  size_t W;               // lp x lp FP32 right factor applied to panels
  size_t W2;              // lp x lp FP32 second right factor
  size_t gpart2, G2;      // Gram partials and Gram of the deferred second CholeskyQR pass
  size_t Tc;              // lp x lp FP64 scratch of W^T G W
  size_t tri;             // tridiagonal eigensolver scratch (FP64, widths <= 128)
  size_t Wpm, Wpn;        // lp x lp FP32 pending right factors of the m- and n-side bases
  size_t Wc;              // lp x lp FP32 product of a pending factor and a first-pass factor
  size_t Ev;              // lp x lp FP64 eigenvectors
  size_t Mj;              // lp x lp FP64 columns of the block Jacobi (widths > 128)
  size_t bjctl;           // kBjMaxSweeps int32 sweep flags of the block Jacobi
  size_t Ls2;             // lp x lp FP64 Cholesky scratch of the side stream (widths > 192)
  size_t lam;             // lp FP64 eigenvalues / singular values
  size_t order;           // lp int32 sort order
  size_t signs;           // k int32 sign-fix argmax
  size_t status;          // kStatusWords int32
  size_t prevS;           // automatic q: previous k singular values + change
  size_t Acast;           // FP32 copy of an FP64 A
  size_t A16;             // BF16 copy of A (when a product runs in BF16)
  size_t Xop16, Mop16;    // BF16 copies of the operand panels
  size_t A8, A8T, sA8;    // FP8 copies of A and A^T, 64 x 64 block scales (FP32)
  size_t Xop8, Mop8;      // FP8 copies of the operand panels
  size_t sX8, sM8;        // their per-column scales
  size_t f8part;          // chunk maxima of the panel FP8 conversion
  // backward (RSVD_FLAG_BACKWARD)
  size_t Pcat, Rcat;      // outer-product factors (ldm x R, ldn x R), R = lp + 2 kp
  size_t gUp, gVp;        // imported cotangents (ldm x kp, ldn x kp)
  size_t Ju, Jv;          // lp x kp FP64
  size_t Sl;              // lp FP64 Ritz values
  size_t coreT, JuW, JvW, sinv;
  size_t slots;           // host-resident A: S tile slots of slot_bytes each
  // CSR input: CSC copy, sort buffers, row-major operand/result, chunk carries
  size_t colptr, rowind, cval, keys0, keys1, pay0, pay1, sort_temp;
  // head columns of the CSC copy: sampled column counts, column -> head index,
  // head index -> column, and the rank sort's buffers
  size_t colcnt, headof, headcol, rk0, rk1, rv0, rv1;
  size_t coo_ptr, coo_col, coo_val;   // CSR arrays built from COO input
  size_t Xr, Yr, carry, first;
  size_t total;
};

struct Plan {
  rsvd_problem prob{};
  rsvd_options opt{};
  int64_t l = 0, lp = 0;        // sketch width, padded width
  int64_t tm = 0, tn = 0;       // tile sizes
  int64_t TI = 0, TJ = 0;       // tile counts (rows, cols)
  int64_t ldm = 0, ldn = 0;     // panel leading dimensions
  int64_t ldac = 0;             // leading dimension of the FP32 cast of A
  int64_t lda16 = 0;            // leading dimension of the BF16 copy of A
  bool any_bf16 = false;        // some product runs in BF16
  bool any_fp8 = false;         // some product runs in FP8 (e4m3)
  int64_t lda8 = 0, ldat8 = 0;  // leading dimensions of the FP8 copies of A and A^T
  bool any_f32 = false;         // some product runs in FP32
  int64_t gram_rows = 0;        // rows per Gram chunk
  int64_t gram_chunks = 0;      // max chunks over the m- and n-side panels
  int64_t kp = 0;               // k rounded up to 32 (backward)
  int64_t rcat = 0;             // columns of the outer-product factors
  bool backward = false;
  bool host = false;            // A in pinned host memory, streamed tile by tile
  bool csr = false;             // A given as CSR (int32 indices, FP32 values), or as COO
  bool coo = false;             // A given as COO (converted to CSR in the workspace)
  bool auto_q = false;          // choose q <= prob.q (RSVD_FLAG_AUTO_Q)
  double q_tol = 0.0;
  int64_t chunks = 0;           // nonzero chunks of the sparse products
  int64_t csc_parts = 1;        // row blocks of the CSC copy (A^T Q gathers within one)
  int64_t head_k = 0;           // head columns of the CSC copy (their own small row blocks)
  int64_t head_parts = 0;       // row blocks of the head columns
  size_t sort_temp = 0;         // scratch reserved for the CSC sort
  int64_t slots = 0;            // HBM tile slots (host-resident A)
  int64_t slot_ld = 0;          // leading dimension (elements) of a slot
  size_t slot_bytes = 0;
  int64_t elem = 4;             // bytes per element of A
  Workspace ws{};
  std::string last_error;
  void* hip_events = nullptr;   // created lazily by the driver
  void* streamer = nullptr;     // copy stream, slot events, slot contents (host A)
  void* side = nullptr;         // side stream + events of the deferred CholeskyQR passes
  void* user_copy = nullptr;    // caller-owned copy / side streams (rsvd_plan_set_streams)
  void* user_side = nullptr;
};

// Fill `plan` or return an error status with plan.last_error set.
rsvd_status make_plan(const rsvd_problem& prob, const rsvd_options* opt, Plan& plan);

// Gram chunking of a panel with `rows` rows.
int64_t gram_chunks_for(const Plan& p, int64_t rows);
inline int64_t gram_nb(const Plan& p) { return ceil_div(p.lp, kGramBlock); }
inline int64_t gram_pairs(const Plan& p) { int64_t nb = gram_nb(p); return nb * (nb + 1) / 2; }
// Lower-triangle Gram (widths up to 192): at most kGramTriChunks row chunks
// of a multiple of 4 rows, one 16 x 16 FP64 partial tile per chunk and tile.
constexpr int64_t kGramTriChunks = 256;
inline bool gram_tri_fits(int64_t lp) { return lp <= 192 && lp % 32 == 0; }
inline int64_t gram_tri_chunk_rows(int64_t rows) {
  return round_up(ceil_div(rows < 1 ? 1 : rows, kGramTriChunks), 4);
}
// Scratch of the global-memory Cholesky (k_chol.hip): the lp x lp square, then
// X_kk and L_kk of up to kWideMax / 16 diagonal blocks and the original
// diagonal.
inline int64_t chol_gm_scratch_doubles(int64_t lp) {
  return lp * lp + (kWideMax / 16) * 16 * (2 * 16 + 1);
}
// Wider panels: the same partial tiles, formed per pair of 128-column slices.
inline bool gram_grp_fits(int64_t lp) { return lp > 192 && lp <= kWideMax && lp % 32 == 0; }
inline size_t gram_tri_bytes(int64_t lp) {
  const int64_t nbk = lp / 16;
  return (size_t)kGramTriChunks * (size_t)(nbk * (nbk + 1) / 2) * 256 * 8;
}

rsvd_options default_options();

// sparse products: nonzero chunks and the scratch reserved for the CSC sort
// (host-side mirrors of the constants in k_sparse.hip)
int64_t spmm_chunk_count(int64_t nnz);
// row blocks of the CSC copy (for the columns outside the head set): the
// rows of Q one block's columns gather from stay within kCscSliceBytes.
// Smaller blocks keep more of those gathers in the last-level cache but add
// a partial result row per (block, column) that is written and read back;
// 1 GiB slices (3 blocks for 2e6 x 352) measured best on a 1e8-entry Zipf
// matrix, against 16 blocks of 128 MiB
int64_t csc_part_count(int64_t m, int64_t n, int64_t lp);
// Head columns of A^T products: the kHeadCols columns with the most nonzeros
// (counted on every kHeadSampleStride-th row) get compressed rows of their
// own per block of kHeadPartRows rows of A; a product stages such a block's
// panel rows in LDS once and runs every head column's entries of the block
// against it.  The other columns keep the csc_part_count row blocks.  256
// rows (68 KB of LDS, two workgroups a compute unit) measured best on a
// 1e8-entry Zipf matrix: 512 rows hide less latency, 128 rows double the
// block results to add.
constexpr int64_t kHeadCols = 512;
constexpr int64_t kHeadPartRows = 256;
constexpr int64_t kHeadSampleStride = 16;
size_t csc_sort_scratch(int64_t nnz);
// Tridiagonal eigensolver of the small SVD (widths up to kTriMaxLp): FP64
// scratch of six kTriMaxLp x kTriMaxLp arrays (the LU factors of the
// inverse iterations and their solutions).
constexpr int64_t kTriMaxLp = 128;
constexpr int64_t kTriScratchDoubles = 6 * kTriMaxLp * kTriMaxLp;

// the small SVD runs the tridiagonal eigensolver first (widths <= kTriMaxLp
// unless RSVD_FLAG_JACOBI_ONLY)
inline bool small_svd_tridiagonal(const Plan& p) {
  return p.lp <= kTriMaxLp && !(p.opt.flags & RSVD_FLAG_JACOBI_ONLY);
}

}  // namespace rsvd
