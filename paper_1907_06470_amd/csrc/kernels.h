// Host-side launchers of the gfx950 kernels.  Every launcher checks nothing
// but the launch itself; shapes are validated by the planner and the driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsvd {

inline int64_t ceil_div_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

// --- Gaussian test matrix (k_philox.hip) ---
hipError_t launch_philox_raw(uint64_t seed, uint32_t stream_id, int64_t row0, int64_t rows,
                             int64_t blocks, uint32_t* out, hipStream_t s);
hipError_t launch_omega_rows(uint64_t seed, int64_t l, int64_t row0, int64_t rows, bool f64,
                             void* out, int64_t ldo, hipStream_t s);
hipError_t launch_omega_panel(uint64_t seed, int64_t n, int64_t l, int64_t lp, float* X,
                              int64_t ld, hipStream_t s);

// --- products with A (k_gemm_f32.hip) ---
// Y(:, 0:lp) (+ partial J at Y + J * part_stride) = A(:, tile J) * X(tile J, 0:lp)
hipError_t launch_nn_f32(const float* A, int64_t lda, int64_t m, int64_t n, int64_t tn, int64_t TJ,
                         const float* X, int64_t ldx, int64_t lp, float* Y, int64_t ldy,
                         int64_t part_stride, hipStream_t s);
// Z(:, 0:lp) (+ partial I) = A(tile I, :)^T * Q(tile I, 0:lp)
hipError_t launch_tn_f32(const float* A, int64_t lda, int64_t m, int64_t n, int64_t tm, int64_t TI,
                         const float* Q, int64_t ldq, int64_t lp, float* Z, int64_t ldz,
                         int64_t part_stride, hipStream_t s);
// out = sum over S partials (fixed order), float4 granularity, count floats
hipError_t launch_reduce_parts(const float* part, int64_t stride, int64_t S, float* out,
                               int64_t count, hipStream_t s);
hipError_t launch_panel_copy(const float* src, int64_t lds, int64_t rows, int64_t cols, float* dst,
                             int64_t ldd, int64_t dst_rows, int64_t dst_cols, hipStream_t s);
hipError_t launch_cast_f64_f32(const double* A, int64_t lda, int64_t m, int64_t n, float* out,
                               int64_t ldo, hipStream_t s);

// --- BF16 products (k_gemm_bf16.hip) ---
hipError_t launch_nn_bf16(const uint16_t* A, int64_t lda, int64_t m, int64_t n, int64_t tn,
                          int64_t TJ, const uint16_t* X, int64_t ldx, int64_t lp, float* Y,
                          int64_t ldy, int64_t part_stride, hipStream_t s);
// The BF16 sketch product straight from the FP32 A (16-byte aligned rows,
// panel width 128), writing the BF16 copy A16 on the way.
hipError_t launch_nn_bf16_cast(const float* A32, int64_t lda, int64_t m, int64_t n, int64_t tn,
                               int64_t TJ, uint16_t* A16, int64_t lda16, const uint16_t* X,
                               int64_t ldx, int64_t lp, float* Y, int64_t ldy,
                               int64_t part_stride, hipStream_t s);
hipError_t launch_tn_bf16(const uint16_t* A, int64_t lda, int64_t m, int64_t n, int64_t tm,
                          int64_t TI, const uint16_t* Q, int64_t ldq, int64_t lp, float* Z,
                          int64_t ldz, int64_t part_stride, hipStream_t s);
hipError_t launch_cast_to_bf16(const void* A, bool f64, int64_t lda, int64_t m, int64_t n,
                               uint16_t* out, int64_t ldo, hipStream_t s);
hipError_t launch_panel_to_bf16(const float* P, uint16_t* P16, int64_t count, hipStream_t s);

// --- FP8 (e4m3) form (k_gemm_fp8.hip) ---
// A8 (m x lda8) and A8T (n x ldat8) FP8 copies of A with one power-of-two
// scale per 64 x 64 block: scale[(i / 64) * ceil(n / 64) + j / 64].
int64_t fp8_scale_blocks(int64_t rows, int64_t cols);
hipError_t launch_cast_fp8(const void* A, bool f64, int64_t lda, int64_t m, int64_t n, uint8_t* A8,
                           int64_t lda8, uint8_t* A8T, int64_t ldat8, float* scale, hipStream_t s);
// P8 = FP8 copy of an FP32 column-major panel (same ld), scale[c] per column.
// part (2 * lp * kPanelFp8Chunks floats, plan.h; or nullptr for the one-pass
// kernel): chunk maxima, so the panel is read by lp x kPanelFp8Chunks
// workgroups.
hipError_t launch_panel_to_fp8(const float* P, int64_t ld, int64_t rows, int64_t lp, uint8_t* P8,
                               float* scale, float* part, hipStream_t s);
// Y (+ partial per reduction tile of tk) = A8 X8 with block scales sA and
// column scales sx (see k_gemm_fp8.hip for the layouts).
hipError_t launch_nn_fp8(const uint8_t* A8, int64_t lda8, int64_t rows, int64_t kdim, int64_t tk,
                         int64_t TK, const float* sA, int64_t sc_r, int64_t sc_k,
                         const uint8_t* X8, int64_t ldx8, const float* sx, int64_t lp, float* Y,
                         int64_t ldy, int64_t part_stride, hipStream_t s);

// --- sparse CSR products (k_sparse.hip) ---
// status[kStBadSparse] = 1 when the CSR arrays are malformed
hipError_t launch_csr_check(const int32_t* ptr, const int32_t* idx, int64_t rows, int64_t cols,
                            int64_t nnz, int32_t* status, hipStream_t s);
// CSC (= CSR of A^T) of each of `parts` row blocks of A (ceil(m / parts) rows
// each), stored one after the other: compressed row b n + j is column j of
// block b.  A stable radix sort of the nonzeros by (block, column) keeps each
// column's row order.  On a scratch shortfall returns hipErrorOutOfMemory with
// the bytes needed in *need.
// Head columns of the CSC copy (plan.h, kHeadCols): counts on sampled rows
// (cnt, n entries), columns ranked by count (rk*, rv*: n-entry sort buffers),
// headof[col] = rank (< head_k) or -1, headcol[rank] = col.
hipError_t launch_head_select(const int32_t* rowptr, const int32_t* colind, int64_t m, int64_t n,
                              int64_t nnz, int64_t head_k, uint32_t* cnt, int32_t* headof,
                              int32_t* headcol, uint32_t* rk0, uint32_t* rk1, int32_t* rv0,
                              int32_t* rv1, void* temp, size_t temp_bytes, size_t* need,
                              hipStream_t s);
// CSC copy with `parts` row blocks for the other columns and, when headof is
// given, head_parts row blocks for the head_k head columns (compressed rows
// parts n + b K + h after the others').
hipError_t launch_build_csc(const int32_t* rowptr, const int32_t* colind, const float* values,
                            int64_t m, int64_t n, int64_t nnz, int64_t parts,
                            const int32_t* headof, int64_t head_k, int64_t head_parts,
                            uint32_t* keys0, uint32_t* keys1, uint64_t* pay0, uint64_t* pay1,
                            void* temp, size_t temp_bytes, int32_t* colptr, int32_t* rowind,
                            float* cval, size_t* need, hipStream_t s);
hipError_t launch_coo_to_csr(const void* rowind, const void* colind, int index_bits,
                             const float* values, int64_t m, int64_t n, int64_t nnz,
                             uint32_t* keys0, uint32_t* keys1, uint64_t* pay0, uint64_t* pay1,
                             void* temp, size_t temp_bytes, int32_t* rowptr, int32_t* col,
                             float* val, int32_t* status, size_t* need, hipStream_t s);
// out (column-major, ldo rows) = S X for S (rows x xrows) in compressed-row
// form and X column-major (ldx); with parts > 1 the compressed rows are parts
// blocks of `rows` rows, and row r of out sums row r of every block in block
// order.  Xr, Yr, carry, first are scratch.
// headcol / head_k / head_parts: the head columns of a CSC copy built with
// them (their block results are added into out rows headcol[h]).
hipError_t launch_spmm(const int32_t* ptr, const int32_t* idx, const float* val, int64_t rows,
                       int64_t parts, int64_t nnz, const float* X, int64_t ldx, int64_t xrows,
                       int64_t lp, float* Xr, float* Yr, float* carry, int32_t* first,
                       float* out, int64_t ldo, hipStream_t s, const int32_t* headcol = nullptr,
                       int64_t head_k = 0, int64_t head_parts = 0);

// --- small dense FP64 steps (k_small.hip) ---
hipError_t launch_gram(const float* P, int64_t ld, int64_t rows, int64_t lp, int64_t chunk_rows,
                       int64_t chunks, double* gpart, double* G, hipStream_t s);
// W = L^-T (FP32, upper triangular) with G = L L^T; dropped directions zero.
// scratch: lp x lp FP64, distinct from G, used for widths above 192 only.
hipError_t launch_chol_inv(const double* G, int64_t lp, int64_t l, float* W, int32_t* status,
                           double tau, double* scratch, hipStream_t s);
// out(:, 0:ncols) = P(:, 0:kdim) * W(0:kdim, 0:ncols); W row-major with ldw;
// `tri`: W upper triangular (skip zero blocks).  Rows [rows, ld) written as 0.
// out = W^T G W (G FP64 symmetric, W FP32, both lp x lp row-major; T is
// lp x lp FP64 scratch distinct from G and out; out may alias G), FP64
// accumulation.
hipError_t launch_congruence(const double* G, const float* W, double* T, double* out, int64_t lp,
                             hipStream_t s);
// C = A B (lp x lp row-major FP32), FP64 accumulation.
hipError_t launch_lp_product(const float* A, const float* B, float* C, int64_t lp, hipStream_t s);
hipError_t launch_apply(const float* P, int64_t ldp, int64_t rows, int64_t kdim, const float* W,
                        int64_t ldw, int64_t lp, int64_t ncols, bool tri, float* out,
                        int64_t ldo, int64_t out_rows_total, hipStream_t s);
// Cholesky factor (L, FP64 row-major, when L != nullptr) or W = L^-T (when
// W != nullptr) of G for lp <= 128 (k_chol.hip); the two launchers above
// route there when the width fits.
bool chol16_fits(int64_t lp);
hipError_t launch_chol16(const double* G, int64_t lp, int64_t l, float* W, double* L,
                         int32_t* status, double tau, hipStream_t s,
                         const int32_t* skip = nullptr);
// W = L^-T for 128 < lp <= 192 (k_chol.hip, lower tiles packed in LDS).
bool chol_tp_fits(int64_t lp);
hipError_t launch_chol_tp(const double* G, int64_t lp, int64_t l, float* W, int32_t* status,
                          double tau, hipStream_t s);
// Cholesky factor (into L = S; 128 < lp <= 512) or W = L^-T (192 < lp <= 512),
// the square in the global scratch S (chol_gm_scratch_doubles(lp) FP64, plan.h;
// not aliasing G; L is its leading lp x lp; k_chol.hip).
bool chol_gm_fits(int64_t lp);
hipError_t launch_chol_gm(const double* G, int64_t lp, int64_t l, double* S, float* W, double* L,
                          int32_t* status, double tau, hipStream_t s);
// Small SVD of sketches wider than 128 (lp <= 512): block one-sided Jacobi on the
// Cholesky factor L (FP64 row-major lp x lp) of C; M (lp x lp FP64) and ctl
// (kBjMaxSweeps int32) are scratch.  Writes lam (|m_c|^2) and Ev (row-major)
// as launch_ojacobi does (k_bjacobi.hip).
bool bjacobi_fits(int64_t lp);
hipError_t launch_bjacobi(const double* L, int64_t lp, int64_t l, double* M, int32_t* ctl,
                          double* lam, double* Ev, int32_t* status, double tol, hipStream_t s);
// Automatic q: prev[k] = max_i<k |S_i - prev_i| / S_i (+inf if first), prev = S.
hipError_t launch_ritz_delta(const double* S, int64_t k, bool first, double* prev, hipStream_t s);
// Small SVD through the Cholesky factor of C and one-sided Jacobi in one
// workgroup (lp <= 128); wider sketches take launch_bjacobi.
bool small_svd_one_sided(int64_t lp);
// L (lp x lp FP64 row-major, distinct from G) with G = L L^T.
// skip (optional): a device word; the kernels return at once when it is
// nonzero (the tridiagonal eigensolver's result passed its checks).
hipError_t launch_chol_factor(const double* G, int64_t lp, int64_t l, double* L, int32_t* status,
                              double tau, hipStream_t s, const int32_t* skip = nullptr);
hipError_t launch_ojacobi(const double* L, int64_t lp, int64_t l, double* lam, double* Ev,
                          int32_t* status, double tol, int max_sweeps, hipStream_t s,
                          const int32_t* skip = nullptr);
// Small SVD through the tridiagonal form of C (k_trieig.hip), lp <=
// kTriMaxLp: writes lam and Ev as launch_ojacobi does and status[kStTriOk]
// (1 when the orthogonality and residual checks held).  scratch:
// kTriScratchDoubles FP64.
hipError_t launch_tri_eig(const double* G, int64_t lp, int64_t l, double* lam, double* Ev,
                          double* scratch, int32_t* status, hipStream_t s);
// sort eigenvalues, form S (k values), Wu = Ev(:, order(0:k)), Wv = Wu / sigma
hipError_t launch_finish_small(const double* lam, const double* Ev, int64_t lp, int64_t l,
                               int64_t k, double* S, float* Wu, float* Wv, int32_t* order,
                               int32_t* status, hipStream_t s);
hipError_t launch_sign_fix(float* U, int64_t ldu, int64_t m, float* V, int64_t ldv, int64_t n,
                           int64_t k, int32_t* work, hipStream_t s);
hipError_t launch_gather_cols(const double* Ev, int64_t lp, int64_t l, const int32_t* order,
                              double* out, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s);

// --- adjoint (k_adjoint.hip) and accuracy pass (k_resid.hip) ---
hipError_t launch_xgram(const float* P, int64_t ldp, int64_t cp, const float* R, int64_t ldr,
                        int64_t cr, int64_t rows, int64_t chunk_rows, int64_t chunks,
                        double* gpart, double* C, hipStream_t s);
hipError_t launch_adj_core(const double* Sl, int64_t lp, int64_t l, int64_t k, int64_t kp,
                           const double* Ju, const double* Jv, const double* gS, float* coreT,
                           float* JuW, float* JvW, float* sinv, int32_t* status, hipStream_t s);
hipError_t launch_colscale(const float* x, int64_t ldx, const float* y, int64_t ldy,
                           const float* sc, int64_t rows, int64_t cols, float* out, int64_t ldo,
                           int64_t out_rows, hipStream_t s);
hipError_t launch_outer(const float* P, int64_t ldp, const float* R, int64_t ldr, int64_t K,
                        int64_t m, int64_t n, float* gA, int64_t ldga, hipStream_t s);
int64_t residual_partials(int64_t m, int64_t n);
hipError_t launch_residual(const void* A, bool f64, int64_t lda, int64_t m, int64_t n,
                           const float* U, int64_t ldu, const double* S, const float* V,
                           int64_t ldv, int64_t k, double* partial, double* out, hipStream_t s);

}  // namespace rsvd
