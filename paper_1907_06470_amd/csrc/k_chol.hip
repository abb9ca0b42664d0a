// Cholesky factor and triangular inverse of the l x l FP64 Gram matrix of a
// CholeskyQR pass (steps 1-3 of the orthonormalisation: G = Y^T Y = L L^T,
// Q = Y L^-T), in one workgroup: k_chol16 for sketch widths up to 128 (below),
// k_chol_tp for widths up to 192 (the same steps on the lower tiles only,
// further down), and for widths up to 512 the same steps on a square in
// global memory over several launches (at the end).
//
// The whole matrix sits in LDS as a 128 x 128 square of doubles whose rows are
// XOR-swizzled in groups of 16 (element (i, c) at i * 128 + (c ^ (i & 15))),
// so that row-wise and column-wise reads of a 16 x 16 tile are both free of
// bank conflicts.  The factorisation is right-looking over 16-column panels:
//   * one wave factors the diagonal block in registers (lane = row; the
//     pivot and the scaled column are broadcast with readlane) and forms its
//     inverse X_kk by forward substitution;
//   * the panel below is L_Ik = A_Ik X_kk^T and the trailing update
//     A_IJ -= L_Ik L_Jk^T, both as 16 x 16 tiles on the FP64 matrix cores;
//   * the wave that factors the next diagonal block first applies that
//     block's own trailing update, so its factorisation overlaps the rest of
//     the update (two workgroup barriers per panel).
// The inverse X = L^-1 proceeds by block rows, X_IJ = -X_II sum_K L_IK
// X_KJ, with the partial sum kept in the accumulator registers and fed back as
// the B operand of the product with X_II.  Block row k needs only block
// columns < k of L and block rows < k of X, so the waves that are not
// factoring make it during panel step k; only the last row follows the
// factorisation.  The off-diagonal blocks of X are
// stored transposed in the upper triangle, which is exactly the layout of the
// upper-triangular W = X^T the apply kernel consumes.
//
// A pivot a_jj <= tau * G_jj (or a non-positive original diagonal) drops the
// direction: column j of L and row and column j of X become zero, so the
// matching column of Q is zero; non-finite pivots are counted separately.
#include <algorithm>

#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace rsvd {

namespace {

constexpr int kB = 16;                  // panel / tile edge
constexpr int kSq = 128;                // square held in LDS
constexpr int kNbMax = kSq / kB;
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ inline int sq(int i, int c) { return i * kSq + (c ^ (i & 15)); }
__device__ inline int xq(int i, int c) { return i * kB + (c ^ i); }   // inside one 16 x 16 block

__device__ inline f64x4 mma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
}

// Register part of a diagonal block (whole wave; every row of 16 lanes holds
// the block, lane r of a row holding row r in d, entries right of the
// diagonal ignored, and od = the original diagonal entry of row r).  Values of
// other rows of the block travel by DPP broadcast inside the 16-lane row, so
// the wave needs no LDS round trip and no scalar registers between steps.  On
// return d[p] (p <= r) is row r of L_kk, dv = 1 / L_kk(r, r) (0 for a dropped
// direction) and x[i] = X_kk(i, r), column r of X_kk = L_kk^-1.
__device__ inline void diag_factor(double (&d)[kB], double od, int g0, int l, double tau,
                                   int& ndrop, int& nbad, double& dv, double (&x)[kB]) {
  const int r = threadIdx.x & 15;
  dv = 0.0;
#pragma unroll
  for (int j = 0; j < kB; ++j) {
    const double a = row16_bcast(d[j], j);
    const double o = row16_bcast(od, j);
    const bool bad = !is_finite_d(a);
    const bool ok = !bad && o > 0.0 && a > tau * o;
    const double rs = fast_rsq(ok ? a : 1.0);
    const double inv = ok ? rs : 0.0;
    d[j] = (r == j) ? a * inv : d[j] * inv;
    dv = (r == j) ? inv : dv;
    const int live = g0 + j < l ? 1 : 0;     // padding columns are not counted
    nbad += bad ? live : 0;
    ndrop += (!bad && !ok) ? live : 0;
    // rank-1 update of the columns to the right (rows above the diagonal
    // collect values that are never read)
#pragma unroll
    for (int c = j + 1; c < kB; ++c) d[c] -= d[j] * row16_bcast(d[j], c);
  }
  // lane r: column r of X_kk = L_kk^-1 by forward substitution, column
  // oriented: once x_p is known it leaves every later row at once (the
  // subtractions of each row keep the order p = 0, 1, ...)
#pragma unroll
  for (int i = 0; i < kB; ++i) x[i] = (i == r) ? 1.0 : 0.0;
#pragma unroll
  for (int p = 0; p < kB; ++p) {
    x[p] *= row16_bcast(dv, p);
#pragma unroll
    for (int i = p + 1; i < kB; ++i) x[i] -= row16_bcast(d[p], i) * x[p];
  }
}

// Factor diagonal block kb in place and write its inverse to Xd[kb] (only
// the first row of 16 lanes stores).
__device__ void diag_block(double* S, double* Xd, double* dinv, const double* d0, int kb, int l,
                           double tau, int& ndrop, int& nbad) {
  const int lane = threadIdx.x & 63, r = lane & 15;
  const int g0 = kb * kB;
  double d[kB], x[kB], dv;
#pragma unroll
  for (int p = 0; p < kB; ++p) {
    const double v = S[sq(g0 + r, g0 + p)];
    d[p] = p <= r ? v : 0.0;
  }
  diag_factor(d, d0[g0 + r], g0, l, tau, ndrop, nbad, dv, x);
  if (lane < kB) {
    // the whole row: entries above the diagonal are never read again
#pragma unroll
    for (int p = 0; p < kB; ++p) S[sq(g0 + r, g0 + p)] = d[p];
    dinv[g0 + r] = dv;
#pragma unroll
    for (int i = 0; i < kB; ++i) Xd[kb * kB * kB + xq(i, r)] = x[i];
  }
}

// L_Ik = A_Ik X_kk^T (one wave, one 16 x 16 tile).
__device__ void panel_tile(double* S, const double* Xd, int kb, int I) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, q = lane >> 4;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = 4 * s + q;
    acc = mma(S[sq(I * kB + l16, kb * kB + k)], Xd[kb * kB * kB + xq(l16, k)], acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) S[sq(I * kB + 4 * r + q, kb * kB + l16)] = acc[r];
}

// A_IJ -= L_Ik L_Jk^T (one wave, one 16 x 16 tile).
__device__ void update_tile(double* S, int kb, int I, int J) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, q = lane >> 4;
  f64x4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = S[sq(I * kB + 4 * r + q, J * kB + l16)];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = kb * kB + 4 * s + q;
    acc = mma(-S[sq(I * kB + l16, k)], S[sq(J * kB + l16, k)], acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) S[sq(I * kB + 4 * r + q, J * kB + l16)] = acc[r];
}

// X_IJ = -X_II sum_{J <= K < I} L_IK X_KJ, stored transposed at block (J, I).
__device__ void inverse_tile(double* S, const double* Xd, int I, int J) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, q = lane >> 4;
  // two accumulators (k-steps 0, 1 and 2, 3 of each block) halve the chain
  // of dependent products
  f64x4 t0 = {0.0, 0.0, 0.0, 0.0}, t1 = t0;
  for (int K = J; K < I; ++K) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + q;
      const double b = (K == J) ? Xd[J * kB * kB + xq(k, l16)] : S[sq(J * kB + l16, K * kB + k)];
      if (s < 2)
        t0 = mma(S[sq(I * kB + l16, K * kB + k)], b, t0);
      else
        t1 = mma(S[sq(I * kB + l16, K * kB + k)], b, t1);
    }
  }
  f64x4 t;
#pragma unroll
  for (int r = 0; r < 4; ++r) t[r] = t0[r] + t1[r];
  // the accumulator register s holds row 4s + q, column l16 of T: exactly the
  // B operand of k-step s
  f64x4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 4; ++s) x = mma(-Xd[I * kB * kB + xq(l16, 4 * s + q)], t[s], x);
#pragma unroll
  for (int r = 0; r < 4; ++r) S[sq(J * kB + l16, I * kB + 4 * r + q)] = x[r];
}

__global__ __launch_bounds__(kThreads) void k_chol16(const double* __restrict__ G, int64_t lp,
                                                     int l, float* __restrict__ W,
                                                     double* __restrict__ Lout,
                                                     int32_t* __restrict__ status, double tau,
                                                     const int32_t* __restrict__ skip) {
  if (skip && *skip) return;   // the whole workgroup: the small SVD is already done
  __shared__ double S[kSq * kSq];
  __shared__ double Xd[kNbMax * kB * kB];
  __shared__ double dinv[kSq];
  __shared__ double d0[kSq];
  // this latency-bound workgroup may share its CU with a bandwidth-bound
  // product running on another stream: its waves take the issue slots first
  __builtin_amdgcn_s_setprio(3);
  const int tid = threadIdx.x, wave = tid >> 6;
  const int n = (int)lp;
  const int nb = (l + kB - 1) / kB;

  // ---- load the leading l x l of G (zeros beyond): pairs of doubles, 16 in
  // flight per thread
  constexpr int kPairs = kSq * kSq / 2, kBatch = 16;
  for (int e0 = tid; e0 < kPairs; e0 += kThreads * kBatch) {
    double2 v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      // every thread loads (from a clamped, in-range address) and then masks,
      // so that the loads of a batch are all in flight together
      const int e = e0 + u * kThreads, i = e >> 6, c = (e & 63) * 2;
      const int ic = min(i, n - 1), cc = min(c, n - 2);
      const double2 w = *reinterpret_cast<const double2*>(G + (int64_t)ic * n + cc);
      v[u].x = (i < l && c < l) ? w.x : 0.0;
      v[u].y = (i < l && c + 1 < l) ? w.y : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = e0 + u * kThreads, i = e >> 6, c = (e & 63) * 2;
      S[sq(i, c)] = v[u].x;
      S[sq(i, c + 1)] = v[u].y;
    }
  }
  for (int i = tid; i < kSq; i += kThreads) d0[i] = i < l ? G[(int64_t)i * n + i] : 0.0;
  lds_barrier();

  int ndrop = 0, nbad = 0;
  if (wave == 0) diag_block(S, Xd, dinv, d0, 0, l, tau, ndrop, nbad);
  lds_barrier();
  for (int kb = 0; kb < nb; ++kb) {
    for (int I = kb + 1 + wave; I < nb; I += kWaves) panel_tile(S, Xd, kb, I);
    lds_barrier();
    if (kb + 1 < nb) {
      const int t = nb - kb - 1, ntile = t * (t + 1) / 2;
      if (wave == 0) {
        update_tile(S, kb, kb + 1, kb + 1);
        wave_lds_fence();
        diag_block(S, Xd, dinv, d0, kb + 1, l, tau, ndrop, nbad);
      } else {
        // tile 0 (the next diagonal block) is wave 0's
        for (int e = wave; e < ntile; e += kWaves - 1) {
          // e -> (i, c), i >= c, in row-major order of the lower triangle
          int i = 0;
          while ((i + 1) * (i + 2) / 2 <= e) ++i;
          const int c = e - i * (i + 1) / 2;
          update_tile(S, kb, kb + 1 + i, kb + 1 + c);
        }
        // block row kb of X = L^-1 while wave 0 factors the next diagonal
        // block: it needs only L's block columns < kb and X's rows < kb
        if (!Lout)
          for (int J = wave - 1; J < kb; J += kWaves - 1) inverse_tile(S, Xd, kb, J);
      }
      lds_barrier();
    }
  }

  if (Lout) {   // factor only: L (FP64, lp x lp row-major, zero above the diagonal)
    for (int e = tid; e < kSq * kSq; e += kThreads) {
      const int i = e >> 7, c = e & (kSq - 1);
      if (i < n && c < n) Lout[(int64_t)i * n + c] = (i < l && c <= i) ? S[sq(i, c)] : 0.0;
    }
  } else {
    // the last block row of X (the others were made during the factorisation)
    for (int J = wave; J < nb - 1; J += kWaves) inverse_tile(S, Xd, nb - 1, J);
    lds_barrier();
    // W(a, c) = X(c, a): the diagonal blocks come from Xd, the rest from the
    // transposed copy in the upper triangle; four columns per thread
    constexpr int kQuads = kSq * kSq / 4;
#pragma unroll 4
    for (int e = tid; e < kQuads; e += kThreads) {
      const int a = e >> 5, c0 = (e & 31) * 4;
      float v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + u;
        const double xd = Xd[(c >> 4) * kB * kB + xq(c & 15, a & 15)];
        const double xs = S[sq(a, c)];
        v[u] = (c < l && a <= c) ? (float)((a >> 4) == (c >> 4) ? xd : xs) : 0.f;
      }
      if (a < n && c0 < n) st4(W + (int64_t)a * n + c0, make_float4(v[0], v[1], v[2], v[3]));
    }
  }
  if (tid == 0) {
    if (ndrop) atomicAdd(status + kStDropped, ndrop);
    if (nbad) atomicAdd(status + kStNonFinite, nbad);
  }
}

// ---- widths 129 .. 192: tile-packed lower triangle ------------------------
// A 192 x 192 square of doubles does not fit in LDS, so only the 78 lower
// 16 x 16 tiles are kept (tile (I, J), I >= J, at I (I + 1) / 2 + J; element
// (r, c) of a tile at r * 16 + (c ^ r)).  The factorisation is the one above;
// the inverse overwrites L in place.  X_kk of a diagonal block keeps its
// diagonal in dinv and its strict lower part transposed in the strict upper
// part of the diagonal tile.  Block row kb of X replaces row kb of L: its
// tiles are formed in registers during panel step kb (they read L_kb,K for
// K >= J, which the in-place stores would destroy) and stored at the start of
// step kb + 1, before anything reads them.
constexpr int kTpMax = 192;
constexpr int kTpNb = kTpMax / kB;
constexpr int kTpTiles = kTpNb * (kTpNb + 1) / 2;
constexpr int kTpSlots = (kTpNb - 1 + kWaves - 2) / (kWaves - 1);   // X tiles per wave and row

__device__ inline int tp(int I, int J, int r, int c) {   // I >= J
  return ((I * (I + 1) / 2 + J) * kB + r) * kB + (c ^ r);
}

// X_kk(a, b) of diagonal block kb
__device__ inline double tp_xkk(const double* S, const double* dinv, int kb, int a, int b) {
  const double up = S[tp(kb, kb, min(a, b), max(a, b))];
  return a == b ? dinv[kb * kB + a] : (a > b ? up : 0.0);
}

__device__ void tp_diag_block(double* S, double* dinv, const double* d0, int kb, int l,
                              double tau, int& ndrop, int& nbad) {
  const int lane = threadIdx.x & 63, r = lane & 15;
  const int g0 = kb * kB;
  double d[kB], x[kB], dv;
#pragma unroll
  for (int p = 0; p < kB; ++p) {
    const double v = S[tp(kb, kb, r, p)];
    d[p] = p <= r ? v : 0.0;
  }
  diag_factor(d, d0[g0 + r], g0, l, tau, ndrop, nbad, dv, x);
  if (lane < kB) {
    // row r of the tile: L_kk(r, p) for p <= r, X_kk(p, r) for p > r
#pragma unroll
    for (int p = 0; p < kB; ++p) S[tp(kb, kb, r, p)] = p <= r ? d[p] : x[p];
    dinv[g0 + r] = dv;
  }
}

// L_Ik = A_Ik X_kk^T
__device__ void tp_panel_tile(double* S, const double* dinv, int kb, int I) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, q = lane >> 4;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = 4 * s + q;
    acc = mma(S[tp(I, kb, l16, k)], tp_xkk(S, dinv, kb, l16, k), acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) S[tp(I, kb, 4 * r + q, l16)] = acc[r];
}

// A_IJ -= L_Ik L_Jk^T
__device__ void tp_update_tile(double* S, int kb, int I, int J) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, q = lane >> 4;
  f64x4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = S[tp(I, J, 4 * r + q, l16)];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = 4 * s + q;
    acc = mma(-S[tp(I, kb, l16, k)], S[tp(J, kb, l16, k)], acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) S[tp(I, J, 4 * r + q, l16)] = acc[r];
}

// X_IJ = -X_II sum_{J <= K < I} L_IK X_KJ, returned in accumulator layout
// (register r of lane (c, q): row 4 r + q, column c); rows < I of X are in
// place, row I still holds L.
__device__ f64x4 tp_inverse_tile(const double* S, const double* dinv, int I, int J) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, q = lane >> 4;
  f64x4 t0 = {0.0, 0.0, 0.0, 0.0}, t1 = t0;
  for (int K = J; K < I; ++K) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + q;
      const double b = (K == J) ? tp_xkk(S, dinv, J, k, l16) : S[tp(K, J, k, l16)];
      if (s < 2)
        t0 = mma(S[tp(I, K, l16, k)], b, t0);
      else
        t1 = mma(S[tp(I, K, l16, k)], b, t1);
    }
  }
  f64x4 t;
#pragma unroll
  for (int r = 0; r < 4; ++r) t[r] = t0[r] + t1[r];
  f64x4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 4; ++s) x = mma(-tp_xkk(S, dinv, I, l16, 4 * s + q), t[s], x);
  return x;
}

__device__ inline void tp_store_tile(double* S, int I, int J, const f64x4& x) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, q = lane >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) S[tp(I, J, 4 * r + q, l16)] = x[r];
}

__global__ __launch_bounds__(kThreads) void k_chol_tp(const double* __restrict__ G, int64_t lp,
                                                      int l, float* __restrict__ W,
                                                      int32_t* __restrict__ status, double tau) {
  __shared__ double S[kTpTiles * kB * kB];
  __shared__ double dinv[kTpMax];
  __shared__ double d0[kTpMax];
  __builtin_amdgcn_s_setprio(3);
  const int tid = threadIdx.x, wave = tid >> 6;
  const int n = (int)lp;
  const int nb = (l + kB - 1) / kB;

  // ---- the lower tiles of the leading l x l of G (zeros beyond); the
  // square is read in pairs of doubles, 16 in flight per thread
  constexpr int kHalf = kTpMax / 2, kPairs = kTpMax * kHalf, kBatch = 16;
  for (int e0 = tid; e0 < kPairs; e0 += kThreads * kBatch) {
    double2 v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = e0 + u * kThreads, i = e / kHalf, c = (e % kHalf) * 2;
      const int ic = min(min(i, n - 1), kTpMax - 1), cc = min(c, n - 2);
      const double2 w = *reinterpret_cast<const double2*>(G + (int64_t)ic * n + cc);
      v[u].x = (e < kPairs && i < l && c < l) ? w.x : 0.0;
      v[u].y = (e < kPairs && i < l && c + 1 < l) ? w.y : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = e0 + u * kThreads, i = e / kHalf, c = (e % kHalf) * 2;
      if (e < kPairs && (i >> 4) >= (c >> 4)) {
        S[tp(i >> 4, c >> 4, i & 15, c & 15)] = v[u].x;
        S[tp(i >> 4, c >> 4, i & 15, (c & 15) + 1)] = v[u].y;
      }
    }
  }
  for (int i = tid; i < kTpMax; i += kThreads) d0[i] = i < l ? G[(int64_t)i * n + i] : 0.0;
  lds_barrier();

  int ndrop = 0, nbad = 0;
  f64x4 xr[kTpSlots];
  if (wave == 0) tp_diag_block(S, dinv, d0, 0, l, tau, ndrop, nbad);
  lds_barrier();
  for (int kb = 0; kb < nb; ++kb) {
    // block row kb - 1 of X, made during the previous step, replaces L
    if (wave > 0 && kb >= 2) {
#pragma unroll
      for (int u = 0; u < kTpSlots; ++u) {
        const int J = wave - 1 + u * (kWaves - 1);
        if (J < kb - 1) tp_store_tile(S, kb - 1, J, xr[u]);
      }
    }
    for (int I = kb + 1 + wave; I < nb; I += kWaves) tp_panel_tile(S, dinv, kb, I);
    lds_barrier();
    if (kb + 1 < nb) {
      const int t = nb - kb - 1, ntile = t * (t + 1) / 2;
      if (wave == 0) {
        tp_update_tile(S, kb, kb + 1, kb + 1);
        wave_lds_fence();
        tp_diag_block(S, dinv, d0, kb + 1, l, tau, ndrop, nbad);
      } else {
        for (int e = wave; e < ntile; e += kWaves - 1) {
          int i = 0;
          while ((i + 1) * (i + 2) / 2 <= e) ++i;
          const int c = e - i * (i + 1) / 2;
          tp_update_tile(S, kb, kb + 1 + i, kb + 1 + c);
        }
#pragma unroll
        for (int u = 0; u < kTpSlots; ++u) {
          const int J = wave - 1 + u * (kWaves - 1);
          if (J < kb) xr[u] = tp_inverse_tile(S, dinv, kb, J);
        }
      }
      lds_barrier();
    }
  }
  // the last block row of X (row nb - 2 was stored at the start of the last
  // step): every wave forms its tiles, then all store
  {
    constexpr int kLast = (kTpNb - 1 + kWaves - 1) / kWaves;
    f64x4 xl[kLast];
#pragma unroll
    for (int u = 0; u < kLast; ++u) {
      const int J = wave + u * kWaves;
      if (J < nb - 1) xl[u] = tp_inverse_tile(S, dinv, nb - 1, J);
    }
    lds_barrier();
#pragma unroll
    for (int u = 0; u < kLast; ++u) {
      const int J = wave + u * kWaves;
      if (J < nb - 1) tp_store_tile(S, nb - 1, J, xl[u]);
    }
    lds_barrier();
  }
  // W(a, c) = X(c, a) (a <= c), FP32; four columns per thread
  const int nq = n / 4;
  for (int e = tid; e < n * nq; e += kThreads) {
    const int a = e / nq, c0 = (e % nq) * 4;
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = c0 + u;
      double xv = 0.0;
      if (c < l && a <= c) {
        const int C = c >> 4, A = a >> 4;
        xv = C == A ? tp_xkk(S, dinv, C, c & 15, a & 15) : S[tp(C, A, c & 15, a & 15)];
      }
      v[u] = (float)xv;
    }
    st4(W + (int64_t)a * n + c0, make_float4(v[0], v[1], v[2], v[3]));
  }
  if (tid == 0) {
    if (ndrop) atomicAdd(status + kStDropped, ndrop);
    if (nbad) atomicAdd(status + kStNonFinite, nbad);
  }
}


// ---- widths 129 .. 512: blocked factorisation over several launches -------
// The steps of k_chol16 on an lp x lp FP64 square in a global scratch buffer
// (row-major, element (i, c) at S[i * lp + c]; at most 2 MiB, so it stays in
// the L2 cache), one launch per phase so that the many trailing tiles of a
// wide matrix are spread over the device:
//   * k_cg_panel(kb): every workgroup factors diagonal block kb (one wave,
//     registers; the same values in each) and forms up to four panel tiles
//     L_Ik = A_Ik X_kk^T; workgroup 0 keeps L_kk and X_kk in the side area;
//   * k_cg_update(kb): one wave per trailing tile, A_IJ -= L_Ik L_Jk^T;
//   * k_cg_inverse: workgroup J forms block column J of X = L^-1 in LDS,
//     X_IJ = -X_II sum_{J <= K < I} L_IK X_KJ for I = J + 1, ... (the sum
//     split over four waves and added in wave order), and writes rows
//     16 J .. 16 J + 15 of W = X^T;
//   * k_cg_lout (factor only): L with its diagonal blocks and zeros above.
// Scratch: S (lp x lp), then the side area: X_kk and L_kk of every diagonal
// block and the original diagonal (chol_gm_scratch_doubles).
constexpr int kGmMaxNb = (int)(kWideMax / 16);   // diagonal blocks: widths up to 512
constexpr int kCgThreads = 256;

__device__ inline int64_t gidx(int64_t ld, int i, int c) { return (int64_t)i * ld + c; }

struct CgSide {
  double* xd;   // X_kk of block kb at xd[kb * 256 + xq(i, r)]
  double* ld;   // L_kk of block kb at ld[kb * 256 + r * 16 + p], p <= r
  double* d0;   // original diagonal
};
__device__ inline CgSide cg_side(double* S, int64_t lp) {
  double* b = S + lp * lp;
  return {b, b + kGmMaxNb * kB * kB, b + 2 * kGmMaxNb * kB * kB};
}

__global__ void k_cg_init(const double* __restrict__ G, int64_t lp, int l, double* __restrict__ S) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const CgSide sd = cg_side(S, lp);
  if (t < lp * lp) {
    const int i = (int)(t / lp), c = (int)(t % lp);
    S[t] = (i < l && c < l) ? G[t] : 0.0;
  }
  if (t < kGmMaxNb * kB) sd.d0[t] = t < l ? G[t * lp + t] : 0.0;
}

__global__ __launch_bounds__(kCgThreads) void k_cg_panel(double* __restrict__ S, int64_t lp,
                                                         int kb, int nb, int l,
                                                         int32_t* __restrict__ status, double tau) {
  __shared__ double Xs[kB * kB];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15;
  const CgSide sd = cg_side(S, lp);
  const int g0 = kb * kB;
  if (wave == 0) {
    double d[kB], x[kB], dv;
#pragma unroll
    for (int p = 0; p < kB; ++p) {
      const double v = S[gidx(lp, g0 + r, g0 + p)];
      d[p] = p <= r ? v : 0.0;
    }
    int ndrop = 0, nbad = 0;
    diag_factor(d, sd.d0[g0 + r], g0, l, tau, ndrop, nbad, dv, x);
    if (lane < kB) {
#pragma unroll
      for (int i = 0; i < kB; ++i) Xs[xq(i, r)] = x[i];
      if (blockIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kB; ++i) sd.xd[kb * kB * kB + xq(i, r)] = x[i];
#pragma unroll
        for (int p = 0; p < kB; ++p) sd.ld[kb * kB * kB + r * kB + p] = d[p];
      }
    }
    if (blockIdx.x == 0 && lane == 0) {
      if (ndrop) atomicAdd(status + kStDropped, ndrop);
      if (nbad) atomicAdd(status + kStNonFinite, nbad);
    }
  }
  __syncthreads();
  // L_Ik = A_Ik X_kk^T, one tile per wave
  const int I = kb + 1 + (int)blockIdx.x * 4 + wave;
  if (I < nb) {
    const int l16 = lane & 15, q = lane >> 4;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + q;
      acc = mma(S[gidx(lp, I * kB + l16, g0 + k)], Xs[xq(l16, k)], acc);
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) S[gidx(lp, I * kB + 4 * rr + q, g0 + l16)] = acc[rr];
  }
}

// A_IJ -= L_Ik L_Jk^T for the trailing tiles I >= J > kb (tile e of the
// lower triangle after kb, one per wave).
__global__ __launch_bounds__(kCgThreads) void k_cg_update(double* __restrict__ S, int64_t lp,
                                                          int kb, int nb) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, l16 = lane & 15, q = lane >> 4;
  const int e = (int)blockIdx.x * 4 + wave, t = nb - kb - 1;
  if (e >= t * (t + 1) / 2) return;
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= e) ++i;
  const int I = kb + 1 + i, J = kb + 1 + (e - i * (i + 1) / 2);
  f64x4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = S[gidx(lp, I * kB + 4 * r + q, J * kB + l16)];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = kb * kB + 4 * s + q;
    acc = mma(-S[gidx(lp, I * kB + l16, k)], S[gidx(lp, J * kB + l16, k)], acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) S[gidx(lp, I * kB + 4 * r + q, J * kB + l16)] = acc[r];
}

// Block column J of X = L^-1 (workgroup J), then rows 16 J .. 16 J + 15 of
// W = X^T (zero below the diagonal, past l and for dropped directions).
__global__ __launch_bounds__(kCgThreads) void k_cg_inverse(const double* __restrict__ S, int64_t lp,
                                                           int nb, int l, float* __restrict__ W) {
  __shared__ double Xc[kGmMaxNb * kB * kB];   // Xc[I * 256 + r * 16 + c] = X_IJ(r, c)
  __shared__ double red[4][kB * kB];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l16 = lane & 15, q = lane >> 4;
  const int J = blockIdx.x;
  const CgSide sd = cg_side(const_cast<double*>(S), lp);
  if (J < nb) {
    for (int e = tid; e < kB * kB; e += kCgThreads) {
      const int i = e >> 4, c = e & 15;
      Xc[J * kB * kB + e] = sd.xd[J * kB * kB + xq(i, c)];
    }
    __syncthreads();
    for (int I = J + 1; I < nb; ++I) {
      f64x4 t = {0.0, 0.0, 0.0, 0.0};
      for (int K = J + wave; K < I; K += 4) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = 4 * s + q;
          t = mma(S[gidx(lp, I * kB + l16, K * kB + k)], Xc[K * kB * kB + k * kB + l16], t);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave][(4 * r + q) * kB + l16] = t[r];
      __syncthreads();
      if (wave == 0) {
        f64x4 tt;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = (4 * r + q) * kB + l16;
          tt[r] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
        }
        // register s of tt holds row 4 s + q, column l16 of T: the B operand
        // of k-step s
        f64x4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) x = mma(-sd.xd[I * kB * kB + xq(l16, 4 * s + q)], tt[s], x);
#pragma unroll
        for (int r = 0; r < 4; ++r) Xc[I * kB * kB + (4 * r + q) * kB + l16] = x[r];
      }
      __syncthreads();
    }
  }
  // W(a, c) = X(c, a) for a in block J, a <= c < l
  const int n = (int)lp;
  for (int e = tid; e < kB * n; e += kCgThreads) {
    const int a = e / n, c = e % n;
    const int ga = J * kB + a, I = c >> 4;
    double v = 0.0;
    if (J < nb && c < l && ga <= c && I >= J) v = Xc[I * kB * kB + (c & 15) * kB + a];
    W[(int64_t)ga * n + c] = (float)v;
  }
}

// Factor only: L in place in S, with the diagonal blocks from the side area
// and zeros above the diagonal and past l.
__global__ void k_cg_lout(double* __restrict__ S, int64_t lp, int l) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= lp * lp) return;
  const CgSide sd = cg_side(S, lp);
  const int i = (int)(t / lp), c = (int)(t % lp);
  double v = 0.0;
  if (i < l && c <= i)
    v = (i >> 4) == (c >> 4) ? sd.ld[(i >> 4) * kB * kB + (i & 15) * kB + (c & 15)] : S[t];
  S[t] = v;
}

}  // namespace

bool chol16_fits(int64_t lp) { return lp <= kSq; }

hipError_t launch_chol16(const double* G, int64_t lp, int64_t l, float* W, double* L,
                         int32_t* status, double tau, hipStream_t s, const int32_t* skip) {
  if (lp > kSq || lp % kB != 0 || l > lp || l < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol16, dim3(1), dim3(kThreads), 0, s, G, lp, (int)l, W, L, status, tau,
                     skip);
  return hipGetLastError();
}

bool chol_tp_fits(int64_t lp) { return lp > kSq && lp <= kTpMax && lp % kB == 0; }

hipError_t launch_chol_tp(const double* G, int64_t lp, int64_t l, float* W, int32_t* status,
                          double tau, hipStream_t s) {
  if (!chol_tp_fits(lp) || l > lp || l < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol_tp, dim3(1), dim3(kThreads), 0, s, G, lp, (int)l, W, status, tau);
  return hipGetLastError();
}

bool chol_gm_fits(int64_t lp) { return lp > kTpMax && lp <= kGmMaxNb * kB && lp % kB == 0; }

hipError_t launch_chol_gm(const double* G, int64_t lp, int64_t l, double* S, float* W, double* L,
                          int32_t* status, double tau, hipStream_t s) {
  // the inverse is taken here only above the widths of the LDS kernels; the
  // factor alone also for 128 < lp (the small SVD of widths 129 .. 192)
  const bool fits = W ? chol_gm_fits(lp) : (lp > kSq && lp <= kGmMaxNb * kB && lp % kB == 0);
  if (!fits || l > lp || l < 1 || !S || S == G || (!W && !L) || (L && L != S))
    return hipErrorInvalidValue;
  const int nb = (int)((l + kB - 1) / kB);
  hipLaunchKernelGGL(k_cg_init, dim3((unsigned)ceil_div_dev(lp * lp, 256)), dim3(256), 0, s, G, lp,
                     (int)l, S);
  hipError_t e = hipGetLastError();
  for (int kb = 0; kb < nb && e == hipSuccess; ++kb) {
    const int below = nb - kb - 1;
    hipLaunchKernelGGL(k_cg_panel, dim3((unsigned)std::max(1, (below + 3) / 4)), dim3(kCgThreads), 0,
                       s, S, lp, kb, nb, (int)l, status, tau);
    if ((e = hipGetLastError()) != hipSuccess) break;
    if (below > 0) {
      hipLaunchKernelGGL(k_cg_update, dim3((unsigned)((below * (below + 1) / 2 + 3) / 4)),
                         dim3(kCgThreads), 0, s, S, lp, kb, nb);
      e = hipGetLastError();
    }
  }
  if (e != hipSuccess) return e;
  if (W)
    hipLaunchKernelGGL(k_cg_inverse, dim3((unsigned)(lp / kB)), dim3(kCgThreads), 0, s, S, lp, nb,
                       (int)l, W);
  else
    hipLaunchKernelGGL(k_cg_lout, dim3((unsigned)ceil_div_dev(lp * lp, 256)), dim3(256), 0, s, S, lp,
                       (int)l);
  return hipGetLastError();
}

}  // namespace rsvd
