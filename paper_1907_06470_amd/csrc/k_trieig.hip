// Small SVD of Section 2.1 step 6 through the symmetric eigenproblem of the
// FP64 Gram C = B B^T (order n = l <= 128; its two triangles are averaged,
// since a congruence Wp^T G Wp is symmetric only to rounding), in one
// workgroup of 512 threads (eight waves: the steps below are bound by what
// every wave repeats, so fewer waves issue less):
//
//   1. Householder reduction Q^T C Q = T (tridiagonal).  C is held in
//      registers on a 32 x 16 thread grid (thread (r, c) owns rows r + 32 i,
//      i < 4, and columns c + 16 j, j < 8); each step forms the reflector
//      from the column below the diagonal, p = tau A v (row sums over a
//      16-lane DPP row), w = p - (tau / 2)(p^T v) v and A -= v w^T + w v^T.
//      The reflectors are kept in LDS.  Sums across lanes go through DPP
//      permutes.  Register blocks whose rows or columns are all <= k (or
//      >= n) drop out of the product and the update; the same holds for the
//      rows of step 4.
//   2. Eigenvalues of T by bisection on the Sturm count (the number of
//      negative pivots of T - x I), four lanes per eigenvalue cutting the
//      interval into five parts per round; 23 rounds take the Gershgorin
//      interval below FP64 resolution.  (The phase is bound by FP64 issue:
//      four lanes do a third less work than eight for the same resolution.)
//   3. Eigenvectors of T by inverse iteration, one lane per eigenvalue: the
//      LU factors of T - lambda I with row interchanges (the LAPACK gttrf
//      pattern) go to a global scratch laid out [array][row][lane], then two
//      solves from a fixed pseudo-random start, normalising in between.
//   4. Back-transformation W = Q Z, the reflectors applied in reverse order
//      (column sums: partials over the thread grid in LDS, then four threads
//      per column).
//   5. Checks: |W^T W - I| <= 1e-12 (the accuracy the one-sided Jacobi path
//      reaches) and, for a fixed pseudo-random y,
//      |C (W y) - W (diag(lambda) y)| <= 1e-12 lambda_max |y|_1, with every
//      value finite.  status[kStTriOk] says whether they held; the Cholesky
//      and Jacobi kernels launched after this one run only when they did
//      not (close or repeated eigenvalues, where independent inverse
//      iterations lose orthogonality, or non-finite input).
//
// Outputs as the Jacobi path writes them: lam[c] = eigenvalue c (zero from n
// on), Ev row-major lp x lp with column c the unit eigenvector (zero rows
// and columns from n on).
#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace rsvd {

namespace {

constexpr int kTeN = (int)kTriMaxLp;             // largest order
constexpr int kTeR = 4;                          // rows per thread (blocks of 32)
constexpr int kTeT = 512;                        // threads: a 32 x 16 grid in phases 1, 4, 5
constexpr int kTeC = 8;                          // columns per thread (blocks of 16)
constexpr int kTeG = 4;                          // lanes per eigenvalue in the bisection
constexpr int kTeRounds = 23;                    // (kTeG + 1)^23 = 5^23 > 2^52
static_assert(kTeG * kTeN == kTeT, "one lane group per eigenvalue");
constexpr int kTePacked = kTeN * (kTeN - 1) / 2; // reflector store (doubles)
constexpr int kTeRed = 33;                       // column stride of the partial sums
static_assert(kTePacked + kTeN * kTeRed <= kTeN * kTeN, "reflectors and partial sums fit");
constexpr double kTeTol = 1e-12;
constexpr int kTeArrays = 6;                     // scratch arrays of the inverse iteration
constexpr int kTeIb = 8;                         // rows per batch of its loads
static_assert(kTeN == 128 && kTeArrays * kTeN * kTeN == kTriScratchDoubles, "scratch layout");

__device__ inline int te_off(int k) { return k * kTeN - k * (k + 1) / 2; }

// Cross-lane sums through DPP lane permutes (no LDS round trips); every lane
// of the 16-lane row (of the wave) ends with the same bits, since each step
// adds the same two operands in every lane.
template <int kCtrl, int kRows = 0xF>   // rows outside kRows get 0
__device__ inline double te_dpp(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, kCtrl, kRows, 0xF, false);
  const int hi =
      __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), kCtrl, kRows, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ inline double te_row_sum(double x) {   // over the 16 lanes of a row
  x += te_dpp<0xB1>(x);    // quad_perm [1, 0, 3, 2]
  x += te_dpp<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  x += te_dpp<0x141>(x);   // row_half_mirror
  x += te_dpp<0x140>(x);   // row_mirror
  return x;
}

__device__ inline double te_lane(double x, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// the four row sums r0..r3 meet in lane 63 as (r3 + r2) + (r1 + r0)
__device__ inline double te_wave_sum(double x) {
  x = te_row_sum(x);
  x += te_dpp<0x142, 0xA>(x);   // row_bcast:15: lane 15 (47) into row 1 (3)
  x += te_dpp<0x143, 0xC>(x);   // row_bcast:31: lane 31 into rows 2 and 3
  return te_lane(x, 63);
}

// 1 / q: the hardware reciprocal and one Newton step
__device__ inline double te_rcp(double q) {
  double r = __builtin_amdgcn_rcp(q);
  return fma(fma(-q, r, 1.0), r, r);
}

// 1 when q < 0: after the pivot floor q is never a zero, so the sign bit
// says it (two instructions instead of a compare, a select and an add)
__device__ inline int te_neg(double q) {
  return (int)(__builtin_bit_cast(uint64_t, q) >> 63);
}

__device__ inline void te_sturm_step(double d, double e2, double x, double pivmin, double& q,
                                     int& cnt) {
  q = (d - x) - e2 * te_rcp(q);
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += te_neg(q);
}

// number of eigenvalues of T below x (negative pivots of T - x I)
__device__ inline int te_sturm(const double* dS, const double* e2S, int n, double x,
                               double pivmin) {
  double q = dS[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = te_neg(q);
  int i = 1;
  for (; i + 4 <= n; i += 4) {
    double d[4], e[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      d[u] = dS[i + u];
      e[u] = e2S[i + u - 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) te_sturm_step(d[u], e[u], x, pivmin, q, cnt);
  }
  for (; i < n; ++i) te_sturm_step(dS[i], e2S[i - 1], x, pivmin, q, cnt);
  return cnt;
}

// fixed pseudo-random start vector entry in [-1, 1)
__device__ inline double te_start(int i, int j) {
  uint32_t h = (uint32_t)(i + 1) * 0x9E3779B1u ^ (uint32_t)(j + 1) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (double)(h >> 8) * (2.0 / 16777216.0) - 1.0;
}

// Step k of the reduction, two barriers.  Thread (tr, tc) of the 32 x 16
// grid holds rows tr + 32 r (r < 4) and columns tc + 16 c (c < 8) of A, so a
// row of the grid is one 16-lane DPP row and its sums need no lane reads.
// Every wave forms the reflector and the scalar K itself (same bits in every
// wave); the column below the diagonal alternates between two buffers so
// that the next step's owner never overwrites one still being read.  Column
// blocks c < CKB (row blocks r < CKB / 2) hold
// indices <= k only, and blocks from NB (2 NB) on indices >= n only; there
// the reflector v and the vector w are zero, the update leaves A as it is
// and the product's terms are zeros, so those blocks are skipped.  (The
// values are those of the full update up to which product each fused
// multiply-add rounds first.)
template <int CKB, int NB>
__device__ __forceinline__ void te_reduce_step(double (&A)[kTeR][kTeC], int k, int n,
                                                double* xsb, double* ps, double* dS,
                                                double* eS, double* tauS, double* vst) {
  constexpr int RKB = CKB / 2, NC = 2 * NB;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15, l64 = tid & 63;
  double* xk = xsb + (k & 1) * kTeN;
  if (tc == (k & 15)) {   // column k: block CKB, or CKB - 1 at the first step of the range
    const bool at = (k >> 4) == CKB;
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const int i = tr + 32 * r;
      const double x = at ? A[r][CKB] : A[r][CKB > 0 ? CKB - 1 : 0];
      if (i < n) xk[i] = i > k ? x : 0.0;   // zeros at rows <= k
      if (i == k) dS[k] = x;
    }
  }
  __syncthreads();
  double tau = 0.0, beta = 0.0, sc = 0.0;
  // v: zero at rows <= k (xk holds zeros there) and >= n (never written,
  // zero from the start), 1 at k + 1, the scaled column below
  auto vof = [&](int i) -> double { return i == k + 1 ? 1.0 : xk[i] * sc; };
  double vi[kTeR], vj[kTeC];
  {
    double sg = 0.0;
    {
      const int i0 = k + 2 + l64, i1 = i0 + 64;
      if (i0 < n) sg += xk[i0] * xk[i0];
      if (i1 < n) sg += xk[i1] * xk[i1];
    }
    sg = te_wave_sum(sg);
    const double al = xk[k + 1];
    beta = al;
    if (sg > 0.0) {
      const double mu = sqrt(al * al + sg);
      beta = al >= 0.0 ? -mu : mu;
      sc = te_rcp(al - beta);   // al - beta and beta are nonzero here (sg > 0)
      tau = (beta - al) * te_rcp(beta);
    }
#pragma unroll
    for (int r = RKB; r < NB; ++r) vi[r] = vof(tr + 32 * r);
    double pr[kTeR] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = CKB; c < NC; ++c) {
      vj[c] = vof(tc + 16 * c);
#pragma unroll
      for (int r = RKB; r < NB; ++r) pr[r] += A[r][c] * vj[c];
    }
#pragma unroll
    for (int r = RKB; r < NB; ++r) pr[r] = te_row_sum(pr[r]);
    if (tc == 0) {
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        const int i = tr + 32 * r;
        if (i < n) ps[i] = (r >= RKB && i > k) ? tau * pr[r] : 0.0;
      }
    }
  }
  __syncthreads();
  {
    double kk = 0.0;
    if (l64 < n) kk += ps[l64] * vof(l64);
    if (l64 + 64 < n) kk += ps[l64 + 64] * vof(l64 + 64);
    const double K = 0.5 * tau * te_wave_sum(kk);
    double wi[kTeR];
#pragma unroll
    for (int r = RKB; r < NB; ++r) {
      const int i = tr + 32 * r;
      wi[r] = i < n ? ps[i] - K * vi[r] : 0.0;
    }
    // the reflector for the back-transformation (xk stays valid until step
    // k + 2 writes it again), stored off the path to the second barrier
    if (tid < 64) {
      for (int i = k + 1 + tid; i < n; i += 64) vst[te_off(k) + i - k - 1] = vof(i);
      if (tid == 0) {
        tauS[k] = tau;
        eS[k] = beta;
      }
    }
#pragma unroll
    for (int c = CKB; c < NC; ++c) {
      const int j = tc + 16 * c;
      const double wj = j < n ? ps[j] - K * vj[c] : 0.0;
#pragma unroll
      for (int r = RKB; r < NB; ++r) A[r][c] -= vi[r] * wj + wi[r] * vj[c];
    }
  }
}

// The steps with first active column block CKB (k = 16 CKB - 1 ...
// 16 CKB + 14), from k on while k + 2 < n, then the next block's.
template <int CKB, int NB>
__device__ __forceinline__ void te_reduce(double (&A)[kTeR][kTeC], int& k, int n,
                                          double* xsb, double* ps, double* dS, double* eS,
                                          double* tauS, double* vst) {
  for (; k + 2 < n && k < 16 * CKB + 15; ++k)
    te_reduce_step<CKB, NB>(A, k, n, xsb, ps, dS, eS, tauS, vst);
  if constexpr (CKB + 1 < 2 * NB) {
    te_reduce<CKB + 1, NB>(A, k, n, xsb, ps, dS, eS, tauS, vst);
  } else {   // the last 2 x 2 block (or the single entry)
    const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
#pragma unroll
    for (int r = 0; r < NB; ++r)
#pragma unroll
      for (int c = 0; c < 2 * NB; ++c) {
        const int i = tr + 32 * r, j = tc + 16 * c;
        if (i == j && i >= n - 2 && i < n) dS[i] = A[r][c];
        if (n >= 2 && i == n - 1 && j == n - 2) eS[n - 2] = A[r][c];
      }
  }
}

// Reflector k of the back-transformation Z -= v (tau v^T Z), Z on the 32 x 16
// grid as A: the grid writes partial column sums over its rows (column-major,
// stride kTeRed), four threads per column add eight partials each and then
// the four through DPP, and every thread updates its entries.  Row blocks
// below KB (rows <= k, where v is zero) and column blocks from 2 NB on
// (columns >= n) are skipped.
template <int KB, int NB>
__device__ __forceinline__ void te_back_step(double (&Z)[kTeR][kTeC], int k, int n,
                                              const double* vst, const double* tauS,
                                              double* red, double* ps) {
  const double tau = tauS[k];
  if (tau == 0.0) return;   // no reflection at this step (the same in every thread)
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  double vi[kTeR];
#pragma unroll
  for (int r = KB; r < NB; ++r) {
    const int i = tr + 32 * r;
    vi[r] = (i > k && i < n) ? vst[te_off(k) + i - k - 1] : 0.0;
  }
#pragma unroll
  for (int c = 0; c < 2 * NB; ++c) {
    double s = 0.0;
#pragma unroll
    for (int r = KB; r < NB; ++r) s += vi[r] * Z[r][c];
    red[(tc + 16 * c) * kTeRed + tr] = s;
  }
  __syncthreads();
  {
    const int col = tid >> 2, q = tid & 3;
    double s = 0.0;
    if (col < n)
#pragma unroll
      for (int t = 0; t < 8; ++t) s += red[col * kTeRed + 8 * q + t];
    s += te_dpp<0xB1>(s);   // quad_perm [1, 0, 3, 2]
    s += te_dpp<0x4E>(s);   // quad_perm [2, 3, 0, 1]
    if (col < n && q == 0) ps[col] = tau * s;
  }
  __syncthreads();
#pragma unroll
  for (int r = KB; r < NB; ++r)
#pragma unroll
    for (int c = 0; c < 2 * NB; ++c) Z[r][c] -= vi[r] * ps[tc + 16 * c];
}

template <int NB>
__device__ __forceinline__ void te_back(double (&Z)[kTeR][kTeC], int n, const double* vst,
                                        const double* tauS, double* red, double* ps) {
  int k = n - 3;
  if constexpr (NB > 3)
    for (; k >= 95; --k) te_back_step<3, NB>(Z, k, n, vst, tauS, red, ps);
  if constexpr (NB > 2)
    for (; k >= 63; --k) te_back_step<2, NB>(Z, k, n, vst, tauS, red, ps);
  if constexpr (NB > 1)
    for (; k >= 31; --k) te_back_step<1, NB>(Z, k, n, vst, tauS, red, ps);
  for (; k >= 0; --k) te_back_step<0, NB>(Z, k, n, vst, tauS, red, ps);
}

__global__ __launch_bounds__(kTeT) void k_tri_eig(const double* __restrict__ G, int64_t lp, int n,
                                                  double* __restrict__ lam,
                                                  double* __restrict__ Ev,
                                                  double* __restrict__ scr,
                                                  int32_t* __restrict__ status) {
  __shared__ double big[kTeN * kTeN];   // reflectors (and column partial sums), then W
  __shared__ double xsb[2 * kTeN], ps[kTeN];
  __shared__ double dS[kTeN], eS[kTeN], e2S[kTeN], tauS[kTeN], lamS[kTeN], znS[kTeN];
  __shared__ double shv[4];
  double* vst = big;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  // scratch arrays: 0 multiplier, 1 reciprocal pivot, 2 and 3 the two super
  // diagonals of U, 4 interchange flag, 5 right-hand side / solution
  double* const sa[kTeArrays] = {scr, scr + kTeN * kTeN, scr + 2 * kTeN * kTeN,
                                 scr + 3 * kTeN * kTeN, scr + 4 * kTeN * kTeN,
                                 scr + 5 * kTeN * kTeN};

  // the thread's share of C: rows tr + 32 r, columns tc + 16 c
  double A[kTeR][kTeC];
#pragma unroll
  for (int r = 0; r < kTeR; ++r)
#pragma unroll
    for (int c = 0; c < kTeC; ++c) {
      const int i = tr + 32 * r, j = tc + 16 * c;
      A[r][c] = (i < n && j < n) ? 0.5 * (G[(int64_t)i * lp + j] + G[(int64_t)j * lp + i]) : 0.0;
    }
  for (int i = tid; i < kTeN; i += kTeT) {
    xsb[i] = 0.0;
    xsb[kTeN + i] = 0.0;
    ps[i] = 0.0;
    eS[i] = 0.0;
    e2S[i] = 0.0;
    tauS[i] = 0.0;
  }
  __syncthreads();

  // 1. tridiagonal reduction (the step is described at te_reduce_step)
  {
    int k = 0;
    switch ((n + 31) >> 5) {
      case 1: te_reduce<0, 1>(A, k, n, xsb, ps, dS, eS, tauS, vst); break;
      case 2: te_reduce<0, 2>(A, k, n, xsb, ps, dS, eS, tauS, vst); break;
      case 3: te_reduce<0, 3>(A, k, n, xsb, ps, dS, eS, tauS, vst); break;
      default: te_reduce<0, 4>(A, k, n, xsb, ps, dS, eS, tauS, vst); break;
    }
  }
  __syncthreads();
  for (int i = tid; i + 1 < n; i += kTeT) e2S[i] = eS[i] * eS[i];
  if (tid < 64) {   // Gershgorin interval, |T| and the pivot floor
    double lo = __builtin_inf(), hi = -__builtin_inf(), em = 0.0;
    for (int i = tid; i < n; i += 64) {
      const double rad = (i > 0 ? fabs(eS[i - 1]) : 0.0) + (i + 1 < n ? fabs(eS[i]) : 0.0);
      lo = fmin(lo, dS[i] - rad);
      hi = fmax(hi, dS[i] + rad);
      if (i + 1 < n) em = fmax(em, eS[i] * eS[i]);
    }
    for (int o = 32; o > 0; o >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, o, 64));
      hi = fmax(hi, __shfl_xor(hi, o, 64));
      em = fmax(em, __shfl_xor(em, o, 64));
    }
    if (tid == 0) {
      const double tn = fmax(fabs(lo), fabs(hi));
      const double w = fmax(tn, 1e-300) * 4.0 * 2.220446049250313e-16;
      shv[0] = lo - w;
      shv[1] = hi + w;
      shv[2] = 2.2250738585072014e-308 * fmax(1.0, em);
      shv[3] = tn;
    }
  }
  __syncthreads();

  // 2. eigenvalues: group of kTeG lanes per eigenvalue j (ascending)
  {
    const int j = tid / kTeG, s = tid % kTeG;
    double a = shv[0], b = shv[1];
    const double pivmin = shv[2];
    for (int round = 0; round < kTeRounds; ++round) {
      const double x = a + (b - a) * (double)(s + 1) * (1.0 / (kTeG + 1));
      const int cnt = j < n ? te_sturm(dS, e2S, n, x, pivmin) : 0;
      int smax = cnt <= j ? s : -1;   // count(a) <= j < count(b)
      for (int o = 1; o < kTeG; o <<= 1) smax = max(smax, __shfl_xor(smax, o, kTeG));
      const double xl = __shfl(x, smax < 0 ? 0 : smax, kTeG);
      const double xh = __shfl(x, smax < kTeG - 1 ? smax + 1 : kTeG - 1, kTeG);
      if (smax >= 0) a = xl;
      if (smax < kTeG - 1) b = xh;
    }
    if (s == 0 && j < n) lamS[j] = 0.5 * (a + b);
  }
  __syncthreads();

  // 3. inverse iteration, lane j = eigenvector j
  if (tid < n) {
    const int j = tid;
    const double lj = lamS[j];
    // only an exactly zero pivot is replaced (by the Sturm pivot floor):
    // raising small pivots to eps |T| caps the growth that makes the
    // iteration converge for eigenvalues far below |T| (their vectors lose
    // orthogonality to ~1e-11); an overflow instead fails the checks
    const double tiny = shv[2];
    double* const dl = sa[0] + j;
    double* const rp = sa[1] + j;
    double* const u1 = sa[2] + j;
    double* const u2 = sa[3] + j;
    double* const pv = sa[4] + j;
    double* const X = sa[5] + j;
    // factor T - lj I = P L U, transforming the start vector on the way
    double dd = dS[0] - lj, du = n > 1 ? eS[0] : 0.0, xi = te_start(0, j);
    for (int i = 0; i + 1 < n; ++i) {
      if (dd == 0.0) dd = tiny;
      const double sub = eS[i], dn = dS[i + 1] - lj, un = i + 2 < n ? eS[i + 1] : 0.0;
      const double bn = te_start(i + 1, j);
      const int o = i * kTeN;
      if (fabs(dd) >= fabs(sub)) {
        const double r = te_rcp(dd), f = sub * r;
        dl[o] = f;
        rp[o] = r;
        u1[o] = du;
        u2[o] = 0.0;
        pv[o] = 0.0;
        X[o] = xi;
        dd = dn - f * du;
        du = un;
        xi = bn - f * xi;
      } else {
        const double r = te_rcp(sub), f = dd * r;
        dl[o] = f;
        rp[o] = r;
        u1[o] = dn;
        u2[o] = un;
        pv[o] = 1.0;
        X[o] = bn;
        const double ndd = du - f * dn;
        du = -f * un;
        xi = xi - f * bn;
        dd = ndd;
      }
    }
    if (dd == 0.0) dd = tiny;
    {
      const int o = (n - 1) * kTeN;
      rp[o] = te_rcp(dd);
      u1[o] = 0.0;
      u2[o] = 0.0;
      X[o] = xi;
    }
    double scale = 1.0;
    for (int it = 0; it < 2; ++it) {
      if (it > 0) {   // forward pass on the normalised previous solution,
                      // kTeIb rows at a time with their loads issued together
                      // (rows i + 1 .. i + kTeIb are read before rows i ..
                      // i + kTeIb - 1 are written)
        double bi = X[0] * scale;
        int i = 0;
        for (; i + kTeIb < n; i += kTeIb) {
          double f[kTeIb], pf[kTeIb], bn[kTeIb];
#pragma unroll
          for (int u = 0; u < kTeIb; ++u) {
            const int o = (i + u) * kTeN;
            f[u] = dl[o];
            pf[u] = pv[o];
            bn[u] = X[o + kTeN] * scale;
          }
#pragma unroll
          for (int u = 0; u < kTeIb; ++u) {
            const int o = (i + u) * kTeN;
            if (pf[u] != 0.0) {
              X[o] = bn[u];
              bi = bi - f[u] * bn[u];
            } else {
              X[o] = bi;
              bi = bn[u] - f[u] * bi;
            }
          }
        }
        for (; i + 1 < n; ++i) {
          const int o = i * kTeN;
          const double f = dl[o], bn = X[o + kTeN] * scale;
          if (pv[o] != 0.0) {
            X[o] = bn;
            bi = bi - f * bn;
          } else {
            X[o] = bi;
            bi = bn - f * bi;
          }
        }
        X[(n - 1) * kTeN] = bi;
      }
      // back substitution with U (reciprocal pivots, super diagonals), kTeIb
      // rows at a time with their loads issued together
      double x1 = 0.0, x2 = 0.0, nrm = 0.0;
      int i = n - 1;
      for (; i >= kTeIb - 1; i -= kTeIb) {
        double b[kTeIb], a1[kTeIb], a2[kTeIb], rr[kTeIb];
#pragma unroll
        for (int u = 0; u < kTeIb; ++u) {
          const int o = (i - u) * kTeN;
          b[u] = X[o];
          a1[u] = u1[o];
          a2[u] = u2[o];
          rr[u] = rp[o];
        }
#pragma unroll
        for (int u = 0; u < kTeIb; ++u) {
          const double x = (b[u] - a1[u] * x1 - a2[u] * x2) * rr[u];
          X[(i - u) * kTeN] = x;
          nrm += x * x;
          x2 = x1;
          x1 = x;
        }
      }
      for (; i >= 0; --i) {
        const int o = i * kTeN;
        const double x = (X[o] - u1[o] * x1 - u2[o] * x2) * rp[o];
        X[o] = x;
        nrm += x * x;
        x2 = x1;
        x1 = x;
      }
      scale = 1.0 / sqrt(nrm);
    }
    znS[j] = scale;
  }
  __syncthreads();

  // 4. W = Q Z, the reflectors in reverse order (te_back_step)
  double* red = big + kTePacked;   // kTeN columns of 32 partial sums
  double Z[kTeR][kTeC];
#pragma unroll
  for (int r = 0; r < kTeR; ++r)
#pragma unroll
    for (int c = 0; c < kTeC; ++c) {
      const int i = tr + 32 * r, j = tc + 16 * c;
      Z[r][c] = (i < n && j < n) ? sa[5][i * kTeN + j] * znS[j] : 0.0;
    }
  switch ((n + 31) >> 5) {
    case 1: te_back<1>(Z, n, vst, tauS, red, ps); break;
    case 2: te_back<2>(Z, n, vst, tauS, red, ps); break;
    case 3: te_back<3>(Z, n, vst, tauS, red, ps); break;
    default: te_back<4>(Z, n, vst, tauS, red, ps); break;
  }
  __syncthreads();   // the reflector store is read for the last time above

  // 5. checks on W (in LDS), then the outputs
#pragma unroll
  for (int r = 0; r < kTeR; ++r)
#pragma unroll
    for (int c = 0; c < kTeC; ++c) big[(tr + 32 * r) * kTeN + tc + 16 * c] = Z[r][c];
  // y of the residual check, in the (now free) column buffer of the reduction
  if (tid < kTeN) xsb[tid] = tid < n ? te_start(tid, 4099) : 0.0;
  __syncthreads();
  double lmax = 0.0;
  for (int j = 0; j < n; ++j) lmax = fmax(lmax, fabs(lamS[j]));
  auto cval = [&](int row, int i) -> double {   // C(row, i), both triangles averaged
    return row < n ? 0.5 * (G[(int64_t)row * lp + i] + G[(int64_t)i * lp + row]) : 0.0;
  };
  bool bad = !(lmax < __builtin_inf());
  {   // W^T W = I; it is symmetric (the two products of a pair are the same
      // bits), so register blocks wholly below the diagonal are left out
    double g[kTeR][kTeC];
#pragma unroll
    for (int r = 0; r < kTeR; ++r)
#pragma unroll
      for (int c = 0; c < kTeC; ++c) g[r][c] = 0.0;
    for (int i = 0; i < n; ++i) {
      double wa[kTeR], wb[kTeC];
#pragma unroll
      for (int r = 0; r < kTeR; ++r) wa[r] = big[i * kTeN + tr + 32 * r];
#pragma unroll
      for (int c = 0; c < kTeC; ++c) wb[c] = big[i * kTeN + tc + 16 * c];
#pragma unroll
      for (int r = 0; r < kTeR; ++r)
#pragma unroll
        for (int c = 2 * r; c < kTeC; ++c) g[r][c] += wa[r] * wb[c];
    }
#pragma unroll
    for (int r = 0; r < kTeR; ++r)
#pragma unroll
      for (int c = 2 * r; c < kTeC; ++c) {
        const int a = tr + 32 * r, b = tc + 16 * c;
        if (a < n && b < n && !(fabs(g[r][c] - (a == b ? 1.0 : 0.0)) <= kTeTol)) bad = true;
      }
  }
  {   // C (W y) = W (diag(lambda) y) for a fixed pseudo-random y: eight
      // threads per row, sixteen entries each, then a sum over the eight;
      // each group of eight takes rows i and i + 64
    const int s8 = tid & 7;
    double tv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = (tid >> 3) + 64 * h;
      double u = 0.0, t = 0.0;
      if (i < n)
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
          const int j = 16 * s8 + q;
          if (j < n) {
            const double y = xsb[j], w = big[i * kTeN + j];
            u += w * y;
            t += w * (lamS[j] * y);
          }
        }
      u += te_dpp<0xB1>(u);
      u += te_dpp<0x4E>(u);
      u += te_dpp<0x141>(u);
      t += te_dpp<0xB1>(t);
      t += te_dpp<0x4E>(t);
      t += te_dpp<0x141>(t);
      if (s8 == 0) ps[i] = i < n ? u : 0.0;
      tv[h] = t;
    }
    __syncthreads();
    const double ysum = te_wave_sum(fabs(xsb[tid & 63]) + fabs(xsb[(tid & 63) + 64]));
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = (tid >> 3) + 64 * h;
      double cu = 0.0;
      if (i < n) {
        double cv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int m = 16 * s8 + q;
          cv[q] = m < n ? cval(i, m) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) cu += cv[q] * ps[16 * s8 + q];
      }
      cu += te_dpp<0xB1>(cu);
      cu += te_dpp<0x4E>(cu);
      cu += te_dpp<0x141>(cu);
      if (i < n && s8 == 0 && !(fabs(cu - tv[h]) <= kTeTol * lmax * ysum)) bad = true;
    }
  }
  const int any_bad = __syncthreads_or(bad ? 1 : 0);
  for (int e = tid; e < lp * lp; e += kTeT) {
    const int i = e / (int)lp, j = e % (int)lp;
    Ev[e] = (i < n && j < n) ? big[i * kTeN + j] : 0.0;
  }
  for (int j = tid; j < lp; j += kTeT) lam[j] = j < n ? lamS[j] : 0.0;
  if (tid == 0) {
    status[kStTriOk] = any_bad ? 0 : 1;
    if (!any_bad) {
      status[kStSweeps] = 0;
      status[kStRounds] = 0;
    }
  }
}

}  // namespace

hipError_t launch_tri_eig(const double* G, int64_t lp, int64_t l, double* lam, double* Ev,
                          double* scratch, int32_t* status, hipStream_t s) {
  if (lp > kTeN || l < 1 || l > lp) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tri_eig, dim3(1), dim3(kTeT), 0, s, G, lp, (int)l, lam, Ev, scratch,
                     status);
  return hipGetLastError();
}

}  // namespace rsvd
