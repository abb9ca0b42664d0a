// Small SVD for sketch widths above what one workgroup holds in LDS (padded
// widths up to 512; Section 2.1, step 6): block one-sided (Hestenes) Jacobi
// on the Cholesky factor L of C = B B^T (C = L L^T, FP64).  The columns of
// M = L are rotated in pairs until mutually orthogonal; then M = U_B diag(s),
// so s_c = |m_c| are the singular values of B and m_c / s_c the eigenvectors
// of C (the same reading as the one-workgroup kernel for narrow sketches).
//
// M is l x l, column-major in global memory (2 MiB at most, so it stays in
// the L2 cache).  Its l columns form nb blocks of 16; a zero block pads an
// odd count.  One launch is one round of the round-robin ("tournament")
// order of the blocks: workgroup x takes the two blocks at positions x and
// nb - 1 - x, loads their 32 columns into LDS and rotates the 256 pairs
// between the two blocks in 16 steps of 16 disjoint pairs, one pair per wave
// (wave w keeps column w of the first block in registers and meets column
// (w + t) mod 16 of the second at step t).  In a sweep's first round it also
// rotates the pairs inside each of its two blocks (15 steps of 8 disjoint
// pairs per block), so the nb - 1 rounds of a sweep rotate every column pair
// of M exactly once, as one sweep of the cyclic method does.
//
// A pair (x, y) with a = |x|^2, b = |y|^2, g = x^T y rotates when
// g^2 > tol^2 a b, by the angle that makes the rotated pair orthogonal:
// zeta = (b - a) / (2 g), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// c = 1 / sqrt(1 + t^2), s = c t, x' = c x - s y, y' = s x + c y.  The
// iteration ends after a sweep in which no pair had |g| / sqrt(a b) (the
// cosine of its angle) above kBjStop: quadratic convergence then leaves an
// off-diagonal mass near kBjStop^2.  The host enqueues kBjMaxSweeps sweeps
// without waiting; every round first reads the flag of the previous sweep
// and returns at once when that sweep was the last one needed.
#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace rsvd {

namespace {

constexpr int kBjW = 16;                 // columns per block
constexpr int kBjThreads = 1024;         // 16 waves, one pair each
constexpr int kBjMaxL = (int)kWideMax;   // rows of a column in LDS
constexpr double kBjStop = 1e-6;

// Position of block slot x in round t of the round-robin order over le
// slots: slot 0 stays, the others rotate.
__device__ inline int bj_pos(int x, int t, int le) {
  if (x == 0) return 0;
  int v = x - 1 + t;
  if (v >= le - 1) v -= le - 1;
  return 1 + v;
}

// Sum over the 64 lanes of a wave; every lane gets the same bits (the four
// row sums are combined as (r0 + r1) + (r2 + r3) in every lane, and IEEE
// addition is commutative).
__device__ inline double bj_sum(double v) {
  v = row16_sum(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Rotate the column pair (x, y) held by one wave (lane holds rows lane + 64 u).
// Every lane computes the same sums, so the branch is uniform.
template <int R>
__device__ inline void bj_rotate(double (&x)[R], double (&y)[R], double tol2, double stop2,
                                 bool& big) {
  double a = 0.0, b = 0.0, g = 0.0;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    a += x[u] * x[u];
    b += y[u] * y[u];
    g += x[u] * y[u];
  }
  a = bj_sum(a);
  b = bj_sum(b);
  g = bj_sum(g);
  const double ab = a * b, g2 = g * g;
  if (!(g2 > tol2 * ab)) return;   // also zero columns and NaN
  big = big || g2 > stop2 * ab;
  const double zeta = (b - a) / (2.0 * g);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const double p = x[u], q = y[u];
    x[u] = c * p - s * q;
    y[u] = s * p + c * q;
  }
}

template <int R>
__device__ inline void bj_load(const double* Ms, int slot, double (&v)[R]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int u = 0; u < R; ++u) v[u] = Ms[slot * kBjMaxL + lane + 64 * u];
}

template <int R>
__device__ inline void bj_store(double* Ms, int slot, const double (&v)[R]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int u = 0; u < R; ++u) Ms[slot * kBjMaxL + lane + 64 * u] = v[u];
}

// One round: R = ceil(l / 64) rows per lane.
template <int R>
__global__ __launch_bounds__(kBjThreads) void k_bj_round(double* __restrict__ M, int64_t lp, int l,
                                                         int nbe, int round, int sweep,
                                                         int32_t* __restrict__ ctl, double tol2,
                                                         double stop2) {
  if (sweep > 0 && ctl[sweep - 1] == 0) return;   // an earlier sweep was the last one needed
  __shared__ double Ms[2 * kBjW * kBjMaxL];
  __shared__ int big_s;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int x0 = bj_pos((int)blockIdx.x, round, nbe);
  const int x1 = bj_pos(nbe - 1 - (int)blockIdx.x, round, nbe);
  const int bI = min(x0, x1), bJ = max(x0, x1);
  if (tid == 0) big_s = 0;
  // slot j < 16: column 16 bI + j; slot 16 + j: column 16 bJ + j; rows and
  // columns at and beyond l are held at zero
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int slot = 2 * wave + h;
    const int c = (slot < kBjW ? bI * kBjW : (bJ - 1) * kBjW) + slot;
    double v[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = lane + 64 * u;
      v[u] = (c < l && i < l) ? M[(int64_t)c * lp + i] : 0.0;
    }
    bj_store<R>(Ms, slot, v);
  }
  lds_barrier();
  bool big = false;
  if (round == 0) {   // pairs inside each block, once per sweep
    const int blk = wave >> 3, pi = wave & 7;
    for (int t = 0; t < kBjW - 1; ++t) {
      const int sa = blk * kBjW + bj_pos(pi, t, kBjW);
      const int sb = blk * kBjW + bj_pos(kBjW - 1 - pi, t, kBjW);
      double xa[R], yb[R];
      bj_load<R>(Ms, sa, xa);
      bj_load<R>(Ms, sb, yb);
      bj_rotate<R>(xa, yb, tol2, stop2, big);
      bj_store<R>(Ms, sa, xa);
      bj_store<R>(Ms, sb, yb);
      lds_barrier();
    }
  }
  // pairs across the two blocks
  double xk[R];
  bj_load<R>(Ms, wave, xk);
  for (int t = 0; t < kBjW; ++t) {
    const int sy = kBjW + ((wave + t) & (kBjW - 1));
    double y[R];
    bj_load<R>(Ms, sy, y);
    bj_rotate<R>(xk, y, tol2, stop2, big);
    bj_store<R>(Ms, sy, y);
    lds_barrier();
  }
  bj_store<R>(Ms, wave, xk);
  if (big) big_s = 1;
  lds_barrier();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int slot = 2 * wave + h;
    const int c = (slot < kBjW ? bI * kBjW : (bJ - 1) * kBjW) + slot;
    if (c < l) {
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int i = lane + 64 * u;
        if (i < l) M[(int64_t)c * lp + i] = Ms[slot * kBjMaxL + i];
      }
    }
  }
  if (tid == 0 && big_s) atomicMax(ctl + sweep, 1);
}

// M (column-major) = L (row-major), the sweep flags cleared.
__global__ void k_bj_init(const double* __restrict__ L, int64_t lp, double* __restrict__ M,
                          int32_t* __restrict__ ctl, int nctl) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < lp * lp) {
    const int64_t c = t / lp, i = t % lp;
    M[t] = L[i * lp + c];
  }
  if (t < nctl) ctl[t] = 0;
}

// lam[c] = |m_c|^2, Ev(i, c) = m_c(i) / |m_c| (row-major lp x lp, zero
// outside l x l); one wave per column.  Block 0 records the sweeps run.
template <int R>
__global__ __launch_bounds__(256) void k_bj_finish(const double* __restrict__ M, int64_t lp, int l,
                                                   const int32_t* __restrict__ ctl, int max_sweeps,
                                                   double* __restrict__ lam,
                                                   double* __restrict__ Ev,
                                                   int32_t* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c < lp) {
    double v[R];
    double ss = 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = lane + 64 * u;
      v[u] = (c < l && i < l) ? M[(int64_t)c * lp + i] : 0.0;
      ss += v[u] * v[u];
    }
    ss = bj_sum(ss);
    const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
    if (lane == 0) lam[c] = c < l ? ss : 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = lane + 64 * u;
      if (i < lp) Ev[(int64_t)i * lp + c] = v[u] * inv;
    }
    for (int i = 64 * R + lane; i < lp; i += 64) Ev[(int64_t)i * lp + c] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int sweeps = max_sweeps;
    for (int sw = 0; sw < max_sweeps; ++sw)
      if (ctl[sw] == 0) {
        sweeps = sw + 1;
        break;
      }
    status[kStSweeps] = sweeps;
    status[kStRounds] = 0;
  }
}

}  // namespace

bool bjacobi_fits(int64_t lp) { return lp <= kWideMax && lp % 32 == 0; }

hipError_t launch_bjacobi(const double* L, int64_t lp, int64_t l, double* M, int32_t* ctl,
                          double* lam, double* Ev, int32_t* status, double tol, hipStream_t s) {
  if (!bjacobi_fits(lp) || l < 1 || l > lp) return hipErrorInvalidValue;
  const int nb = (int)((l + kBjW - 1) / kBjW);
  const int nbe = nb < 2 ? 2 : nb + (nb & 1);
  const int R = (int)((l + 63) / 64);
  hipLaunchKernelGGL(k_bj_init, dim3((unsigned)ceil_div_dev(lp * lp, 256)), dim3(256), 0, s, L, lp,
                     M, ctl, (int)kBjMaxSweeps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double tol2 = tol * tol, stop2 = kBjStop * kBjStop;
  for (int sw = 0; sw < (int)kBjMaxSweeps; ++sw)
    for (int r = 0; r < nbe - 1; ++r) {
#define BJ(RR)                                                                                   \
  hipLaunchKernelGGL(k_bj_round<RR>, dim3((unsigned)(nbe / 2)), dim3(kBjThreads), 0, s, M, lp, \
                     (int)l, nbe, r, sw, ctl, tol2, stop2)
      switch (R) {
        case 1: BJ(1); break;
        case 2: BJ(2); break;
        case 3: BJ(3); break;
        case 4: BJ(4); break;
        case 5: BJ(5); break;
        case 6: BJ(6); break;
        case 7: BJ(7); break;
        default: BJ(8); break;
      }
#undef BJ
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  const dim3 gf((unsigned)ceil_div_dev(lp, 4));
#define BF(RR)                                                                                  \
  hipLaunchKernelGGL(k_bj_finish<RR>, gf, dim3(256), 0, s, M, lp, (int)l, ctl,                 \
                     (int)kBjMaxSweeps, lam, Ev, status)
  switch (R) {
    case 1: BF(1); break;
    case 2: BF(2); break;
    case 3: BF(3); break;
    case 4: BF(4); break;
    case 5: BF(5); break;
    case 6: BF(6); break;
    case 7: BF(7); break;
    default: BF(8); break;
  }
#undef BF
  return hipGetLastError();
}

}  // namespace rsvd
