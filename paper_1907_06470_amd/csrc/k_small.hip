// Small dense steps of the randomized SVD, FP64 where the conditioning needs
// it:
//  * Gram matrices P^T P of tall-skinny FP32 panels on the FP64 matrix cores
//    (v_mfma_f64_16x16x4_f64), split over row chunks and summed in chunk
//    order (deterministic).  Used by the QR of steps 3-4 (Section 2.1) as
//    CholeskyQR, and for B B^T of step 6 ("SVD0 preparation", Section 4.1).
//  * Routing of the Cholesky factor and W = L^-T to the kernels of
//    k_chol.hip (a pivot at or below tau times its original diagonal drops
//    the direction: the basis gets a zero column).
//  * Panel times small matrix on the FP32 matrix cores (Q = Y W, U = Q U_B,
//    V = B^T U_B S^-1; step 7 of Section 2.1).
//  * One-sided Jacobi on the Cholesky factor of B B^T (step 6) in one
//    workgroup for sketch widths up to 128 (wider ones: k_bjacobi.hip), and
//    the sort, scaling and sign convention that finish the small SVD.
#include "device.h"
#include "kernels.h"
#include "plan.h"
#include "rank.h"

namespace rsvd {

namespace {

constexpr int kMaxLp = 192;




__device__ inline f64x4 mfma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- Gram ----
// gpart[(chunk * npairs + pair) * 64 * 64 + r * 64 + c] =
//   sum over rows i of the chunk of P(i, 64*ab + r) * P(i, 64*bb + c),
// pair = ab * (ab + 1) / 2 + bb, ab >= bb.  4 waves in a 2 x 2 grid, each a
// 32 x 32 block as 2 x 2 MFMA tiles of 16 x 16.
__global__ __launch_bounds__(256) void k_gram_part(const float* __restrict__ P, int64_t ld,
                                                   int64_t rows, int64_t lp, int64_t chunk_rows,
                                                   double* __restrict__ gpart, int npairs) {
  __shared__ __attribute__((aligned(16))) float Pa[64][68];
  __shared__ __attribute__((aligned(16))) float Pb[64][68];
  const int pair = blockIdx.x;
  const int64_t chunk = blockIdx.y;
  int ab = 0;
  while ((ab + 1) * (ab + 2) / 2 <= pair) ++ab;
  const int bb = pair - ab * (ab + 1) / 2;
  const int64_t r0 = chunk * chunk_rows;
  const int64_t r1 = min(rows, r0 + chunk_rows);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wa = wave >> 1, wb = wave & 1, l16 = lane & 15, q = lane >> 4;
  const int lrow = tid >> 4, lcol = (tid & 15) * 4;

  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

  for (int64_t it = r0; it < r1; it += 64) {
    const int64_t i = it + lcol;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t ca = (int64_t)ab * 64 + lrow + 16 * s;
      const int64_t cb = (int64_t)bb * 64 + lrow + 16 * s;
      float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
      if (ca < lp && i < r1) va = ld4_masked(P + ca * ld, i, r1);
      if (cb < lp && i < r1) vb = ld4_masked(P + cb * ld, i, r1);
      *reinterpret_cast<float4*>(&Pa[lrow + 16 * s][lcol]) = va;
      *reinterpret_cast<float4*>(&Pb[lrow + 16 * s][lcol]) = vb;
    }
    __syncthreads();
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      float4 av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = *reinterpret_cast<const float4*>(&Pa[wa * 32 + t * 16 + l16][q * 16 + s4 * 4]);
        bv[t] = *reinterpret_cast<const float4*>(&Pb[wb * 32 + t * 16 + l16][q * 16 + s4 * 4]);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int ta = 0; ta < 2; ++ta)
#pragma unroll
          for (int tb = 0; tb < 2; ++tb)
            acc[ta][tb] = mfma64((double)av[ta][e], (double)bv[tb][e], acc[ta][tb]);
      }
    }
    __syncthreads();
  }
  // FP64 16x16 accumulators: lane (l16, q) register r holds row q + 4 r of
  // column l16 (rows strided by 4, unlike the FP32 layouts where a lane's
  // registers are consecutive rows).
  double* out = gpart + ((int64_t)chunk * npairs + pair) * 4096;
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wa * 32 + ta * 16 + q + 4 * r;
        const int col = wb * 32 + tb * 16 + l16;
        out[row * 64 + col] = acc[ta][tb][r];
      }
}

// Lower-triangle Gram for sketch widths up to 192 (lp = 16 NBK): the 16 x 16
// tiles (I, J), I >= J, of P^T P, tile t = I (I + 1) / 2 + J handled by wave
// t mod 4 in accumulator t / 4, over one row chunk per workgroup.  Each 64-row
// slab of the chunk is staged in LDS column by column (the panel is
// column-major) and the next slab is prefetched into registers meanwhile.
// Lane (i, q) of a k-step takes rows 4 q + s of a 16-row group, so one
// 16-byte LDS read gives a lane its values for four k-steps; both MFMA
// operands of a tile come from the same read (A and B are both columns of
// P).  gpart[(chunk * ntile + t) * 256 + r * 16 + c] = tile t's (r, c).
constexpr int kGtSlab = 64;
constexpr int kGtLd = kGtSlab + 4;          // floats per staged column

// Wave W's share of k_gram_tri (tiles t = W mod 4, chosen at compile time so
// that the MFMA sequence has no branches).  Every wave runs the same slab
// loop, so the workgroup barriers match.
template <int NBK, int W>
__device__ inline void gram_tri_wave(const float* __restrict__ P, int64_t ld, int64_t r0,
                                     int64_t r1, double* __restrict__ out, float* T) {
  constexpr int NT = NBK * (NBK + 1) / 2, NA = (NT + 3 - W) / 4 > 0 ? (NT + 3 - W) / 4 : 1;
  constexpr int LP = 16 * NBK;
  constexpr int NQ = LP * (kGtSlab / 4) / 256;   // float4 loads per thread per slab
  const int tid = threadIdx.x, lane = tid & 63;
  const int i16 = lane & 15, kq = lane >> 4;
  f64x4 acc[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) acc[a] = f64x4{0.0, 0.0, 0.0, 0.0};
  float4 pre[NQ];
  auto gload = [&](int64_t rb) {
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      const int idx = tid + 256 * u, c = idx / (kGtSlab / 4), q = idx % (kGtSlab / 4);
      const int64_t i = rb + 4 * q;
      pre[u] = i < r1 ? ld4_masked(P + (int64_t)c * ld, i, r1) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  if (r0 < r1) gload(r0);
  for (int64_t rb = r0; rb < r1; rb += kGtSlab) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      const int idx = tid + 256 * u, c = idx / (kGtSlab / 4), q = idx % (kGtSlab / 4);
      *reinterpret_cast<float4*>(&T[c * kGtLd + 4 * q]) = pre[u];
    }
    __syncthreads();
    if (rb + kGtSlab < r1) gload(rb + kGtSlab);
    // 16-row groups past the chunk's end hold zeros: skip them
    const int ng = (int)min<int64_t>(kGtSlab / 16, (r1 - rb + 15) / 16);
#pragma unroll
    for (int g = 0; g < kGtSlab / 16; ++g) {
      if (g < ng) {
        float4 v[NBK];
#pragma unroll
        for (int b = 0; b < NBK; ++b)
          v[b] = *reinterpret_cast<const float4*>(&T[(b * 16 + i16) * kGtLd + g * 16 + 4 * kq]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          double d[NBK];
#pragma unroll
          for (int b = 0; b < NBK; ++b) d[b] = (double)v[b][s];
#pragma unroll
          for (int I = 0, t = 0; I < NBK; ++I)
#pragma unroll
            for (int J = 0; J <= I; ++J, ++t)
              if ((t & 3) == W) acc[t >> 2] = mfma64(d[I], d[J], acc[t >> 2]);
        }
      }
    }
  }
  // accumulator register r of lane (c, q) holds row q + 4 r, column c
#pragma unroll
  for (int t = W; t < NT; t += 4)
#pragma unroll
    for (int r = 0; r < 4; ++r) out[t * 256 + (kq + 4 * r) * 16 + i16] = acc[t >> 2][r];
}

template <int NBK>
__global__ __launch_bounds__(256) void k_gram_tri(const float* __restrict__ P, int64_t ld,
                                                  int64_t rows, int64_t chunk_rows,
                                                  double* __restrict__ gpart) {
  constexpr int NT = NBK * (NBK + 1) / 2;
  __shared__ __attribute__((aligned(16))) float T[16 * NBK * kGtLd];
  const int64_t r0 = (int64_t)blockIdx.x * chunk_rows;
  const int64_t r1 = min(rows, r0 + chunk_rows);
  double* out = gpart + (int64_t)blockIdx.x * NT * 256;
  switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
    case 0: gram_tri_wave<NBK, 0>(P, ld, r0, r1, out, T); break;
    case 1: gram_tri_wave<NBK, 1>(P, ld, r0, r1, out, T); break;
    case 2: gram_tri_wave<NBK, 2>(P, ld, r0, r1, out, T); break;
    default: gram_tri_wave<NBK, 3>(P, ld, r0, r1, out, T); break;
  }
}

// Lower-triangle Gram for wider panels (lp > 192): the lp columns are cut
// into slices of 128 (8 blocks of 16; the last may have 2, 4 or 6), and one
// launch forms the tiles of one slice pair (s, t), s >= t: the lower
// triangle of slice s with itself (DIAG) or the NA x NB rectangle of slice s
// against slice t.  The inner loop is that of k_gram_tri, with the two
// slices' columns staged side by side; tiles are stored at their places in
// the whole lower triangle, so k_gram_tri_reduce sums them as for k_gram_tri.
// Each slice pair reads its slices of the panel once: nS slice pairs per
// slice, i.e. the panel nS times for nS slices (3 at width 352).
template <int NA, int NB, bool DIAG, int W>
__device__ inline void gram_grp_wave(const float* __restrict__ P, int64_t ld, int64_t r0,
                                     int64_t r1, int ca, int cb, int ia, int ib,
                                     double* __restrict__ out, float* T) {
  constexpr int NC = DIAG ? NA : NA + NB;              // staged 16-column blocks
  constexpr int NT = DIAG ? NA * (NA + 1) / 2 : NA * NB;
  constexpr int NACC = (NT + 3 - W) / 4 > 0 ? (NT + 3 - W) / 4 : 1;
  constexpr int NQ = 16 * NC * (kGtSlab / 4) / 256;    // float4 loads per thread per slab
  const int tid = threadIdx.x, lane = tid & 63;
  const int i16 = lane & 15, kq = lane >> 4;
  f64x4 acc[NACC];
#pragma unroll
  for (int a = 0; a < NACC; ++a) acc[a] = f64x4{0.0, 0.0, 0.0, 0.0};
  float4 pre[NQ];
  auto gload = [&](int64_t rb) {
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      const int idx = tid + 256 * u, c = idx / (kGtSlab / 4), q = idx % (kGtSlab / 4);
      const int gc = c < 16 * NA ? ca + c : cb + (c - 16 * NA);
      const int64_t i = rb + 4 * q;
      pre[u] = i < r1 ? ld4_masked(P + (int64_t)gc * ld, i, r1) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  if (r0 < r1) gload(r0);
  for (int64_t rb = r0; rb < r1; rb += kGtSlab) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      const int idx = tid + 256 * u, c = idx / (kGtSlab / 4), q = idx % (kGtSlab / 4);
      *reinterpret_cast<float4*>(&T[c * kGtLd + 4 * q]) = pre[u];
    }
    __syncthreads();
    if (rb + kGtSlab < r1) gload(rb + kGtSlab);
    const int ng = (int)min<int64_t>(kGtSlab / 16, (r1 - rb + 15) / 16);
#pragma unroll
    for (int g = 0; g < kGtSlab / 16; ++g) {
      if (g < ng) {
        float4 v[NC];
#pragma unroll
        for (int b = 0; b < NC; ++b)
          v[b] = *reinterpret_cast<const float4*>(&T[(b * 16 + i16) * kGtLd + g * 16 + 4 * kq]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          double d[NC];
#pragma unroll
          for (int b = 0; b < NC; ++b) d[b] = (double)v[b][s];
          if constexpr (DIAG) {
#pragma unroll
            for (int I = 0, t = 0; I < NA; ++I)
#pragma unroll
              for (int J = 0; J <= I; ++J, ++t)
                if ((t & 3) == W) acc[t >> 2] = mfma64(d[I], d[J], acc[t >> 2]);
          } else {
#pragma unroll
            for (int I = 0, t = 0; I < NA; ++I)
#pragma unroll
              for (int J = 0; J < NB; ++J, ++t)
                if ((t & 3) == W) acc[t >> 2] = mfma64(d[I], d[NA + J], acc[t >> 2]);
          }
        }
      }
    }
  }
  // local tile t -> its place I (I + 1) / 2 + J in the whole lower triangle
#pragma unroll
  for (int t = W; t < NT; t += 4) {
    int I, J;
    if constexpr (DIAG) {
      I = 0;
      while ((I + 1) * (I + 2) / 2 <= t) ++I;
      J = t - I * (I + 1) / 2;
      I += ia;
      J += ia;
    } else {
      I = ia + t / NB;
      J = ib + t % NB;
    }
    const int tg = I * (I + 1) / 2 + J;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[tg * 256 + (kq + 4 * r) * 16 + i16] = acc[t >> 2][r];
  }
}

// One slice pair over one row chunk per workgroup; gpart as for k_gram_tri
// (ntile = the tiles of the whole lower triangle).
template <int NA, int NB, bool DIAG>
__global__ __launch_bounds__(256) void k_gram_grp(const float* __restrict__ P, int64_t ld,
                                                  int64_t rows, int64_t chunk_rows, int ca, int cb,
                                                  int ia, int ib, int ntile,
                                                  double* __restrict__ gpart) {
  constexpr int NC = DIAG ? NA : NA + NB;
  __shared__ __attribute__((aligned(16))) float T[16 * NC * kGtLd];
  const int64_t r0 = (int64_t)blockIdx.x * chunk_rows;
  const int64_t r1 = min(rows, r0 + chunk_rows);
  double* out = gpart + (int64_t)blockIdx.x * ntile * 256;
  switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
    case 0: gram_grp_wave<NA, NB, DIAG, 0>(P, ld, r0, r1, ca, cb, ia, ib, out, T); break;
    case 1: gram_grp_wave<NA, NB, DIAG, 1>(P, ld, r0, r1, ca, cb, ia, ib, out, T); break;
    case 2: gram_grp_wave<NA, NB, DIAG, 2>(P, ld, r0, r1, ca, cb, ia, ib, out, T); break;
    default: gram_grp_wave<NA, NB, DIAG, 3>(P, ld, r0, r1, ca, cb, ia, ib, out, T); break;
  }
}

// G (lp x lp, full symmetric) from the k_gram_tri partials: 16 threads per
// element, thread j summing chunks j, j + 16, ... in order, then the 16
// partial sums in a fixed tree (deterministic).
__global__ __launch_bounds__(256) void k_gram_tri_reduce(const double* __restrict__ gpart,
                                                         int64_t chunks, int ntile, int64_t lp,
                                                         double* __restrict__ G) {
  __shared__ double red[256];
  const int tid = threadIdx.x, j = tid & 15;
  const int64_t e = (int64_t)blockIdx.x * 16 + (tid >> 4);
  const int64_t total = (int64_t)ntile * 256;
  double v = 0.0;
  if (e < total) {
    int64_t c = j;
    for (; c + 48 < chunks; c += 64) {
      const double x0 = gpart[c * total + e], x1 = gpart[(c + 16) * total + e];
      const double x2 = gpart[(c + 32) * total + e], x3 = gpart[(c + 48) * total + e];
      v += x0;
      v += x1;
      v += x2;
      v += x3;
    }
    for (; c < chunks; c += 16) v += gpart[c * total + e];
  }
  red[tid] = v;
  __syncthreads();
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) {
    if (j < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (j == 0 && e < total) {
    const int t = (int)(e / 256), w = (int)(e % 256);
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = t - I * (I + 1) / 2;
    const int64_t row = I * 16 + w / 16, col = J * 16 + w % 16;
    if (row < lp && col < lp) {
      G[row * lp + col] = red[tid];
      G[col * lp + row] = red[tid];
    }
  }
}

// G (lp x lp, full symmetric) from the chunk partials, summed in chunk order.
__global__ void k_gram_reduce(const double* __restrict__ gpart, int64_t chunks, int npairs,
                              int64_t lp, double* __restrict__ G) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)npairs * 4096) return;
  const int pair = (int)(t / 4096), e = (int)(t % 4096);
  int ab = 0;
  while ((ab + 1) * (ab + 2) / 2 <= pair) ++ab;
  const int bb = pair - ab * (ab + 1) / 2;
  const int64_t row = (int64_t)ab * 64 + e / 64, col = (int64_t)bb * 64 + e % 64;
  if (row >= lp || col >= lp) return;
  if (ab == bb && row < col) return;      // diagonal block: lower half writes both
  double v = 0.0;
  for (int64_t c = 0; c < chunks; ++c) v += gpart[(c * npairs + pair) * 4096 + e];
  G[row * lp + col] = v;
  G[col * lp + row] = v;
}

// ------------------------------------------------------ panel x matrix ----
// Accumulator tile of output column c for rows rbase .. rbase + 31 in the
// 32 x 32 matrix-core layout (register 4 g + e holds row rbase + 8 g +
// 4 half + e): zero, or (accum) the values already in out, so that a product
// split over row ranges of W adds its parts in a fixed order.
__device__ inline f32x16 apply_acc_init(const float* out, int64_t ldo, int64_t out_rows,
                                        int64_t rbase, int c, int half, int ncols, int accum) {
  f32x16 a = f32x16{};
  if (accum && c < ncols) {
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t r = rbase + 8 * g + 4 * half + e;
        if (r < out_rows) a[4 * g + e] = out[(int64_t)c * ldo + r];
      }
  }
  return a;
}

// out(i, c) = sum_a P(i, a) W(a, c) for c < ncols; rows [rows, out_rows)
// receive zeros.  One wave per 32 rows, all lp output columns.
template <int NT, bool TRI>
__global__ __launch_bounds__(256) void k_apply(const float* __restrict__ P, int64_t ldp,
                                               int64_t rows, int kdim, const float* __restrict__ W,
                                               int64_t ldw, int ncols, float* __restrict__ out,
                                               int64_t ldo, int64_t out_rows, int vec_ok,
                                               int accum) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int64_t rbase = (int64_t)blockIdx.x * 128 + wave * 32;
  const int64_t i = rbase + l32;
  const bool iok = i < rows;
  f32x16 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = apply_acc_init(out, ldo, out_rows, rbase, t * 32 + l32, half,
                                                       ncols, accum);
  const int kd2 = (kdim + 1) & ~1;
  for (int a0 = 0; a0 < kd2; a0 += 16) {
    float av[8];
    float bv[NT][8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int a = a0 + 2 * s + half;
      av[s] = (iok && a < kdim) ? P[(int64_t)a * ldp + i] : 0.f;
#pragma unroll
      for (int t = 0; t < NT; ++t) bv[t][s] = (a < kdim) ? W[(int64_t)a * ldw + t * 32 + l32] : 0.f;
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (a0 + 2 * s >= kd2) break;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (TRI && a0 + 2 * s >= (t + 1) * 32) continue;
        acc[t] = mfma32(av[s], bv[t][s], acc[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = t * 32 + l32;
    if (c >= ncols) continue;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int64_t r = rbase + 8 * g + 4 * half;
      float* dst = out + (int64_t)c * ldo + r;
      if (vec_ok && r + 3 < out_rows) {
        st4(dst, make_float4(acc[t][4 * g], acc[t][4 * g + 1], acc[t][4 * g + 2], acc[t][4 * g + 3]));
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (r + e < out_rows) dst[e] = acc[t][4 * g + e];
      }
    }
  }
}

// The same product for tall panels: W (kdim x 32 NT, kdim <= KR) is staged in
// LDS once per workgroup, and each wave then takes 32-row blocks in turn
// (grid stride), with the next 16 rows of P's k-range loaded while the
// current ones go through the matrix cores.  Reading W through the caches
// for every 32-row block costs more than the product at width 192 and
// millions of rows; on short panels the staging is not repaid.
constexpr int kApThreads = 512;

template <int NT, bool TRI, int KR>
__global__ __launch_bounds__(kApThreads) void k_apply_staged(const float* __restrict__ P,
                                                             int64_t ldp, int64_t rows, int kdim,
                                                             const float* __restrict__ W,
                                                             int64_t ldw, int ncols,
                                                             float* __restrict__ out, int64_t ldo,
                                                             int64_t out_rows, int vec_ok,
                                                             int accum) {
  constexpr int WC = NT * 32;
  __shared__ __attribute__((aligned(16))) float Ws[KR * WC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int kd2 = (kdim + 1) & ~1;
  if ((ldw & 3) == 0 && (((uintptr_t)W) & 15) == 0) {
    // 16-byte pieces, eight in flight per thread
    constexpr int WQ = WC / 4;
#pragma unroll 8
    for (int e = tid; e < kd2 * WQ; e += blockDim.x) {
      const int a = e / WQ, c = (e % WQ) * 4;
      const float4 v = a < kdim ? *reinterpret_cast<const float4*>(W + (int64_t)a * ldw + c)
                                : make_float4(0.f, 0.f, 0.f, 0.f);
      *reinterpret_cast<float4*>(&Ws[a * WC + c]) = v;
    }
  } else {
    for (int e = tid; e < kd2 * WC; e += blockDim.x) {
      const int a = e / WC, c = e % WC;
      Ws[e] = a < kdim ? W[(int64_t)a * ldw + c] : 0.f;
    }
  }
  __syncthreads();
  const int kWaves = blockDim.x / 64;
  const int64_t nblk = (out_rows + 31) / 32;
  for (int64_t blk = (int64_t)blockIdx.x * kWaves + wave; blk < nblk;
       blk += (int64_t)gridDim.x * kWaves) {
    const int64_t rbase = blk * 32;
    const int64_t i = rbase + l32;
    const bool iok = i < rows;
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
      acc[t] = apply_acc_init(out, ldo, out_rows, rbase, t * 32 + l32, half, ncols, accum);
    float av[8], an[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int a = 2 * s + half;
      av[s] = (iok && a < kdim) ? P[(int64_t)a * ldp + i] : 0.f;
    }
    for (int a0 = 0; a0 < kd2; a0 += 16) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int a = a0 + 16 + 2 * s + half;
        an[s] = (iok && a < kdim) ? P[(int64_t)a * ldp + i] : 0.f;
      }
      // triangular W: output block t takes k < 32 (t + 1) only
      const int tlo = TRI ? a0 >> 5 : 0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t < tlo) continue;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int a = a0 + 2 * s;
          if (a < kd2) acc[t] = mfma32(av[s], Ws[(a + half) * WC + t * 32 + l32], acc[t]);
        }
      }
#pragma unroll
      for (int s = 0; s < 8; ++s) av[s] = an[s];
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int c = t * 32 + l32;
      if (c >= ncols) continue;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t r = rbase + 8 * g + 4 * half;
        float* dst = out + (int64_t)c * ldo + r;
        if (vec_ok && r + 3 < out_rows) {
          st4(dst, make_float4(acc[t][4 * g], acc[t][4 * g + 1], acc[t][4 * g + 2],
                               acc[t][4 * g + 3]));
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (r + e < out_rows) dst[e] = acc[t][4 * g + e];
        }
      }
    }
  }
}

// One-sided (Hestenes) Jacobi on the Cholesky factor L of C = B B^T
// (C = L L^T), for sketch widths up to 128: the columns of M = L are rotated
// in pairs until mutually orthogonal; then M = U_B diag(s), so s_c = |m_c|
// and U_B(:, c) = m_c / s_c are the singular values of B and the
// eigenvectors of C.
//
// Block form with two-column blocks in the odd-even order: the nb blocks sit
// at positions 0..nb-1; a round of parity par pairs positions (2i + par,
// 2i + par + 1), rotates the four cross pairs of columns of each pair (two
// steps of two independent rotations; the pairs inside the blocks once per
// sweep), and the two blocks trade positions.  nb such rounds make a sweep in
// which every two blocks meet exactly once (the exchanges of odd-even
// transposition sort on a reversed sequence).  Group i of 16 lanes always
// holds the block at position 2i + 1 in registers (8 rows each per lane),
// so a round moves only one block per group through LDS (half the traffic of
// an order in which both blocks move); LDS traffic, FP64 issue and the round
// barrier bound this one-workgroup kernel.  Blocks end in permuted positions;
// the output columns follow the original order.
//
// A rotation is kept short: its tangent comes from FP32 arithmetic on the
// exponent-normalised pair (accurate to ~1e-7, which only changes by how much
// the pair's cosine drops), while the cosine is cs = (1 + t^2)^-1/2 in FP64
// for that t, so every applied rotation is orthogonal to FP64 rounding.  The
// rotate/skip test |g| > tol sqrt(a b) runs beside it as g^2 > tol^2 a b.  The
// sweep loop ends after a sweep in which no column pair had the cosine of its
// angle above kOjStop in magnitude:
// quadratic convergence leaves the remaining off-diagonal mass near kOjStop^2,
// far below what the FP64 rotations themselves leave on the singular values.
constexpr int kOjMaxLp = 128;
constexpr int kOjLd = kOjMaxLp + 1;      // odd stride in doubles: no bank conflicts
constexpr int kOjG = 16;                 // lanes per block pair
constexpr int kOjThreads = kOjG * (kOjMaxLp / 4);
constexpr int kOjRows = kOjMaxLp / kOjG;
constexpr double kOjStop = 1e-6;

__device__ inline double oj_norm2(const double (&x)[kOjRows]) {
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int u = 0; u < kOjRows; u += 2) {
    s0 += x[u] * x[u];
    s1 += x[u + 1] * x[u + 1];
  }
  return row16_sum(s0 + s1);
}

// Rotate column pairs (x1, y1) and (x2, y2), four distinct columns, side by
// side: the two inner products, angles and updates are independent, so their
// dependent chains (16-lane sums, the angle, the updates) overlap.  The
// squared norms are carried along: only the inner product g of each pair is
// summed from the data, and the norms of a rotated pair follow from the
// rotation actually applied, a' = c^2 a - 2 c s g + s^2 b and
// b' = s^2 a + 2 c s g + c^2 b.  An updated norm below 1/100 of the old one
// (nearly parallel columns: the update cancels) sets `stale`, and the caller
// sums it afresh.  A pair rotates when g^2 > tol2 a b and its enable flag is
// set.
__device__ inline void oj_angle(double gg, double aa, double bb, bool en, double tol2,
                                double stop2, double& cs, double& sn, bool& any, bool& big) {
  const double ab = aa * bb, g2 = gg * gg;
  const bool rot = en && g2 > tol2 * ab;
  // tangent of the Hestenes angle, t = sign(d) 2g / (|d| + sqrt(d^2 + 4g^2))
  // with d = b - a, on the pair scaled by a power of two
  const double dd = bb - aa, tg = 2.0 * gg;
  const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(dd), fabs(tg)));
  const float d32 = (float)__builtin_amdgcn_ldexp(dd, -ex);
  const float g32 = (float)__builtin_amdgcn_ldexp(tg, -ex);
  const float den = fabsf(d32) + __builtin_amdgcn_sqrtf(d32 * d32 + g32 * g32);
  const float t32 = (d32 >= 0.f ? g32 : -g32) * __builtin_amdgcn_rcpf(den);
  const double tt = rot ? (double)t32 : 0.0;
  cs = fast_rsq(1.0 + tt * tt);
  sn = cs * tt;
  any = any || rot;
  big = big || (rot && g2 > stop2 * ab);
}

__device__ inline void oj_norms(double cs, double sn, double gg, double& na, double& nb,
                                bool& stale) {
  const double aa = na, bb = nb;
  const double c2 = cs * cs, s2 = sn * sn, cg = 2.0 * cs * sn * gg;
  const double a2 = c2 * aa - cg + s2 * bb;
  const double b2 = s2 * aa + cg + c2 * bb;
  stale = stale || a2 < 0.01 * aa || b2 < 0.01 * bb;
  na = a2;
  nb = b2;
}

__device__ inline void oj_rotate2(double (&x1)[kOjRows], double (&y1)[kOjRows], double& na1,
                                  double& nb1, bool en1, double (&x2)[kOjRows],
                                  double (&y2)[kOjRows], double& na2, double& nb2, bool en2,
                                  bool& stale, double tol2, double stop2, bool& any, bool& big) {
  double g10 = 0.0, g11 = 0.0, g20 = 0.0, g21 = 0.0;
#pragma unroll
  for (int u = 0; u < kOjRows; u += 2) {
    g10 += x1[u] * y1[u];
    g20 += x2[u] * y2[u];
    g11 += x1[u + 1] * y1[u + 1];
    g21 += x2[u + 1] * y2[u + 1];
  }
  const double gg1 = row16_sum(g10 + g11), gg2 = row16_sum(g20 + g21);
  double c1, s1, c2, s2;
  oj_angle(gg1, na1, nb1, en1, tol2, stop2, c1, s1, any, big);
  oj_angle(gg2, na2, nb2, en2, tol2, stop2, c2, s2, any, big);
#pragma unroll
  for (int u = 0; u < kOjRows; ++u) {
    const double p1 = x1[u], q1 = y1[u], p2 = x2[u], q2 = y2[u];
    x1[u] = c1 * p1 - s1 * q1;
    y1[u] = s1 * p1 + c1 * q1;
    x2[u] = c2 * p2 - s2 * q2;
    y2[u] = s2 * p2 + c2 * q2;
  }
  oj_norms(c1, s1, gg1, na1, nb1, stale);
  oj_norms(c2, s2, gg2, na2, nb2, stale);
}

// Position p of the odd-even order is idle in a round of parity par when no
// pair (2i + par, 2i + par + 1) of the nb positions covers it.
__device__ inline bool oj_idle(int pos, int par, int nb) {
  if (par == 0) return pos == nb - 1 && (nb & 1);
  return pos == 0 || (pos == nb - 1 && !(nb & 1));
}

__global__ __launch_bounds__(kOjThreads) void k_ojacobi(const double* __restrict__ L, int64_t lp,
                                                        int l, double* __restrict__ lam,
                                                        double* __restrict__ Ev, int32_t* status,
                                                        double tol, int max_sweeps,
                                                        const int32_t* __restrict__ skip) {
  if (skip && *skip) return;   // the whole workgroup: the small SVD is already done
  __shared__ double M[kOjMaxLp * kOjLd];   // block at position p: columns 2p, 2p + 1
  __shared__ int blk[kOjMaxLp / 2];        // block (pair of original columns) at position p
  __shared__ double nrm[kOjMaxLp];         // squared column norms of the block at position p
  __shared__ int pos_of[kOjMaxLp / 2];
  __shared__ int any_s, big_s;
  const int tid = threadIdx.x, grp = tid / kOjG, sub = tid % kOjG;
  const int nb = max((l + 1) / 2, 2);            // two-column blocks (a zero block pads l <= 2)
  const int ng = nb / 2;                          // group i keeps the block at position 2i + 1
  const double tol2 = tol * tol, stop2 = kOjStop * kOjStop;
  // rows and columns at and beyond l are held at zero: a zero column never
  // passes the rotate test and a zero row stays zero, so no load or store
  // below needs a bound
  for (int e = tid; e < kOjMaxLp * kOjMaxLp; e += kOjThreads) {
    const int i = e / kOjMaxLp, c = e % kOjMaxLp;
    M[c * kOjLd + i] = (i < l && c < l) ? L[(int64_t)i * lp + c] : 0.0;
  }
  for (int p = tid; p < kOjMaxLp / 2; p += kOjThreads) blk[p] = p;
  lds_barrier();
  const bool owner = grp < ng;
  const int kpos = 2 * grp + 1;
  double xk[2][kOjRows];                          // the kept block, in registers
  int idk = kpos;
  if (owner) {
#pragma unroll
    for (int u = 0; u < kOjRows; ++u) {
      xk[0][u] = M[(2 * kpos) * kOjLd + sub + kOjG * u];
      xk[1][u] = M[(2 * kpos + 1) * kOjLd + sub + kOjG * u];
    }
  }
  int sweeps = 0, rnd = 0;
  double nk[2];
  for (int sw = 0; sw < max_sweeps && l > 1; ++sw) {
    // the norms carried through the rotations restart from the data each sweep
    if (owner) {
      nk[0] = oj_norm2(xk[0]);
      nk[1] = oj_norm2(xk[1]);
    }
    for (int c = grp; c < kOjMaxLp; c += kOjThreads / kOjG) {
      double v[kOjRows];
#pragma unroll
      for (int u = 0; u < kOjRows; ++u) v[u] = M[c * kOjLd + sub + kOjG * u];
      const double ss = oj_norm2(v);
      if (sub == 0) nrm[c] = ss;
    }
    if (tid == 0) {
      any_s = 0;
      big_s = 0;
    }
    lds_barrier();
    const int par0 = rnd & 1;
    for (int t = 0; t < nb; ++t, ++rnd) {
      // round of parity par: positions (2i + par, 2i + par + 1) meet, then
      // trade places.  Group i's kept block sits at 2i + 1 (the upper one of
      // an even round, the lower one of an odd round); the other block, at
      // slot position sp, comes from LDS, and after the exchange the kept
      // block's data goes to sp while the slot block's data stays in
      // registers as the new block at 2i + 1.
      const int par = rnd & 1;
      const int sp = par ? kpos + 1 : kpos - 1;
      if (owner && sp < nb) {
        double* ms = M + 2 * sp * kOjLd + sub;
        double xs[2][kOjRows];
#pragma unroll
        for (int u = 0; u < kOjRows; ++u) {
          xs[0][u] = ms[kOjG * u];
          xs[1][u] = ms[kOjLd + kOjG * u];
        }
        const int ids = blk[sp];
        double ns[2] = {nrm[2 * sp], nrm[2 * sp + 1]};
        bool any = false, big = false, stale = false;
        // the pairs inside a block, once per sweep: in the sweep's first
        // round, or in its second for a block idle in the first
        const bool ik = t == 0 || (t == 1 && oj_idle(kpos, par0, nb));
        const bool is = t == 0 || (t == 1 && oj_idle(sp, par0, nb));
        // the two inner pairs side by side, then the four cross pairs as two
        // side-by-side steps of disjoint pairs
        if (ik || is)
          oj_rotate2(xk[0], xk[1], nk[0], nk[1], ik, xs[0], xs[1], ns[0], ns[1], is, stale, tol2,
                     stop2, any, big);
        oj_rotate2(xk[0], xs[0], nk[0], ns[0], true, xk[1], xs[1], nk[1], ns[1], true, stale, tol2,
                   stop2, any, big);
        oj_rotate2(xk[0], xs[1], nk[0], ns[1], true, xk[1], xs[0], nk[1], ns[0], true, stale, tol2,
                   stop2, any, big);
        if (stale) {   // rare: sum all four norms afresh
          nk[0] = oj_norm2(xk[0]);
          nk[1] = oj_norm2(xk[1]);
          ns[0] = oj_norm2(xs[0]);
          ns[1] = oj_norm2(xs[1]);
        }
#pragma unroll
        for (int u = 0; u < kOjRows; ++u) {
          ms[kOjG * u] = xk[0][u];
          ms[kOjLd + kOjG * u] = xk[1][u];
          xk[0][u] = xs[0][u];
          xk[1][u] = xs[1][u];
        }
        if (sub == 0) {
          nrm[2 * sp] = nk[0];
          nrm[2 * sp + 1] = nk[1];
          blk[sp] = idk;
          if (any) {
            any_s = 1;
            if (big) big_s = 1;
          }
        }
        idk = ids;
        nk[0] = ns[0];
        nk[1] = ns[1];
      }
      lds_barrier();
    }
    ++sweeps;
    const int any = any_s, big = big_s;
    lds_barrier();
    if (!any || !big) break;
  }
  // kept blocks back to their positions, then the inverse of blk
  if (owner) {
#pragma unroll
    for (int u = 0; u < kOjRows; ++u) {
      M[(2 * kpos) * kOjLd + sub + kOjG * u] = xk[0][u];
      M[(2 * kpos + 1) * kOjLd + sub + kOjG * u] = xk[1][u];
    }
    if (sub == 0) blk[kpos] = idk;
  }
  lds_barrier();
  for (int p = tid; p < kOjMaxLp / 2; p += kOjThreads) pos_of[blk[p]] = p;
  lds_barrier();
  // s_c = |m_c| (one group per original column c), U_B(:, c) = m_c / s_c
  for (int c = grp; c < lp; c += kOjThreads / kOjG) {
    const int mc = 2 * pos_of[c >> 1] + (c & 1);
    double ss = 0.0;
    if (c < l)
      for (int i = sub; i < l; i += kOjG) ss += M[mc * kOjLd + i] * M[mc * kOjLd + i];
    ss = row16_sum(ss);
    const double sv = sqrt(ss);
    if (sub == 0) lam[c] = c < l ? ss : 0.0;
    const double inv = sv > 0.0 ? 1.0 / sv : 0.0;
    for (int i = sub; i < lp; i += kOjG)
      Ev[(int64_t)i * lp + c] = (c < l && i < l) ? M[mc * kOjLd + i] * inv : 0.0;
  }
  if (tid == 0) {
    status[kStSweeps] = sweeps;
    status[kStRounds] = 0;
  }
}

// Automatic iteration parameter: largest relative change of the k leading
// singular values from the previous power step (prev[k] receives it; +inf on
// the first step), then prev = S.
__global__ __launch_bounds__(256) void k_ritz_delta(const double* __restrict__ S, int k, int first,
                                                    double* __restrict__ prev) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double d = 0.0;
  for (int i = tid; i < k; i += 256) {
    const double a = S[i], b = prev[i];
    if (a > 0.0) d = fmax(d, fabs(a - b) / a);
    else if (b != 0.0) d = fmax(d, 1.0);
    if (!(a == a)) d = __builtin_inf();
  }
  red[tid] = d;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] = fmax(red[tid], red[tid + off]);
    __syncthreads();
  }
  for (int i = tid; i < k; i += 256) prev[i] = S[i];
  if (tid == 0) prev[k] = first ? __builtin_inf() : red[0];
}

// Sort eigenvalues descending (ties by index), S = sqrt(lambda) for the first
// k, Wu(a, c) = Ev(a, order c), Wv(a, c) = Wu(a, c) (1 / sigma_c) (0 if sigma_c is
// negligible), both lp x lp row-major FP32 with zero columns from k on.
__global__ __launch_bounds__(1024) void k_finish_small(const double* __restrict__ lam,
                                                       const double* __restrict__ Ev, int64_t lp,
                                                       int l, int k, double* __restrict__ S,
                                                       float* __restrict__ Wu,
                                                       float* __restrict__ Wv,
                                                       int32_t* __restrict__ order_out,
                                                       int32_t* status) {
  __shared__ int order[kWideMax];
  __shared__ double lv[kWideMax], sig[kWideMax], inv[kWideMax];
  __shared__ double smax_s;
  __shared__ int nzero;
  const int tid = threadIdx.x;
  if (tid == 0) nzero = 0;
  for (int i = tid; i < l; i += blockDim.x) lv[i] = nan_as_low(lam[i]);
  __syncthreads();
  // Rank by a strict total order: NaN counts as -inf and ties go by index,
  // so the ranks are a permutation of [0, l) whatever the values are.
  for (int i = tid; i < l; i += blockDim.x) order[desc_rank(lv, l, i)] = i;
  if (tid == 0) {
    double mx = 0.0;
    for (int j = 0; j < l; ++j) mx = fmax(mx, lv[j]);
    smax_s = sqrt(fmax(mx, 0.0));
  }
  __syncthreads();
  const double smax = smax_s;
  for (int c = tid; c < l; c += blockDim.x) {
    const double s = sqrt(fmax(lam[order[c]], 0.0));
    sig[c] = s;
    inv[c] = s > 1e-12 * smax ? 1.0 / s : 0.0;
    if (c < k) {
      S[c] = s;
      if (!(s > 1e-12 * smax)) atomicAdd(&nzero, 1);
    }
    order_out[c] = order[c];
  }
  __syncthreads();
#pragma unroll 4
  for (int e = tid; e < lp * lp; e += blockDim.x) {
    const int a = e / (int)lp, c = e % (int)lp;
    float u = 0.f, v = 0.f;
    if (a < l && c < k) {
      const double ev = Ev[(int64_t)a * lp + order[c]];
      u = (float)ev;
      v = (float)(ev * inv[c]);
    }
    Wu[e] = u;
    Wv[e] = v;
  }
  if (tid == 0) status[kStRankSmall] = nzero;
}

// Sign convention: in every column c < k of V the entry of largest magnitude
// (lowest row on ties) becomes positive; U's column flips with it.  One
// workgroup per column finds the entry and records the flip in flip[c]; a
// second, wide kernel negates the flipped columns of U and V.
__global__ __launch_bounds__(256) void k_sign_find(const float* __restrict__ V, int64_t ldv,
                                                   int64_t n, int32_t* __restrict__ flip) {
  __shared__ float bv[256];
  __shared__ int64_t bi[256];
  const int c = blockIdx.x, tid = threadIdx.x;
  float best = -1.f;
  int64_t bidx = 0;
  const float* col = V + (int64_t)c * ldv;
  // eight independent loads per iteration; each thread keeps its first maximum
  for (int64_t j0 = (int64_t)tid * 8; j0 < n; j0 += 8 * (int64_t)blockDim.x) {
    float a[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = j0 + e < n ? fabsf(col[j0 + e]) : -1.f;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (a[e] > best) {
        best = a[e];
        bidx = j0 + e;
      }
  }
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      const float ob = bv[tid + off];
      const int64_t oi = bi[tid + off];
      if (ob > bv[tid] || (ob == bv[tid] && oi < bi[tid])) {
        bv[tid] = ob;
        bi[tid] = oi;
      }
    }
    __syncthreads();
  }
  if (tid == 0) flip[c] = col[bi[0]] < 0.f ? 1 : 0;
}

// Negate column c of U (rows < m) and of V (rows < n) where flip[c]; block
// (x, c) covers rows [1024 x, 1024 x + 1024) of both.
__global__ __launch_bounds__(256) void k_sign_apply(float* __restrict__ U, int64_t ldu, int64_t m,
                                                    float* __restrict__ V, int64_t ldv, int64_t n,
                                                    const int32_t* __restrict__ flip) {
  const int c = blockIdx.y;
  if (!flip[c]) return;
  const int64_t r0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  float* u = U + (int64_t)c * ldu;
  float* v = V + (int64_t)c * ldv;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t r = r0 + 256 * e;
    if (r < m) u[r] = -u[r];
    if (r < n) v[r] = -v[r];
  }
}

// out(a, c) = Ev(a, order c) for a, c < l (row-major l x l, FP64).
__global__ void k_gather_cols(const double* __restrict__ Ev, int64_t lp, int l,
                              const int32_t* __restrict__ order, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)l * l) return;
  const int a = (int)(t / l), c = (int)(t % l);
  const int oc = min(max(order[c], 0), l - 1);
  out[t] = Ev[(int64_t)a * lp + oc];
}

// C = op(A) B for lp x lp row-major matrices (lp a multiple of 16, at most
// KM), FP64 accumulation in index order: one 16 x 16 tile of C per
// workgroup; the tile's 16 rows of op(A) and 16 columns of B are loaded to
// LDS in one batch (every load in flight at once), then each thread sums
// its element.
constexpr int kLpMax = (int)kWideMax;
template <typename TA, typename TB, typename TC, bool TRANS_A, int KM>
__global__ __launch_bounds__(256) void k_lp_gemm(const TA* __restrict__ A, const TB* __restrict__ B,
                                                 TC* __restrict__ C, int lp) {
  __shared__ double As[16][KM + 1], Bs[KM][17];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int r0 = blockIdx.y * 16, c0 = blockIdx.x * 16;
#pragma unroll 12
  for (int e = tid; e < 16 * lp; e += 256) {
    // As[i][k] = op(A)(r0 + i, k); Bs[k][j] = B(k, c0 + j)
    const int i = TRANS_A ? e % 16 : e / lp, k = TRANS_A ? e / 16 : e % lp;
    As[i][k] = TRANS_A ? (double)A[(int64_t)k * lp + r0 + i] : (double)A[(int64_t)(r0 + i) * lp + k];
    const int kb = e / 16, j = e % 16;
    Bs[kb][j] = (double)B[(int64_t)kb * lp + c0 + j];
  }
  __syncthreads();
  double acc = 0.0;
  for (int k = 0; k < lp; ++k) acc += As[ty][k] * Bs[k][tx];
  C[(int64_t)(r0 + ty) * lp + c0 + tx] = (TC)acc;
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = v;
}

}  // namespace

hipError_t launch_gram(const float* P, int64_t ld, int64_t rows, int64_t lp, int64_t chunk_rows,
                       int64_t chunks, double* gpart, double* G, hipStream_t s) {
  if (gram_grp_fits(lp) && (ld % 4) == 0 && (((uintptr_t)P) & 15) == 0) {
    const int64_t crow = gram_tri_chunk_rows(rows);
    const int64_t nch = ceil_div_dev(rows, crow);
    const int nbk = (int)(lp / 16), ntile = nbk * (nbk + 1) / 2;
    const int nsl = (nbk + 7) / 8;
    for (int sa = 0; sa < nsl; ++sa) {
      const int na = min(8, nbk - 8 * sa);
      for (int sb = 0; sb <= sa; ++sb) {
        const int ia = 8 * sa, ib = 8 * sb;
#define GG(A, B, D)                                                                          \
  hipLaunchKernelGGL((k_gram_grp<A, B, D>), dim3((unsigned)nch), dim3(256), 0, s, P, ld, rows, \
                     crow, 16 * ia, 16 * ib, ia, ib, ntile, gpart)
        if (sa == sb) {
          switch (na) {
            case 2: GG(2, 1, true); break;
            case 4: GG(4, 1, true); break;
            case 6: GG(6, 1, true); break;
            default: GG(8, 1, true); break;
          }
        } else {
          switch (na) {
            case 2: GG(2, 8, false); break;
            case 4: GG(4, 8, false); break;
            case 6: GG(6, 8, false); break;
            default: GG(8, 8, false); break;
          }
        }
#undef GG
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
    }
    hipLaunchKernelGGL(k_gram_tri_reduce, dim3((unsigned)ceil_div_dev((int64_t)ntile * 256, 16)),
                       dim3(256), 0, s, gpart, nch, ntile, lp, G);
    return hipGetLastError();
  }
  if (gram_tri_fits(lp) && (ld % 4) == 0 && (((uintptr_t)P) & 15) == 0) {
    const int64_t crow = gram_tri_chunk_rows(rows);
    const int64_t nch = ceil_div_dev(rows, crow);
    const int nbk = (int)(lp / 16), ntile = nbk * (nbk + 1) / 2;
#define GT(NBK)                                                                              \
  hipLaunchKernelGGL(k_gram_tri<NBK>, dim3((unsigned)nch), dim3(256), 0, s, P, ld, rows, crow, \
                     gpart)
    switch (nbk) {
      case 2: GT(2); break;
      case 4: GT(4); break;
      case 6: GT(6); break;
      case 8: GT(8); break;
      case 10: GT(10); break;
      case 12: GT(12); break;
      default: return hipErrorInvalidValue;
    }
#undef GT
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_tri_reduce, dim3((unsigned)ceil_div_dev((int64_t)ntile * 256, 16)),
                       dim3(256), 0, s, gpart, nch, ntile, lp, G);
    return hipGetLastError();
  }
  const int nb = (int)ceil_div_dev(lp, 64);
  const int npairs = nb * (nb + 1) / 2;
  hipLaunchKernelGGL(k_gram_part, dim3((unsigned)npairs, (unsigned)chunks), dim3(256), 0, s, P, ld,
                     rows, lp, chunk_rows, gpart, npairs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)ceil_div_dev((int64_t)npairs * 4096, 256)),
                     dim3(256), 0, s, gpart, chunks, npairs, lp, G);
  return hipGetLastError();
}

hipError_t launch_chol_inv(const double* G, int64_t lp, int64_t l, float* W, int32_t* status,
                           double tau, double* scratch, hipStream_t s) {
  if (chol_gm_fits(lp)) return launch_chol_gm(G, lp, l, scratch, W, nullptr, status, tau, s);
  if (lp > kMaxLp) return hipErrorInvalidValue;
  if (chol16_fits(lp)) return launch_chol16(G, lp, l, W, nullptr, status, tau, s);
  if (chol_tp_fits(lp)) return launch_chol_tp(G, lp, l, W, status, tau, s);
  return hipErrorInvalidValue;
}

namespace {
hipError_t apply_one(const float* P, int64_t ldp, int64_t rows, int64_t kdim, const float* W,
                     int64_t ldw, int64_t lp, int64_t ncols, bool tri, float* out, int64_t ldo,
                     int64_t out_rows_total, int accum, hipStream_t s) {
  if (kdim < 0 || kdim > kMaxLp) return hipErrorInvalidValue;
  const int vec_ok = ((ldo % 4) == 0 && (((uintptr_t)out) & 15) == 0) ? 1 : 0;
  const int64_t nblk = ceil_div_dev(out_rows_total, 32);
  // tall panels (4096 or more 32-row blocks): W staged in LDS, 8 waves per
  // workgroup, at most 1024 workgroups; otherwise one wave per 32-row block
  const bool tall = nblk >= 4096;
  const bool wide = kdim > lp;   // W has more rows than columns (the adjoint's factors)
  const dim3 grid_s((unsigned)std::min<int64_t>(1024, ceil_div_dev(nblk, kApThreads / 64)));
  const dim3 grid((unsigned)ceil_div_dev(out_rows_total, 128));
#define AP_ST(NT, TRI, KR)                                                                  \
  hipLaunchKernelGGL((k_apply_staged<NT, TRI, KR>), grid_s, dim3(kApThreads), 0, s, P, ldp, \
                     rows, (int)kdim, W, ldw, (int)ncols, out, ldo, out_rows_total, vec_ok, accum)
#define AP_CALL(NT)                                                                         \
  do {                                                                                      \
    if (tall && tri && !wide)                                                               \
      AP_ST(NT, true, NT * 32);                                                             \
    else if (tall && !wide)                                                                 \
      AP_ST(NT, false, NT * 32);                                                            \
    else if (tall)                                                                          \
      AP_ST(NT, false, kMaxLp);                                                             \
    else if (tri)                                                                           \
      hipLaunchKernelGGL((k_apply<NT, true>), grid, dim3(256), 0, s, P, ldp, rows, (int)kdim, \
                         W, ldw, (int)ncols, out, ldo, out_rows_total, vec_ok, accum);      \
    else                                                                                    \
      hipLaunchKernelGGL((k_apply<NT, false>), grid, dim3(256), 0, s, P, ldp, rows,         \
                         (int)kdim, W, ldw, (int)ncols, out, ldo, out_rows_total, vec_ok,   \
                         accum);                                                            \
  } while (0)
  switch (lp / 32) {
    case 1: AP_CALL(1); break;
    case 2: AP_CALL(2); break;
    case 3: AP_CALL(3); break;
    case 4: AP_CALL(4); break;
    case 5: AP_CALL(5); break;
    case 6: AP_CALL(6); break;
    default: return hipErrorInvalidValue;
  }
#undef AP_CALL
#undef AP_ST
  return hipGetLastError();
}
}  // namespace

// Widths above kMaxLp: W (kdim x lp) is taken in sub-blocks of at most
// kMaxLp x kMaxLp, column slices of equal width (a multiple of 32) and row
// slices on the same boundaries, so that every sub-block fits the kernels
// above (W staged in LDS on tall panels).  The row slices of one column slice
// add into the output in increasing order (the first writes, the others
// accumulate); with triangular W the slices below the diagonal are skipped.
hipError_t launch_apply(const float* P, int64_t ldp, int64_t rows, int64_t kdim, const float* W,
                        int64_t ldw, int64_t lp, int64_t ncols, bool tri, float* out, int64_t ldo,
                        int64_t out_rows_total, hipStream_t s) {
  if (kdim < 0 || lp < 32 || lp % 32) return hipErrorInvalidValue;
  if (lp <= kMaxLp && kdim <= kMaxLp)
    return apply_one(P, ldp, rows, kdim, W, ldw, lp, ncols, tri, out, ldo, out_rows_total, 0, s);
  if (lp > kWideMax || kdim > kWideMax) return hipErrorInvalidValue;
  const int64_t nslice = ceil_div_dev(std::max(lp, kdim), kMaxLp);
  const int64_t cw = ceil_div_dev(ceil_div_dev(std::max(lp, kdim), nslice), 32) * 32;
  for (int64_t c0 = 0; c0 < lp && c0 < ncols; c0 += cw) {
    const int64_t wc = std::min(cw, lp - c0), nc = std::min(wc, ncols - c0);
    const int64_t kend = tri ? std::min(kdim, c0 + wc) : kdim;
    int accum = 0;
    for (int64_t k0 = 0; k0 < kend || (k0 == 0 && kend == 0); k0 += cw) {
      const int64_t kw = std::min(cw, kend - k0);
      hipError_t e = apply_one(P + k0 * ldp, ldp, rows, kw, W + k0 * ldw + c0, ldw, wc, nc,
                               tri && k0 == c0, out + c0 * ldo, ldo, out_rows_total, accum, s);
      if (e != hipSuccess) return e;
      accum = 1;
      if (kend == 0) break;
    }
  }
  return hipSuccess;
}

bool small_svd_one_sided(int64_t lp) { return lp <= kOjMaxLp; }

hipError_t launch_chol_factor(const double* G, int64_t lp, int64_t l, double* L, int32_t* status,
                              double tau, hipStream_t s, const int32_t* skip) {
  if (chol16_fits(lp)) return launch_chol16(G, lp, l, nullptr, L, status, tau, s, skip);
  if (skip) return hipErrorInvalidValue;   // the tridiagonal path covers widths <= 128 only
  return launch_chol_gm(G, lp, l, L, nullptr, L, status, tau, s);
}

hipError_t launch_ojacobi(const double* L, int64_t lp, int64_t l, double* lam, double* Ev,
                          int32_t* status, double tol, int max_sweeps, hipStream_t s,
                          const int32_t* skip) {
  if (lp > kOjMaxLp) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ojacobi, dim3(1), dim3(kOjThreads), 0, s, L, lp, (int)l, lam, Ev, status,
                     tol, max_sweeps, skip);
  return hipGetLastError();
}

// The LDS tiles are sized for the plan's width class: kMaxLp, or kLpMax for
// wide sketches (135 KB, one workgroup per CU).
hipError_t launch_congruence(const double* G, const float* W, double* T, double* out, int64_t lp,
                             hipStream_t s) {
  if (lp % 16 || lp > kLpMax) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(lp / 16), (unsigned)(lp / 16));
  if (T == G || T == out) return hipErrorInvalidValue;
  if (lp <= kMaxLp)
    hipLaunchKernelGGL((k_lp_gemm<double, float, double, false, kMaxLp>), grid, dim3(256), 0, s, G,
                       W, T, (int)lp);
  else
    hipLaunchKernelGGL((k_lp_gemm<double, float, double, false, kLpMax>), grid, dim3(256), 0, s, G,
                       W, T, (int)lp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (lp <= kMaxLp)
    hipLaunchKernelGGL((k_lp_gemm<float, double, double, true, kMaxLp>), grid, dim3(256), 0, s, W,
                       T, out, (int)lp);
  else
    hipLaunchKernelGGL((k_lp_gemm<float, double, double, true, kLpMax>), grid, dim3(256), 0, s, W,
                       T, out, (int)lp);
  return hipGetLastError();
}

hipError_t launch_lp_product(const float* A, const float* B, float* C, int64_t lp, hipStream_t s) {
  if (lp % 16 || lp > kLpMax) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(lp / 16), (unsigned)(lp / 16));
  if (lp <= kMaxLp)
    hipLaunchKernelGGL((k_lp_gemm<float, float, float, false, kMaxLp>), grid, dim3(256), 0, s, A, B,
                       C, (int)lp);
  else
    hipLaunchKernelGGL((k_lp_gemm<float, float, float, false, kLpMax>), grid, dim3(256), 0, s, A, B,
                       C, (int)lp);
  return hipGetLastError();
}

hipError_t launch_finish_small(const double* lam, const double* Ev, int64_t lp, int64_t l,
                               int64_t k, double* S, float* Wu, float* Wv, int32_t* order,
                               int32_t* status, hipStream_t s) {
  if (lp > kWideMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finish_small, dim3(1), dim3(1024), 0, s, lam, Ev, lp, (int)l, (int)k, S, Wu,
                     Wv, order, status);
  return hipGetLastError();
}

hipError_t launch_ritz_delta(const double* S, int64_t k, bool first, double* prev,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_ritz_delta, dim3(1), dim3(256), 0, s, S, (int)k, first ? 1 : 0, prev);
  return hipGetLastError();
}

hipError_t launch_sign_fix(float* U, int64_t ldu, int64_t m, float* V, int64_t ldv, int64_t n,
                           int64_t k, int32_t* work, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sign_find, dim3((unsigned)k), dim3(256), 0, s, V, ldv, n, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t rows = m > n ? m : n;
  hipLaunchKernelGGL(k_sign_apply, dim3((unsigned)ceil_div_dev(rows, 1024), (unsigned)k),
                     dim3(256), 0, s, U, ldu, m, V, ldv, n, work);
  return hipGetLastError();
}

hipError_t launch_gather_cols(const double* Ev, int64_t lp, int64_t l, const int32_t* order,
                              double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)ceil_div_dev(l * l, 256)), dim3(256), 0, s, Ev,
                     lp, (int)l, order, out);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div_dev(count, 256)), dim3(256), 0, s, p,
                     count, v);
  return hipGetLastError();
}

}  // namespace rsvd
