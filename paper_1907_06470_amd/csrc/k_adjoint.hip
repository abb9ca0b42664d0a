// Kernels of the truncated-SVD adjoint (the backward pass of the randomized
// SVD; the paper has no derivative).  With the l Ritz triplets (U_l, S_l, V_l)
// recomputed by the forward schedule:
//   J_u = U_l^T gU, J_v = V_l^T gV              FP64 cross Gram matrices
//   core = (F o skew(J_u)) S + S (F o skew(J_v)) + diag(gS),
//          F_ij = 1 / (s_j^2 - s_i^2)          FP64, one workgroup
//   gA = [U_l | P2 | P3] [V_l core^T | V_k | R3]^T      one outer product
// with P2 = (gU - U_l J_u) S_k^-1, P3 = U_k S_k^-1, R3 = gV - V_l J_v, written
// tile by tile on the FP32 matrix cores (the dense m x n output is the bulk of
// the traffic).
#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace rsvd {

namespace {

__device__ inline f64x4 mfma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// gpart[(chunk * nbq + bq) * nbp + bp][64 x 64] = P(chunk rows, 64 bp + r)^T
// R(chunk rows, 64 bq + c).  Same tiling as the Gram kernel, with the second
// operand from R and every block pair computed.
__global__ __launch_bounds__(256) void k_xgram_part(const float* __restrict__ P, int64_t ldp,
                                                    int64_t cp, const float* __restrict__ R,
                                                    int64_t ldr, int64_t cr, int64_t rows,
                                                    int64_t chunk_rows, double* __restrict__ gpart,
                                                    int nbp) {
  __shared__ __attribute__((aligned(16))) float Pa[64][68];
  __shared__ __attribute__((aligned(16))) float Pb[64][68];
  const int bp = blockIdx.x % nbp, bq = blockIdx.x / nbp;
  const int64_t chunk = blockIdx.y;
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
      const int64_t ca = (int64_t)bp * 64 + lrow + 16 * s;
      const int64_t cb = (int64_t)bq * 64 + lrow + 16 * s;
      float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
      if (ca < cp && i < r1) va = ld4_masked(P + ca * ldp, i, r1);
      if (cb < cr && i < r1) vb = ld4_masked(R + cb * ldr, i, r1);
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
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int ta = 0; ta < 2; ++ta)
#pragma unroll
          for (int tb = 0; tb < 2; ++tb)
            acc[ta][tb] = mfma64((double)av[ta][e], (double)bv[tb][e], acc[ta][tb]);
    }
    __syncthreads();
  }
  // FP64 accumulators: register r of lane (l16, q) is row q + 4 r, column l16
  double* out = gpart + ((int64_t)chunk * gridDim.x + blockIdx.x) * 4096;
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(wa * 32 + ta * 16 + q + 4 * r) * 64 + wb * 32 + tb * 16 + l16] = acc[ta][tb][r];
}

// C (cp x cr, row-major) = sum over chunks (in chunk order) of the blocks.
__global__ void k_xgram_reduce(const double* __restrict__ gpart, int64_t chunks, int nblocks,
                               int nbp, int64_t cp, int64_t cr, double* __restrict__ C) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nblocks * 4096) return;
  const int blk = (int)(t / 4096), e = (int)(t % 4096);
  const int bp = blk % nbp, bq = blk / nbp;
  const int64_t row = (int64_t)bp * 64 + e / 64, col = (int64_t)bq * 64 + e % 64;
  if (row >= cp || col >= cr) return;
  double v = 0.0;
  for (int64_t c = 0; c < chunks; ++c) v += gpart[(c * nblocks + blk) * 4096 + e];
  C[row * cr + col] = v;
}

// The l x l core and the small factors of the outer product (one workgroup).
//   coreT(a, c) = core(c, a)          (lp x lp, FP32; R1 = V_l coreT)
//   JuW = J_u, JvW = J_v              (lp x kp, FP32; for U_l J_u, V_l J_v)
//   sinv(c) = 1 / s_c for c < k       (kp, FP32)
__global__ __launch_bounds__(256) void k_adj_core(const double* __restrict__ Sl, int64_t lp,
                                                  int l, int k, int64_t kp,
                                                  const double* __restrict__ Ju,
                                                  const double* __restrict__ Jv,
                                                  const double* __restrict__ gS,
                                                  float* __restrict__ coreT,
                                                  float* __restrict__ JuW,
                                                  float* __restrict__ JvW,
                                                  float* __restrict__ sinv, int32_t* status) {
  __shared__ int ntie;
  const int tid = threadIdx.x;
  if (tid == 0) ntie = 0;
  __syncthreads();
  double s1 = 0.0;
  for (int a = 0; a < l; ++a) s1 = fmax(s1, Sl[a]);
  const double s1sq = s1 * s1;
  for (int e = tid; e < lp * lp; e += 256) {
    const int a = e / (int)lp, b = e % (int)lp;   // core(a, b)
    double v = 0.0;
    if (a < l && b < l) {
      if (a == b) {
        v = (gS && a < k) ? gS[a] : 0.0;
      } else {
        const double sa = Sl[a], sb = Sl[b];
        const double diff = sb * sb - sa * sa;
        double f = 0.0;
        if (fabs(diff) > 1e-12 * s1sq) {
          f = 1.0 / diff;
        } else if (a < k || b < k) {
          atomicAdd(&ntie, 1);
        }
        const double jab = (b < k) ? Ju[(int64_t)a * kp + b] : 0.0;
        const double jba = (a < k) ? Ju[(int64_t)b * kp + a] : 0.0;
        const double vab = (b < k) ? Jv[(int64_t)a * kp + b] : 0.0;
        const double vba = (a < k) ? Jv[(int64_t)b * kp + a] : 0.0;
        v = f * (jab - jba) * sb + sa * f * (vab - vba);
      }
    }
    coreT[(int64_t)b * lp + a] = (float)v;
  }
  for (int e = tid; e < lp * kp; e += 256) {
    const int a = e / (int)kp, c = e % (int)kp;
    const bool ok = a < l && c < k;
    JuW[e] = ok ? (float)Ju[e] : 0.f;
    JvW[e] = ok ? (float)Jv[e] : 0.f;
  }
  for (int c = tid; c < kp; c += 256) {
    const double sc = c < k ? Sl[c] : 0.0;
    sinv[c] = (c < k && sc > 1e-12 * s1) ? (float)(1.0 / sc) : 0.f;
  }
  __syncthreads();
  if (tid == 0) status[kStTies] = ntie;
}

// out(i, c) = (x(i, c) - y(i, c)) * sc(c) for i < rows (y, sc optional);
// rows [rows, out_rows) zero.
__global__ void k_colscale(const float* __restrict__ x, int64_t ldx, const float* __restrict__ y,
                           int64_t ldy, const float* __restrict__ sc, int64_t rows, int64_t cols,
                           float* __restrict__ out, int64_t ldo, int64_t out_rows) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= out_rows * cols) return;
  const int64_t c = t / out_rows, i = t % out_rows;
  float v = 0.f;
  if (i < rows) {
    v = x ? x[c * ldx + i] : 0.f;
    if (y) v -= y[c * ldy + i];
    if (sc) v *= sc[c];
  }
  out[c * ldo + i] = v;
}

// gA (m x n, row-major) = P R^T with P (m x K), R (n x K) column-major.
// 128 x 128 output tile per workgroup, K staged through LDS in slabs of 16;
// each wave owns a 64 x 64 quarter as 2 x 2 MFMA 32x32 tiles.
constexpr int OT = 128, OK = 16;
__global__ __launch_bounds__(256) void k_outer(const float* __restrict__ P, int64_t ldp,
                                               const float* __restrict__ R, int64_t ldr, int64_t K,
                                               int64_t m, int64_t n, float* __restrict__ gA,
                                               int64_t ldga) {
  __shared__ __attribute__((aligned(16))) float Ps[OK][OT + 4];
  __shared__ __attribute__((aligned(16))) float Rs[OK][OT + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int64_t i0 = (int64_t)blockIdx.y * OT, j0 = (int64_t)blockIdx.x * OT;
  const int wi = (wave >> 1) * 64, wj = (wave & 1) * 64;
  f32x16 acc[2][2] = {{f32x16{}, f32x16{}}, {f32x16{}, f32x16{}}};
  const int lr = tid >> 5, lc = (tid & 31) * 4;     // 8 rows x 32 float4 per pass
  for (int64_t r0 = 0; r0 < K; r0 += OK) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int rr = lr + 8 * s;
      const int64_t r = r0 + rr;
      float4 vp = make_float4(0.f, 0.f, 0.f, 0.f), vr = vp;
      if (r < K) {
        const int64_t ii = i0 + lc, jj = j0 + lc;
        vp = ld4_scalar(P + r * ldp, ii, m);
        vr = ld4_scalar(R + r * ldr, jj, n);
      }
      *reinterpret_cast<float4*>(&Ps[rr][lc]) = vp;
      *reinterpret_cast<float4*>(&Rs[rr][lc]) = vr;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < OK / 2; ++s) {
      const int kk = 2 * s + half;
      float a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = Ps[kk][wi + t * 32 + l32];
        b[t] = Rs[kk][wj + t * 32 + l32];
      }
#pragma unroll
      for (int ta = 0; ta < 2; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) acc[ta][tb] = mfma32(a[ta], b[tb], acc[ta][tb]);
    }
    __syncthreads();
  }
  // lane holds D(8g + 4 half + e, l32): rows i, column j; row-major stores
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb) {
      const int64_t j = j0 + wj + tb * 32 + l32;
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t i = i0 + wi + ta * 32 + 8 * g + 4 * half + e;
          if (i < m && j < n) gA[i * ldga + j] = acc[ta][tb][4 * g + e];
        }
    }
}

}  // namespace

hipError_t launch_xgram(const float* P, int64_t ldp, int64_t cp, const float* R, int64_t ldr,
                        int64_t cr, int64_t rows, int64_t chunk_rows, int64_t chunks,
                        double* gpart, double* C, hipStream_t s) {
  const int nbp = (int)ceil_div_dev(cp, 64), nbq = (int)ceil_div_dev(cr, 64);
  hipLaunchKernelGGL(k_xgram_part, dim3((unsigned)(nbp * nbq), (unsigned)chunks), dim3(256), 0, s,
                     P, ldp, cp, R, ldr, cr, rows, chunk_rows, gpart, nbp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_xgram_reduce, dim3((unsigned)ceil_div_dev((int64_t)nbp * nbq * 4096, 256)),
                     dim3(256), 0, s, gpart, chunks, nbp * nbq, nbp, cp, cr, C);
  return hipGetLastError();
}

hipError_t launch_adj_core(const double* Sl, int64_t lp, int64_t l, int64_t k, int64_t kp,
                           const double* Ju, const double* Jv, const double* gS, float* coreT,
                           float* JuW, float* JvW, float* sinv, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_core, dim3(1), dim3(256), 0, s, Sl, lp, (int)l, (int)k, kp, Ju, Jv, gS,
                     coreT, JuW, JvW, sinv, status);
  return hipGetLastError();
}

hipError_t launch_colscale(const float* x, int64_t ldx, const float* y, int64_t ldy,
                           const float* sc, int64_t rows, int64_t cols, float* out, int64_t ldo,
                           int64_t out_rows, hipStream_t s) {
  const int64_t total = out_rows * cols;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_colscale, dim3((unsigned)ceil_div_dev(total, 256)), dim3(256), 0, s, x, ldx,
                     y, ldy, sc, rows, cols, out, ldo, out_rows);
  return hipGetLastError();
}

hipError_t launch_outer(const float* P, int64_t ldp, const float* R, int64_t ldr, int64_t K,
                        int64_t m, int64_t n, float* gA, int64_t ldga, hipStream_t s) {
  dim3 grid((unsigned)ceil_div_dev(n, OT), (unsigned)ceil_div_dev(m, OT));
  if (grid.y > 65535u) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_outer, grid, dim3(256), 0, s, P, ldp, R, ldr, K, m, n, gA, ldga);
  return hipGetLastError();
}

}  // namespace rsvd
