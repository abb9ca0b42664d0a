// Products of A with a tall-skinny panel on the FP32 matrix cores of gfx950
// (v_mfma_f32_32x32x2_f32, FP32 accumulation).
//
// These are the passes over A of the randomized SVD: the sketch A O
// (Section 2.1, step 2), the power-iteration products with A and A^T
// (Section 2.2, Eq. (2)) and the projection A^T Q (step 5).  Each launch
// covers every block-cyclic tile of A (Section 2.3, Eq. (3); Section 3.1):
// grid.y is the tile index along the reduced dimension and each tile's
// contribution goes to its own partial panel, summed afterwards in tile order
// (a deterministic split-K).  Panels are column-major (element (i, c) at
// P[c * ld + i]); the sketch width is padded to a multiple of 32 with zero
// columns, so one workgroup owns all lp columns of its rows and A is read
// from HBM exactly once per pass.
#include <algorithm>

#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace rsvd {

namespace {

constexpr int BM = 128;     // rows of A (NN) or columns of A (TN) per workgroup
constexpr int BK = 32;      // reduction slab
constexpr int PADK = BK + 4;

__device__ inline f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Lane (l32, half) of an MFMA 32x32x2 step holds operand row/column l32 and
// reduction slot `half`.  Within a 32-deep slab the two halves take the
// reduction indices [0, 16) and [16, 32) in order: any assignment works as
// long as both operands use the same one.

// Store the 32x32 accumulator block of one wave: lane holds, for g = 0..3,
// output rows 8g + 4*half + (0..3) of column l32.
__device__ inline void store_acc(float* out, int64_t ld, int64_t row_base, int col,
                                 const f32x16& acc, int half) {
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int64_t r = row_base + 8 * g + 4 * half;
    st4(out + (int64_t)col * ld + r,
        make_float4(acc[4 * g + 0], acc[4 * g + 1], acc[4 * g + 2], acc[4 * g + 3]));
  }
}

template <int NT, bool VEC>
__global__ __launch_bounds__(256) void k_nn_f32(const float* __restrict__ A, int64_t lda, int64_t m,
                                                int64_t n, int64_t tn, const float* __restrict__ X,
                                                int64_t ldx, float* __restrict__ Y, int64_t ldy,
                                                int64_t part_stride) {
  constexpr int LP = NT * 32;
  __shared__ __attribute__((aligned(16))) float As[2][BM][PADK];
  __shared__ __attribute__((aligned(16))) float Xs[2][LP][PADK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int64_t i0 = (int64_t)blockIdx.x * BM;
  const int64_t k0 = (int64_t)blockIdx.y * tn;
  const int64_t k1 = min(n, k0 + tn);
  float* Yp = Y + (int64_t)blockIdx.y * part_stride;

  const int lr = tid >> 3;          // 0..31
  const int lc = (tid & 7) * 4;     // 0..28

  float4 ra[4];
  float4 rx[NT];
  auto gload = [&](int64_t kt) {
    const int64_t kk = kt + lc;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t i = i0 + lr + 32 * s;
      if (i < m && kk < k1)
        ra[s] = VEC ? ld4_masked(A + i * lda, kk, k1) : ld4_scalar(A + i * lda, kk, k1);
      else
        ra[s] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int s = 0; s < NT; ++s) {
      const int c = lr + 32 * s;
      rx[s] = (kk < k1) ? ld4_masked(X + (int64_t)c * ldx, kk, k1) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int s = 0; s < 4; ++s) *reinterpret_cast<float4*>(&As[buf][lr + 32 * s][lc]) = ra[s];
#pragma unroll
    for (int s = 0; s < NT; ++s) *reinterpret_cast<float4*>(&Xs[buf][lr + 32 * s][lc]) = rx[s];
  };

  f32x16 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x16{};

  gload(k0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int64_t kt = k0; kt < k1; kt += BK) {
    const bool more = kt + BK < k1;
    if (more) gload(kt + BK);
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
      float a[8];
      const float* ap = &As[buf][wave * 32 + l32][half * 16 + sg * 8];
      *reinterpret_cast<float4*>(&a[0]) = *reinterpret_cast<const float4*>(ap);
      *reinterpret_cast<float4*>(&a[4]) = *reinterpret_cast<const float4*>(ap + 4);
      float b[NT][8];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const float* bp = &Xs[buf][t * 32 + l32][half * 16 + sg * 8];
        *reinterpret_cast<float4*>(&b[t][0]) = *reinterpret_cast<const float4*>(bp);
        *reinterpret_cast<float4*>(&b[t][4]) = *reinterpret_cast<const float4*>(bp + 4);
      }
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma32(a[s], b[t][s], acc[t]);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) store_acc(Yp, ldy, i0 + wave * 32, t * 32 + l32, acc[t], half);
}

template <int NT>
__global__ __launch_bounds__(256) void k_tn_f32(const float* __restrict__ A, int64_t lda, int64_t m,
                                                int64_t n, int64_t tm, const float* __restrict__ Q,
                                                int64_t ldq, float* __restrict__ Z, int64_t ldz,
                                                int64_t part_stride) {
  constexpr int LP = NT * 32;
  __shared__ __attribute__((aligned(16))) float Qs[2][LP][PADK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int64_t j0 = (int64_t)blockIdx.x * BM;
  const int64_t ib0 = (int64_t)blockIdx.y * tm;
  const int64_t ib1 = min(m, ib0 + tm);
  float* Zp = Z + (int64_t)blockIdx.y * part_stride;
  const int64_t j = j0 + wave * 32 + l32;     // column of A this lane feeds
  const bool jok = j < n;

  const int lr = tid >> 3;
  const int lc = (tid & 7) * 4;

  float ra[16];
  float4 rq[NT];
  // A^T operand straight from HBM: lanes 0-31 read 32 consecutive columns of
  // one row of A (128 bytes), lanes 32-63 the row 16 below.
  auto gload = [&](int64_t it) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int64_t i = it + half * 16 + s;
      ra[s] = (jok && i < ib1) ? A[i * lda + j] : 0.f;
    }
    const int64_t kk = it + lc;
#pragma unroll
    for (int s = 0; s < NT; ++s) {
      const int c = lr + 32 * s;
      rq[s] = (kk < ib1) ? ld4_masked(Q + (int64_t)c * ldq, kk, ib1) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };

  f32x16 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x16{};

  float cur[16];
  gload(ib0);
#pragma unroll
  for (int s = 0; s < NT; ++s) *reinterpret_cast<float4*>(&Qs[0][lr + 32 * s][lc]) = rq[s];
#pragma unroll
  for (int s = 0; s < 16; ++s) cur[s] = ra[s];
  __syncthreads();
  int buf = 0;
  for (int64_t it = ib0; it < ib1; it += BK) {
    const bool more = it + BK < ib1;
    if (more) gload(it + BK);
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
      float b[NT][8];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const float* bp = &Qs[buf][t * 32 + l32][half * 16 + sg * 8];
        *reinterpret_cast<float4*>(&b[t][0]) = *reinterpret_cast<const float4*>(bp);
        *reinterpret_cast<float4*>(&b[t][4]) = *reinterpret_cast<const float4*>(bp + 4);
      }
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma32(cur[sg * 8 + s], b[t][s], acc[t]);
    }
    if (more) {
#pragma unroll
      for (int s = 0; s < NT; ++s) *reinterpret_cast<float4*>(&Qs[buf ^ 1][lr + 32 * s][lc]) = rq[s];
#pragma unroll
      for (int s = 0; s < 16; ++s) cur[s] = ra[s];
    }
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) store_acc(Zp, ldz, j0 + wave * 32, t * 32 + l32, acc[t], half);
}

__global__ void k_reduce_parts(const float* __restrict__ part, int64_t stride, int64_t S,
                               float* __restrict__ out, int64_t count4) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count4) return;
  float4 acc = ld4(part + 4 * t);
  for (int64_t s = 1; s < S; ++s) {
    const float4 v = ld4(part + s * stride + 4 * t);
    acc.x += v.x;
    acc.y += v.y;
    acc.z += v.z;
    acc.w += v.w;
  }
  st4(out + 4 * t, acc);
}

__global__ void k_cast_f64_f32(const double* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                               float* __restrict__ out, int64_t ldo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * ldo) return;
  const int64_t i = t / ldo, jj = t % ldo;
  out[t] = jj < n ? (float)A[i * lda + jj] : 0.f;
}

}  // namespace

#define RSVD_NT_SWITCH(NTV, CALL) \
  switch (NTV) {                  \
    case 1: CALL(1); break;       \
    case 2: CALL(2); break;       \
    case 3: CALL(3); break;       \
    case 4: CALL(4); break;       \
    case 5: CALL(5); break;       \
    case 6: CALL(6); break;       \
    default: return hipErrorInvalidValue; \
  }

static hipError_t launch_nn_f32_slice(const float* A, int64_t lda, int64_t m, int64_t n, int64_t tn, int64_t TJ,
                         const float* X, int64_t ldx, int64_t lp, float* Y, int64_t ldy,
                         int64_t part_stride, hipStream_t s) {
  dim3 grid((unsigned)ceil_div_dev(m, BM), (unsigned)TJ);
  const bool vec = (lda % 4) == 0 && (((uintptr_t)A) & 15) == 0;
#define NN_CALL(NT)                                                                          \
  do {                                                                                       \
    if (vec)                                                                                 \
      hipLaunchKernelGGL((k_nn_f32<NT, true>), grid, dim3(256), 0, s, A, lda, m, n, tn, X,   \
                         ldx, Y, ldy, part_stride);                                          \
    else                                                                                     \
      hipLaunchKernelGGL((k_nn_f32<NT, false>), grid, dim3(256), 0, s, A, lda, m, n, tn, X,  \
                         ldx, Y, ldy, part_stride);                                          \
  } while (0)
  RSVD_NT_SWITCH(lp / 32, NN_CALL)
#undef NN_CALL
  return hipGetLastError();
}

static hipError_t launch_tn_f32_slice(const float* A, int64_t lda, int64_t m, int64_t n, int64_t tm, int64_t TI,
                         const float* Q, int64_t ldq, int64_t lp, float* Z, int64_t ldz,
                         int64_t part_stride, hipStream_t s) {
  dim3 grid((unsigned)ceil_div_dev(n, BM), (unsigned)TI);
#define TN_CALL(NT)                                                                               \
  hipLaunchKernelGGL(k_tn_f32<NT>, grid, dim3(256), 0, s, A, lda, m, n, tm, Q, ldq, Z, ldz, \
                     part_stride)
  RSVD_NT_SWITCH(lp / 32, TN_CALL)
#undef TN_CALL
  return hipGetLastError();
}

hipError_t launch_reduce_parts(const float* part, int64_t stride, int64_t S, float* out,
                               int64_t count, hipStream_t s) {
  const int64_t c4 = count / 4;
  hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)ceil_div_dev(c4, 256)), dim3(256), 0, s, part,
                     stride, S, out, c4);
  return hipGetLastError();
}

hipError_t launch_cast_f64_f32(const double* A, int64_t lda, int64_t m, int64_t n, float* out,
                               int64_t ldo, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f64_f32, dim3((unsigned)ceil_div_dev(m * ldo, 256)), dim3(256), 0, s, A,
                     lda, m, n, out, ldo);
  return hipGetLastError();
}

}  // namespace rsvd

namespace rsvd {
namespace {
// dst(i, c) = src(i, c) for i < rows, c < cols; 0 elsewhere in [0, dst_rows) x [0, dst_cols).
__global__ void k_panel_copy(const float* __restrict__ src, int64_t lds, int64_t rows, int64_t cols,
                             float* __restrict__ dst, int64_t ldd, int64_t dst_rows,
                             int64_t dst_cols) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= dst_rows * dst_cols) return;
  const int64_t c = t / dst_rows, i = t % dst_rows;
  dst[c * ldd + i] = (i < rows && c < cols) ? src[c * lds + i] : 0.f;
}
}  // namespace

hipError_t launch_panel_copy(const float* src, int64_t lds, int64_t rows, int64_t cols, float* dst,
                             int64_t ldd, int64_t dst_rows, int64_t dst_cols, hipStream_t s) {
  const int64_t total = dst_rows * dst_cols;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_panel_copy, dim3((unsigned)ceil_div_dev(total, 256)), dim3(256), 0, s, src,
                     lds, rows, cols, dst, ldd, dst_rows, dst_cols);
  return hipGetLastError();
}

// Panels wider than kSliceMax columns are multiplied in column slices
// (plan.h, slice_width): one launch per slice, each reading A once more;
// the slices' columns are independent, so results equal a single launch.
hipError_t launch_nn_f32(const float* A, int64_t lda, int64_t m, int64_t n, int64_t tn, int64_t TJ,
                         const float* X, int64_t ldx, int64_t lp, float* Y, int64_t ldy,
                         int64_t part_stride, hipStream_t s) {
  const int64_t cw = slice_width(lp);
  for (int64_t c0 = 0; c0 < lp; c0 += cw) {
    const hipError_t e = launch_nn_f32_slice(A, lda, m, n, tn, TJ, X + c0 * ldx, ldx,
                                             std::min(cw, lp - c0), Y + c0 * ldy, ldy,
                                             part_stride, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_tn_f32(const float* A, int64_t lda, int64_t m, int64_t n, int64_t tm, int64_t TI,
                         const float* Q, int64_t ldq, int64_t lp, float* Z, int64_t ldz,
                         int64_t part_stride, hipStream_t s) {
  const int64_t cw = slice_width(lp);
  for (int64_t c0 = 0; c0 < lp; c0 += cw) {
    const hipError_t e = launch_tn_f32_slice(A, lda, m, n, tm, TI, Q + c0 * ldq, ldq,
                                             std::min(cw, lp - c0), Z + c0 * ldz, ldz,
                                             part_stride, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rsvd
