// Accuracy pass: ||A - U diag(S) V^T||_F, computed directly, tile by tile.
// Each workgroup rebuilds a 64 x 128 tile of U S V^T on the FP32 matrix cores
// (reduction over the k columns), subtracts it from the matching tile of A in
// FP64 and sums the squares in FP64; workgroup partials are then summed in a
// fixed order (deterministic).  One more pass over A; the randomized SVD
// itself does not need it.
#include "device.h"
#include "kernels.h"

namespace rsvd {

namespace {

__device__ inline f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

constexpr int kResidWGs = 2048;

template <typename TA>
__global__ __launch_bounds__(256) void k_residual(const TA* __restrict__ A, int64_t lda, int64_t m,
                                                  int64_t n, const float* __restrict__ U,
                                                  int64_t ldu, const double* __restrict__ S,
                                                  const float* __restrict__ V, int64_t ldv, int k,
                                                  double* __restrict__ partial) {
  __shared__ double red[256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int64_t tiles_j = (n + 127) / 128, tiles = tiles_j * ((m + 63) / 64);
  double sum = 0.0;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t rb = (tile / tiles_j) * 64 + (wave >> 1) * 32;   // rows of this wave
    const int64_t cb = (tile % tiles_j) * 128 + (wave & 1) * 64;   // columns of this wave
    const int64_t i = rb + l32;
    f32x16 acc[2] = {f32x16{}, f32x16{}};
    for (int c0 = 0; c0 < k; c0 += 2) {
      const int c = c0 + half;
      const float a = (i < m && c < k) ? U[(int64_t)c * ldu + i] * (float)S[c] : 0.f;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int64_t j = cb + t * 32 + l32;
        const float b = (j < n && c < k) ? V[(int64_t)c * ldv + j] : 0.f;
        acc[t] = mfma32(a, b, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int64_t j = cb + t * 32 + l32;
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t r = rb + 8 * g + 4 * half + e;
          if (r < m && j < n) {
            const double d = (double)A[r * lda + j] - (double)acc[t][4 * g + e];
            sum += d * d;
          }
        }
    }
  }
  red[tid] = sum;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_sqrt(const double* __restrict__ partial, int64_t count,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int64_t e = tid; e < count; e += 256) s += partial[e];
  red[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) out[0] = sqrt(red[0]);
}

}  // namespace

int64_t residual_partials(int64_t, int64_t) { return kResidWGs; }

hipError_t launch_residual(const void* A, bool f64, int64_t lda, int64_t m, int64_t n,
                           const float* U, int64_t ldu, const double* S, const float* V,
                           int64_t ldv, int64_t k, double* partial, double* out, hipStream_t s) {
  dim3 grid(kResidWGs);
  if (f64)
    hipLaunchKernelGGL(k_residual<double>, grid, dim3(256), 0, s, (const double*)A, lda, m, n, U,
                       ldu, S, V, ldv, (int)k, partial);
  else
    hipLaunchKernelGGL(k_residual<float>, grid, dim3(256), 0, s, (const float*)A, lda, m, n, U, ldu,
                       S, V, ldv, (int)k, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_sqrt, dim3(1), dim3(256), 0, s, partial, (int64_t)kResidWGs, out);
  return hipGetLastError();
}

}  // namespace rsvd
