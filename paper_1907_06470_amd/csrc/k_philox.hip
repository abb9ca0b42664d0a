// Gaussian test matrix O of step 1 of the randomized SVD (Section 2.1): every
// entry independently N(0, 1).  Entry (j, c) is a pure function of
// (seed, j, c): Philox-4x32-10 (Salmon et al., SC'11) on the counter
// (c / 4, j mod 2^32, j / 2^32, stream) with key (seed mod 2^32, seed / 2^32);
// the four words become uniforms (x + 1/2) 2^-32, and Box-Muller maps the pair
// (u0, u1) to columns 4b, 4b+1 and (u2, u3) to 4b+2, 4b+3.  Any row block is
// generated on its own, which the block-wise passes need (Section 2.3).
#include "device.h"
#include "kernels.h"

namespace rsvd {

__device__ inline void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;   // Weyl increments of the key schedule
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, x0), lo0 = 0xD2511F53u * x0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, x2), lo1 = 0xCD9E8D57u * x2;
    const uint32_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
    x0 = n0;
    x1 = lo1;
    x2 = n2;
    x3 = lo0;
  }
}

__device__ inline void philox_block(uint64_t seed, uint32_t stream, int64_t j, uint32_t b,
                                    uint32_t w[4]) {
  uint32_t x0 = b, x1 = (uint32_t)((uint64_t)j & 0xFFFFFFFFu), x2 = (uint32_t)((uint64_t)j >> 32),
           x3 = stream;
  philox4x32_10(x0, x1, x2, x3, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32));
  w[0] = x0;
  w[1] = x1;
  w[2] = x2;
  w[3] = x3;
}

// Four Gaussians of column block b of row j.
__device__ inline void gauss4(uint64_t seed, int64_t j, uint32_t b, double g[4]) {
  uint32_t w[4];
  philox_block(seed, 0u, j, b, w);
  const double two_pi = 6.283185307179586476925286766559;
  const double scale = 2.3283064365386962890625e-10;   // 2^-32
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double ua = ((double)w[2 * h] + 0.5) * scale;
    const double ub = ((double)w[2 * h + 1] + 0.5) * scale;
    const double rho = sqrt(-2.0 * log(ua));
    const double t = two_pi * ub;
    g[2 * h] = rho * cos(t);
    g[2 * h + 1] = rho * sin(t);
  }
}

__global__ void k_philox_raw(uint64_t seed, uint32_t stream, int64_t row0, int64_t rows,
                             int64_t blocks, uint32_t* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * blocks) return;
  const int64_t r = t / blocks, b = t % blocks;
  uint32_t w[4];
  philox_block(seed, stream, row0 + r, (uint32_t)b, w);
  uint4 v = make_uint4(w[0], w[1], w[2], w[3]);
  *reinterpret_cast<uint4*>(out + 4 * t) = v;
}

template <typename T>
__global__ void k_omega_rows(uint64_t seed, int64_t l, int64_t row0, int64_t rows, T* out,
                             int64_t ldo) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t b = blockIdx.y;
  if (r >= rows) return;
  double g[4];
  gauss4(seed, row0 + r, b, g);
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int64_t c = 4 * (int64_t)b + w;
    if (c < l) out[r * ldo + c] = (T)g[w];
  }
}

// O as a column-major FP32 panel (n x lp, leading dimension ld): columns
// [l, lp) and rows [n, ld) are zero.
__global__ void k_omega_panel(uint64_t seed, int64_t n, int64_t l, int64_t lp, float* X,
                              int64_t ld) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t b = blockIdx.y;
  if (j >= ld) return;
  double g[4] = {0.0, 0.0, 0.0, 0.0};
  if (j < n && 4 * (int64_t)b < l) gauss4(seed, j, b, g);
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int64_t c = 4 * (int64_t)b + w;
    if (c < lp) X[c * ld + j] = (j < n && c < l) ? (float)g[w] : 0.f;
  }
}

hipError_t launch_philox_raw(uint64_t seed, uint32_t stream_id, int64_t row0, int64_t rows,
                             int64_t blocks, uint32_t* out, hipStream_t s) {
  const int64_t total = rows * blocks;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_raw, dim3((unsigned)ceil_div_dev(total, 256)), dim3(256), 0, s, seed,
                     stream_id, row0, rows, blocks, out);
  return hipGetLastError();
}

hipError_t launch_omega_rows(uint64_t seed, int64_t l, int64_t row0, int64_t rows, bool f64,
                             void* out, int64_t ldo, hipStream_t s) {
  if (rows <= 0 || l <= 0) return hipSuccess;
  dim3 grid((unsigned)ceil_div_dev(rows, 256), (unsigned)ceil_div_dev(l, 4));
  if (f64)
    hipLaunchKernelGGL(k_omega_rows<double>, grid, dim3(256), 0, s, seed, l, row0, rows,
                       (double*)out, ldo);
  else
    hipLaunchKernelGGL(k_omega_rows<float>, grid, dim3(256), 0, s, seed, l, row0, rows,
                       (float*)out, ldo);
  return hipGetLastError();
}

hipError_t launch_omega_panel(uint64_t seed, int64_t n, int64_t l, int64_t lp, float* X,
                              int64_t ld, hipStream_t s) {
  dim3 grid((unsigned)ceil_div_dev(ld, 256), (unsigned)ceil_div_dev(lp, 4));
  hipLaunchKernelGGL(k_omega_panel, grid, dim3(256), 0, s, seed, n, l, lp, X, ld);
  return hipGetLastError();
}

}  // namespace rsvd
