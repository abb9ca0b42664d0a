// Device-side helpers shared by the CDNA4 (gfx950) kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsvd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Launch-time description of a column-major panel: element (i, c) at
// base[c * ld + i], rows valid, lp columns.
struct PanelF32 {
  float* p;
  int64_t ld;
};

__device__ inline float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ inline void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }

// Load 4 consecutive floats from row-major storage with a per-element bound.
__device__ inline float4 ld4_masked(const float* row, int64_t k, int64_t kend) {
  if (k + 4 <= kend) return ld4(row + k);
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (k + 0 < kend) v.x = row[k + 0];
  if (k + 1 < kend) v.y = row[k + 1];
  if (k + 2 < kend) v.z = row[k + 2];
  return v;
}

// Same, element by element (rows that are not 16-byte aligned).
__device__ inline float4 ld4_scalar(const float* row, int64_t k, int64_t kend) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (k + 0 < kend) v.x = row[k + 0];
  if (k + 1 < kend) v.y = row[k + 1];
  if (k + 2 < kend) v.z = row[k + 2];
  if (k + 3 < kend) v.w = row[k + 3];
  return v;
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline int is_finite_d(double x) { return __builtin_isfinite(x); }

// Lane exchange inside rows of 16 lanes through DPP (one VALU instruction per
// 32-bit half; no LDS round trip).
template <int CTRL>
__device__ inline double dpp_d(double v) {
  int lo, hi;
  __builtin_memcpy(&lo, &v, 4);
  __builtin_memcpy(&hi, reinterpret_cast<const char*>(&v) + 4, 4);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  double r;
  __builtin_memcpy(&r, &lo, 4);
  __builtin_memcpy(reinterpret_cast<char*>(&r) + 4, &hi, 4);
  return r;
}

// Sum over each row of 16 lanes, the same bits in every lane of the row:
// swap neighbours, swap pairs, mirror within 8, mirror within 16.
__device__ inline double row16_sum(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);   // row_half_mirror
  v += dpp_d<0x140>(v);   // row_mirror
  return v;
}

// Reciprocal and reciprocal square root from the hardware estimates plus two
// Newton steps (relative error ~1e-16; enough for Jacobi rotations, whose
// parameters need not be correctly rounded).
__device__ inline double fast_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * (2.0 - x * y);
  return y * (2.0 - x * y);
}
__device__ inline double fast_rsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  return y * (1.5 - 0.5 * x * y * y);
}

__device__ inline double readlane_d(double v, int lane) {
  int lo, hi;
  __builtin_memcpy(&lo, &v, 4);
  __builtin_memcpy(&hi, reinterpret_cast<const char*>(&v) + 4, 4);
  lo = __builtin_amdgcn_readlane(lo, lane);
  hi = __builtin_amdgcn_readlane(hi, lane);
  double r;
  __builtin_memcpy(&r, &lo, 4);
  __builtin_memcpy(reinterpret_cast<char*>(&r) + 4, &hi, 4);
  return r;
}

// Value of lane n of each row of 16 lanes, in every lane of that row (DPP
// row_newbcast; n must fold to a constant).
__device__ inline double row16_bcast(double v, int n) {
  int lo, hi;
  __builtin_memcpy(&lo, &v, 4);
  __builtin_memcpy(&hi, reinterpret_cast<const char*>(&v) + 4, 4);
  switch (n) {
#define RSVD_BC(N)                                          \
  case N:                                                   \
    lo = __builtin_amdgcn_mov_dpp(lo, 0x150 + N, 0xF, 0xF, false); \
    hi = __builtin_amdgcn_mov_dpp(hi, 0x150 + N, 0xF, 0xF, false); \
    break;
    RSVD_BC(0) RSVD_BC(1) RSVD_BC(2) RSVD_BC(3) RSVD_BC(4) RSVD_BC(5) RSVD_BC(6) RSVD_BC(7)
    RSVD_BC(8) RSVD_BC(9) RSVD_BC(10) RSVD_BC(11) RSVD_BC(12) RSVD_BC(13) RSVD_BC(14) RSVD_BC(15)
#undef RSVD_BC
    default: break;
  }
  double r;
  __builtin_memcpy(&r, &lo, 4);
  __builtin_memcpy(reinterpret_cast<char*>(&r) + 4, &hi, 4);
  return r;
}

// Workgroup barrier that orders LDS only: global stores issued before it stay
// in flight (a plain __syncthreads() would wait for them to reach memory).
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace rsvd
