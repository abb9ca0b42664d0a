// FP8 (OCP e4m3) form of the passes over A: A is stored once as FP8 with one
// power-of-two scale per 64 x 64 block, in two layouts (A8 row-major for the
// products A X, A8T = A^T row-major for A^T Q), and each panel operand is
// stored as FP8 with one power-of-two scale per column.  The products run on
// the gfx950 matrix cores (v_mfma_scale_f32_32x32x64_f8f6f4, FP32
// accumulation).  The power-of-two block scale of A is the instruction's A
// scale (an E8M0 exponent byte per lane, applied to that lane's 32 values of
// the 64-deep slab), so the accumulators run across the slabs of a tile with
// no rescaling; the column scale of the panel is applied in the epilogue.
//
// This extends the half-precision storage of Section 3.2 one step further:
// A costs one byte per entry, a quarter of its FP32 size, and every pass over
// A streams half the bytes of the BF16 form.  Quantisation (per value):
//   s = 2^ceil(log2(amax / 448)) over the value's block (s = 1 for an all-zero
//   block), q = round-to-nearest-even(x / s) in e4m3 (|x / s| <= 448, so the
//   conversion never overflows).
#include <algorithm>

#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace rsvd {

namespace {

typedef int v8i __attribute__((ext_vector_type(8)));
typedef uint8_t u8;

constexpr int kQB = 64;          // quantisation block edge (rows and columns)
constexpr float kFp8Max = 448.f;

// 16 bytes of A that is read once (non-temporal: leaves the caches to others)
__device__ inline float4 ld4_nt(const float* p) {
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
  return make_float4(v[0], v[1], v[2], v[3]);
}

// 2^ceil(log2(amax / 448)), at least 2^-126 (a normal FP32 value, so that its
// exponent field is the E8M0 byte of the matrix-core scale; only blocks with
// amax below 448 * 2^-126 are affected, and they still fit e4m3)
__device__ inline float pow2_scale(float amax) {
  if (!(amax > 0.f)) return 1.f;                        // all-zero block
  const float r = amax / kFp8Max;
  int e;
  const float f = __builtin_frexpf(r, &e);              // r = f 2^e, f in [0.5, 1)
  return __builtin_ldexpf(1.f, max(f == 0.5f ? e - 1 : e, -126));
}

// two FP32 values -> two e4m3 bytes (round to nearest even) in the low half
__device__ inline uint32_t cvt2(float a, float b) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
}

__device__ inline float wave_max(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// One workgroup per 64 x 64 block: amax, scale, A8 rows, and the transposed
// block through LDS for A8T.  Thread t covers rows t/16 + 16u (u < 4) and
// columns 4 (t % 16) .. +3 of the block.
template <typename T>
__global__ __launch_bounds__(256) void k_cast_fp8(const T* __restrict__ A, int64_t lda, int64_t m,
                                                  int64_t n, u8* __restrict__ A8, int64_t lda8,
                                                  u8* __restrict__ A8T, int64_t ldat8,
                                                  float* __restrict__ scale, int64_t nbk) {
  __shared__ float red[8];
  __shared__ __attribute__((aligned(16))) u8 Tt[kQB][kQB + 16];   // [column][row]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * kQB, j0 = (int64_t)blockIdx.x * kQB;
  const int cr = tid >> 4, cc = (tid & 15) * 4;
  float x[4][4];
  float amax = 0.f, bad = 0.f;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t i = i0 + cr + 16 * u;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t j = j0 + cc + e;
      x[u][e] = (i < m && j < n) ? (float)A[i * lda + j] : 0.f;
      amax = fmaxf(amax, fabsf(x[u][e]));
      bad = fmaxf(bad, __builtin_isfinite(x[u][e]) ? 0.f : 1.f);
    }
  }
  amax = wave_max(amax);
  bad = wave_max(bad);
  if (lane == 0) {
    red[wave] = amax;
    red[4 + wave] = bad;
  }
  __syncthreads();
  amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  bad = fmaxf(fmaxf(red[4], red[5]), fmaxf(red[6], red[7]));
  // a non-finite value makes the whole block NaN, so the factorisation reports it
  const float s = bad > 0.f ? __builtin_nanf("") : pow2_scale(amax);
  const float inv = 1.f / s;   // exact: s is a power of two
  if (tid == 0) scale[blockIdx.y * nbk + blockIdx.x] = s;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = cr + 16 * u;
    const uint32_t w = cvt2(x[u][0] * inv, x[u][1] * inv) | (cvt2(x[u][2] * inv, x[u][3] * inv) << 16);
    const int64_t i = i0 + r, j = j0 + cc;
    if (i < m && j < n) {
      if (j + 4 <= n && (lda8 & 3) == 0) {
        *reinterpret_cast<uint32_t*>(A8 + i * lda8 + j) = w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (j + e < n) A8[i * lda8 + j + e] = (u8)(w >> (8 * e));
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) Tt[cc + e][r] = (u8)(w >> (8 * e));
  }
  __syncthreads();
  // A8T rows j0 + c, 16 bytes (rows i0 + 16 q ..) per thread
  {
    const int c = tid >> 2, q = (tid & 3) * 16;
    const int64_t j = j0 + c, i = i0 + q;
    if (j < n && i < m) {
      if (i + 16 <= m && (ldat8 & 15) == 0) {
        *reinterpret_cast<uint4*>(A8T + j * ldat8 + i) = *reinterpret_cast<const uint4*>(&Tt[c][q]);
      } else {
        for (int e = 0; e < 16 && i + e < m; ++e) A8T[j * ldat8 + i + e] = Tt[c][q + e];
      }
    }
  }
}

// Same cast for FP32 input, one workgroup per 128 x 256 strip (2 x 4 blocks):
// wave w reads rows 16 w .. 16 w + 15 of the strip, lane L columns 4 L ..
// 4 L + 3 (block L / 16) as 16-byte loads (1 KB per row and wave), so A8 rows
// go out as 256 contiguous bytes and A8T rows (through LDS) as 128.  Each
// thread packs the 16 bytes of one column over its 16 rows and writes them to
// the transposed staging in one store; staging column p holds strip column
// 4 (p % 64) + p / 64, which spreads a store's 64 lanes over all banks.
// Same scales and values as the one-block kernel.
__global__ __launch_bounds__(512) void k_cast_fp8_strip(const float* __restrict__ A, int64_t lda,
                                                        int64_t m, int64_t n,
                                                        u8* __restrict__ A8, int64_t lda8,
                                                        u8* __restrict__ A8T, int64_t ldat8,
                                                        float* __restrict__ scale, int64_t nbk) {
  constexpr int SR = 128, SC = 256, TLD = SR + 16;
  __shared__ float red[2][8][4];                                 // [amax / bad][wave][block column]
  __shared__ __attribute__((aligned(16))) u8 Tt[SC * TLD];       // staging column p, row r
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * SR, j0 = (int64_t)blockIdx.x * SC;
  const int bc = lane >> 4, br = wave >> 2;
  const int64_t jc = j0 + 4 * lane;
  const bool full = i0 + SR <= m && j0 + SC <= n;
  float4 x[16];
  float amax = 0.f, bad = 0.f;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int64_t i = i0 + 16 * wave + u;
    if (full)   // A is read once: a non-temporal load leaves the caches to others
      x[u] = ld4_nt(A + i * lda + jc);
    else
      x[u] = (i < m && jc < n) ? ld4_masked(A + i * lda, jc, n) : make_float4(0.f, 0.f, 0.f, 0.f);
    amax = fmaxf(amax, fmaxf(fmaxf(fabsf(x[u].x), fabsf(x[u].y)), fmaxf(fabsf(x[u].z), fabsf(x[u].w))));
    const bool fin = __builtin_isfinite(x[u].x) && __builtin_isfinite(x[u].y) &&
                     __builtin_isfinite(x[u].z) && __builtin_isfinite(x[u].w);
    bad = fmaxf(bad, fin ? 0.f : 1.f);
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) {        // within the 16 lanes of a block column
    amax = fmaxf(amax, __shfl_xor(amax, off, 64));
    bad = fmaxf(bad, __shfl_xor(bad, off, 64));
  }
  if ((lane & 15) == 0) {
    red[0][wave][bc] = amax;
    red[1][wave][bc] = bad;
  }
  __syncthreads();
  amax = fmaxf(fmaxf(red[0][4 * br][bc], red[0][4 * br + 1][bc]),
               fmaxf(red[0][4 * br + 2][bc], red[0][4 * br + 3][bc]));
  bad = fmaxf(fmaxf(red[1][4 * br][bc], red[1][4 * br + 1][bc]),
              fmaxf(red[1][4 * br + 2][bc], red[1][4 * br + 3][bc]));
  const float sc = bad > 0.f ? __builtin_nanf("") : pow2_scale(amax);
  const float inv = 1.f / sc;   // exact: a power of two
  if ((lane & 15) == 0 && (wave & 3) == 0) {
    const int64_t gbr = blockIdx.y * 2 + br, gbc = blockIdx.x * 4 + bc;
    if (gbr * kQB < m && gbc * kQB < n) scale[gbr * nbk + gbc] = sc;
  }
  uint32_t w[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    w[u] = cvt2(x[u].x * inv, x[u].y * inv) | (cvt2(x[u].z * inv, x[u].w * inv) << 16);
    const int64_t i = i0 + 16 * wave + u;
    if (full) {
      __builtin_nontemporal_store(w[u], reinterpret_cast<uint32_t*>(A8 + i * lda8 + jc));
    } else if (i < m && jc < n) {
      if (jc + 4 <= n && (lda8 & 3) == 0) {
        *reinterpret_cast<uint32_t*>(A8 + i * lda8 + jc) = w[u];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (jc + e < n) A8[i * lda8 + jc + e] = (u8)(w[u] >> (8 * e));
      }
    }
  }
  // column 4 lane + e of the strip, rows 16 wave .. + 15: 16 bytes
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    uint32_t q[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
      q[v] = ((w[4 * v + 0] >> (8 * e)) & 0xffu) | (((w[4 * v + 1] >> (8 * e)) & 0xffu) << 8) |
             (((w[4 * v + 2] >> (8 * e)) & 0xffu) << 16) | (((w[4 * v + 3] >> (8 * e)) & 0xffu) << 24);
    const int p = e * 64 + lane;
    *reinterpret_cast<uint4*>(&Tt[p * TLD + 16 * wave]) = make_uint4(q[0], q[1], q[2], q[3]);
  }
  __syncthreads();
  // A8T rows j0 + c: 8 threads per column, 16 bytes (rows i0 + 16 t8 ..) each
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int id = tid + 512 * k, c = id >> 3, t8 = id & 7;
    const int p = (c & 3) * 64 + (c >> 2);
    const int64_t j = j0 + c, i = i0 + 16 * t8;
    const uint4 v = *reinterpret_cast<const uint4*>(&Tt[p * TLD + 16 * t8]);
    if (full) {
      typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
      __builtin_nontemporal_store(u32x4{v.x, v.y, v.z, v.w}, reinterpret_cast<u32x4*>(A8T + j * ldat8 + i));
    } else if (j < n && i < m) {
      if (i + 16 <= m && (ldat8 & 15) == 0) {
        *reinterpret_cast<uint4*>(A8T + j * ldat8 + i) = v;
      } else {
        const uint32_t vv[4] = {v.x, v.y, v.z, v.w};
        for (int e = 0; e < 16 && i + e < m; ++e) A8T[j * ldat8 + i + e] = (u8)(vv[e >> 2] >> (8 * (e & 3)));
      }
    }
  }
}

// FP8 copy of an FP32 panel, one workgroup per column: amax over the column,
// power-of-two scale, e4m3 values over the whole leading dimension.
__global__ __launch_bounds__(256) void k_panel_to_fp8(const float* __restrict__ P, int64_t ld,
                                                      int64_t rows, u8* __restrict__ P8,
                                                      float* __restrict__ sc) {
  __shared__ float red[8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t c = blockIdx.x;
  const float* col = P + c * ld;
  float amax = 0.f, bad = 0.f;
  for (int64_t i = 4 * tid; i < rows; i += 1024) {
    const float4 v = ld4_masked(col, i, rows);
    amax = fmaxf(amax, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    const bool fin = __builtin_isfinite(v.x) && __builtin_isfinite(v.y) &&
                     __builtin_isfinite(v.z) && __builtin_isfinite(v.w);
    bad = fmaxf(bad, fin ? 0.f : 1.f);
  }
  amax = wave_max(amax);
  bad = wave_max(bad);
  if (lane == 0) {
    red[wave] = amax;
    red[4 + wave] = bad;
  }
  __syncthreads();
  amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  bad = fmaxf(fmaxf(red[4], red[5]), fmaxf(red[6], red[7]));
  const float s = bad > 0.f ? __builtin_nanf("") : pow2_scale(amax), inv = 1.f / s;
  if (tid == 0) sc[c] = s;
  for (int64_t i = 4 * tid; i < ld; i += 1024) {
    const float4 v = i < rows ? ld4_masked(col, i, rows) : make_float4(0.f, 0.f, 0.f, 0.f);
    const uint32_t w = cvt2(v.x * inv, v.y * inv) | (cvt2(v.z * inv, v.w * inv) << 16);
    *reinterpret_cast<uint32_t*>(P8 + c * ld + i) = w;
  }
}

// c + (2^(sa - 127) a) b on e4m3 operands: sa is the E8M0 scale byte of this
// lane's A values, sb that of its B values.  Both are passed in registers
// (a scale the compiler sees as a constant would be encoded as an FP32
// inline constant instead of a byte).
__device__ inline f32x16 mfma_fp8(const v8i& a, const v8i& b, f32x16 c, int sa, int sb) {
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
}

// E8M0 byte of a power-of-two FP32 scale (its exponent field; NaN gives 0xFF,
// the E8M0 NaN, so a non-finite block still poisons its products)
__device__ inline int e8m0_of(float s) { return (int)((__builtin_bit_cast(uint32_t, s) >> 23) & 0xffu); }

// 127 (scale 1) in a register the compiler cannot fold
__device__ inline int e8m0_one() {
  int v = 127;
  asm volatile("" : "+v"(v));
  return v;
}

// 16 consecutive bytes of a row from index k, zero past kend.
__device__ inline uint4 ld16_masked(const u8* row, int64_t k, int64_t kend) {
  if (k + 16 <= kend) return *reinterpret_cast<const uint4*>(row + k);
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  for (int e = 0; e < 16; ++e)
    if (k + e < kend) w[e >> 2] |= (uint32_t)row[k + e] << (8 * (e & 3));
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Y (+ partial per reduction tile) = A8 X8 with the block scales of A and the
// column scales of X.  A8: rows x kdim row-major FP8 (lda8 % 16 == 0); X8:
// column-major FP8 (element (k, c) at X8[c * ldx8 + k]); the reduction tile of
// blockIdx.y covers [y tk, (y + 1) tk) with tk % 64 == 0.  Block scale of rows
// [64 r, 64 r + 64) and reduction slab [64 b, 64 b + 64): sA[r sc_r + b sc_k].
// 4 waves; wave w owns rows [w WR, (w + 1) WR) of BM = 4 WR and all NT * 32
// panel columns; a 128-deep stage holds two 64-deep slabs.
constexpr int BKB = 128;
constexpr int PADB = BKB + 16;
template <int NT, int MT>
__global__ __launch_bounds__(256) void k_nn_fp8(const u8* __restrict__ A, int64_t lda, int64_t rows,
                                                int64_t kdim, int64_t tk,
                                                const float* __restrict__ sA, int64_t sc_r,
                                                int64_t sc_k, const u8* __restrict__ X, int64_t ldx,
                                                const float* __restrict__ sx, float* __restrict__ Y,
                                                int64_t ldy, int64_t part_stride) {
  constexpr int LP = NT * 32, WR = MT * 32, BM = 4 * WR, AS = BM / 32;
  __shared__ __attribute__((aligned(16))) u8 As[2][BM][PADB];
  __shared__ __attribute__((aligned(16))) u8 Xs[2][LP][PADB];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int64_t i0 = (int64_t)blockIdx.x * BM;
  const int64_t k0 = (int64_t)blockIdx.y * tk;
  const int64_t k1 = min(kdim, k0 + tk);
  float* Yp = Y + (int64_t)blockIdx.y * part_stride;
  const int lr = tid >> 3, lc = (tid & 7) * 16;

  uint4 ra[AS];
  uint4 rx[NT];
  auto gload = [&](int64_t kt) {
    const int64_t kk = kt + lc;
#pragma unroll
    for (int s = 0; s < AS; ++s) {
      const int64_t i = i0 + lr + 32 * s;
      ra[s] = (i < rows && kk < k1) ? ld16_masked(A + i * lda, kk, k1) : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int s = 0; s < NT; ++s) {
      const int c = lr + 32 * s;
      rx[s] = kk < k1 ? ld16_masked(X + (int64_t)c * ldx, kk, k1) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int s = 0; s < AS; ++s) *reinterpret_cast<uint4*>(&As[buf][lr + 32 * s][lc]) = ra[s];
#pragma unroll
    for (int s = 0; s < NT; ++s) *reinterpret_cast<uint4*>(&Xs[buf][lr + 32 * s][lc]) = rx[s];
  };

  const int one = e8m0_one();
  f32x16 acc[MT][NT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[a][t] = f32x16{};
  // row block (of the 64-row quantisation grid) of each M tile of this wave
  int64_t rblk[MT];
#pragma unroll
  for (int a = 0; a < MT; ++a) rblk[a] = min(i0 + wave * WR + a * 32, rows - 1) / kQB;

  gload(k0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int64_t kt = k0; kt < k1; kt += BKB) {
    const bool more = kt + BKB < k1;
    if (more) gload(kt + BKB);
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const int64_t kb = kt / kQB + s2;
      if (kb * kQB >= k1) break;
      v8i av[MT], bv[NT];
#pragma unroll
      for (int a = 0; a < MT; ++a) {
        const u8* p = &As[buf][wave * WR + a * 32 + l32][s2 * 64 + half * 32];
        const uint4 lo = *reinterpret_cast<const uint4*>(p);
        const uint4 hi = *reinterpret_cast<const uint4*>(p + 16);
        av[a] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const u8* p = &Xs[buf][t * 32 + l32][s2 * 64 + half * 32];
        const uint4 lo = *reinterpret_cast<const uint4*>(p);
        const uint4 hi = *reinterpret_cast<const uint4*>(p + 16);
        bv[t] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      }
#pragma unroll
      for (int a = 0; a < MT; ++a) {
        const int sa = e8m0_of(sA[rblk[a] * sc_r + kb * sc_k]);
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[a][t] = mfma_fp8(av[a], bv[t], acc[a][t], sa, one);
      }
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = t * 32 + l32;
    const float cs = sx[col];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      const int64_t rb = i0 + wave * WR + a * 32;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t r = rb + 8 * g + 4 * half;
        st4(Yp + (int64_t)col * ldy + r,
            make_float4(acc[a][t][4 * g + 0] * cs, acc[a][t][4 * g + 1] * cs,
                        acc[a][t][4 * g + 2] * cs, acc[a][t][4 * g + 3] * cs));
      }
    }
  }
}

// Direct-to-LDS form for panel width 128 (the same byte geometry and slab
// schedule as the BF16 direct-to-LDS A X kernel): 8 waves, a 256 x 128 output
// block per workgroup (4 x 2 waves of 64 x 64); the A slabs (256 rows x 128
// FP8 = 32 KB, two 64-deep quantisation slabs) stream from HBM into a 4-deep
// LDS ring with buffer_load ... lds, three in flight; the panel slabs (128
// columns x 128) go through registers two slabs ahead into a double buffer.
// Row r of a slab stores its 16-byte chunk c at slot c ^ (r & 7) (the source
// addresses make the swizzle).  Each wave's 64 rows are one quantisation row
// block, so one block scale per wave and 64-deep slab; the per-slab products
// and their scaling are those of the register-staged kernel, in the same
// order.  A partial last slab goes through registers with masked loads.
// Needs 256 * lda and LP * ldx bytes within a 31-bit offset.
//
// NT = 5 (panel width 160), as for the BF16 form: each of the 8 waves takes 32
// rows (half of one quantisation row block) and all five 32-column tiles, the
// A ring has three stages (the panel slab is 20 KB), and the 20 panel runs of
// a slab go to waves w, w + 8, w + 16 (waves 4-7 load their second run once
// more into rows 160-191 of the panel buffer, which nothing reads).
constexpr int F8_BM = 256, F8_ARUN = 4;

template <int NT>
__global__ __launch_bounds__(512) void k_nn_fp8_dl(const u8* __restrict__ A, int64_t lda,
                                                   int64_t rows, int64_t kdim, int64_t tk,
                                                   const float* __restrict__ sA, int64_t sc_r,
                                                   int64_t sc_k, const u8* __restrict__ X,
                                                   int64_t ldx, const float* __restrict__ sx,
                                                   float* __restrict__ Y, int64_t ldy,
                                                   int64_t part_stride) {
  static_assert(NT == 4 || NT == 5, "panel widths 128 and 160");
  constexpr int LP = 32 * NT;
  constexpr int NS = NT == 4 ? 4 : 3;           // A ring stages
  constexpr int XR = NT == 4 ? 2 : 3;           // panel loads per lane and slab
  constexpr int XB = 64 * XR;                   // panel buffer rows (192 at width 160: the
                                                // unused third runs of waves 4-7 land past 160)
  constexpr int MT = NT == 4 ? 2 : 1;           // 32-row tiles per wave
  constexpr int NW = NT == 4 ? 2 : 5;           // 32-column tiles per wave
  __shared__ __attribute__((aligned(1024))) u8 As0[F8_BM * 128], As1[F8_BM * 128];
  __shared__ __attribute__((aligned(1024))) u8 As2[F8_BM * 128], As3[NS == 4 ? F8_BM * 128 : 1];
  __shared__ __attribute__((aligned(1024))) u8 Xs0[XB * 128], Xs1[XB * 128];
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l32 = lane & 31, half = lane >> 5;
  const int wrow = NT == 4 ? (wave & 3) * 64 : wave * 32;
  const int wcol = NT == 4 ? (wave >> 2) * 64 : 0;
  const int64_t i0 = (int64_t)blockIdx.x * F8_BM;
  const int64_t k0 = (int64_t)blockIdx.y * tk;
  const int64_t k1 = min(kdim, k0 + tk);
  float* Yp = Y + (int64_t)blockIdx.y * part_stride;
  const int64_t nfull = (k1 - k0) / 128;
  const bool tail = k0 + nfull * 128 < k1;
  const int rr = lane >> 3, sl = lane & 7;
  const int nrow = (int)min((int64_t)F8_BM, rows - i0);
  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(A + i0 * lda), (short)0, (int)((int64_t)(nrow - 1) * lda + kdim), 0x00020000);
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
      (void*)X, (short)0, (int)((int64_t)(LP - 1) * ldx + kdim), 0x00020000);
  // quantisation row block of this wave's rows (rows past the end: the last)
  const int64_t rblk = min(i0 + wrow, rows - 1) / kQB;

  auto issue_a = [&](u8* st, int64_t t) {   // past the last slab: panel re-reads
    const bool real = t < nfull;
    const __amdgpu_buffer_rsrc_t rs = real ? ra : rx;
    const int kk = (int)(k0 + t * 128);
#pragma unroll
    for (int j = 0; j < F8_ARUN; ++j) {
      const int r = (wave * F8_ARUN + j) * 8 + rr;
      const int rc = min(r, nrow - 1);
      const int c = r % LP;
      const int off = real ? rc * (int)lda + kk + 16 * (sl ^ (r & 7)) : c * (int)ldx + (int)k0 + 16 * sl;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, st + (wave * F8_ARUN + j) * 1024, 16, off, 0, 0, 2);
    }
  };
  // panel runs of this wave (8 panel columns each): 2 w, 2 w + 1 (width 128)
  // or w, w + 8, w + 16 (width 160; runs past the 20 re-read run w + 8 and
  // land in the unread rows 160-191)
  auto xrun = [&](int u) { return NT == 4 ? wave * 2 + u : wave + 8 * u; };
  auto xrun_ld = [&](int u) {
    const int j = xrun(u);
    return j < LP / 8 ? j : xrun(1);
  };
  auto load_x = [&](v4u (&x)[XR], int64_t t) {
    const int kk = (int)(k0 + (t < nfull ? t : 0) * 128);
#pragma unroll
    for (int u = 0; u < XR; ++u) {
      const int c = xrun_ld(u) * 8 + rr;
      x[u] = __builtin_amdgcn_raw_buffer_load_b128(rx, c * (int)ldx + kk + 16 * (sl ^ (c & 7)), 0, 0);
    }
  };
  auto store_x = [&](u8* st, const v4u (&x)[XR]) {
#pragma unroll
    for (int u = 0; u < XR; ++u)
      *reinterpret_cast<v4u*>(st + xrun(u) * 1024 + lane * 16) = x[u];
  };

  const int one = e8m0_one();
  f32x16 acc[MT][NW];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int t = 0; t < NW; ++t) acc[a][t] = f32x16{};

  // 64-deep quantisation slabs nq (1 or 2) of a 128-deep slab from column kb
  auto compute = [&](const u8* as, const u8* xs, int64_t kb, int nq) {
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      if (s2 >= nq) break;
      const int q = 4 * s2 + 2 * half;             // this lane's two 16-byte chunks
      v8i av[MT], bv[NW];
#pragma unroll
      for (int a = 0; a < MT; ++a) {
        const int r = wrow + a * 32 + l32;
        const v4u lo = *reinterpret_cast<const v4u*>(as + r * 128 + 16 * (q ^ (r & 7)));
        const v4u hi = *reinterpret_cast<const v4u*>(as + r * 128 + 16 * ((q + 1) ^ (r & 7)));
        av[a] = v8i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
      }
#pragma unroll
      for (int t = 0; t < NW; ++t) {
        const int c = wcol + t * 32 + l32;
        const v4u lo = *reinterpret_cast<const v4u*>(xs + c * 128 + 16 * (q ^ (c & 7)));
        const v4u hi = *reinterpret_cast<const v4u*>(xs + c * 128 + 16 * ((q + 1) ^ (c & 7)));
        bv[t] = v8i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
      }
      const int sa = e8m0_of(sA[rblk * sc_r + (kb / kQB + s2) * sc_k]);
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int t = 0; t < NW; ++t) acc[a][t] = mfma_fp8(av[a], bv[t], acc[a][t], sa, one);
    }
  };

  // the slab schedule of the BF16 direct-to-LDS kernel
  constexpr int kWaitStep = 0x0f70 | ((NS - 2) * F8_ARUN + XR);
  auto step = [&](int64_t t, u8* as, u8* xs, u8* xs_next, u8* as_refill, v4u (&xp)[XR],
                  v4u (&xn)[XR]) {
    load_x(xn, t + 2);
    issue_a(as_refill, t + NS - 1);
    __builtin_amdgcn_sched_barrier(0);
    compute(as, xs, k0 + t * 128, 2);
    __builtin_amdgcn_s_waitcnt(kWaitStep);
    store_x(xs_next, xp);
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_s_barrier();
  };

  v4u xa[XR], xb[XR];
  if (nfull > 0) {
    load_x(xa, 0);
    __builtin_amdgcn_s_waitcnt(0x0f70);
    store_x(Xs0, xa);
    load_x(xb, 1);
    issue_a(As0, 0);
    issue_a(As1, 1);
    if (NS == 4) issue_a(As2, 2);
    __builtin_amdgcn_s_waitcnt(0x0f70 | ((NS - 2) * F8_ARUN));
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_s_barrier();
  }
  int64_t tb = 0;
  if constexpr (NS == 4) {
    for (; tb + 3 < nfull; tb += 4) {
      step(tb, As0, Xs0, Xs1, As3, xb, xa);
      step(tb + 1, As1, Xs1, Xs0, As0, xa, xb);
      step(tb + 2, As2, Xs0, Xs1, As1, xb, xa);
      step(tb + 3, As3, Xs1, Xs0, As2, xa, xb);
    }
    if (tb < nfull) {
      step(tb, As0, Xs0, Xs1, As3, xb, xa);
      if (tb + 1 < nfull) {
        step(tb + 1, As1, Xs1, Xs0, As0, xa, xb);
        if (tb + 2 < nfull) step(tb + 2, As2, Xs0, Xs1, As1, xb, xa);
      }
    }
  } else {
    for (; tb + 5 < nfull; tb += 6) {
      step(tb, As0, Xs0, Xs1, As2, xb, xa);
      step(tb + 1, As1, Xs1, Xs0, As0, xa, xb);
      step(tb + 2, As2, Xs0, Xs1, As1, xb, xa);
      step(tb + 3, As0, Xs1, Xs0, As2, xa, xb);
      step(tb + 4, As1, Xs0, Xs1, As0, xb, xa);
      step(tb + 5, As2, Xs1, Xs0, As1, xa, xb);
    }
    if (tb < nfull) step(tb, As0, Xs0, Xs1, As2, xb, xa);
    if (tb + 1 < nfull) step(tb + 1, As1, Xs1, Xs0, As0, xa, xb);
    if (tb + 2 < nfull) step(tb + 2, As2, Xs0, Xs1, As1, xb, xa);
    if (tb + 3 < nfull) step(tb + 3, As0, Xs1, Xs0, As2, xa, xb);
    if (tb + 4 < nfull) step(tb + 4, As1, Xs0, Xs1, As0, xb, xa);
  }
  __builtin_amdgcn_s_waitcnt(0x0f70);
  if (tail) {   // last, partial slab: masked loads through registers
    __syncthreads();
    const int64_t kk = k0 + nfull * 128;
    for (int e = tid; e < F8_BM * 8; e += 512) {
      const int r = e >> 3, c = e & 7;
      const int64_t gi = min(i0 + r, rows - 1);
      *reinterpret_cast<uint4*>(As0 + r * 128 + 16 * (c ^ (r & 7))) =
          ld16_masked(A + gi * lda, kk + 16 * c, k1);
    }
    for (int e = tid; e < LP * 8; e += 512) {
      const int r = e >> 3, c = e & 7;
      *reinterpret_cast<uint4*>(Xs0 + r * 128 + 16 * (c ^ (r & 7))) =
          ld16_masked(X + (int64_t)r * ldx, kk + 16 * c, k1);
    }
    __syncthreads();
    compute(As0, Xs0, kk, (int)((k1 - kk + kQB - 1) / kQB));
  }
  // column scales; rows [rows, rows rounded up to 128) stored as zeros, as by
  // the register-staged kernel
  const int64_t rz = (rows + 127) / 128 * 128;
#pragma unroll
  for (int t = 0; t < NW; ++t) {
    const int col = wcol + t * 32 + l32;
    const float cs = sx[col];
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      const int64_t rb = i0 + wrow + a * 32;
      if (rb >= rz) continue;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t r = rb + 8 * g + 4 * half;
        st4(Yp + (int64_t)col * ldy + r,
            make_float4(r + 0 < rows ? acc[a][t][4 * g + 0] * cs : 0.f,
                        r + 1 < rows ? acc[a][t][4 * g + 1] * cs : 0.f,
                        r + 2 < rows ? acc[a][t][4 * g + 2] * cs : 0.f,
                        r + 3 < rows ? acc[a][t][4 * g + 3] * cs : 0.f));
      }
    }
  }
}

// The same conversion split over kPanelFp8Chunks row chunks per column (lp x
// chunks workgroups instead of lp): the chunk maxima and non-finite flags go
// to `part`, and every converting workgroup takes the maximum of its column's
// chunks, so the scale is that of the one-pass kernel (a maximum does not
// depend on its order) and so are the bytes.
__global__ __launch_bounds__(256) void k_panel_amax(const float* __restrict__ P, int64_t ld,
                                                    int64_t rows, int64_t crow,
                                                    float* __restrict__ part) {
  __shared__ float red[8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t c = blockIdx.x, q = blockIdx.y, nq = gridDim.y;
  const float* col = P + c * ld;
  const int64_t r0 = q * crow, r1 = min(rows, r0 + crow);
  float amax = 0.f, bad = 0.f;
  for (int64_t i = r0 + 4 * tid; i < r1; i += 1024) {
    const float4 v = ld4_masked(col, i, r1);
    amax = fmaxf(amax, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    const bool fin = __builtin_isfinite(v.x) && __builtin_isfinite(v.y) &&
                     __builtin_isfinite(v.z) && __builtin_isfinite(v.w);
    bad = fmaxf(bad, fin ? 0.f : 1.f);
  }
  amax = wave_max(amax);
  bad = wave_max(bad);
  if (lane == 0) {
    red[wave] = amax;
    red[4 + wave] = bad;
  }
  __syncthreads();
  if (tid == 0) {
    part[c * nq + q] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    part[(gridDim.x + c) * nq + q] = fmaxf(fmaxf(red[4], red[5]), fmaxf(red[6], red[7]));
  }
}

__global__ __launch_bounds__(256) void k_panel_conv_fp8(const float* __restrict__ P, int64_t ld,
                                                        int64_t rows, int64_t cld,
                                                        const float* __restrict__ part,
                                                        u8* __restrict__ P8,
                                                        float* __restrict__ sc) {
  const int tid = threadIdx.x;
  const int64_t c = blockIdx.x, q = blockIdx.y, nq = gridDim.y;
  // every wave gathers the column's chunk maxima (lane j % nq) and reduces them
  const int64_t j = (tid & 63) % nq;
  const float amax = wave_max(part[c * nq + j]);
  const float bad = wave_max(part[(gridDim.x + c) * nq + j]);
  const float s = bad > 0.f ? __builtin_nanf("") : pow2_scale(amax), inv = 1.f / s;
  if (q == 0 && tid == 0) sc[c] = s;
  const float* col = P + c * ld;
  const int64_t i0 = q * cld, i1 = min(ld, i0 + cld);
  for (int64_t i = i0 + 4 * tid; i < i1; i += 1024) {
    const float4 v = i < rows ? ld4_masked(col, i, rows) : make_float4(0.f, 0.f, 0.f, 0.f);
    const uint32_t w = cvt2(v.x * inv, v.y * inv) | (cvt2(v.z * inv, v.w * inv) << 16);
    *reinterpret_cast<uint32_t*>(P8 + c * ld + i) = w;
  }
}

}  // namespace

int64_t fp8_scale_blocks(int64_t rows, int64_t cols) {
  return ceil_div_dev(rows, kQB) * ceil_div_dev(cols, kQB);
}

hipError_t launch_cast_fp8(const void* A, bool f64, int64_t lda, int64_t m, int64_t n, uint8_t* A8,
                           int64_t lda8, uint8_t* A8T, int64_t ldat8, float* scale,
                           hipStream_t s) {
  if (lda8 < n || ldat8 < m) return hipErrorInvalidValue;
  const int64_t nbk = ceil_div_dev(n, kQB);
  dim3 grid((unsigned)nbk, (unsigned)ceil_div_dev(m, kQB));
  if (!f64 && (lda % 4) == 0 && ((uintptr_t)A & 15) == 0 && (lda8 % 4) == 0 &&
      (ldat8 % 16) == 0 && ((uintptr_t)A8 & 3) == 0 && ((uintptr_t)A8T & 15) == 0) {
    dim3 g2((unsigned)ceil_div_dev(n, 256), (unsigned)ceil_div_dev(m, 128));
    hipLaunchKernelGGL(k_cast_fp8_strip, g2, dim3(512), 0, s, (const float*)A, lda, m, n, A8, lda8,
                       A8T, ldat8, scale, nbk);
  } else if (f64)
    hipLaunchKernelGGL(k_cast_fp8<double>, grid, dim3(256), 0, s, (const double*)A, lda, m, n, A8,
                       lda8, A8T, ldat8, scale, nbk);
  else
    hipLaunchKernelGGL(k_cast_fp8<float>, grid, dim3(256), 0, s, (const float*)A, lda, m, n, A8,
                       lda8, A8T, ldat8, scale, nbk);
  return hipGetLastError();
}

hipError_t launch_panel_to_fp8(const float* P, int64_t ld, int64_t rows, int64_t lp, uint8_t* P8,
                               float* scale, float* part, hipStream_t s) {
  if (ld % 4 != 0 || rows > ld) return hipErrorInvalidValue;
  if (part == nullptr) {
    hipLaunchKernelGGL(k_panel_to_fp8, dim3((unsigned)lp), dim3(256), 0, s, P, ld, rows, P8, scale);
    return hipGetLastError();
  }
  const int64_t crow = ceil_div_dev(ceil_div_dev(rows, kPanelFp8Chunks), 4) * 4;
  const int64_t cld = ceil_div_dev(ceil_div_dev(ld, kPanelFp8Chunks), 4) * 4;
  const dim3 grid((unsigned)lp, (unsigned)kPanelFp8Chunks);
  hipLaunchKernelGGL(k_panel_amax, grid, dim3(256), 0, s, P, ld, rows, crow, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_panel_conv_fp8, grid, dim3(256), 0, s, P, ld, rows, cld, part, P8, scale);
  return hipGetLastError();
}

static hipError_t launch_nn_fp8_slice(const uint8_t* A8, int64_t lda8, int64_t rows, int64_t kdim, int64_t tk,
                         int64_t TK, const float* sA, int64_t sc_r, int64_t sc_k,
                         const uint8_t* X8, int64_t ldx8, const float* sx, int64_t lp, float* Y,
                         int64_t ldy, int64_t part_stride, hipStream_t s) {
  if (tk % kQB != 0 || lda8 % 16 != 0 || ldx8 % 16 != 0 || ldy % 4 != 0)
    return hipErrorInvalidValue;
  const int nt = (int)(lp / 32);
  // direct-to-LDS form: panel widths 128 and 160, 16-byte aligned operands,
  // 31-bit buffer offsets over 256 rows of A and the panel columns
  if ((nt == 4 || nt == 5) && ((uintptr_t)A8 & 15) == 0 && ((uintptr_t)X8 & 15) == 0 &&
      (int64_t)F8_BM * lda8 <= INT32_MAX && lp * ldx8 <= INT32_MAX) {
    dim3 grid((unsigned)ceil_div_dev(rows, F8_BM), (unsigned)TK);
    if (nt == 4)
      hipLaunchKernelGGL(k_nn_fp8_dl<4>, grid, dim3(512), 0, s, A8, lda8, rows, kdim, tk, sA, sc_r,
                         sc_k, X8, ldx8, sx, Y, ldy, part_stride);
    else
      hipLaunchKernelGGL(k_nn_fp8_dl<5>, grid, dim3(512), 0, s, A8, lda8, rows, kdim, tk, sA, sc_r,
                         sc_k, X8, ldx8, sx, Y, ldy, part_stride);
    return hipGetLastError();
  }
  dim3 grid((unsigned)ceil_div_dev(rows, 128), (unsigned)TK);
#define NN8(NT) hipLaunchKernelGGL((k_nn_fp8<NT, 1>), grid, dim3(256), 0, s, A8, lda8, rows, kdim, tk, sA, sc_r, sc_k, X8, ldx8, sx, Y, ldy, part_stride)
  switch (nt) {
    case 1: NN8(1); break;
    case 2: NN8(2); break;
    case 3: NN8(3); break;
    case 4: NN8(4); break;
    case 5: NN8(5); break;
    case 6: NN8(6); break;
    default: return hipErrorInvalidValue;
  }
#undef NN8
  return hipGetLastError();
}

// Panels wider than kSliceMax columns are multiplied in column slices
// (plan.h, slice_width): one launch per slice, each reading A once more;
// the slices' columns are independent, so results equal a single launch.
hipError_t launch_nn_fp8(const uint8_t* A8, int64_t lda8, int64_t rows, int64_t kdim, int64_t tk,
                         int64_t TK, const float* sA, int64_t sc_r, int64_t sc_k,
                         const uint8_t* X8, int64_t ldx8, const float* sx, int64_t lp, float* Y,
                         int64_t ldy, int64_t part_stride, hipStream_t s) {
  const int64_t cw = slice_width(lp);
  for (int64_t c0 = 0; c0 < lp; c0 += cw) {
    const hipError_t e = launch_nn_fp8_slice(A8, lda8, rows, kdim, tk, TK, sA, sc_r, sc_k,
                                             X8 + c0 * ldx8, ldx8, sx + c0,
                                             std::min(cw, lp - c0), Y + c0 * ldy, ldy,
                                             part_stride, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rsvd
