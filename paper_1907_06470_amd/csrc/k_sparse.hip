// Sparse A (CSR, int32 indices, FP32 values): the products of Section 2.1
// steps 2 and 5 and of the power steps (Section 2.2 Eq. (2)) as sparse x
// tall-skinny products, with A^T applied through a CSC copy (the CSR of A^T)
// built once per call by a stable sort of the nonzeros by column.
//
// Product Y = S X, S in compressed-row form (rows of A, or rows of A^T):
//   * X is first copied row-major (n x lp), so the row of X a nonzero needs
//     is one contiguous run of lp floats: a wave gathers it with lanes over
//     the columns (coalesced) and accumulates a * X(col, :) in registers.
//   * Work is split by nonzeros, not by rows: chunk c covers nonzeros
//     [c C, (c + 1) C) (one wave each), so a column of A^T with millions of
//     entries (a Zipf head column) is spread over many waves.  A row that
//     starts inside a chunk is written by that chunk (complete, or its first
//     part); every later chunk the row reaches writes its part to carry[c];
//     a fix-up pass adds the carries to the row in chunk order.  The result
//     does not depend on scheduling: runs are bitwise reproducible.
//   * The result is written row-major and transposed into the column-major
//     panel the orthonormalisation uses; empty rows become zero there.
#include <algorithm>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace rsvd {

namespace {

constexpr int kChunk = (int)kSpmmChunk;   // nonzeros per wave
constexpr int kMaxCW = 3;        // columns per lane: slices of up to 192 = 3 x 64 columns
constexpr int kGather = 8;       // nonzeros whose rows of X are loaded together

// first row of each chunk: largest r with ptr[r] <= c C
__global__ void k_chunk_rows(const int32_t* __restrict__ ptr, int64_t rows, int64_t nnz,
                             int64_t chunks, int32_t* __restrict__ first) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= chunks) return;
  const int64_t e = c * kChunk;
  int64_t lo = 0, hi = rows - 1;   // ptr[lo] <= e always (ptr[0] = 0)
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (ptr[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  // skip empty rows that also start at e (the row holding nonzero e is the
  // last r with ptr[r] <= e, which is what the search returns)
  first[c] = (int32_t)lo;
  (void)nnz;
}

template <int CW>
__device__ inline void flush_row(float* __restrict__ Yr, int64_t ldyr, float* __restrict__ carry,
                                 int64_t c, int64_t r, bool continued, const float (&acc)[kMaxCW],
                                 int lane, int lp) {
  float* dst = continued ? carry + c * ldyr : Yr + r * ldyr;
#pragma unroll
  for (int u = 0; u < CW; ++u) {
    const int col = lane + 64 * u;
    if (col < lp) dst[col] = acc[u];
  }
}

// One wave per chunk of nonzeros; 4 waves per workgroup.
template <int CW>
__global__ __launch_bounds__(256) void k_spmm_chunk(const int32_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ idx,
                                                    const float* __restrict__ val, int64_t rows,
                                                    int64_t nnz, const int32_t* __restrict__ first,
                                                    int64_t chunks, const float* __restrict__ Xr,
                                                    int64_t ldxr, int64_t xrows, int lp,
                                                    float* __restrict__ Yr, int64_t ldyr,
                                                    float* __restrict__ carry) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= chunks) return;
  const int64_t e0 = c * kChunk, e1 = min(nnz, e0 + kChunk);
  int64_t r = first[c];
  int64_t rend = ptr[r + 1];
  while (rend <= e0 && r + 1 < rows) {   // empty rows at the chunk start
    ++r;
    rend = ptr[r + 1];
  }
  bool continued = ptr[r] < e0;
  float acc[kMaxCW] = {0.f, 0.f, 0.f};
  for (int64_t g = e0; g < e1; g += 64) {
    const int cnt = (int)min<int64_t>(64, e1 - g);
    // out-of-range indices (flagged by the input check) are clamped
    const int32_t mycol = lane < cnt ? (int32_t)min<uint32_t>((uint32_t)idx[g + lane], (uint32_t)(xrows - 1)) : 0;
    const float myval = lane < cnt ? val[g + lane] : 0.f;
    // kGather nonzeros at a time: their rows of X are loaded together, then
    // added in nonzero order, closing a row of the result wherever one ends
    // (so short rows keep as many loads in flight as long ones)
    for (int t = 0; t < cnt; t += kGather) {
      float v[kGather], x[kGather][kMaxCW];
#pragma unroll
      for (int q = 0; q < kGather; ++q) {
        const int tq = min(t + q, cnt - 1);
        const int32_t col = __builtin_amdgcn_readlane(mycol, tq);
        v[q] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, myval), tq));
#pragma unroll
        for (int u = 0; u < CW; ++u) {
          const int cc = lane + 64 * u;
          x[q][u] = cc < lp ? Xr[(int64_t)col * ldxr + cc] : 0.f;
        }
      }
      if (t + kGather <= cnt && g + t + kGather <= rend) {   // all in row r
#pragma unroll
        for (int q = 0; q < kGather; ++q)
#pragma unroll
          for (int u = 0; u < CW; ++u) acc[u] += v[q] * x[q][u];
        continue;
      }
#pragma unroll
      for (int q = 0; q < kGather; ++q) {
        if (t + q >= cnt) break;
        const int64_t e = g + t + q;
        if (e >= rend) {   // row r is done
          flush_row<CW>(Yr, ldyr, carry, c, r, continued, acc, lane, lp);
#pragma unroll
          for (int u = 0; u < kMaxCW; ++u) acc[u] = 0.f;
          continued = false;
          // next row holding nonzero e (malformed pointers, flagged by the
          // input check, end at the last row)
          while (r + 1 < rows) {
            ++r;
            rend = ptr[r + 1];
            if (rend > e) break;
          }
        }
#pragma unroll
        for (int u = 0; u < CW; ++u) acc[u] += v[q] * x[q][u];
      }
    }
  }
  // the chunk's last row: complete, or the first part of a row that goes on
  flush_row<CW>(Yr, ldyr, carry, c, r, continued, acc, lane, lp);
}

// For every row that continues into later chunks: add their carries in chunk
// order.  Chunk c handles row first[c] when the row started inside chunk c-1.
__global__ __launch_bounds__(256) void k_spmm_fixup(const int32_t* __restrict__ ptr,
                                                    int64_t rows, const int32_t* __restrict__ first,
                                                    int64_t chunks, const float* __restrict__ carry,
                                                    int lp, float* __restrict__ Yr, int64_t ldyr) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= chunks || c == 0) return;
  // the row that owns chunk c's carry: the first non-empty row reaching past c C
  int64_t r = first[c];
  const int64_t e0 = c * kChunk;
  while (ptr[r + 1] <= e0 && r + 1 < rows) ++r;
  if (ptr[r] >= e0) return;                 // row starts in chunk c: no carry
  if (ptr[r] < e0 - kChunk) return;         // row started before chunk c-1: handled earlier
  for (int u = 0; u < kMaxCW; ++u) {
    const int col = lane + 64 * u;
    if (col >= lp) continue;
    float s = Yr[r * ldyr + col];
    for (int64_t c2 = c; c2 < chunks; ++c2) {
      const int64_t f0 = c2 * kChunk;
      if (c2 > c && f0 >= ptr[r + 1]) break;
      s += carry[c2 * ldyr + col];
    }
    Yr[r * ldyr + col] = s;
  }
}

// Panel layout changes around the products, 64 x 64 tiles through LDS with
// 16-byte accesses on both sides (ld, ldr multiples of 4, lp a multiple of 4,
// 16-byte aligned pointers; a row index r < ld that is a multiple of 4 keeps
// r + 3 < ld).  t[c][r] holds column c, row r of the tile; its odd stride
// keeps the column-wise and the row-wise element accesses free of bank
// conflicts.
constexpr int kTT = 64;

// column-major panel (ld) -> row-major copy (rows x lp, ldr)
__global__ __launch_bounds__(256) void k_to_rows(const float* __restrict__ P, int64_t ld,
                                                 int64_t rows, int lp, float* __restrict__ R,
                                                 int64_t ldr) {
  __shared__ float t[kTT][kTT + 1];
  const int64_t r0 = (int64_t)blockIdx.x * kTT;
  const int c0 = blockIdx.y * kTT;
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u, c = e >> 4, q = e & 15;
    const int64_t r = r0 + 4 * q;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (c0 + c < lp && r < rows) {
      v = *reinterpret_cast<const float4*>(P + (int64_t)(c0 + c) * ld + r);
      if (r + 1 >= rows) v.y = 0.f;
      if (r + 2 >= rows) v.z = 0.f;
      if (r + 3 >= rows) v.w = 0.f;
    }
    t[c][4 * q] = v.x;
    t[c][4 * q + 1] = v.y;
    t[c][4 * q + 2] = v.z;
    t[c][4 * q + 3] = v.w;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u, r = e >> 4, c = (e & 15) * 4;
    if (r0 + r < rows && c0 + c < lp)
      st4(R + (r0 + r) * ldr + c0 + c, make_float4(t[c][r], t[c + 1][r], t[c + 2][r], t[c + 3][r]));
  }
}

// row-major result -> column-major panel (ld rows, padding rows zero).  The
// result holds `parts` row sets of `rows` rows each (the products of the row
// blocks of A); row r of the panel is their sum, taken in part order.  Rows
// without nonzeros are zero.
__global__ __launch_bounds__(256) void k_from_rows(const float* __restrict__ R, int64_t ldr,
                                                   const int32_t* __restrict__ ptr, int64_t rows,
                                                   int64_t parts, int lp, float* __restrict__ P,
                                                   int64_t ld) {
  __shared__ float t[kTT][kTT + 1];
  const int64_t r0 = (int64_t)blockIdx.x * kTT;
  const int c0 = blockIdx.y * kTT;
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u, r = e >> 4, c = (e & 15) * 4;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r0 + r < rows && c0 + c < lp)
      for (int64_t b = 0; b < parts; ++b) {
        const int64_t rv = b * rows + r0 + r;
        if (ptr[rv + 1] > ptr[rv]) {
          const float4 w = *reinterpret_cast<const float4*>(R + rv * ldr + c0 + c);
          v.x += w.x;
          v.y += w.y;
          v.z += w.z;
          v.w += w.w;
        }
      }
    t[c][r] = v.x;
    t[c + 1][r] = v.y;
    t[c + 2][r] = v.z;
    t[c + 3][r] = v.w;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u, c = e >> 4, q = e & 15;
    const int64_t r = r0 + 4 * q;
    if (r < ld && c0 + c < lp)
      st4(P + (int64_t)(c0 + c) * ld + r,
          make_float4(t[c][4 * q], t[c][4 * q + 1], t[c][4 * q + 2], t[c][4 * q + 3]));
  }
}

// CSC build: keys = column, payload = (row << 32) | value bits
__global__ void k_csc_keys(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                           const float* __restrict__ values, int64_t m, int64_t n, int64_t nnz,
                           int64_t block_rows, uint32_t* __restrict__ keys,
                           uint64_t* __restrict__ payload) {
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= m) return;
  const int lane = threadIdx.x & 63;
  const int64_t lo = max<int64_t>(0, rowptr[i]), hi = min<int64_t>(nnz, rowptr[i + 1]);
  const uint32_t base = (uint32_t)((i / block_rows) * n);
  for (int64_t e = lo + lane; e < hi; e += 64) {
    keys[e] = base + min<uint32_t>((uint32_t)colind[e], (uint32_t)(n - 1));
    payload[e] = ((uint64_t)(uint32_t)i << 32) | (uint64_t)__builtin_bit_cast(uint32_t, values[e]);
  }
}

__global__ void k_fill_keys(int64_t nnz, uint32_t key, uint32_t* __restrict__ keys,
                            uint64_t* __restrict__ payload) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) {
    keys[e] = key;
    payload[e] = 0;
  }
}

// Input check of a CSR matrix: pointers start at 0, end at nnz, never
// decrease; column indices in [0, n).  Any violation sets the status word.
__global__ void k_csr_check(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                            int64_t rows, int64_t cols, int64_t nnz, int32_t* __restrict__ status) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (t <= rows) {
    const int64_t p = ptr[t];
    if (t == 0 && p != 0) bad = true;
    if (t == rows && p != nnz) bad = true;
    if (t < rows && ptr[t + 1] < p) bad = true;
    if (p < 0 || p > nnz) bad = true;
  }
  for (int64_t e = t; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = idx[e];
    if (j < 0 || j >= cols) bad = true;
  }
  if (bad) atomicOr(status + kStBadSparse, 1);
}

// column pointers from the sorted keys, then the row indices and values
__global__ void k_csc_finish(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ payload,
                             int64_t nnz, int64_t n, int32_t* __restrict__ colptr,
                             int32_t* __restrict__ rowind, float* __restrict__ cval) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e > nnz) return;
  if (e == nnz) {   // trailing empty columns (and n == 0 guard)
    const int64_t last = nnz ? (int64_t)keys[nnz - 1] : -1;
    for (int64_t j = last + 1; j <= n; ++j) colptr[j] = (int32_t)nnz;
    return;
  }
  const int64_t k = keys[e];
  const int64_t prev = e ? (int64_t)keys[e - 1] : -1;
  for (int64_t j = prev + 1; j <= k; ++j) colptr[j] = (int32_t)e;
  const uint64_t p = payload[e];
  rowind[e] = (int32_t)(p >> 32);
  cval[e] = __builtin_bit_cast(float, (uint32_t)(p & 0xffffffffu));
}

// COO to CSR: keys = row, payload = (column << 32) | value bits.  Indices
// outside [0, m) x [0, n) are clamped (every later access stays in bounds)
// and flagged in the status word.
template <typename IT>
__global__ void k_coo_keys(const IT* __restrict__ ri, const IT* __restrict__ ci,
                           const float* __restrict__ values, int64_t m, int64_t n, int64_t nnz,
                           uint32_t* __restrict__ keys, uint64_t* __restrict__ payload,
                           int32_t* __restrict__ status) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const int64_t r = (int64_t)ri[e], c = (int64_t)ci[e];
  if (r < 0 || r >= m || c < 0 || c >= n) atomicOr(status + kStBadSparse, 1);
  const int64_t rc = min<int64_t>(max<int64_t>(r, 0), m - 1);
  const int64_t cc = min<int64_t>(max<int64_t>(c, 0), n - 1);
  keys[e] = (uint32_t)rc;
  payload[e] = ((uint64_t)(uint32_t)cc << 32) | (uint64_t)__builtin_bit_cast(uint32_t, values[e]);
}

// row pointers from the sorted keys, then the column indices and values
__global__ void k_coo_finish(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ payload,
                             int64_t nnz, int64_t m, int32_t* __restrict__ rowptr,
                             int32_t* __restrict__ colind, float* __restrict__ val) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e > nnz) return;
  if (e == nnz) {   // trailing empty rows
    const int64_t last = nnz ? (int64_t)keys[nnz - 1] : -1;
    for (int64_t r = last + 1; r <= m; ++r) rowptr[r] = (int32_t)nnz;
    return;
  }
  const int64_t k = keys[e];
  const int64_t prev = e ? (int64_t)keys[e - 1] : -1;
  for (int64_t r = prev + 1; r <= k; ++r) rowptr[r] = (int32_t)e;
  const uint64_t p = payload[e];
  colind[e] = (int32_t)(p >> 32);
  val[e] = __builtin_bit_cast(float, (uint32_t)(p & 0xffffffffu));
}

}  // namespace


hipError_t launch_csr_check(const int32_t* ptr, const int32_t* idx, int64_t rows, int64_t cols,
                            int64_t nnz, int32_t* status, hipStream_t s) {
  const int64_t threads = std::max<int64_t>(rows + 1, 1);
  hipLaunchKernelGGL(k_csr_check, dim3((unsigned)ceil_div_dev(threads, 256)), dim3(256), 0, s, ptr,
                     idx, rows, cols, nnz, status);
  return hipGetLastError();
}


hipError_t launch_build_csc(const int32_t* rowptr, const int32_t* colind, const float* values,
                            int64_t m, int64_t n, int64_t nnz, int64_t parts, uint32_t* keys0,
                            uint32_t* keys1, uint64_t* pay0, uint64_t* pay1, void* temp,
                            size_t temp_bytes, int32_t* colptr, int32_t* rowind, float* cval,
                            size_t* need, hipStream_t s) {
  *need = 0;
  const int64_t nv = parts * n;   // columns of the row blocks, block-major
  if (parts < 1 || nv > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
  const int64_t block_rows = ceil_div_dev(m > 0 ? m : 1, parts);
  if (nnz > 0) {
    // entries no row covers (malformed pointers) keep defined keys
    hipLaunchKernelGGL(k_fill_keys, dim3((unsigned)ceil_div_dev(nnz, 256)), dim3(256), 0, s, nnz,
                       (uint32_t)(nv - 1), keys0, pay0);
    hipLaunchKernelGGL(k_csc_keys, dim3((unsigned)ceil_div_dev(m, 4)), dim3(256), 0, s, rowptr,
                       colind, values, m, n, nnz, block_rows, keys0, pay0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned bits = 1;
    while (bits < 32 && (int64_t(1) << bits) < nv) ++bits;
    // ping-pong buffers owned by the workspace: the sort's own scratch is
    // only its histograms and look-back state
    rocprim::double_buffer<uint32_t> kb(keys0, keys1);
    rocprim::double_buffer<uint64_t> vb(pay0, pay1);
    size_t want = 0;
    e = rocprim::radix_sort_pairs(nullptr, want, kb, vb, (size_t)nnz, 0, bits, s);
    if (e != hipSuccess) return e;
    if (want > temp_bytes) {
      *need = want;
      return hipErrorOutOfMemory;
    }
    e = rocprim::radix_sort_pairs(temp, want, kb, vb, (size_t)nnz, 0, bits, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_csc_finish, dim3((unsigned)ceil_div_dev(nnz + 1, 256)), dim3(256), 0, s,
                       kb.current(), vb.current(), nnz, nv, colptr, rowind, cval);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_csc_finish, dim3(1), dim3(256), 0, s, keys1, pay1, nnz, nv, colptr, rowind,
                     cval);
  return hipGetLastError();
}

hipError_t launch_coo_to_csr(const void* rowind, const void* colind, int index_bits,
                             const float* values, int64_t m, int64_t n, int64_t nnz,
                             uint32_t* keys0, uint32_t* keys1, uint64_t* pay0, uint64_t* pay1,
                             void* temp, size_t temp_bytes, int32_t* rowptr, int32_t* col,
                             float* val, int32_t* status, size_t* need, hipStream_t s) {
  *need = 0;
  if (nnz == 0) {
    hipLaunchKernelGGL(k_coo_finish, dim3(1), dim3(256), 0, s, keys1, pay1, nnz, m, rowptr, col,
                       val);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)ceil_div_dev(nnz, 256));
  if (index_bits == 64)
    hipLaunchKernelGGL(k_coo_keys<int64_t>, grid, dim3(256), 0, s, (const int64_t*)rowind,
                       (const int64_t*)colind, values, m, n, nnz, keys0, pay0, status);
  else
    hipLaunchKernelGGL(k_coo_keys<int32_t>, grid, dim3(256), 0, s, (const int32_t*)rowind,
                       (const int32_t*)colind, values, m, n, nnz, keys0, pay0, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  unsigned bits = 1;
  while (bits < 32 && (int64_t(1) << bits) < m) ++bits;
  rocprim::double_buffer<uint32_t> kb(keys0, keys1);
  rocprim::double_buffer<uint64_t> vb(pay0, pay1);
  size_t want = 0;
  e = rocprim::radix_sort_pairs(nullptr, want, kb, vb, (size_t)nnz, 0, bits, s);
  if (e != hipSuccess) return e;
  if (want > temp_bytes) {
    *need = want;
    return hipErrorOutOfMemory;
  }
  e = rocprim::radix_sort_pairs(temp, want, kb, vb, (size_t)nnz, 0, bits, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_coo_finish, dim3((unsigned)ceil_div_dev(nnz + 1, 256)), dim3(256), 0, s,
                     kb.current(), vb.current(), nnz, m, rowptr, col, val);
  return hipGetLastError();
}

hipError_t launch_spmm(const int32_t* ptr, const int32_t* idx, const float* val, int64_t rows,
                       int64_t parts, int64_t nnz, const float* X, int64_t ldx, int64_t xrows,
                       int64_t lp, float* Xr, float* Yr, float* carry, int32_t* first,
                       float* out, int64_t ldo, hipStream_t s) {
  if (parts < 1) return hipErrorInvalidValue;
  const int64_t out_rows = rows;
  rows *= parts;   // the compressed rows the product walks
  const int64_t chunks = spmm_chunk_count(nnz);
  // the layout kernels move 16-byte pieces
  if (lp % 4 || ldx % 4 || ldo % 4 || (((uintptr_t)X | (uintptr_t)Xr | (uintptr_t)Yr |
                                         (uintptr_t)out) & 15))
    return hipErrorInvalidValue;
  hipError_t e;
  if (nnz > 0) {
    hipLaunchKernelGGL(k_chunk_rows, dim3((unsigned)ceil_div_dev(chunks, 256)), dim3(256), 0, s,
                       ptr, rows, nnz, chunks, first);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // Panels wider than a lane's kMaxCW columns go in column slices: each slice
  // gathers only its own columns of X, so the gathered bytes do not grow;
  // only the compressed arrays are read once more per slice.
  constexpr int64_t kSlice = 64 * kMaxCW;
  for (int64_t c0 = 0; c0 < lp; c0 += kSlice) {
    const int64_t cw = std::min<int64_t>(kSlice, lp - c0);
    const int64_t ldr = cw;
    dim3 gx((unsigned)ceil_div_dev(xrows, kTT), (unsigned)ceil_div_dev(cw, kTT));
    hipLaunchKernelGGL(k_to_rows, gx, dim3(256), 0, s, X + c0 * ldx, ldx, xrows, (int)cw, Xr, ldr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (nnz > 0) {
      dim3 g((unsigned)ceil_div_dev(chunks, 4));
      switch ((cw + 63) / 64) {
        case 1: hipLaunchKernelGGL(k_spmm_chunk<1>, g, dim3(256), 0, s, ptr, idx, val, rows, nnz, first, chunks, Xr, ldr, xrows, (int)cw, Yr, ldr, carry); break;
        case 2: hipLaunchKernelGGL(k_spmm_chunk<2>, g, dim3(256), 0, s, ptr, idx, val, rows, nnz, first, chunks, Xr, ldr, xrows, (int)cw, Yr, ldr, carry); break;
        default: hipLaunchKernelGGL(k_spmm_chunk<3>, g, dim3(256), 0, s, ptr, idx, val, rows, nnz, first, chunks, Xr, ldr, xrows, (int)cw, Yr, ldr, carry); break;
      }
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_spmm_fixup, g, dim3(256), 0, s, ptr, rows, first, chunks, carry,
                         (int)cw, Yr, ldr);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    dim3 gy((unsigned)ceil_div_dev(ldo, kTT), (unsigned)ceil_div_dev(cw, kTT));
    hipLaunchKernelGGL(k_from_rows, gy, dim3(256), 0, s, Yr, ldr, ptr, out_rows, parts, (int)cw,
                       out + c0 * ldo, ldo);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rsvd
