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
//   * A^T Q gathers rows of Q in the order of each column's rows; with
//     millions of rows of Q in random order those gathers come from HBM or
//     the last-level cache, never twice from L2.  The head columns (the most
//     frequent, found from counts on a sample of the rows) hold about half of
//     a Zipf matrix's entries and are handled apart: their entries are keyed
//     to compressed rows hbase + b K + h per block b of kHeadPartRows rows of
//     A, after the P n compressed rows of the other columns' P row blocks in
//     the same sorted copy.  One workgroup per (block, 64 columns) copies the
//     block's rows of Q into LDS once and runs every head column's entries of
//     the block against that copy; a last pass adds each head column's block
//     results in block order into its output row.  The chunked product walks
//     only the other columns' compressed rows.  Every sum keeps a fixed
//     order.
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
  // the product covers compressed rows [0, rows): entries up to ptr[rows]
  const int64_t ne = min<int64_t>(nnz, ptr[rows]);
  const int64_t e0 = c * kChunk, e1 = min(ne, e0 + kChunk);
  if (e0 >= ne) return;
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
                                                    int64_t rows, int64_t nnz,
                                                    const int32_t* __restrict__ first,
                                                    int64_t chunks, const float* __restrict__ carry,
                                                    int lp, float* __restrict__ Yr, int64_t ldyr) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= chunks || c == 0) return;
  // the row that owns chunk c's carry: the first non-empty row reaching past c C
  int64_t r = first[c];
  const int64_t e0 = c * kChunk;
  if (e0 >= min<int64_t>(nnz, ptr[rows])) return;   // no entries of rows [0, rows) here
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

// CSC build: keys = compressed row, payload = (row << 32) | value bits.  An
// entry of a head column h (headof[col] = h >= 0) goes to compressed row
// hbase + (i / head_rows) K + h, any other to (i / block_rows) n + col.
__global__ void k_csc_keys(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                           const float* __restrict__ values, int64_t m, int64_t n, int64_t nnz,
                           int64_t block_rows, const int32_t* __restrict__ headof, int64_t hbase,
                           int64_t head_rows, int64_t head_k, uint32_t* __restrict__ keys,
                           uint64_t* __restrict__ payload) {
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= m) return;
  const int lane = threadIdx.x & 63;
  const int64_t lo = max<int64_t>(0, rowptr[i]), hi = min<int64_t>(nnz, rowptr[i + 1]);
  const uint32_t base = (uint32_t)((i / block_rows) * n);
  const uint32_t hb = (uint32_t)(hbase + (i / head_rows) * head_k);
  for (int64_t e = lo + lane; e < hi; e += 64) {
    const uint32_t c = min<uint32_t>((uint32_t)colind[e], (uint32_t)(n - 1));
    const int32_t h = headof ? headof[c] : -1;
    keys[e] = h >= 0 ? hb + (uint32_t)h : base + c;
    payload[e] = ((uint64_t)(uint32_t)i << 32) | (uint64_t)__builtin_bit_cast(uint32_t, values[e]);
  }
}

// Column counts on every stride-th row (one wave per sampled row; the entries
// of a row have distinct columns).  Integer sums: the counts do not depend on
// the order of the additions.
__global__ void k_col_count_sample(const int32_t* __restrict__ rowptr,
                                   const int32_t* __restrict__ colind, int64_t m, int64_t n,
                                   int64_t nnz, int64_t stride, uint32_t* __restrict__ cnt) {
  const int64_t i = ((int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)) * stride;
  if (i >= m) return;
  const int lane = threadIdx.x & 63;
  const int64_t lo = max<int64_t>(0, rowptr[i]), hi = min<int64_t>(nnz, rowptr[i + 1]);
  for (int64_t e = lo + lane; e < hi; e += 64)
    atomicAdd(cnt + min<uint32_t>((uint32_t)colind[e], (uint32_t)(n - 1)), 1u);
}

// Rank keys: ascending sort of ~count with the column as payload orders the
// columns by count, descending, ties by column (the sort is stable).
__global__ void k_rank_keys(const uint32_t* __restrict__ cnt, int64_t n, uint32_t* __restrict__ keys,
                            int32_t* __restrict__ vals, int32_t* __restrict__ headof) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  keys[j] = ~cnt[j];
  vals[j] = (int32_t)j;
  headof[j] = -1;
}

__global__ void k_head_map(const int32_t* __restrict__ ranked, int64_t k, int32_t* __restrict__ headof,
                           int32_t* __restrict__ headcol) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= k) return;
  const int32_t c = ranked[h];
  headof[c] = (int32_t)h;
  headcol[h] = c;
}

// Head columns' entries of A^T Q.  Workgroup (b, g) copies rows
// [b R, b R + R) of panel columns [64 g, 64 g + 64) of the slice into LDS
// (column-major with stride R + 1, so a wave reading one row across its 64
// columns hits 64 different banks), and the block's K + 1 compressed-row
// pointers.  The block's head entries are one contiguous run, compressed row
// hbase + b K + h after another; a wave takes a piece (whole compressed
// rows [h_p, h_p+1)) and walks it as a flat stream, 512 entries loaded at a
// time and summed 8 at a time, lane = column.  Each compressed row's sum of
// value * Q(row, :), in stored order, goes to that row of the result; rows
// without entries get zeros.
constexpr int kHeadR = (int)kHeadPartRows;
constexpr int kHeadS = kHeadR + 1;
constexpr int kHeadWaves = 16;
static_assert(kHeadCols + 1 <= 64 * kHeadWaves, "one block pointer per thread");
static_assert((64 * (kHeadR / 4)) % (64 * kHeadWaves) == 0, "whole staging loads per thread");

// A block's work is cut into kHeadPieces pieces of whole compressed rows,
// balanced on the cost lp[h] + kHeadRowCost h up to compressed row h
// (entries, plus a charge per row for closing it: many short rows cost more
// per entry than a few long ones); the waves take pieces from an LDS counter
// until none is left.  head_split returns the first h in [0, K] whose cost
// is >= t (the cost grows with h).
constexpr int64_t kHeadRowCost = 16;
constexpr int kHeadPieces = 32;

__device__ inline int head_split(const int* lp, int K, int64_t t, int lane) {
  int cnt = 0;
  for (int h0 = 0; h0 < K; h0 += 64) {
    const int h = h0 + lane;
    cnt += __popcll(__ballot(h < K && (int64_t)lp[h] + kHeadRowCost * h < t));
  }
  return cnt;
}

__global__ __launch_bounds__(1024) void k_head_spmm(const int32_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ idx,
                                                    const float* __restrict__ val, int64_t nnz,
                                                    int64_t hbase, int64_t head_k,
                                                    const float* __restrict__ X, int64_t ldx,
                                                    int64_t xrows, int cw, float* __restrict__ Yr,
                                                    int64_t ldr) {
  __shared__ float qs[64 * kHeadS];
  __shared__ int lp[kHeadCols + 1];
  __shared__ int next;
  const int64_t b = blockIdx.x;
  const int g0 = blockIdx.y * 64;
  const int64_t r0 = b * kHeadR;
  const int K = (int)head_k;
  const int64_t vbase = hbase + b * head_k;   // compressed row of h = 0
  const int tid = threadIdx.x;
  // 16-byte loads down each column, all issued before the first LDS store
  // (ldx and r0 are multiples of 4, so a row r < xrows keeps r + 3 < ldx)
  // (loads from clamped addresses, masked afterwards, so none waits for
  // another); the block's K + 1 <= 1024 pointers go first
  const int pk = ptr[vbase + min(tid, K)];
  constexpr int kLoads = 64 * (kHeadR / 4) / 1024;
  const int64_t rlast = ((xrows - 1) / 4) * 4;
  float4 v[kLoads];
#pragma unroll
  for (int i = 0; i < kLoads; ++i) {
    const int e = tid + 1024 * i, c = e / (kHeadR / 4), q = e % (kHeadR / 4);
    const int64_t r = r0 + 4 * q;
    v[i] = *reinterpret_cast<const float4*>(X + (int64_t)min(g0 + c, cw - 1) * ldx + min(r, rlast));
  }
#pragma unroll
  for (int i = 0; i < kLoads; ++i) {
    const int e = tid + 1024 * i, c = e / (kHeadR / 4), q = e % (kHeadR / 4);
    const int64_t r = r0 + 4 * q;
    if (g0 + c >= cw || r >= xrows) v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r + 1 >= xrows) v[i].y = 0.f;
    if (r + 2 >= xrows) v[i].z = 0.f;
    if (r + 3 >= xrows) v[i].w = 0.f;
  }
  if (tid <= K)   // entries past nnz (malformed input) are cut off
    lp[tid] = pk < 0 ? 0 : (pk > nnz ? (int)nnz : pk);
  if (tid == 0) next = 0;
#pragma unroll
  for (int i = 0; i < kLoads; ++i) {
    const int e = tid + 1024 * i, c = e / (kHeadR / 4), q = e % (kHeadR / 4);
    float* d = qs + c * kHeadS + 4 * q;
    d[0] = v[i].x;
    d[1] = v[i].y;
    d[2] = v[i].z;
    d[3] = v[i].w;
  }
  __syncthreads();
  const int lane = tid & 63;
  const int E0 = __builtin_amdgcn_readfirstlane(lp[0]);
  const int E1 = __builtin_amdgcn_readfirstlane(lp[K]);
  const int64_t cost = (int64_t)(E1 - E0) + kHeadRowCost * K;
  const float* qc = qs + lane * kHeadS;
  float* yr = Yr + vbase * ldr + g0 + lane;
  const bool st = g0 + lane < cw;
  const int r0i = (int)r0;
  for (;;) {
    int piece = 0;
    if (lane == 0) piece = atomicAdd(&next, 1);
    piece = __builtin_amdgcn_readfirstlane(piece);
    if (piece >= kHeadPieces) break;
    const int hb =
        __builtin_amdgcn_readfirstlane(head_split(lp, K, E0 + cost * piece / kHeadPieces, lane));
    const int he = piece == kHeadPieces - 1
                       ? K
                       : __builtin_amdgcn_readfirstlane(
                             head_split(lp, K, E0 + cost * (piece + 1) / kHeadPieces, lane));
    if (hb >= he) continue;
    int r = hb;
    int rend = __builtin_amdgcn_readfirstlane(lp[r + 1]);
    float acc = 0.f;
    const int ebeg = __builtin_amdgcn_readfirstlane(lp[hb]);
    const int eend = __builtin_amdgcn_readfirstlane(lp[he]);
    // kWin windows of 64 entries are loaded together (rows outside the
    // block, from malformed input, are clamped into it)
    constexpr int kWin = 8;
    for (int eb = ebeg; eb < eend; eb += 64 * kWin) {
      int cr[kWin];
      float cv[kWin];
#pragma unroll
      for (int j = 0; j < kWin; ++j) {   // lanes past the end reload the last entry
        const int e = min(eb + 64 * j + lane, eend - 1);
        cr[j] = idx[e];
        cv[j] = val[e];
      }
#pragma unroll
      for (int j = 0; j < kWin; ++j) {
        const int d = cr[j] - r0i;
        cr[j] = d < 0 ? 0 : (d > kHeadR - 1 ? kHeadR - 1 : d);
      }
#pragma unroll
      for (int j = 0; j < kWin; ++j) {
        const int e0 = eb + 64 * j;
        if (e0 >= eend) break;
        const int cnt = min(64, eend - e0);
        // eight entries at a time: their rows of Q are read from LDS
        // together (lanes past the end hold valid rows), then added in
        // order, closing a row wherever one ends (t <= 56, so t + u stays a
        // lane index)
        for (int t = 0; t < cnt; t += 8) {
          float q[8], a[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            q[u] = qc[__builtin_amdgcn_readlane(cr[j], t + u)];
            a[u] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, cv[j]), t + u));
          }
          if (t + 8 <= cnt && e0 + t + 8 <= rend) {   // all in row r
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += a[u] * q[u];
            continue;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (t + u >= cnt) break;
            while (e0 + t + u >= rend) {   // row r is done (e0 + t + u < eend keeps r + 1 < he)
              if (st) yr[(int64_t)r * ldr] = acc;
              acc = 0.f;
              ++r;
              rend = __builtin_amdgcn_readfirstlane(lp[r + 1]);
            }
            acc += a[u] * q[u];
          }
        }
      }
    }
    for (; r < he; ++r) {   // the last row with entries, then the empty ones after it
      if (st) yr[(int64_t)r * ldr] = acc;
      acc = 0.f;
    }
  }
}

// Head results, first pass: for each group of kHeadGroup consecutive row
// blocks, the sum of the group's rows (in block order) replaces the group's
// first row.  Thread = (group, head column, 4 columns).
constexpr int64_t kHeadGroup = 64;

__global__ __launch_bounds__(256) void k_head_groups(float* __restrict__ R, int64_t ldr,
                                                     int64_t hbase, int64_t head_k,
                                                     int64_t head_parts, int cw) {
  const int64_t c4n = cw / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t groups = (head_parts + kHeadGroup - 1) / kHeadGroup;
  if (t >= groups * head_k * c4n) return;
  const int64_t c4 = t % c4n, h = (t / c4n) % head_k, g = t / (c4n * head_k);
  const int64_t b0 = g * kHeadGroup, b1 = min(head_parts, b0 + kHeadGroup);
  float* p = R + (hbase + b0 * head_k + h) * ldr + 4 * c4;
  const int64_t step = head_k * ldr;
  float4 s = *reinterpret_cast<const float4*>(p);
  int64_t b = b0 + 1;
  for (; b + 8 <= b1; b += 8) {
    float4 x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = *reinterpret_cast<const float4*>(p + (b - b0 + u) * step);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      s.x += x[u].x;
      s.y += x[u].y;
      s.z += x[u].z;
      s.w += x[u].w;
    }
  }
  for (; b < b1; ++b) {
    const float4 x = *reinterpret_cast<const float4*>(p + (b - b0) * step);
    s.x += x.x;
    s.y += x.y;
    s.z += x.z;
    s.w += x.w;
  }
  *reinterpret_cast<float4*>(p) = s;
}

// Head columns' rows of the result: out(col h, :) = the group sums of head
// column h, added in group order.  The other-column pass left these rows
// zero.
__global__ __launch_bounds__(256) void k_from_head(const float* __restrict__ R, int64_t ldr,
                                                   int64_t hbase, int64_t head_k,
                                                   int64_t head_parts,
                                                   const int32_t* __restrict__ headcol, int cw,
                                                   float* __restrict__ P, int64_t ld) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= head_k * cw) return;
  const int64_t h = t / cw;
  const int c = (int)(t % cw);
  const float* p = R + (hbase + h) * ldr + c;
  const int64_t step = kHeadGroup * head_k * ldr;
  const int64_t groups = (head_parts + kHeadGroup - 1) / kHeadGroup;
  float v = 0.f;
  int64_t g = 0;
  for (; g + 8 <= groups; g += 8) {
    float x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = p[(g + u) * step];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += x[u];
  }
  for (; g < groups; ++g) v += p[g * step];
  P[(int64_t)c * ld + headcol[h]] = v;
}

__global__ __launch_bounds__(256) void k_zero_head(int64_t head_k, const int32_t* __restrict__ headcol,
                                                   int cw, float* __restrict__ P, int64_t ld) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= head_k * cw) return;
  P[(t % cw) * ld + headcol[t / cw]] = 0.f;
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


hipError_t launch_head_select(const int32_t* rowptr, const int32_t* colind, int64_t m, int64_t n,
                              int64_t nnz, int64_t head_k, uint32_t* cnt, int32_t* headof,
                              int32_t* headcol, uint32_t* rk0, uint32_t* rk1, int32_t* rv0,
                              int32_t* rv1, void* temp, size_t temp_bytes, size_t* need,
                              hipStream_t s) {
  *need = 0;
  if (head_k < 1 || head_k > n) return hipErrorInvalidValue;
  hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(cnt), n, 0, s);
  if (e != hipSuccess) return e;
  const int64_t sampled = ceil_div_dev(m, kHeadSampleStride);
  if (nnz > 0 && sampled > 0) {
    hipLaunchKernelGGL(k_col_count_sample, dim3((unsigned)ceil_div_dev(sampled, 4)), dim3(256), 0,
                       s, rowptr, colind, m, n, nnz, kHeadSampleStride, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_rank_keys, dim3((unsigned)ceil_div_dev(n, 256)), dim3(256), 0, s, cnt, n, rk0,
                     rv0, headof);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  rocprim::double_buffer<uint32_t> kb(rk0, rk1);
  rocprim::double_buffer<int32_t> vb(rv0, rv1);
  size_t want = 0;
  e = rocprim::radix_sort_pairs(nullptr, want, kb, vb, (size_t)n, 0, 32, s);
  if (e != hipSuccess) return e;
  if (want > temp_bytes) {
    *need = want;
    return hipErrorOutOfMemory;
  }
  e = rocprim::radix_sort_pairs(temp, want, kb, vb, (size_t)n, 0, 32, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_head_map, dim3((unsigned)ceil_div_dev(head_k, 256)), dim3(256), 0, s,
                     vb.current(), head_k, headof, headcol);
  return hipGetLastError();
}

hipError_t launch_build_csc(const int32_t* rowptr, const int32_t* colind, const float* values,
                            int64_t m, int64_t n, int64_t nnz, int64_t parts,
                            const int32_t* headof, int64_t head_k, int64_t head_parts,
                            uint32_t* keys0, uint32_t* keys1, uint64_t* pay0, uint64_t* pay1,
                            void* temp, size_t temp_bytes, int32_t* colptr, int32_t* rowind,
                            float* cval, size_t* need, hipStream_t s) {
  *need = 0;
  if (!headof) head_k = head_parts = 0;
  // compressed rows: the row blocks' columns, block-major, then the head
  // columns of the head row blocks
  const int64_t nv = parts * n + head_parts * head_k;
  if (parts < 1 || nv > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
  const int64_t block_rows = ceil_div_dev(m > 0 ? m : 1, parts);
  const int64_t head_rows = kHeadPartRows;
  if (head_parts > 0 && head_parts * head_rows < m) return hipErrorInvalidValue;
  if (nnz > 0) {
    // entries no row covers (malformed pointers) keep defined keys
    hipLaunchKernelGGL(k_fill_keys, dim3((unsigned)ceil_div_dev(nnz, 256)), dim3(256), 0, s, nnz,
                       (uint32_t)(nv - 1), keys0, pay0);
    hipLaunchKernelGGL(k_csc_keys, dim3((unsigned)ceil_div_dev(m, 4)), dim3(256), 0, s, rowptr,
                       colind, values, m, n, nnz, block_rows, head_k > 0 ? headof : nullptr,
                       parts * n, head_rows, head_k, keys0, pay0);
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
                       float* out, int64_t ldo, hipStream_t s, const int32_t* headcol,
                       int64_t head_k, int64_t head_parts) {
  if (parts < 1) return hipErrorInvalidValue;
  if (!headcol) head_k = head_parts = 0;
  if (head_k > kHeadCols || (head_k > 0 && head_parts < 1)) return hipErrorInvalidValue;
  const int64_t out_rows = rows;
  // the chunked product walks the compressed rows [0, hbase); the head
  // columns' rows follow
  const int64_t hbase = rows * parts;
  rows = hbase;
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
      hipLaunchKernelGGL(k_spmm_fixup, g, dim3(256), 0, s, ptr, rows, nnz, first, chunks, carry,
                         (int)cw, Yr, ldr);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (head_k > 0) {
        hipLaunchKernelGGL(k_head_spmm, dim3((unsigned)head_parts, (unsigned)ceil_div_dev(cw, 64)),
                           dim3(64 * kHeadWaves), 0, s, ptr, idx, val, nnz, hbase, head_k, X + c0 * ldx, ldx,
                           xrows, (int)cw, Yr, ldr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
    }
    dim3 gy((unsigned)ceil_div_dev(ldo, kTT), (unsigned)ceil_div_dev(cw, kTT));
    hipLaunchKernelGGL(k_from_rows, gy, dim3(256), 0, s, Yr, ldr, ptr, out_rows, parts, (int)cw,
                       out + c0 * ldo, ldo);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (head_k > 0) {
      if (nnz > 0) {
        const int64_t gt = ceil_div_dev(head_parts, kHeadGroup) * head_k * (cw / 4);
        hipLaunchKernelGGL(k_head_groups, dim3((unsigned)ceil_div_dev(gt, 256)), dim3(256), 0, s,
                           Yr, ldr, hbase, head_k, head_parts, (int)cw);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_from_head, dim3((unsigned)ceil_div_dev(head_k * cw, 256)), dim3(256),
                           0, s, Yr, ldr, hbase, head_k, head_parts, headcol, (int)cw,
                           out + c0 * ldo, ldo);
      } else {   // no entries: the head rows of the result are zero
        hipLaunchKernelGGL(k_zero_head, dim3((unsigned)ceil_div_dev(head_k * cw, 256)), dim3(256),
                           0, s, head_k, headcol, (int)cw, out + c0 * ldo, ldo);
      }
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace rsvd
