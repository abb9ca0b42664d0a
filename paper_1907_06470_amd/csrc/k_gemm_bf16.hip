// Products of A with a tall-skinny panel in BF16 on the gfx950 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation): the same passes over A as
// the FP32 kernels (Section 2.1 steps 2 and 5, Section 2.2 Eq. (2)) with A and
// the panel stored in BF16, which halves the bytes streamed from HBM.  The
// paper stores half precision and computes in single (Section 3.2); here the
// matrix cores multiply BF16 operands exactly and accumulate in FP32.
//
// Operands: A16 row-major (leading dimension a multiple of 8, rows 16-byte
// aligned); panels column-major BF16 (element (i, c) at P[c * ld + i]).
// Like the FP32 kernels, grid.y runs over the block-cyclic tiles of the
// reduced dimension and each tile writes its own FP32 partial panel.
#include <algorithm>

#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace rsvd {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16;

constexpr int BK = 64;          // reduction slab (elements)
constexpr int PADK = BK + 8;    // LDS row of a k-contiguous tile: 144 bytes

__device__ inline f32x16 mfma_bf16(const bf16x8& a, const bf16x8& b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// 8 consecutive BF16 of a row from index k, zero past kend.
__device__ inline uint4 ld8_masked(const u16* row, int64_t k, int64_t kend) {
  if (k + 8 <= kend) return *reinterpret_cast<const uint4*>(row + k);
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int e = 0; e < 8; ++e)
    if (k + e < kend) w[e >> 1] |= (uint32_t)row[k + e] << (16 * (e & 1));
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Same, with a non-temporal hint for the full 16-byte case (A is streamed
// once per pass; keeping it out of the way leaves the caches to the panel).
__device__ inline uint4 ld8_masked_nt(const u16* row, int64_t k, int64_t kend) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  if (k + 8 <= kend) {
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(row + k));
    return make_uint4(v[0], v[1], v[2], v[3]);
  }
  return ld8_masked(row, k, kend);
}

__device__ inline void store_acc16(float* out, int64_t ld, int64_t row_base, int col,
                                   const f32x16& acc, int half) {
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int64_t r = row_base + 8 * g + 4 * half;
    st4(out + (int64_t)col * ld + r,
        make_float4(acc[4 * g + 0], acc[4 * g + 1], acc[4 * g + 2], acc[4 * g + 3]));
  }
}

// Same, with the rows at and past `valid` stored as zeros.
__device__ inline void store_acc16_rows(float* out, int64_t ld, int64_t row_base, int col,
                                        const f32x16& acc, int half, int64_t valid) {
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int64_t r = row_base + 8 * g + 4 * half;
    st4(out + (int64_t)col * ld + r,
        make_float4(r + 0 < valid ? acc[4 * g + 0] : 0.f, r + 1 < valid ? acc[4 * g + 1] : 0.f,
                    r + 2 < valid ? acc[4 * g + 2] : 0.f, r + 3 < valid ? acc[4 * g + 3] : 0.f));
  }
}

// Direct-to-LDS form of the A X product for panel width 128: 8 waves, a
// 256 x 128 output block per workgroup (4 x 2 waves of 64 x 64).  The A slabs
// (256 rows x 64 BF16) travel from HBM straight into a 4-deep LDS ring with
// buffer_load ... lds (no registers in between), so three slabs (32 KB each)
// are in flight per workgroup while one is multiplied.  Lane i of a 16-byte
// load lands at LDS offset 16 i of its 1 KB run, so the XOR swizzle of
// 16-byte chunks within a row (chunk c of row r at slot c ^ (r & 7);
// conflict-free MFMA operand reads) is made by the choice of source
// addresses.  The panel slabs (128 columns x 64, from the caches) are loaded
// into registers two slabs ahead and written to a double buffer in LDS.
// Loads complete in issue order, so waiting for a panel load also waits for
// every A slab issued before it: the panel slab t + 1 is waited for at the
// end of slab t, when A slab t + 1 (issued before it) is due anyway, and
// three A slabs stay in flight.  Buffer (not global) loads: the compiler
// counts them in order too, so its own waits stay at that depth.  One
// workgroup barrier per slab.  A partial last slab (k1 not a multiple of 64)
// goes through registers with masked loads, so padding beyond n is never
// read.  Needs 256 * lda and LP * ldx BF16 elements to fit a 31-bit byte
// offset (the launcher checks).  CP: cache-policy bits of the A loads (2 =
// non-temporal: A is streamed once per pass).
//
// NT = 5 (panel width 160): each of the 8 waves takes 32 rows and all five
// 32-column tiles (one A operand read and five panel reads per step).  The
// panel slab is 20 KB, so the A ring has three stages (3 x 32 + 2 x 20 KB of
// LDS): two A slabs in flight while one is multiplied.  The 20 panel runs of
// a slab go to waves w, w + 8, w + 16; waves 4-7 load their second run once
// more into rows 160-191 of the panel buffer, which nothing reads, so every
// wave issues and stores the same number of runs (same wait counts, no
// branch).
constexpr int DL_BM = 256, DL_ARUN = DL_BM / 8 / 8;

template <int CP, int NT>
__global__ __launch_bounds__(512) void k_nn_bf16_dl(const u16* __restrict__ A, int64_t lda,
                                                    int64_t m, int64_t n, int64_t tn,
                                                    const u16* __restrict__ X, int64_t ldx,
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
  // one LDS object per stage: the compiler then sees that reading one stage
  // does not depend on the loads still landing in the others
  __shared__ __attribute__((aligned(1024))) u16 As0[DL_BM * 64], As1[DL_BM * 64];
  __shared__ __attribute__((aligned(1024))) u16 As2[DL_BM * 64], As3[NS == 4 ? DL_BM * 64 : 1];
  __shared__ __attribute__((aligned(1024))) u16 Xs0[XB * 64], Xs1[XB * 64];
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l32 = lane & 31, half = lane >> 5;
  // this wave's first row and column within the block
  const int wrow = NT == 4 ? (wave & 3) * 64 : wave * 32;
  const int wcol = NT == 4 ? (wave >> 2) * 64 : 0;
  const int64_t i0 = (int64_t)blockIdx.x * DL_BM;
  const int64_t k0 = (int64_t)blockIdx.y * tn;
  const int64_t k1 = min(n, k0 + tn);
  float* Yp = Y + (int64_t)blockIdx.y * part_stride;
  const int64_t nfull = (k1 - k0) / 64;               // whole 64-deep slabs
  const bool tail = k0 + nfull * 64 < k1;
  // this lane's 16-byte source within a 1 KB run: row rr of the run, slot sl
  const int rr = lane >> 3, sl = lane & 7;
  const int rows = (int)min((int64_t)DL_BM, m - i0);  // valid rows of this block
  // buffer descriptors (data format 32 in the fourth word); the byte extents
  // end at the last element either matrix holds, so the hardware range check
  // returns zeros rather than reading past it
  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(A + i0 * lda), (short)0, (int)(((int64_t)(rows - 1) * lda + n) * 2), 0x00020000);
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
      (void*)X, (short)0, (int)(((int64_t)(LP - 1) * ldx + n) * 2), 0x00020000);

  // A slab t into LDS stage st, or past the last slab a re-read of panel
  // slab 0 (from the caches) so that every slab issues the same loads.  One
  // instruction sequence for both (descriptor and offsets are selected).
  auto issue_a = [&](u16* st, int64_t t) {
    const bool real = t < nfull;
    const __amdgpu_buffer_rsrc_t rs = real ? ra : rx;
    const int kk = (int)(k0 + t * 64);
#pragma unroll
    for (int j = 0; j < DL_ARUN; ++j) {
      const int r = (wave * DL_ARUN + j) * 8 + rr;   // row within the block
      const int rc = min(r, rows - 1);                // rows past m: any valid row
      const int c = r % LP;
      const int off = real ? (rc * (int)lda + kk + 8 * (sl ^ (r & 7))) * 2
                           : (c * (int)ldx + (int)k0 + 8 * sl) * 2;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, st + (wave * DL_ARUN + j) * 512, 16, off, 0, 0, CP);
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
  // panel slab t (slab 0 past the last) into registers, and registers -> LDS
  auto load_x = [&](v4u (&x)[XR], int64_t t) {
    const int kk = (int)(k0 + (t < nfull ? t : 0) * 64);
#pragma unroll
    for (int u = 0; u < XR; ++u) {
      const int c = xrun_ld(u) * 8 + rr;
      x[u] = __builtin_amdgcn_raw_buffer_load_b128(rx, (c * (int)ldx + kk + 8 * (sl ^ (c & 7))) * 2, 0, 0);
    }
  };
  auto store_x = [&](u16* st, const v4u (&x)[XR]) {
#pragma unroll
    for (int u = 0; u < XR; ++u)
      *reinterpret_cast<v4u*>(st + xrun(u) * 512 + lane * 8) = x[u];
  };

  f32x16 acc[MT][NW];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int t = 0; t < NW; ++t) acc[a][t] = f32x16{};

  auto compute = [&](const u16* as, const u16* xs) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int q = half * 4 + s;                    // 16-byte chunk of the 64-deep slab
      bf16x8 av[MT], bv[NW];
#pragma unroll
      for (int a = 0; a < MT; ++a) {
        const int r = wrow + a * 32 + l32;
        av[a] = *reinterpret_cast<const bf16x8*>(as + r * 64 + 8 * (q ^ (r & 7)));
      }
#pragma unroll
      for (int t = 0; t < NW; ++t) {
        const int c = wcol + t * 32 + l32;
        bv[t] = *reinterpret_cast<const bf16x8*>(xs + c * 64 + 8 * (q ^ (c & 7)));
      }
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int t = 0; t < NW; ++t) acc[a][t] = mfma_bf16(av[a], bv[t], acc[a][t]);
    }
  };

  // Slab t: A stage t % NS, panel buffer t % 2.  Every slab issues the same
  // loads (dummies past the end), so the wait counts are constants.  Issue
  // order of slab t: panel registers of slab t + 2 (XR loads), then A slab
  // t + NS - 1 (DL_ARUN loads).  One step, entered after a barrier that
  // follows every wave's A slab t and panel slab t landing in LDS:
  //   issue panel slab t + 2 -> registers xn, A slab t + NS - 1 -> the stage
  //   slab t - 1 used; compute slab t; wait for the panel registers xp of
  //   slab t + 1 (the loads issued since: this step's, and with four stages
  //   also the previous step's A slab), which also means this wave's A slab
  //   t + 1 has landed; write them to the panel buffer slab t - 1 used;
  //   barrier.
  // s_waitcnt immediates: vmcnt in bits 3:0 and 15:14, expcnt 6:4 and
  // lgkmcnt 11:8 (0xc07f: lgkmcnt(0) only).
  constexpr int kWaitStep = 0x0f70 | ((NS - 2) * DL_ARUN + XR);
  auto step = [&](int64_t t, u16* as, u16* xs, u16* xs_next, u16* as_refill, v4u (&xp)[XR],
                  v4u (&xn)[XR]) {
    load_x(xn, t + 2);
    issue_a(as_refill, t + NS - 1);
    __builtin_amdgcn_sched_barrier(0);          // loads go out before the compute
    compute(as, xs);
    __builtin_amdgcn_s_waitcnt(kWaitStep);
    store_x(xs_next, xp);
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_s_barrier();
  };

  v4u xa[XR], xb[XR];                           // panel registers, two slabs
  if (nfull > 0) {
    load_x(xa, 0);
    __builtin_amdgcn_s_waitcnt(0x0f70);
    store_x(Xs0, xa);
    load_x(xb, 1);
    issue_a(As0, 0);
    issue_a(As1, 1);
    if (NS == 4) issue_a(As2, 2);
    // A slab 0 (and the panel registers of slab 1) are older than A slabs
    // 1 .. NS - 2
    __builtin_amdgcn_s_waitcnt(0x0f70 | ((NS - 2) * DL_ARUN));
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_s_barrier();
  }
  // slab t holds its panel registers: slab t + 1 in xb when t is even, else xa
  int64_t tb = 0;
  if constexpr (NS == 4) {
    for (; tb + 3 < nfull; tb += 4) {   // four whole steps: no branch between them
      step(tb, As0, Xs0, Xs1, As3, xb, xa);
      step(tb + 1, As1, Xs1, Xs0, As0, xa, xb);
      step(tb + 2, As2, Xs0, Xs1, As1, xb, xa);
      step(tb + 3, As3, Xs1, Xs0, As2, xa, xb);
    }
    if (tb < nfull) {                     // up to three remaining slabs
      step(tb, As0, Xs0, Xs1, As3, xb, xa);
      if (tb + 1 < nfull) {
        step(tb + 1, As1, Xs1, Xs0, As0, xa, xb);
        if (tb + 2 < nfull) step(tb + 2, As2, Xs0, Xs1, As1, xb, xa);
      }
    }
  } else {
    for (; tb + 5 < nfull; tb += 6) {   // six whole steps: stages and buffers realign
      step(tb, As0, Xs0, Xs1, As2, xb, xa);
      step(tb + 1, As1, Xs1, Xs0, As0, xa, xb);
      step(tb + 2, As2, Xs0, Xs1, As1, xb, xa);
      step(tb + 3, As0, Xs1, Xs0, As2, xa, xb);
      step(tb + 4, As1, Xs0, Xs1, As0, xb, xa);
      step(tb + 5, As2, Xs1, Xs0, As1, xa, xb);
    }
    if (tb < nfull) step(tb, As0, Xs0, Xs1, As2, xb, xa);   // up to five remaining slabs
    if (tb + 1 < nfull) step(tb + 1, As1, Xs1, Xs0, As0, xa, xb);
    if (tb + 2 < nfull) step(tb + 2, As2, Xs0, Xs1, As1, xb, xa);
    if (tb + 3 < nfull) step(tb + 3, As0, Xs1, Xs0, As2, xa, xb);
    if (tb + 4 < nfull) step(tb + 4, As1, Xs0, Xs1, As0, xb, xa);
  }
  __builtin_amdgcn_s_waitcnt(0x0f70);   // the last (dummy) loads land before LDS is reused or freed
  if (tail) {   // last, partial slab: masked loads through registers
    __syncthreads();
    const int64_t kk = k0 + nfull * 64;
    for (int e = tid; e < DL_BM * 8; e += 512) {
      const int r = e >> 3, c = e & 7;
      const int64_t gi = min(i0 + r, m - 1);
      *reinterpret_cast<uint4*>(As0 + r * 64 + 8 * (c ^ (r & 7))) =
          ld8_masked(A + gi * lda, kk + 8 * c, k1);
    }
    for (int e = tid; e < LP * 8; e += 512) {
      const int r = e >> 3, c = e & 7;
      *reinterpret_cast<uint4*>(Xs0 + r * 64 + 8 * (c ^ (r & 7))) =
          ld8_masked(X + (int64_t)r * ldx, kk + 8 * c, k1);
    }
    __syncthreads();
    compute(As0, Xs0);
  }
  // rows [m, m rounded up to 128) are written as zeros, as by the
  // register-staged form (rows past m of the block hold sums of the clamped
  // row m - 1)
  const int64_t mz = (m + 127) / 128 * 128;
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int t = 0; t < NW; ++t) {
      const int64_t rb = i0 + wrow + a * 32;
      if (rb < mz) store_acc16_rows(Yp, ldy, rb, wcol + t * 32 + l32, acc[a][t], half, m);
    }
}

// Y (+ partial J) = A16(:, tile J) X16(tile J, :).  4 waves; wave w owns rows
// [w*WR, (w+1)*WR) of the BM = 4*WR rows and all NT*32 panel columns.
// Within a 64-deep slab, lane half h takes reduction indices h*32 + 8s + v at
// MFMA step s, so every lane reads 16-byte runs of both LDS tiles.
template <int NT, int MT>
__global__ __launch_bounds__(256) void k_nn_bf16(const u16* __restrict__ A, int64_t lda, int64_t m,
                                                 int64_t n, int64_t tn, const u16* __restrict__ X,
                                                 int64_t ldx, float* __restrict__ Y, int64_t ldy,
                                                 int64_t part_stride) {
  constexpr int LP = NT * 32, WR = MT * 32, BM = 4 * WR, AS = BM / 32;
  __shared__ __attribute__((aligned(16))) u16 As[2][BM][PADK];
  __shared__ __attribute__((aligned(16))) u16 Xs[2][LP][PADK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int64_t i0 = (int64_t)blockIdx.x * BM;
  const int64_t k0 = (int64_t)blockIdx.y * tn;
  const int64_t k1 = min(n, k0 + tn);
  float* Yp = Y + (int64_t)blockIdx.y * part_stride;
  const int lr = tid >> 3, lc = (tid & 7) * 8;

  uint4 ra[AS];
  uint4 rx[NT];
  auto gload = [&](int64_t kt) {
    const int64_t kk = kt + lc;
#pragma unroll
    for (int s = 0; s < AS; ++s) {
      const int64_t i = i0 + lr + 32 * s;
      ra[s] = (i < m && kk < k1) ? ld8_masked(A + i * lda, kk, k1) : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int s = 0; s < NT; ++s) {
      const int c = lr + 32 * s;
      rx[s] = kk < k1 ? ld8_masked(X + (int64_t)c * ldx, kk, k1) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int s = 0; s < AS; ++s) *reinterpret_cast<uint4*>(&As[buf][lr + 32 * s][lc]) = ra[s];
#pragma unroll
    for (int s = 0; s < NT; ++s) *reinterpret_cast<uint4*>(&Xs[buf][lr + 32 * s][lc]) = rx[s];
  };

  f32x16 acc[MT][NT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[a][t] = f32x16{};

  gload(k0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int64_t kt = k0; kt < k1; kt += BK) {
    const bool more = kt + BK < k1;
    if (more) gload(kt + BK);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      bf16x8 av[MT], bv[NT];
#pragma unroll
      for (int a = 0; a < MT; ++a)
        av[a] = *reinterpret_cast<const bf16x8*>(&As[buf][wave * WR + a * 32 + l32][half * 32 + s * 8]);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        bv[t] = *reinterpret_cast<const bf16x8*>(&Xs[buf][t * 32 + l32][half * 32 + s * 8]);
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[a][t] = mfma_bf16(av[a], bv[t], acc[a][t]);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int t = 0; t < NT; ++t)
      store_acc16(Yp, ldy, i0 + wave * WR + a * 32, t * 32 + l32, acc[a][t], half);
}

// Square wave tiles: the 128 x 128 output block of a workgroup is split 2 x 2
// over the waves (64 rows x 64 panel columns each), so a wave reads 64 rows
// of A and 64 columns of the panel from LDS per slab instead of 32 rows and
// all 128 columns.  One LDS stage (37 KB, several workgroups per CU); the
// next DEPTH slabs are in flight in registers while the current one is
// multiplied, and A is loaded with a non-temporal hint (it is streamed once
// per pass; the caches stay with the panel).  Panel width 128.
//
// CAST: A is the FP32 input (rows 16-byte aligned) instead of its BF16 copy;
// each 8-value chunk is rounded to BF16 (nearest even) in registers, written
// to A16 (the copy the later passes read) and multiplied, so the sketch pass
// also produces the BF16 copy: one read of the FP32 matrix instead of two.
// Every element of A belongs to exactly one workgroup, so A16 is written once.
__device__ inline uint32_t pack_bf16(float a, float b);

template <int DEPTH, int MR = 2, bool CAST = false>
__global__ __launch_bounds__(256) void k_nn_bf16_sq(const u16* __restrict__ A, int64_t lda,
                                                    int64_t m, int64_t n, int64_t tn,
                                                    const u16* __restrict__ X, int64_t ldx,
                                                    float* __restrict__ Y, int64_t ldy,
                                                    int64_t part_stride,
                                                    const float* __restrict__ A32 = nullptr,
                                                    u16* __restrict__ A16 = nullptr,
                                                    int64_t lda16 = 0) {
  constexpr int BM = 64 * MR, LP = 128, CPR = BK / 8, RPI = 256 / CPR, AS = BM / RPI, XS = LP / RPI;
  __shared__ __attribute__((aligned(16))) u16 As[BM][PADK];
  __shared__ __attribute__((aligned(16))) u16 Xs[LP][PADK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int wr = wave & 1, wc = wave >> 1;
  const int64_t i0 = (int64_t)blockIdx.x * BM;
  const int64_t k0 = (int64_t)blockIdx.y * tn;
  const int64_t k1 = min(n, k0 + tn);
  float* Yp = Y + (int64_t)blockIdx.y * part_stride;
  const int lr = tid / CPR, lc = (tid % CPR) * 8;

  uint4 ra[DEPTH][AS];
  uint4 rx[DEPTH][XS];
  auto gload = [&](int d, int64_t kt) {
    const int64_t kk = kt + lc;
#pragma unroll
    for (int s = 0; s < AS; ++s) {
      const int64_t i = i0 + lr + RPI * s;
      if (CAST) {
        uint4 w = make_uint4(0u, 0u, 0u, 0u);
        if (i < m && kk < k1) {
          const float* row = A32 + i * lda;
          const float4 x0 = ld4_masked(row, kk, k1), x1 = ld4_masked(row, kk + 4, k1);
          w = make_uint4(pack_bf16(x0.x, x0.y), pack_bf16(x0.z, x0.w), pack_bf16(x1.x, x1.y),
                         pack_bf16(x1.z, x1.w));
          u16* dst = A16 + i * lda16 + kk;
          if (kk + 8 <= k1) {
            *reinterpret_cast<uint4*>(dst) = w;
          } else {
            const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
            for (int e = 0; kk + e < k1; ++e) dst[e] = (u16)(ww[e >> 1] >> (16 * (e & 1)));
          }
        }
        ra[d][s] = w;
      } else {
        ra[d][s] = (i < m && kk < k1) ? ld8_masked_nt(A + i * lda, kk, k1) : make_uint4(0u, 0u, 0u, 0u);
      }
    }
#pragma unroll
    for (int s = 0; s < XS; ++s) {
      const int c = lr + RPI * s;
      rx[d][s] = kk < k1 ? ld8_masked(X + (int64_t)c * ldx, kk, k1) : make_uint4(0u, 0u, 0u, 0u);
    }
  };

  f32x16 acc[MR][2];
#pragma unroll
  for (int a = 0; a < MR; ++a)
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[a][t] = f32x16{};

  auto step = [&](int d, int64_t kt) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < AS; ++s) *reinterpret_cast<uint4*>(&As[lr + RPI * s][lc]) = ra[d][s];
#pragma unroll
    for (int s = 0; s < XS; ++s) *reinterpret_cast<uint4*>(&Xs[lr + RPI * s][lc]) = rx[d][s];
    __syncthreads();
    if (kt + DEPTH * BK < k1) gload(d, kt + DEPTH * BK);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kc = half * 32 + s * 8;
      bf16x8 av[MR], bv[2];
#pragma unroll
      for (int a = 0; a < MR; ++a)
        av[a] = *reinterpret_cast<const bf16x8*>(&As[wr * 32 * MR + a * 32 + l32][kc]);
#pragma unroll
      for (int t = 0; t < 2; ++t)
        bv[t] = *reinterpret_cast<const bf16x8*>(&Xs[wc * 64 + t * 32 + l32][kc]);
#pragma unroll
      for (int a = 0; a < MR; ++a)
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[a][t] = mfma_bf16(av[a], bv[t], acc[a][t]);
    }
  };

#pragma unroll
  for (int d = 0; d < DEPTH; ++d)
    if (k0 + d * BK < k1) gload(d, k0 + d * BK);
  for (int64_t kt = k0; kt < k1; kt += DEPTH * BK) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d)
      if (kt + d * BK < k1) step(d, kt + d * BK);
  }
#pragma unroll
  for (int a = 0; a < MR; ++a)
#pragma unroll
    for (int t = 0; t < 2; ++t)
      store_acc16(Yp, ldy, i0 + wr * 32 * MR + a * 32, wc * 64 + t * 32 + l32, acc[a][t], half);
}

// Direct-to-LDS form of the sketch pass with the cast (panel width 128): A is
// the FP32 input, and the pass both multiplies it and writes its BF16 copy.
// 8 waves, a 128 x 128 output block per workgroup (4 x 2 waves of 32 x 64).
// The FP32 slabs (128 rows x 64 values = 32 KB, 256-byte row pieces) stream
// into a 4-deep LDS ring with buffer_load ... lds; each lane reads its 8
// values per matrix-core step from LDS and rounds them to BF16 (nearest even,
// as the register form) before multiplying, and the slab is also read once
// more, row-contiguously, to write the copy (128 bytes per row and slab).
// Layout of a slab in LDS: row r at 256 r bytes, its 16-byte chunk c (4
// values) at slot c ^ (r & 7), which keeps the 8 rows read per LDS cycle on
// distinct banks.  The panel slabs go through registers two slabs ahead, as
// in the BF16 form, with the same slab schedule (the copy stores enter the
// wait counts).  A partial last slab goes through registers with masked
// loads and masked copy writes.  Needs 128 * lda FP32 values, 128 * ldx and
// 128 * lda16 BF16 values within a 31-bit byte offset (the launcher checks).
constexpr int DC_BM = 128, DC_LP = 128, DC_ARUN = 4, DC_XRUN = 2;

__global__ __launch_bounds__(512) void k_nn_bf16_dl_cast(const float* __restrict__ A32, int64_t lda,
                                                         int64_t m, int64_t n, int64_t tn,
                                                         const u16* __restrict__ X, int64_t ldx,
                                                         float* __restrict__ Y, int64_t ldy,
                                                         int64_t part_stride,
                                                         u16* __restrict__ A16, int64_t lda16) {
  __shared__ __attribute__((aligned(1024))) float As0[DC_BM * 64], As1[DC_BM * 64];
  __shared__ __attribute__((aligned(1024))) float As2[DC_BM * 64], As3[DC_BM * 64];
  __shared__ __attribute__((aligned(1024))) u16 Xs0[DC_LP * 64], Xs1[DC_LP * 64];
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l32 = lane & 31, half = lane >> 5;
  const int wr = wave & 3, wc = wave >> 2;
  const int64_t i0 = (int64_t)blockIdx.x * DC_BM;
  const int64_t k0 = (int64_t)blockIdx.y * tn;
  const int64_t k1 = min(n, k0 + tn);
  float* Yp = Y + (int64_t)blockIdx.y * part_stride;
  const int64_t nfull = (k1 - k0) / 64;
  const bool tail = k0 + nfull * 64 < k1;
  const int rows = (int)min((int64_t)DC_BM, m - i0);
  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(A32 + i0 * lda), (short)0, (int)(((int64_t)(rows - 1) * lda + n) * 4), 0x00020000);
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
      (void*)X, (short)0, (int)(((int64_t)(DC_LP - 1) * ldx + n) * 2), 0x00020000);

  // A slab t: wave w fills the 1 KB runs 4 w .. 4 w + 3, run b = rows 4 b ..
  // 4 b + 3; lane i writes slot i & 15 of row 4 b + (i >> 4), which holds
  // chunk (i & 15) ^ (row & 7).  Past the last slab: panel re-reads.
  auto issue_a = [&](float* st, int64_t t) {
    const bool real = t < nfull;
    const __amdgpu_buffer_rsrc_t rs = real ? ra : rx;
    const int kk = (int)(k0 + t * 64);
#pragma unroll
    for (int j = 0; j < DC_ARUN; ++j) {
      const int b = wave * DC_ARUN + j;
      const int r = 4 * b + (lane >> 4), slot = lane & 15;
      const int rc = min(r, rows - 1);
      const int off = (rc * (int)lda + kk + 4 * (slot ^ (r & 7))) * 4;
      const int c = (4 * b + (lane >> 4)) & (DC_LP - 1);
      const int doff = (c * (int)ldx + (int)k0 + 8 * (slot & 7)) * 2;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, st + b * 256, 16, real ? off : doff, 0, 0, 2);
    }
  };
  const int rr = lane >> 3, sl = lane & 7;
  const int xc0 = (wave * DC_XRUN) * 8 + rr, xc1 = xc0 + 8;
  auto load_x = [&](v4u& x0, v4u& x1, int64_t t) {
    const int kk = (int)(k0 + (t < nfull ? t : 0) * 64);
    x0 = __builtin_amdgcn_raw_buffer_load_b128(rx, (xc0 * (int)ldx + kk + 8 * (sl ^ (xc0 & 7))) * 2, 0, 0);
    x1 = __builtin_amdgcn_raw_buffer_load_b128(rx, (xc1 * (int)ldx + kk + 8 * (sl ^ (xc1 & 7))) * 2, 0, 0);
  };
  auto store_x = [&](u16* st, const v4u& x0, const v4u& x1) {
    *reinterpret_cast<v4u*>(st + (wave * DC_XRUN) * 512 + lane * 8) = x0;
    *reinterpret_cast<v4u*>(st + (wave * DC_XRUN + 1) * 512 + lane * 8) = x1;
  };

  f32x16 acc[2];
  acc[0] = f32x16{};
  acc[1] = f32x16{};
  const int row = wr * 32 + l32;                   // this lane's A row in the block
  // the copy's rows of this block; rows past m fall outside the extent, so
  // their stores are dropped by the range check
  const __amdgpu_buffer_rsrc_t rc16 = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(A16 + i0 * lda16), (short)0, (int)((int64_t)rows * lda16 * 2), 0x00020000);
  // slab in LDS -> BF16 copy: thread e / 8-value chunk: 8 threads per row,
  // 128 contiguous bytes per row and slab, two 16-byte stores per thread
  // (rows past m: offsets past the extent, dropped).  The partial slab stores
  // element by element up to k1.
  auto copy_out = [&](const float* as, int64_t kb, bool masked) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int e = tid + 512 * j, r = e >> 3, c8 = e & 7;
      const float4 f0 = *reinterpret_cast<const float4*>(as + r * 64 + 4 * ((2 * c8) ^ (r & 7)));
      const float4 f1 = *reinterpret_cast<const float4*>(as + r * 64 + 4 * ((2 * c8 + 1) ^ (r & 7)));
      const v4u w = {pack_bf16(f0.x, f0.y), pack_bf16(f0.z, f0.w), pack_bf16(f1.x, f1.y),
                     pack_bf16(f1.z, f1.w)};
      const int64_t kk = kb + 8 * c8;
      if (!masked) {
        __builtin_amdgcn_raw_buffer_store_b128(w, rc16, (int)((r * lda16 + kk) * 2), 0, 2);
      } else if (i0 + r < m) {
        u16* dst = A16 + (i0 + r) * lda16 + kk;
        for (int q = 0; q < 8 && kk + q < k1; ++q) dst[q] = (u16)(w[q >> 1] >> (16 * (q & 1)));
      }
    }
  };
  // the matrix-core steps of a slab: lane half h takes the values 32 h + 8 s
  // .. + 7 at step s (the order of the register form), rounded to BF16
  auto compute = [&](const float* as, const u16* xs) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int q = 8 * half + 2 * s;              // first 16-byte chunk of this lane's 8 values
      const float4 f0 = *reinterpret_cast<const float4*>(as + row * 64 + 4 * (q ^ (row & 7)));
      const float4 f1 = *reinterpret_cast<const float4*>(as + row * 64 + 4 * ((q + 1) ^ (row & 7)));
      const uint4 w = make_uint4(pack_bf16(f0.x, f0.y), pack_bf16(f0.z, f0.w),
                                 pack_bf16(f1.x, f1.y), pack_bf16(f1.z, f1.w));
      bf16x8 av;
      __builtin_memcpy(&av, &w, 16);
      const int qx = 4 * half + s;                 // panel chunk (8 values) of this step
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int c = wc * 64 + t * 32 + l32;
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(xs + c * 64 + 8 * (qx ^ (c & 7)));
        acc[t] = mfma_bf16(av, bv, acc[t]);
      }
    }
  };

  // the slab schedule of the BF16 form, with this pass's copy stores in the
  // count: issue order of slab t is panel t + 2 (DC_XRUN), A t + 3
  // (DC_ARUN), the copy stores of slab t (4).  Waiting for the panel
  // registers of t + 1 at the end of slab t allows the A slab t + 2, the
  // stores of t - 1 and everything of t to stay in flight; at the end of slab
  // 0 nothing of slab -1 exists, so the wait is shorter there (A slab 1 must
  // have landed for slab 1).
  auto vmwait = [](int cnt) { return 0x0f70 | (cnt & 15) | ((cnt >> 4) << 14); };
  constexpr int kStores = 2;
  auto step = [&](int64_t t, float* as, u16* xs, u16* xs_next, float* as_refill, v4u& xp0,
                  v4u& xp1, v4u& xn0, v4u& xn1, bool first) {
    load_x(xn0, xn1, t + 2);
    issue_a(as_refill, t + 3);
    __builtin_amdgcn_sched_barrier(0);
    copy_out(as, k0 + t * 64, false);
    compute(as, xs);
    __builtin_amdgcn_sched_barrier(0);
    if (first)
      __builtin_amdgcn_s_waitcnt(vmwait(2 * DC_ARUN + DC_XRUN + kStores));
    else
      __builtin_amdgcn_s_waitcnt(vmwait(2 * DC_ARUN + DC_XRUN + 2 * kStores));
    store_x(xs_next, xp0, xp1);
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_s_barrier();
  };

  v4u xa0, xa1, xb0, xb1;
  if (nfull > 0) {
    load_x(xa0, xa1, 0);
    __builtin_amdgcn_s_waitcnt(0x0f70);
    store_x(Xs0, xa0, xa1);
    load_x(xb0, xb1, 1);
    issue_a(As0, 0);
    issue_a(As1, 1);
    issue_a(As2, 2);
    __builtin_amdgcn_s_waitcnt(0x0f70 | (2 * DC_ARUN));
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_s_barrier();
    step(0, As0, Xs0, Xs1, As3, xb0, xb1, xa0, xa1, true);
  }
  int64_t tb = 1;
  for (; tb + 3 < nfull; tb += 4) {     // four whole steps: no branch between them
    step(tb, As1, Xs1, Xs0, As0, xa0, xa1, xb0, xb1, false);
    step(tb + 1, As2, Xs0, Xs1, As1, xb0, xb1, xa0, xa1, false);
    step(tb + 2, As3, Xs1, Xs0, As2, xa0, xa1, xb0, xb1, false);
    step(tb + 3, As0, Xs0, Xs1, As3, xb0, xb1, xa0, xa1, false);
  }
  if (tb < nfull) {                     // up to three remaining slabs
    step(tb, As1, Xs1, Xs0, As0, xa0, xa1, xb0, xb1, false);
    if (tb + 1 < nfull) {
      step(tb + 1, As2, Xs0, Xs1, As1, xb0, xb1, xa0, xa1, false);
      if (tb + 2 < nfull) step(tb + 2, As3, Xs1, Xs0, As2, xa0, xa1, xb0, xb1, false);
    }
  }
  __builtin_amdgcn_s_waitcnt(0x0f70);
  if (tail) {   // last, partial slab: masked loads through registers
    __syncthreads();
    const int64_t kk = k0 + nfull * 64;
    for (int e = tid; e < DC_BM * 16; e += 512) {
      const int r = e >> 4, c = e & 15;
      const int64_t gi = min(i0 + r, m - 1);
      *reinterpret_cast<float4*>(As0 + r * 64 + 4 * (c ^ (r & 7))) =
          ld4_masked(A32 + gi * lda, kk + 4 * c, k1);
    }
    for (int e = tid; e < DC_LP * 8; e += 512) {
      const int r = e >> 3, c = e & 7;
      *reinterpret_cast<uint4*>(Xs0 + r * 64 + 8 * (c ^ (r & 7))) =
          ld8_masked(X + (int64_t)r * ldx, kk + 8 * c, k1);
    }
    __syncthreads();
    copy_out(As0, kk, true);
    compute(As0, Xs0);
  }
  const int64_t mz = (m + 127) / 128 * 128;
  const int64_t rb = i0 + wr * 32;
  if (rb < mz) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
      store_acc16_rows(Yp, ldy, rb, wc * 64 + t * 32 + l32, acc[t], half, m);
  }
}

// Z (+ partial I) = A16(tile I, :)^T Q16(tile I, :).  The A tile is staged
// row-major as loaded ([i][j], coalesced 16-byte loads); each lane gathers
// its A^T fragment (8 consecutive i of one column j) with 16-bit LDS reads,
// so no transposed copy of A is ever stored.
constexpr int TBN = 128;
constexpr int TPAD = TBN + 8;
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;

template <int NT, bool NTL = false>
__global__ __launch_bounds__(256) void k_tn_bf16(const u16* __restrict__ A, int64_t lda, int64_t m,
                                                 int64_t n, int64_t tm, const u16* __restrict__ Q,
                                                 int64_t ldq, float* __restrict__ Z, int64_t ldz,
                                                 int64_t part_stride) {
  constexpr int LP = NT * 32;
  __shared__ __attribute__((aligned(16))) u16 As[2][BK][TPAD];
  __shared__ __attribute__((aligned(16))) u16 Qs[2][LP][PADK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int64_t j0 = (int64_t)blockIdx.x * TBN;
  const int64_t ib0 = (int64_t)blockIdx.y * tm;
  const int64_t ib1 = min(m, ib0 + tm);
  float* Zp = Z + (int64_t)blockIdx.y * part_stride;
  const int ar = tid >> 4, ac = (tid & 15) * 8;      // A tile: 16 chunks of 8 per row
  const int qr = tid >> 3, qc = (tid & 7) * 8;       // Q tile: 8 chunks of 8 per row

  uint4 ra[4];
  uint4 rq[NT];
  auto gload = [&](int64_t it) {
    const int64_t j = j0 + ac;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t i = it + ar + 16 * s;
      ra[s] = (i < ib1 && j < n) ? (NTL ? ld8_masked_nt(A + i * lda, j, n) : ld8_masked(A + i * lda, j, n))
                                 : make_uint4(0u, 0u, 0u, 0u);
    }
    const int64_t kk = it + qc;
#pragma unroll
    for (int s = 0; s < NT; ++s) {
      const int c = qr + 32 * s;
      rq[s] = kk < ib1 ? ld8_masked(Q + (int64_t)c * ldq, kk, ib1) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int s = 0; s < 4; ++s) *reinterpret_cast<uint4*>(&As[buf][ar + 16 * s][ac]) = ra[s];
#pragma unroll
    for (int s = 0; s < NT; ++s) *reinterpret_cast<uint4*>(&Qs[buf][qr + 32 * s][qc]) = rq[s];
  };

  f32x16 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x16{};

  gload(ib0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  const int jl = wave * 32 + l32;
  for (int64_t it = ib0; it < ib1; it += BK) {
    const bool more = it + BK < ib1;
    if (more) gload(it + BK);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      // reduction indices of this step: 16 s + 8 half + v
      bf16x8 av;
      uint32_t w[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const uint32_t lo = As[buf][s * 16 + half * 8 + 2 * v][jl];
        const uint32_t hi = As[buf][s * 16 + half * 8 + 2 * v + 1][jl];
        w[v] = lo | (hi << 16);
      }
      __builtin_memcpy(&av, w, 16);
      bf16x8 bv[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t)
        bv[t] = *reinterpret_cast<const bf16x8*>(&Qs[buf][t * 32 + l32][s * 16 + half * 8]);
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = mfma_bf16(av, bv[t], acc[t]);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) store_acc16(Zp, ldz, j0 + wave * 32, t * 32 + l32, acc[t], half);
}

// Direct-to-LDS form of Z (+ partial I) = A16(tile I, :)^T Q16(tile I, :) for
// panel width 128: 8 waves, a 256 x 128 output block per workgroup (4 x 2
// waves of 64 x 64), the reduction running over the rows of the tile.  The A
// slabs (64 rows x 256 BF16 columns = 32 KB) stream from HBM into a 4-deep LDS
// ring with buffer_load ... lds and the panel slabs (128 columns x 64 rows)
// go through registers two slabs ahead into a double buffer, as in the A X
// form above.  The matrix-core A operand needs 8 consecutive rows of one
// column per lane: ds_read_tr16_b64 transposes 4 rows x 16 columns across a
// 16-lane group, so two such reads give each lane its 8 rows.  Layout of an A
// slab in LDS: row r at 512 r bytes, its 16-byte chunk c at slot
// c ^ 2 (r & 3), so the 4 rows of a transposed read fall on distinct banks
// (the DMA writes lane i at offset 16 i, so the swizzle is in the source
// addresses).  Rows past the tile read zeros through the buffer range check
// (offsets past the descriptor's extent), so the reduction needs no tail
// path; panel rows past the tile are zeroed the same way.  Columns past n
// re-read the block's last chunk: with n a multiple of 32 their sums fill
// only whole 32-row groups of the output past n, which are stored as zeros.
// Needs n a multiple of 32, m a multiple of 8, tm * lda and LP * ldq BF16
// elements within a 31-bit byte offset (the launcher checks).
//
// NT = 5 (panel width 160), as for the A X form: each of the 8 waves takes 32
// output rows and all five 32-column tiles, the A ring has three stages, and
// the 20 panel runs of a slab go to waves w, w + 8, w + 16 (waves 4-7 load
// their second run once more into rows 160-191 of the panel buffer, which
// nothing reads).
constexpr int DT_BN = 256, DT_ARUN = 64 * DT_BN / 512 / 8;

template <int CP, int NT>
__global__ __launch_bounds__(512) void k_tn_bf16_dl(const u16* __restrict__ A, int64_t lda,
                                                    int64_t m, int64_t n, int64_t tm,
                                                    const u16* __restrict__ Q, int64_t ldq,
                                                    float* __restrict__ Z, int64_t ldz,
                                                    int64_t part_stride) {
  static_assert(DT_ARUN == 4, "four 1 KB runs per wave and slab");
  static_assert(NT == 4 || NT == 5, "panel widths 128 and 160");
  constexpr int LP = 32 * NT;
  constexpr int NS = NT == 4 ? 4 : 3;           // A ring stages
  constexpr int XR = NT == 4 ? 2 : 3;           // panel loads per lane and slab
  constexpr int XB = 64 * XR;                   // panel buffer rows (192 at width 160: the
                                                // unused third runs of waves 4-7 land past 160)
  constexpr int MT = NT == 4 ? 2 : 1;           // 32-row output tiles per wave
  constexpr int NW = NT == 4 ? 2 : 5;           // 32-column tiles per wave
  __shared__ __attribute__((aligned(1024))) u16 As0[64 * DT_BN], As1[64 * DT_BN];
  __shared__ __attribute__((aligned(1024))) u16 As2[64 * DT_BN], As3[NS == 4 ? 64 * DT_BN : 1];
  __shared__ __attribute__((aligned(1024))) u16 Qs0[XB * 64], Qs1[XB * 64];
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l32 = lane & 31, half = lane >> 5;
  const int wrow = NT == 4 ? (wave & 3) * 64 : wave * 32;   // first output row (column of A)
  const int wcol = NT == 4 ? (wave >> 2) * 64 : 0;          // first panel column
  const int64_t j0 = (int64_t)blockIdx.x * DT_BN;
  const int64_t ib0 = (int64_t)blockIdx.y * tm;
  const int64_t ib1 = min(m, ib0 + tm);
  float* Zp = Z + (int64_t)blockIdx.y * part_stride;
  const int64_t ns = (ib1 - ib0 + 63) / 64;            // slabs, the last one maybe partial
  // columns of this block that exist; chunks past them re-read the last one
  // (their sums land only in output rows past n, which are stored as zeros)
  const int ncol = (int)min((int64_t)DT_BN, n - j0);
  constexpr int kOob = 0x7ffffff0;                      // past every extent below: reads zero
  // A rows [ib0, ib1) from column j0; the extent ends with row ib1 - 1
  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(A + ib0 * lda + j0), (short)0, (int)((ib1 - ib0) * lda * 2), 0x00020000);
  const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc(
      (void*)Q, (short)0, (int)(((int64_t)(LP - 1) * ldq + m) * 2), 0x00020000);

  // A slab t: wave w fills the 1 KB runs 4 w .. 4 w + 3, run b = rows 2 b and
  // 2 b + 1; lane i writes slot i & 31 of row 2 b + (i >> 5), which holds
  // chunk (i & 31) ^ 2 (row & 3).  Past the last slab: a re-read of panel
  // slab 0 (cached), so every slab issues the same loads.
  auto issue_a = [&](u16* st, int64_t t) {
    const bool real = t < ns;
    const __amdgpu_buffer_rsrc_t rs = real ? ra : rq;
#pragma unroll
    for (int j = 0; j < DT_ARUN; ++j) {
      const int b = wave * DT_ARUN + j;
      const int r = 2 * b + (lane >> 5), slot = lane & 31;
      const int ch = slot ^ (2 * (r & 3));
      const int row = (int)(t * 64) + r;               // within the tile
      const int off = (row * (int)lda + min(8 * ch, ncol - 8)) * 2;
      const int c = (b * 2 + (lane >> 5)) % LP;
      const int doff = (c * (int)ldq + (int)ib0 + 8 * (slot & 7)) * 2;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, st + b * 512, 16, real ? off : doff, 0, 0, CP);
    }
  };
  // panel runs of this wave (8 panel columns each): 2 w, 2 w + 1 (width 128)
  // or w, w + 8, w + 16 (width 160; runs past the 20 re-read run w + 8 and
  // land in the unread rows 160-191); rows
  // past the tile read zero
  const int rr = lane >> 3, sl = lane & 7;
  auto qrun = [&](int u) { return NT == 4 ? wave * 2 + u : wave + 8 * u; };
  auto qrun_ld = [&](int u) {
    const int j = qrun(u);
    return j < LP / 8 ? j : qrun(1);
  };
  auto load_q = [&](v4u (&x)[XR], int64_t t) {
    const int64_t i0 = ib0 + (t < ns ? t : 0) * 64;
#pragma unroll
    for (int u = 0; u < XR; ++u) {
      const int qc = qrun_ld(u) * 8 + rr;
      const int64_t r0 = i0 + 8 * (sl ^ (qc & 7));
      x[u] = __builtin_amdgcn_raw_buffer_load_b128(rq, r0 < ib1 ? (int)((qc * ldq + r0) * 2) : kOob, 0, 0);
    }
  };
  auto store_q = [&](u16* st, const v4u (&x)[XR]) {
#pragma unroll
    for (int u = 0; u < XR; ++u)
      *reinterpret_cast<v4u*>(st + qrun(u) * 512 + lane * 8) = x[u];
  };

  f32x16 acc[MT][NW];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int t = 0; t < NW; ++t) acc[a][t] = f32x16{};

  // transposed-read coordinates of this lane: 16-lane group g, row a4 of the
  // four, columns 4 b4 .. 4 b4 + 3 of the group's sixteen
  const int g = lane >> 4, a4 = (lane >> 2) & 3, b4 = lane & 3;
  auto compute = [&](const u16* as, const u16* qs) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      bf16x8 av[MT], bv[NW];
#pragma unroll
      for (int a = 0; a < MT; ++a) {
        const int col = wrow + a * 32 + (g & 1) * 16 + 4 * b4;
        const int r0 = s * 16 + half * 8 + a4, r1 = r0 + 4;    // r0 & 3 == r1 & 3 == a4
        const int cs = ((col >> 3) ^ (2 * a4)) * 8 + (col & 7);
        const s16x4 lo4 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(as + r0 * DT_BN + cs));
        const s16x4 hi4 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(as + r1 * DT_BN + cs));
        __builtin_memcpy(&av[a], &lo4, 8);
        __builtin_memcpy(reinterpret_cast<char*>(&av[a]) + 8, &hi4, 8);
      }
      const int q = s * 2 + half;                   // 16-byte chunk of the 64-row slab
#pragma unroll
      for (int t = 0; t < NW; ++t) {
        const int c = wcol + t * 32 + l32;
        bv[t] = *reinterpret_cast<const bf16x8*>(qs + c * 64 + 8 * (q ^ (c & 7)));
      }
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int t = 0; t < NW; ++t) acc[a][t] = mfma_bf16(av[a], bv[t], acc[a][t]);
    }
  };

  // the same slab schedule as the A X form: issue panel t + 2 and A
  // t + NS - 1, compute t, wait for the panel registers of t + 1 (and so A
  // t + 1), write them to LDS, barrier
  constexpr int kWaitStep = 0x0f70 | ((NS - 2) * DT_ARUN + XR);
  auto step = [&](int64_t t, u16* as, u16* qs, u16* qs_next, u16* as_refill, v4u (&xp)[XR],
                  v4u (&xn)[XR]) {
    load_q(xn, t + 2);
    issue_a(as_refill, t + NS - 1);
    __builtin_amdgcn_sched_barrier(0);
    compute(as, qs);
    __builtin_amdgcn_s_waitcnt(kWaitStep);
    store_q(qs_next, xp);
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_s_barrier();
  };

  v4u xa[XR], xb[XR];
  load_q(xa, 0);
  __builtin_amdgcn_s_waitcnt(0x0f70);
  store_q(Qs0, xa);
  load_q(xb, 1);
  issue_a(As0, 0);
  issue_a(As1, 1);
  if (NS == 4) issue_a(As2, 2);
  __builtin_amdgcn_s_waitcnt(0x0f70 | ((NS - 2) * DT_ARUN));
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_s_barrier();
  int64_t tb = 0;
  if constexpr (NS == 4) {
    for (; tb + 3 < ns; tb += 4) {
      step(tb, As0, Qs0, Qs1, As3, xb, xa);
      step(tb + 1, As1, Qs1, Qs0, As0, xa, xb);
      step(tb + 2, As2, Qs0, Qs1, As1, xb, xa);
      step(tb + 3, As3, Qs1, Qs0, As2, xa, xb);
    }
    if (tb < ns) {
      step(tb, As0, Qs0, Qs1, As3, xb, xa);
      if (tb + 1 < ns) {
        step(tb + 1, As1, Qs1, Qs0, As0, xa, xb);
        if (tb + 2 < ns) step(tb + 2, As2, Qs0, Qs1, As1, xb, xa);
      }
    }
  } else {
    for (; tb + 5 < ns; tb += 6) {
      step(tb, As0, Qs0, Qs1, As2, xb, xa);
      step(tb + 1, As1, Qs1, Qs0, As0, xa, xb);
      step(tb + 2, As2, Qs0, Qs1, As1, xb, xa);
      step(tb + 3, As0, Qs1, Qs0, As2, xa, xb);
      step(tb + 4, As1, Qs0, Qs1, As0, xb, xa);
      step(tb + 5, As2, Qs1, Qs0, As1, xa, xb);
    }
    if (tb < ns) step(tb, As0, Qs0, Qs1, As2, xb, xa);
    if (tb + 1 < ns) step(tb + 1, As1, Qs1, Qs0, As0, xa, xb);
    if (tb + 2 < ns) step(tb + 2, As2, Qs0, Qs1, As1, xb, xa);
    if (tb + 3 < ns) step(tb + 3, As0, Qs1, Qs0, As2, xa, xb);
    if (tb + 4 < ns) step(tb + 4, As1, Qs0, Qs1, As0, xb, xa);
  }
  __builtin_amdgcn_s_waitcnt(0x0f70);   // the last (dummy) loads land before LDS is freed
  // output rows [n, n rounded up to 128) are written as zeros, as by the
  // register-staged form
  const int64_t nz = (n + 127) / 128 * 128;
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int t = 0; t < NW; ++t) {
      const int64_t jb = j0 + wrow + a * 32;
      if (jb < nz) store_acc16_rows(Zp, ldz, jb, wcol + t * 32 + l32, acc[a][t], half, n);
    }
}

// A16 (m x ldo, BF16, round to nearest even) = A (m x n FP32 or FP64, lda);
// columns [n, ldo) zero.  8 elements per thread; rows that are 16-byte aligned
// take two 16-byte loads.
__device__ inline uint32_t pack_bf16(float a, float b) {
  const __bf16 x = (__bf16)a, y = (__bf16)b;
  uint16_t u0, u1;
  __builtin_memcpy(&u0, &x, 2);
  __builtin_memcpy(&u1, &y, 2);
  return (uint32_t)u0 | ((uint32_t)u1 << 16);
}

template <typename T, bool VEC>
__global__ void k_cast_to_bf16(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                               u16* __restrict__ out, int64_t ldo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per_row = ldo / 8;
  if (t >= m * per_row) return;
  const int64_t i = t / per_row, j0 = (t % per_row) * 8;
  float x[8];
  if (VEC && j0 + 8 <= n) {
    const float4 a = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(A) + i * lda + j0);
    const float4 b = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(A) + i * lda + j0 + 4);
    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = j0 + e < n ? (float)A[i * lda + j0 + e] : 0.f;
  }
  uint32_t w[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) w[e] = pack_bf16(x[2 * e], x[2 * e + 1]);
  *reinterpret_cast<uint4*>(out + i * ldo + j0) = make_uint4(w[0], w[1], w[2], w[3]);
}

// FP64 source: each value rounded once, FP64 -> BF16 (nearest even).
__global__ void k_cast_f64_to_bf16(const double* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                   u16* __restrict__ out, int64_t ldo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per_row = ldo / 8;
  if (t >= m * per_row) return;
  const int64_t i = t / per_row, j0 = (t % per_row) * 8;
  uint32_t w[4];
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const __bf16 b0 = (__bf16)(j0 + e < n ? A[i * lda + j0 + e] : 0.0);
    const __bf16 b1 = (__bf16)(j0 + e + 1 < n ? A[i * lda + j0 + e + 1] : 0.0);
    uint16_t u0, u1;
    __builtin_memcpy(&u0, &b0, 2);
    __builtin_memcpy(&u1, &b1, 2);
    w[e >> 1] = (uint32_t)u0 | ((uint32_t)u1 << 16);
  }
  *reinterpret_cast<uint4*>(out + i * ldo + j0) = make_uint4(w[0], w[1], w[2], w[3]);
}

// BF16 copy of an FP32 panel (same leading dimension), 4 elements per thread.
__global__ void k_panel_to_bf16(const float* __restrict__ P, u16* __restrict__ P16, int64_t count4) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count4) return;
  const float4 v = ld4(P + 4 * t);
  const __bf16 b[4] = {(__bf16)v.x, (__bf16)v.y, (__bf16)v.z, (__bf16)v.w};
  uint2 o;
  __builtin_memcpy(&o, b, 8);
  *reinterpret_cast<uint2*>(P16 + 4 * t) = o;
}

}  // namespace

static hipError_t launch_nn_bf16_slice(const uint16_t* A, int64_t lda, int64_t m, int64_t n, int64_t tn,
                          int64_t TJ, const uint16_t* X, int64_t ldx, int64_t lp, float* Y,
                          int64_t ldy, int64_t part_stride, hipStream_t s) {
  const int nt = (int)(lp / 32);
  // direct-to-LDS form (widths 128 and 160): 16-byte aligned rows and 31-bit
  // buffer offsets over 256 rows of A and the panel columns
  const bool dl = (nt == 4 || nt == 5) && (lda % 8) == 0 && (ldx % 8) == 0 && (tn % 8) == 0 &&
                  ((uintptr_t)A & 15) == 0 && ((uintptr_t)X & 15) == 0 &&
                  (int64_t)DL_BM * lda * 2 <= INT32_MAX && lp * ldx * 2 <= INT32_MAX;
  if (dl) {
    dim3 grid((unsigned)ceil_div_dev(m, DL_BM), (unsigned)TJ);
    if (nt == 4)
      hipLaunchKernelGGL((k_nn_bf16_dl<2, 4>), grid, dim3(512), 0, s, A, lda, m, n, tn, X, ldx, Y,
                         ldy, part_stride);
    else
      hipLaunchKernelGGL((k_nn_bf16_dl<2, 5>), grid, dim3(512), 0, s, A, lda, m, n, tn, X, ldx, Y,
                         ldy, part_stride);
    return hipGetLastError();
  }
  if (nt == 4) {   // square wave tiles, 128 rows per workgroup
    dim3 grid((unsigned)ceil_div_dev(m, 128), (unsigned)TJ);
    hipLaunchKernelGGL((k_nn_bf16_sq<1, 2>), grid, dim3(256), 0, s, A, lda, m, n, tn, X, ldx, Y,
                       ldy, part_stride);
    return hipGetLastError();
  }
  dim3 grid((unsigned)ceil_div_dev(m, 128), (unsigned)TJ);
#define NN16(NT) hipLaunchKernelGGL((k_nn_bf16<NT, 1>), grid, dim3(256), 0, s, A, lda, m, n, tn, X, ldx, Y, ldy, part_stride)
  switch (nt) {
    case 1: NN16(1); break;
    case 2: NN16(2); break;
    case 3: NN16(3); break;
    case 5: NN16(5); break;
    case 6: NN16(6); break;
    default: return hipErrorInvalidValue;
  }
#undef NN16
  return hipGetLastError();
}

hipError_t launch_nn_bf16_cast(const float* A32, int64_t lda, int64_t m, int64_t n, int64_t tn,
                               int64_t TJ, uint16_t* A16, int64_t lda16, const uint16_t* X,
                               int64_t ldx, int64_t lp, float* Y, int64_t ldy,
                               int64_t part_stride, hipStream_t s) {
  if (lp != 128 || (lda % 4) != 0 || (((uintptr_t)A32) & 15) != 0 || (lda16 % 8) != 0)
    return hipErrorInvalidValue;
  // direct-to-LDS form: 16-byte aligned copy rows and panel, 31-bit offsets
  if ((tn % 8) == 0 && (ldx % 8) == 0 && ((uintptr_t)X & 15) == 0 && ((uintptr_t)A16 & 15) == 0 &&
      (int64_t)DC_BM * lda * 4 <= INT32_MAX && (int64_t)DC_LP * ldx * 2 <= INT32_MAX &&
      (int64_t)DC_BM * lda16 * 2 <= INT32_MAX) {
    dim3 grid((unsigned)ceil_div_dev(m, DC_BM), (unsigned)TJ);
    hipLaunchKernelGGL(k_nn_bf16_dl_cast, grid, dim3(512), 0, s, A32, lda, m, n, tn, X, ldx, Y, ldy,
                       part_stride, A16, lda16);
    return hipGetLastError();
  }
  dim3 grid((unsigned)ceil_div_dev(m, 128), (unsigned)TJ);
  hipLaunchKernelGGL((k_nn_bf16_sq<1, 2, true>), grid, dim3(256), 0, s, (const u16*)nullptr, lda, m,
                     n, tn, X, ldx, Y, ldy, part_stride, A32, A16, lda16);
  return hipGetLastError();
}

static hipError_t launch_tn_bf16_slice(const uint16_t* A, int64_t lda, int64_t m, int64_t n, int64_t tm,
                          int64_t TI, const uint16_t* Q, int64_t ldq, int64_t lp, float* Z,
                          int64_t ldz, int64_t part_stride, hipStream_t s) {
  // direct-to-LDS form: whole 16-byte chunks at both ends of every row and
  // tile (n a multiple of 32, m of 8), 16-byte aligned rows, 31-bit offsets
  const bool dl = (lp == 128 || lp == 160) && (n % 32) == 0 && (m % 8) == 0 && (tm % 8) == 0 &&
                  (lda % 8) == 0 && (ldq % 8) == 0 && ((uintptr_t)A & 15) == 0 &&
                  ((uintptr_t)Q & 15) == 0 && (tm + 64) * lda * 2 <= INT32_MAX &&
                  lp * ldq * 2 <= INT32_MAX;
  if (dl) {
    dim3 grid((unsigned)ceil_div_dev(n, DT_BN), (unsigned)TI);
    if (lp == 128)
      hipLaunchKernelGGL((k_tn_bf16_dl<2, 4>), grid, dim3(512), 0, s, A, lda, m, n, tm, Q, ldq, Z,
                         ldz, part_stride);
    else
      hipLaunchKernelGGL((k_tn_bf16_dl<2, 5>), grid, dim3(512), 0, s, A, lda, m, n, tm, Q, ldq, Z,
                         ldz, part_stride);
    return hipGetLastError();
  }
  dim3 grid((unsigned)ceil_div_dev(n, TBN), (unsigned)TI);
#define TN16(NT) hipLaunchKernelGGL((k_tn_bf16<NT, true>), grid, dim3(256), 0, s, A, lda, m, n, tm, Q, ldq, Z, ldz, part_stride)
  switch (lp / 32) {
    case 1: TN16(1); break;
    case 2: TN16(2); break;
    case 3: TN16(3); break;
    case 4: TN16(4); break;
    case 5: TN16(5); break;
    case 6: TN16(6); break;
    default: return hipErrorInvalidValue;
  }
#undef TN16
  return hipGetLastError();
}

hipError_t launch_cast_to_bf16(const void* A, bool f64, int64_t lda, int64_t m, int64_t n,
                               uint16_t* out, int64_t ldo, hipStream_t s) {
  if (ldo % 8) return hipErrorInvalidValue;
  const int64_t total = m * (ldo / 8);
  dim3 grid((unsigned)ceil_div_dev(total, 256));
  if (f64) {
    hipLaunchKernelGGL(k_cast_f64_to_bf16, grid, dim3(256), 0, s, (const double*)A, lda, m, n, out,
                       ldo);
  } else if ((lda % 4) == 0 && (((uintptr_t)A) & 15) == 0) {
    hipLaunchKernelGGL((k_cast_to_bf16<float, true>), grid, dim3(256), 0, s, (const float*)A, lda,
                       m, n, out, ldo);
  } else {
    hipLaunchKernelGGL((k_cast_to_bf16<float, false>), grid, dim3(256), 0, s, (const float*)A, lda,
                       m, n, out, ldo);
  }
  return hipGetLastError();
}

hipError_t launch_panel_to_bf16(const float* P, uint16_t* P16, int64_t count, hipStream_t s) {
  const int64_t c4 = count / 4;
  hipLaunchKernelGGL(k_panel_to_bf16, dim3((unsigned)ceil_div_dev(c4, 256)), dim3(256), 0, s, P,
                     P16, c4);
  return hipGetLastError();
}

// Panels wider than kSliceMax columns are multiplied in column slices
// (plan.h, slice_width): one launch per slice, each reading A once more;
// the slices' columns are independent, so results equal a single launch.
hipError_t launch_nn_bf16(const uint16_t* A, int64_t lda, int64_t m, int64_t n, int64_t tn,
                          int64_t TJ, const uint16_t* X, int64_t ldx, int64_t lp, float* Y,
                          int64_t ldy, int64_t part_stride, hipStream_t s) {
  const int64_t cw = slice_width(lp);
  for (int64_t c0 = 0; c0 < lp; c0 += cw) {
    const hipError_t e = launch_nn_bf16_slice(A, lda, m, n, tn, TJ, X + c0 * ldx, ldx,
                                              std::min(cw, lp - c0), Y + c0 * ldy, ldy,
                                              part_stride, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_tn_bf16(const uint16_t* A, int64_t lda, int64_t m, int64_t n, int64_t tm,
                          int64_t TI, const uint16_t* Q, int64_t ldq, int64_t lp, float* Z,
                          int64_t ldz, int64_t part_stride, hipStream_t s) {
  const int64_t cw = slice_width(lp);
  for (int64_t c0 = 0; c0 < lp; c0 += cw) {
    const hipError_t e = launch_tn_bf16_slice(A, lda, m, n, tm, TI, Q + c0 * ldq, ldq,
                                              std::min(cw, lp - c0), Z + c0 * ldz, ldz,
                                              part_stride, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rsvd
