// Host-only planner: validation, block-cyclic tiles, splits, workspace layout.
#include "plan.h"

#include <algorithm>
#include <cstdio>

namespace rsvd {

rsvd_options default_options() {
  rsvd_options o{};
  o.prec_sketch = o.prec_power = o.prec_project = RSVD_F32;
  o.ortho = RSVD_ORTHO_EACH;
  o.tile_m = o.tile_n = 0;
  o.grid_p = o.grid_q = 1;
  o.hbm_budget_bytes = 0;
  o.flags = 0;
  o.a_budget_bytes = o.new_budget_bytes = 0;
  return o;
}

static rsvd_status fail(Plan& p, rsvd_status s, const char* fmt, long long a = 0, long long b = 0,
                        long long c = 0) {
  char buf[512];
  std::snprintf(buf, sizeof buf, fmt, a, b, c);
  p.last_error = buf;
  return s;
}

int64_t spmm_chunk_count(int64_t nnz) { return std::max<int64_t>(1, ceil_div(nnz, kSpmmChunk)); }

int64_t csc_part_count(int64_t m, int64_t n, int64_t lp) {
  constexpr int64_t kCscSliceBytes = int64_t(1024) << 20;
  constexpr int64_t kMaxParts = 16;
  int64_t parts = std::max<int64_t>(1, ceil_div(m * lp * 4, kCscSliceBytes));
  parts = std::min(parts, kMaxParts);
  // compressed rows b n + j are 32-bit sort keys and int32 row indices of the
  // product's chunk table
  while (parts > 1 && parts * n > (int64_t)INT32_MAX - 1) --parts;
  return parts;
}

size_t csc_sort_scratch(int64_t nnz) { return (size_t)64 * 1024 * 1024 + (size_t)nnz * 4; }

int64_t gram_chunks_for(const Plan& p, int64_t rows) {
  return std::max<int64_t>(1, ceil_div(rows, p.gram_rows));
}

// Auto tile size along a dimension of `len` so that `other_blocks` x tiles
// workgroups fill the device several times, with at most 64 tiles.
static int64_t auto_tile(int64_t len, int64_t other_blocks) {
  const int64_t want_wgs = 1024;
  int64_t tiles = std::min<int64_t>(64, std::max<int64_t>(1, ceil_div(want_wgs, other_blocks)));
  int64_t t = round_up(ceil_div(len, tiles), 256);
  return std::max<int64_t>(t, 256);
}

rsvd_status make_plan(const rsvd_problem& prob, const rsvd_options* optp, Plan& p) {
  p.prob = prob;
  p.opt = optp ? *optp : default_options();
  const rsvd_options& o = p.opt;
  const int64_t m = prob.m, n = prob.n, k = prob.k, pp = prob.p, q = prob.q;

  if (m < 1 || n < 1) return fail(p, RSVD_E_INVALID_ARG, "m=%lld and n=%lld must be >= 1", m, n);
  if (k < 1) return fail(p, RSVD_E_INVALID_ARG, "k=%lld must be >= 1", k);
  if (pp < 0) return fail(p, RSVD_E_INVALID_ARG, "p=%lld must be >= 0", pp);
  if (q < 0 || q > 64) return fail(p, RSVD_E_INVALID_ARG, "q=%lld must be in [0, 64]", q);
  if (k + pp > std::min(m, n))
    return fail(p, RSVD_E_INVALID_ARG, "k + p = %lld exceeds min(m, n) = %lld", k + pp,
                std::min(m, n));
  if (prob.format != RSVD_DENSE && prob.format != RSVD_CSR && prob.format != RSVD_COO)
    return fail(p, RSVD_E_INVALID_ARG, "unknown format %lld", prob.format);
  p.coo = prob.format == RSVD_COO;
  p.csr = prob.format == RSVD_CSR || p.coo;
  if (p.csr && (m >= 2147483647ll || n >= 2147483647ll))
    return fail(p, RSVD_E_UNSUPPORTED, "sparse input needs m, n < 2^31 - 1 (int32 CSR indices)");
  if (p.csr) {
    if (prob.nnz < 0 || prob.nnz > 2147483647ll)
      return fail(p, RSVD_E_INVALID_ARG, "nnz=%lld must be in [0, 2^31) (int32 indices)", prob.nnz);
    if (prob.dtype != RSVD_F32)
      return fail(p, RSVD_E_UNSUPPORTED, "CSR values must be FP32");
    if (prob.loc != RSVD_LOC_DEVICE)
      return fail(p, RSVD_E_UNSUPPORTED, "CSR input must be in device memory");
    if (o.prec_sketch != RSVD_F32 || o.prec_power != RSVD_F32 || o.prec_project != RSVD_F32)
      return fail(p, RSVD_E_UNSUPPORTED, "CSR products run in FP32");
    if (o.flags & RSVD_FLAG_BACKWARD)
      return fail(p, RSVD_E_UNSUPPORTED, "the adjoint needs dense A");
  }
  if (prob.dtype != RSVD_F32 && prob.dtype != RSVD_F64 && prob.dtype != RSVD_BF16) {
    if (prob.dtype == RSVD_FP8E4M3)
      return fail(p, RSVD_E_UNSUPPORTED, "A stored as dtype %lld is not implemented", prob.dtype);
    return fail(p, RSVD_E_INVALID_ARG, "unknown dtype %lld", prob.dtype);
  }
  if (prob.loc != RSVD_LOC_DEVICE && prob.loc != RSVD_LOC_HOST_PINNED)
    return fail(p, RSVD_E_INVALID_ARG, "unknown location %lld", prob.loc);
  p.host = prob.loc == RSVD_LOC_HOST_PINNED;
  for (int32_t pr : {o.prec_sketch, o.prec_power, o.prec_project}) {
    if (pr != RSVD_F32 && pr != RSVD_BF16 && pr != RSVD_FP8E4M3)
      return fail(p, RSVD_E_INVALID_ARG, "unknown product precision %lld", pr);
  }
  p.any_bf16 = o.prec_sketch == RSVD_BF16 || o.prec_project == RSVD_BF16 ||
               (o.prec_power == RSVD_BF16 && prob.q > 0);
  p.any_f32 = o.prec_sketch == RSVD_F32 || o.prec_project == RSVD_F32 ||
              (o.prec_power == RSVD_F32 && prob.q > 0);
  p.any_fp8 = o.prec_sketch == RSVD_FP8E4M3 || o.prec_project == RSVD_FP8E4M3 ||
              (o.prec_power == RSVD_FP8E4M3 && prob.q > 0);
  if (prob.dtype == RSVD_BF16 && (p.any_f32 || p.any_fp8))
    return fail(p, RSVD_E_UNSUPPORTED, "A stored in BF16 needs BF16 products throughout");
  if (p.host) {
    // streamed tiles are multiplied in their storage precision
    const int32_t want = prob.dtype == RSVD_BF16 ? RSVD_BF16 : RSVD_F32;
    if (prob.dtype == RSVD_F64)
      return fail(p, RSVD_E_UNSUPPORTED, "host-resident A must be FP32 or BF16");
    for (int32_t pr : {o.prec_sketch, o.prec_power, o.prec_project})
      if (pr != want)
        return fail(p, RSVD_E_UNSUPPORTED,
                    want == RSVD_BF16
                        ? "host-resident A is multiplied in its storage precision (BF16 products)"
                        : "host-resident A is multiplied in its storage precision (FP32 products)");
    if (o.flags & RSVD_FLAG_BACKWARD)
      return fail(p, RSVD_E_UNSUPPORTED, "the adjoint needs A in device memory");
  }
  if (o.ortho != RSVD_ORTHO_EACH && o.ortho != RSVD_ORTHO_FINAL_ONLY)
    return fail(p, RSVD_E_INVALID_ARG, "unknown ortho schedule %lld", o.ortho);
  if (o.ortho == RSVD_ORTHO_FINAL_ONLY)
    return fail(p, RSVD_E_UNSUPPORTED, "ortho FINAL_ONLY is not implemented");
  if (o.grid_p < 1 || o.grid_q < 1)
    return fail(p, RSVD_E_INVALID_ARG, "process grid %lld x %lld must be >= 1", o.grid_p, o.grid_q);
  if (o.tile_m < 0 || o.tile_n < 0 || o.tile_m % 32 || o.tile_n % 32)
    return fail(p, RSVD_E_INVALID_ARG, "tile sizes %lld x %lld must be >= 0 and multiples of 32",
                o.tile_m, o.tile_n);
  if (o.flags & ~(RSVD_FLAG_NO_SIGN_FIX | RSVD_FLAG_CHOLQR1 | RSVD_FLAG_BACKWARD | RSVD_FLAG_AUTO_Q |
                  RSVD_FLAG_JACOBI_ONLY))
    return fail(p, RSVD_E_INVALID_ARG, "unknown flags 0x%llx", o.flags);
  p.auto_q = (o.flags & RSVD_FLAG_AUTO_Q) != 0;
  if (p.auto_q) {
    if (!(o.q_tol >= 0.0) || o.q_tol >= 1.0)
      return fail(p, RSVD_E_INVALID_ARG, "q_tol must be in [0, 1)");
    if (o.prec_power != o.prec_project)
      return fail(p, RSVD_E_INVALID_ARG, "automatic q needs the same precision for the power steps "
                                          "and the projection");
    if (o.flags & RSVD_FLAG_BACKWARD)
      return fail(p, RSVD_E_UNSUPPORTED, "automatic q with the adjoint is not implemented");
    p.q_tol = o.q_tol > 0.0 ? o.q_tol : 1e-4;
  }

  p.l = k + pp;
  p.lp = round_up(p.l, kColAlign);
  if (p.lp > kWideMax)
    return fail(p, RSVD_E_UNSUPPORTED, "k + p = %lld: sketch widths above %lld are not implemented",
                p.l, kWideMax);
  p.ldm = round_up(m, kPanelAlign);
  p.ldn = round_up(n, kPanelAlign);

  // block-cyclic tiles over A; one tile spans the whole dimension at most
  p.tm = o.tile_m ? std::min<int64_t>(o.tile_m, round_up(m, 32)) : auto_tile(m, ceil_div(n, 128));
  p.tn = o.tile_n ? std::min<int64_t>(o.tile_n, round_up(n, 32)) : auto_tile(n, ceil_div(m, 128));
  if (p.host) {   // streamed tiles start on product-kernel row/column block boundaries
    p.tm = round_up(p.tm, 256);
    p.tn = round_up(p.tn, 256);
  }
  if (p.any_fp8) {   // FP8 scale blocks are 64 x 64: tiles must not split one
    if ((o.tile_m && o.tile_m % 64) || (o.tile_n && o.tile_n % 64))
      return fail(p, RSVD_E_INVALID_ARG, "FP8 products need tile sizes that are multiples of 64");
    p.tm = round_up(p.tm, 64);
    p.tn = round_up(p.tn, 64);
  }
  p.TI = ceil_div(m, p.tm);
  p.TJ = ceil_div(n, p.tn);

  // Gram chunking: enough chunks that the Gram kernels fill the device
  {
    const int64_t pairs = gram_pairs(p);
    const int64_t want = 256;
    const int64_t rows = std::max(m, n);
    int64_t chunks = std::max<int64_t>(1, ceil_div(want, pairs));
    p.gram_rows = std::max<int64_t>(256, round_up(ceil_div(rows, chunks), 64));
    p.gram_chunks = gram_chunks_for(p, rows);
  }
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += (size_t)round_up((int64_t)bytes, 256);
    return at;
  };
  const size_t lp = (size_t)p.lp;
  Workspace& w = p.ws;
  w.Xop = take((size_t)p.ldn * lp * 4);
  w.Mop = take((size_t)p.ldm * lp * 4);
  w.M0 = take((size_t)p.ldm * lp * 4);
  w.M1 = take((size_t)p.ldm * lp * 4);
  w.N0 = take((size_t)p.ldn * lp * 4);
  w.N1 = take((size_t)p.ldn * lp * 4);
  {
    size_t a = p.TJ > 1 ? (size_t)p.TJ * p.ldm * lp * 4 : 0;
    size_t b = p.TI > 1 ? (size_t)p.TI * p.ldn * lp * 4 : 0;
    w.part = take(std::max<size_t>(std::max(a, b), 256));
  }
  p.backward = (o.flags & RSVD_FLAG_BACKWARD) != 0;
  p.kp = round_up(k, kColAlign);
  p.rcat = p.lp + 2 * p.kp;
  {
    // Gram partial blocks: lower pairs of lp x lp, or lp x kp cross blocks
    const int64_t cross = ceil_div(p.lp, kGramBlock) * ceil_div(p.kp, kGramBlock);
    const int64_t blocks = std::max<int64_t>(gram_pairs(p), p.backward ? cross : 0);
    // also holds the 2048 partial sums of the accuracy pass
    size_t gbytes = std::max<size_t>((size_t)p.gram_chunks * blocks * kGramBlock * kGramBlock * 8,
                                     2048 * 8);
    if (gram_tri_fits(p.lp) || gram_grp_fits(p.lp)) gbytes = std::max(gbytes, gram_tri_bytes(p.lp));
    w.gpart = take(gbytes);
    w.gpart2 = take(gbytes);
  }
  w.G2 = take(lp * lp * 8);
  w.Tc = take(lp * lp * 8);
  w.Wpm = take(lp * lp * 4);
  w.Wpn = take(lp * lp * 4);
  w.Wc = take(lp * lp * 4);
  w.G = take(lp * lp * 8);
  // above 128 also the scratch of the global-memory Cholesky (the square plus
  // its side area)
  w.L = take((size_t)(p.lp > 128 ? chol_gm_scratch_doubles(p.lp) : p.lp * p.lp) * 8);
  w.W = take(lp * lp * 4);
  w.W2 = take(lp * lp * 4);
  w.Ev = take(lp * lp * 8);
  w.tri = small_svd_tridiagonal(p) ? take((size_t)kTriScratchDoubles * 8) : off;
  const bool bj = p.lp > 128, wide = p.lp > kSliceMax;   // block Jacobi; Cholesky in global memory
  w.Mj = bj ? take(lp * lp * 8) : off;
  w.bjctl = bj ? take((size_t)kBjMaxSweeps * 4) : off;
  w.Ls2 = wide ? take((size_t)chol_gm_scratch_doubles(p.lp) * 8) : off;
  w.lam = take(lp * 8);
  w.order = take(lp * 4);
  w.signs = take(lp * 4);
  w.status = take(kStatusWords * 4);
  w.prevS = take((size_t)k * 8 + 8);
  p.ldac = round_up(n, 64);
  p.lda16 = round_up(n, 64);
  w.Acast = (prob.dtype == RSVD_F64 && p.any_f32) ? take((size_t)m * p.ldac * 4) : off;
  w.A16 = (p.any_bf16 && prob.dtype != RSVD_BF16) ? take((size_t)m * p.lda16 * 2) : off;
  w.Xop16 = p.any_bf16 ? take((size_t)p.ldn * lp * 2) : off;
  w.Mop16 = p.any_bf16 ? take((size_t)p.ldm * lp * 2) : off;
  p.lda8 = round_up(n, 64);
  p.ldat8 = round_up(m, 64);
  w.A8 = p.any_fp8 ? take((size_t)m * p.lda8) : off;
  w.A8T = p.any_fp8 ? take((size_t)n * p.ldat8) : off;
  w.sA8 = p.any_fp8 ? take((size_t)ceil_div(m, 64) * ceil_div(n, 64) * 4) : off;
  w.Xop8 = p.any_fp8 ? take((size_t)p.ldn * lp) : off;
  w.Mop8 = p.any_fp8 ? take((size_t)p.ldm * lp) : off;
  w.sX8 = p.any_fp8 ? take(lp * 4) : off;
  w.sM8 = p.any_fp8 ? take(lp * 4) : off;
  w.f8part = p.any_fp8 ? take((size_t)2 * lp * kPanelFp8Chunks * 4) : off;
  if (p.backward) {
    const size_t kp = (size_t)p.kp, rc = (size_t)p.rcat;
    w.Pcat = take((size_t)p.ldm * rc * 4);
    w.Rcat = take((size_t)p.ldn * rc * 4);
    w.gUp = take((size_t)p.ldm * kp * 4);
    w.gVp = take((size_t)p.ldn * kp * 4);
    w.Ju = take(lp * kp * 8);
    w.Jv = take(lp * kp * 8);
    w.Sl = take(lp * 8);
    w.coreT = take(lp * lp * 4);
    w.JuW = take(lp * kp * 4);
    w.JvW = take(lp * kp * 4);
    w.sinv = take(kp * 4);
  } else {
    w.Pcat = w.Rcat = w.gUp = w.gVp = w.Ju = w.Jv = w.Sl = w.coreT = w.JuW = w.JvW = w.sinv = off;
  }
  if (p.csr) {
    p.chunks = spmm_chunk_count(prob.nnz);
    p.csc_parts = csc_part_count(m, n, p.lp);
    p.head_k = std::min<int64_t>(kHeadCols, n);
    p.head_parts = ceil_div(m, kHeadPartRows);
    // compressed rows of the CSC copy: b n + j for the other columns, then
    // P n + b' K + h for the head columns (32-bit sort keys, int32 rows); a
    // matrix too tall for the head blocks goes without them
    if (p.head_k < 1 || p.head_parts < 1 ||
        p.csc_parts * n + p.head_parts * p.head_k > (int64_t)INT32_MAX - 1)
      p.head_k = p.head_parts = 0;
    if (p.csc_parts * n > (int64_t)INT32_MAX - 1)
      return fail(p, RSVD_E_UNSUPPORTED, "sparse A with %lld columns is too wide for 32-bit keys",
                  (long long)n);
    const int64_t nv = p.csc_parts * n + p.head_parts * p.head_k;
    const size_t nnz = (size_t)prob.nnz;
    // Xr: the row-major operand (n rows for A X, m for A^T Q); Yr: the
    // compressed rows of the result (m, or the CSC copy's compressed rows)
    const size_t xrows = (size_t)std::max<int64_t>(m, n);
    const size_t yrows = (size_t)std::max<int64_t>(m, nv);
    w.colptr = take((size_t)(nv + 1) * 4);
    w.colcnt = take((size_t)n * 4);
    w.headof = take((size_t)n * 4);
    w.headcol = take((size_t)p.head_k * 4);
    w.rk0 = take((size_t)n * 4);
    w.rk1 = take((size_t)n * 4);
    w.rv0 = take((size_t)n * 4);
    w.rv1 = take((size_t)n * 4);
    w.rowind = take(nnz * 4);
    w.cval = take(nnz * 4);
    w.keys0 = take(nnz * 4);
    w.keys1 = take(nnz * 4);
    w.pay0 = take(nnz * 8);
    w.pay1 = take(nnz * 8);
    p.sort_temp = csc_sort_scratch(prob.nnz);
    w.sort_temp = take(p.sort_temp);
    w.Xr = take(xrows * lp * 4);
    w.Yr = take(yrows * lp * 4);
    w.carry = take((size_t)p.chunks * lp * 4);
    w.first = take((size_t)p.chunks * 4);
  } else {
    w.colptr = w.rowind = w.cval = w.keys0 = w.keys1 = w.pay0 = w.pay1 = w.sort_temp = off;
    w.colcnt = w.headof = w.headcol = w.rk0 = w.rk1 = w.rv0 = w.rv1 = off;
    w.Xr = w.Yr = w.carry = w.first = off;
  }
  if (p.coo) {
    w.coo_ptr = take((size_t)(m + 1) * 4);
    w.coo_col = take((size_t)prob.nnz * 4);
    w.coo_val = take((size_t)prob.nnz * 4);
  } else {
    w.coo_ptr = w.coo_col = w.coo_val = off;
  }
  // Section 3.5's limits: per matrix (the tiles of A), new matrices (all of
  // the above), global; an unset one takes the next one's value
  const uint64_t lim_new = o.new_budget_bytes ? o.new_budget_bytes : o.hbm_budget_bytes;
  const uint64_t lim_a = o.a_budget_bytes ? o.a_budget_bytes : lim_new;
  const size_t own = off;
  if (lim_new && own > lim_new)
    return fail(p, RSVD_E_BUDGET, "the plan's own matrices need %lld bytes, the limit is %lld",
                (long long)own, (long long)lim_new);
  if (!p.host && o.a_budget_bytes) {
    const int64_t a_bytes = p.csr ? prob.nnz * 8 + (m + 1) * 4
                                  : m * n * (prob.dtype == RSVD_F64 ? 8 : prob.dtype == RSVD_BF16 ? 2 : 4);
    if ((uint64_t)a_bytes > o.a_budget_bytes)
      return fail(p, RSVD_E_BUDGET,
                  "device-resident A holds %lld bytes, above its limit of %lld (plan it "
                  "host-resident to stream it)",
                  (long long)a_bytes, (long long)o.a_budget_bytes);
  }
  if (p.host) {
    // tile slots: as many as the limit on A allows (at least two, so copies
    // and products overlap), at most one per tile; four when there is no limit
    p.elem = prob.dtype == RSVD_BF16 ? 2 : 4;
    p.slot_ld = round_up(p.tn, 64);
    p.slot_bytes = (size_t)round_up((int64_t)p.tm * p.slot_ld * p.elem, 256);
    const int64_t tiles = p.TI * p.TJ;
    int64_t S = std::min<int64_t>(tiles, 4);
    if (lim_a) {
      // with only the global limit set, the slots share it with the rest
      const bool own_limit = o.a_budget_bytes || o.new_budget_bytes;
      const uint64_t avail = own_limit ? lim_a : (lim_a > own ? lim_a - own : 0);
      if (avail < 2 * p.slot_bytes)
        return fail(p, RSVD_E_BUDGET,
                    "host-resident A needs two %lld-byte tile slots (%lld bytes); its limit leaves "
                    "%lld",
                    (long long)p.slot_bytes, (long long)(2 * p.slot_bytes), (long long)avail);
      S = std::min<int64_t>(tiles, (int64_t)(avail / p.slot_bytes));
    }
    p.slots = std::max<int64_t>(S, std::min<int64_t>(tiles, 2));
    w.slots = take((size_t)p.slots * p.slot_bytes);
  } else {
    w.slots = off;
  }
  w.total = off;

  if (o.hbm_budget_bytes && w.total > o.hbm_budget_bytes)
    return fail(p, RSVD_E_BUDGET, "workspace needs %lld bytes, budget is %lld", (long long)w.total,
                (long long)o.hbm_budget_bytes);
  p.last_error.clear();
  return RSVD_OK;
}

}  // namespace rsvd
