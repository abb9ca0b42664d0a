// C ABI and pass schedule of the randomized SVD on one MI355X.
//
// Schedule (Section 2.1 steps 1-7 on the power matrix of Section 2.2):
//   O (n x l) Gaussian                         step 1
//   Y = A O, Q = orth(Y)                        steps 2-4
//   q times: Z = A^T Q, Z = orth(Z),            Eq. (2), right to left,
//            Y = A Z,   Q = orth(Y)             re-orthonormalised
//   B^T = A^T Q                                 step 5 (computed transposed)
//   C = B B^T (FP64), C = E diag(lambda) E^T    step 6 (Jacobi)
//   U = Q E_k, S = sqrt(lambda_k), V = B^T E_k S^-1,  sign convention  step 7
// orth() is CholeskyQR2 with an FP64 Gram and Cholesky.  Everything is
// enqueued on one stream; the host waits only when a report is requested.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "plan.h"

struct rsvd_plan_s {
  rsvd::Plan p;
};

namespace {

thread_local std::string g_last_error;

constexpr double kCholTau = 1e-10;    // pivot / original diagonal below which a direction drops
constexpr double kJacobiTol = 1e-14;  // relative off-diagonal size that ends a rotation
constexpr int kNumEvents = 9;

// Stage events plus one start/stop pair per product-kernel launch.
struct Events {
  hipEvent_t ev[kNumEvents];
  std::vector<hipEvent_t> kern;   // 2 per product launch
  bool made = false;
};

hipError_t make_events(Events& e, size_t kernel_pairs) {
  if (!e.made) {
    for (int i = 0; i < kNumEvents; ++i) {
      hipError_t err = hipEventCreate(&e.ev[i]);
      if (err != hipSuccess) {
        for (int j = 0; j < i; ++j) (void)hipEventDestroy(e.ev[j]);
        return err;
      }
    }
    e.made = true;
  }
  while (e.kern.size() < 2 * kernel_pairs) {
    hipEvent_t x;
    hipError_t err = hipEventCreate(&x);
    if (err != hipSuccess) return err;
    e.kern.push_back(x);
  }
  return hipSuccess;
}

void destroy_events(Events* e) {
  if (!e) return;
  if (e->made)
    for (int i = 0; i < kNumEvents; ++i) (void)hipEventDestroy(e->ev[i]);
  for (hipEvent_t x : e->kern) (void)hipEventDestroy(x);
  delete e;
}

// Host-resident A (Section 3.5, out of core): a copy stream moves tiles from
// pinned host memory into S HBM slots while the compute stream multiplies the
// tiles already there.  Slot j is reused only after the product that read it
// has finished (event free[j]); a product waits for its tile (event ready[j]).
// Every pass visits every tile, so a least-recently-used cache smaller than A
// would thrash; instead, with S slots and T > S tiles, tiles 0 .. S-3 own a
// slot each and stay resident across the passes of a call (loaded once),
// and the other tiles stream through the last two slots (double buffering;
// a pass that starts where the previous one ended, serpentine order, still
// finds that tile in its streaming slot).  Loads per call:
// T + (passes - 1) (T - S + 2) - (passes - 1).
struct Streamer {
  hipStream_t copy = nullptr;
  bool own_copy = false;          // created here (else the caller's)
  std::vector<hipEvent_t> ready, freed;
  std::vector<int64_t> tile;       // tile held by each slot (-1: none)
  std::vector<int64_t> last_use;
  int64_t clock = 0;
  double h2d_bytes = 0.0;
  int64_t loads = 0;
};

void destroy_streamer(Streamer* st) {
  if (!st) return;
  for (hipEvent_t e : st->ready) (void)hipEventDestroy(e);
  for (hipEvent_t e : st->freed) (void)hipEventDestroy(e);
  if (st->copy && st->own_copy) (void)hipStreamDestroy(st->copy);
  delete st;
}

hipError_t make_streamer(rsvd::Plan& P, Streamer*& out) {
  out = static_cast<Streamer*>(P.streamer);
  if (out) return hipSuccess;
  Streamer* st = new (std::nothrow) Streamer;
  if (!st) return hipErrorOutOfMemory;
  hipError_t e = hipSuccess;
  if (P.user_copy) {
    st->copy = static_cast<hipStream_t>(P.user_copy);
  } else {
    e = hipStreamCreateWithFlags(&st->copy, hipStreamNonBlocking);
    st->own_copy = e == hipSuccess;
  }
  for (int64_t j = 0; e == hipSuccess && j < P.slots; ++j) {
    hipEvent_t a, b;
    e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
    if (e != hipSuccess) break;
    st->ready.push_back(a);
    e = hipEventCreateWithFlags(&b, hipEventDisableTiming);
    if (e != hipSuccess) break;
    st->freed.push_back(b);
  }
  if (e != hipSuccess) {
    destroy_streamer(st);
    return e;
  }
  st->tile.assign((size_t)P.slots, -1);
  st->last_use.assign((size_t)P.slots, 0);
  P.streamer = st;
  out = st;
  return hipSuccess;
}

rsvd_status set_err(rsvd_plan_t h, rsvd_status s, const std::string& msg) {
  if (h)
    h->p.last_error = msg;
  else
    g_last_error = msg;
  return s;
}

rsvd_status hip_err(rsvd_plan_t h, hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  return set_err(h, RSVD_E_HIP, msg);
}

#define RSVD_HIP(call)                                   \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_err(h, e_, #call);  \
  } while (0)

struct Buffers {
  float *Xop, *Mop, *M0, *M1, *N0, *N1, *part, *W, *W2, *Acast;
  uint16_t *A16, *Xop16, *Mop16;
  uint8_t *A8, *A8T, *Xop8, *Mop8;
  float *sA8, *sX8, *sM8, *f8part;
  char* slots;
  int32_t *colptr, *rowind, *first, *headof, *headcol, *rv0, *rv1;
  uint32_t *colcnt, *rk0, *rk1;
  float *cval, *Xr, *Yr, *carry;
  uint32_t *keys0, *keys1;
  uint64_t *pay0, *pay1;
  void* sort_temp;
  int32_t *coo_ptr, *coo_col;
  float* coo_val;
  float *Pcat, *Rcat, *gUp, *gVp, *coreT, *JuW, *JvW, *sinv;
  double *Ju, *Jv, *Sl;
  double *gpart, *G, *L, *Ev, *lam, *Mj, *Ls2;
  double* tri;   // tridiagonal eigensolver scratch, or null (Jacobi only)
  int32_t* bjctl;
  double *gpart2, *G2, *Tc;
  float *Wpm, *Wpn, *Wc;
  int32_t *order, *signs, *status;
  double* prevS;
};

Buffers carve(const rsvd::Plan& P, void* ws) {
  char* b = static_cast<char*>(ws);
  const rsvd::Workspace& w = P.ws;
  Buffers B;
  B.Xop = (float*)(b + w.Xop);
  B.Mop = (float*)(b + w.Mop);
  B.M0 = (float*)(b + w.M0);
  B.M1 = (float*)(b + w.M1);
  B.N0 = (float*)(b + w.N0);
  B.N1 = (float*)(b + w.N1);
  B.part = (float*)(b + w.part);
  B.W = (float*)(b + w.W);
  B.W2 = (float*)(b + w.W2);
  B.Acast = (float*)(b + w.Acast);
  B.A16 = (uint16_t*)(b + w.A16);
  B.Xop16 = (uint16_t*)(b + w.Xop16);
  B.Mop16 = (uint16_t*)(b + w.Mop16);
  B.A8 = (uint8_t*)(b + w.A8);
  B.A8T = (uint8_t*)(b + w.A8T);
  B.Xop8 = (uint8_t*)(b + w.Xop8);
  B.Mop8 = (uint8_t*)(b + w.Mop8);
  B.sA8 = (float*)(b + w.sA8);
  B.sX8 = (float*)(b + w.sX8);
  B.sM8 = (float*)(b + w.sM8);
  B.f8part = (float*)(b + w.f8part);
  B.slots = b + w.slots;
  B.colptr = (int32_t*)(b + w.colptr);
  B.headof = (int32_t*)(b + w.headof);
  B.headcol = (int32_t*)(b + w.headcol);
  B.rv0 = (int32_t*)(b + w.rv0);
  B.rv1 = (int32_t*)(b + w.rv1);
  B.colcnt = (uint32_t*)(b + w.colcnt);
  B.rk0 = (uint32_t*)(b + w.rk0);
  B.rk1 = (uint32_t*)(b + w.rk1);
  B.rowind = (int32_t*)(b + w.rowind);
  B.first = (int32_t*)(b + w.first);
  B.cval = (float*)(b + w.cval);
  B.Xr = (float*)(b + w.Xr);
  B.Yr = (float*)(b + w.Yr);
  B.carry = (float*)(b + w.carry);
  B.keys0 = (uint32_t*)(b + w.keys0);
  B.keys1 = (uint32_t*)(b + w.keys1);
  B.pay0 = (uint64_t*)(b + w.pay0);
  B.pay1 = (uint64_t*)(b + w.pay1);
  B.sort_temp = b + w.sort_temp;
  B.coo_ptr = (int32_t*)(b + w.coo_ptr);
  B.coo_col = (int32_t*)(b + w.coo_col);
  B.coo_val = (float*)(b + w.coo_val);
  B.Pcat = (float*)(b + w.Pcat);
  B.Rcat = (float*)(b + w.Rcat);
  B.gUp = (float*)(b + w.gUp);
  B.gVp = (float*)(b + w.gVp);
  B.coreT = (float*)(b + w.coreT);
  B.JuW = (float*)(b + w.JuW);
  B.JvW = (float*)(b + w.JvW);
  B.sinv = (float*)(b + w.sinv);
  B.Ju = (double*)(b + w.Ju);
  B.Jv = (double*)(b + w.Jv);
  B.Sl = (double*)(b + w.Sl);
  B.gpart = (double*)(b + w.gpart);
  B.G = (double*)(b + w.G);
  B.gpart2 = (double*)(b + w.gpart2);
  B.G2 = (double*)(b + w.G2);
  B.Tc = (double*)(b + w.Tc);
  B.Wpm = (float*)(b + w.Wpm);
  B.Wpn = (float*)(b + w.Wpn);
  B.Wc = (float*)(b + w.Wc);
  B.L = (double*)(b + w.L);
  B.Ev = (double*)(b + w.Ev);
  B.Mj = (double*)(b + w.Mj);
  B.tri = rsvd::small_svd_tridiagonal(P) ? (double*)(b + w.tri) : nullptr;
  B.Ls2 = (double*)(b + w.Ls2);
  B.bjctl = (int32_t*)(b + w.bjctl);
  B.lam = (double*)(b + w.lam);
  B.order = (int32_t*)(b + w.order);
  B.signs = (int32_t*)(b + w.signs);
  B.status = (int32_t*)(b + w.status);
  B.prevS = (double*)(b + w.prevS);
  return B;
}

// Side stream of the deferred second CholeskyQR passes (default priority,
// non-blocking), with the fork and join events; owned by the plan.
struct Side {
  hipStream_t s = nullptr;
  bool own = false;               // created here (else the caller's)
  hipEvent_t fork = nullptr, join = nullptr;
};

void destroy_side(Side* d) {
  if (!d) return;
  if (d->fork) (void)hipEventDestroy(d->fork);
  if (d->join) (void)hipEventDestroy(d->join);
  if (d->s && d->own) (void)hipStreamDestroy(d->s);
  delete d;
}

hipError_t make_side(rsvd::Plan& P, Side*& out) {
  out = static_cast<Side*>(P.side);
  if (out) return hipSuccess;
  Side* d = new (std::nothrow) Side;
  if (!d) return hipErrorOutOfMemory;
  hipError_t e = hipSuccess;
  if (P.user_side) {
    d->s = static_cast<hipStream_t>(P.user_side);
  } else {
    e = hipStreamCreateWithFlags(&d->s, hipStreamNonBlocking);
    d->own = e == hipSuccess;
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&d->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&d->join, hipEventDisableTiming);
  if (e != hipSuccess) {
    destroy_side(d);
    return e;
  }
  P.side = d;
  out = d;
  return hipSuccess;
}

// ---- checkpoint layout (rsvd_factor_resumable) ---------------------------
// side of the state after pass t of npass: 0 the m-side basis, 1 the n-side
// panel, 2 (after the projection) the basis over B^T.
int ckpt_side(int64_t t, int64_t npass) { return t == npass ? 2 : (t % 2 == 1 ? 0 : 1); }

// Panel rows: the state panel(s), then lp rows holding the pending right
// factor of the basis (row-major lp x lp factor, column c below column c).
int64_t ckpt_rows(const rsvd::Plan& P, int side) {
  return (side == 0 ? P.prob.m : side == 1 ? P.prob.n : P.prob.m + P.prob.n) + P.lp;
}

// 64-bit FNV-1a over 32-bit words (each word is one unit of the hash).
uint64_t ckpt_hash(const float* p, size_t words) {
  const uint32_t* w = reinterpret_cast<const uint32_t*>(p);
  uint64_t h = 0xcbf29ce484222325ull;
  for (size_t i = 0; i < words; ++i) {
    h ^= w[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

// The runner holds everything one call needs.
struct Runner {
  rsvd_plan_t h;
  const rsvd::Plan& P;
  Buffers B;
  hipStream_t s;
  const float* A32 = nullptr;
  int64_t lda32 = 0;
  const uint16_t* A16 = nullptr;
  int64_t lda16 = 0;
  Events* ev = nullptr;        // non-null: time every product kernel
  std::vector<int> nn_idx, tn_idx;
  int next_pair = 0;
  const int32_t* rowptr = nullptr;   // CSR input
  const int32_t* colind = nullptr;
  const float* values = nullptr;
  const float* cast_src = nullptr;   // FP32 A whose BF16 copy the sketch pass will write
  int64_t cast_lda = 0;
  const char* Ahost = nullptr; // host-resident A (pinned), streamed tile by tile
  int64_t ldh = 0;
  Streamer* st8 = nullptr;
  int64_t pass_no = 0;         // passes over A so far in this call
  int64_t q_used = 0;          // power steps run
  double q_delta = 0.0;        // automatic q: last relative change
  // per-pass persistence (rsvd_factor_resumable); null for the plain calls
  struct Ckpt {
    const rsvd_checkpoint* resume;
    const float* resume_panel;
    int32_t stop_after;
    rsvd_checkpoint* out;
    float* out_panel;
  };
  const Ckpt* ck = nullptr;
  // Deferred second CholeskyQR pass: a basis Q1 = Y W1 is handed to the next
  // product at once, while Q1's own Gram and Cholesky run on the side stream
  // and give its pending right factor W2 (Q = Q1 W2).  Every consumer folds
  // W2 in on its lp x lp side (the next Gram is W2^T G W2, the next right
  // factor W2 W1, the final small factors W2 U_B), so W2 never touches a
  // tall panel.  pend[0] / pend[1]: the m- / n-side basis has one.
  Side* side = nullptr;
  bool allow_defer = true;     // false: both passes on the caller's stream (no side stream)
  bool pend[2] = {false, false};
  bool side_busy = false;
  double* gsmall = nullptr;    // the l x l Gram the small SVD factors (B.G, or its congruence)
  float* Wpend(int sd) const { return sd ? B.Wpn : B.Wpm; }

  hipError_t tick(bool nn, bool start) {
    if (!ev) return hipSuccess;
    if (start) {
      (nn ? nn_idx : tn_idx).push_back(next_pair);
      return hipEventRecord(ev->kern[2 * next_pair], s);
    }
    return hipEventRecord(ev->kern[2 * (next_pair++) + 1], s);
  }

  Runner(rsvd_plan_t hh, void* ws, hipStream_t ss) : h(hh), P(hh->p), B(carve(hh->p, ws)), s(ss) {}

  // Operand copies of A the products need: FP32 (FP64 input is rounded once)
  // and/or BF16 (rounded to nearest even once per call).
  bool fuse_cast = true;       // allow the sketch pass to produce the BF16 copy
  int coo_bits = 0;            // index width of the caller's COO arrays

  // The BF16 copy if it is still owed (a BF16 product other than the sketch
  // comes first).
  rsvd_status settle_cast() {
    if (!cast_src) return RSVD_OK;
    RSVD_HIP(rsvd::launch_cast_to_bf16(cast_src, false, cast_lda, P.prob.m, P.prob.n, B.A16,
                                       P.lda16, s));
    cast_src = nullptr;
    return RSVD_OK;
  }

  rsvd_status bind_A(const void* A, int64_t lda) {
    const int32_t dt = P.prob.dtype;
    if (P.host) {
      Ahost = static_cast<const char*>(A);
      ldh = lda;
      RSVD_HIP(make_streamer(h->p, st8));
      std::fill(st8->tile.begin(), st8->tile.end(), -1);   // A may have changed since the last call
      st8->h2d_bytes = 0.0;
      st8->loads = 0;
      return RSVD_OK;
    }
    if (P.any_f32) {
      if (dt == RSVD_F64) {
        RSVD_HIP(rsvd::launch_cast_f64_f32((const double*)A, lda, P.prob.m, P.prob.n, B.Acast,
                                           P.ldac, s));
        A32 = B.Acast;
        lda32 = P.ldac;
      } else {
        A32 = (const float*)A;
        lda32 = lda;
      }
    }
    if (P.any_bf16) {
      if (dt == RSVD_BF16) {
        A16 = (const uint16_t*)A;
        lda16 = lda;
      } else if (dt == RSVD_F32 && fuse_cast && P.opt.prec_sketch == RSVD_BF16 && P.lp == 128 &&
                 lda % 4 == 0 && (((uintptr_t)A) & 15) == 0) {
        // the BF16 sketch product writes the copy while it reads A (one read)
        cast_src = (const float*)A;
        cast_lda = lda;
        A16 = B.A16;
        lda16 = P.lda16;
      } else {
        RSVD_HIP(rsvd::launch_cast_to_bf16(A, dt == RSVD_F64, lda, P.prob.m, P.prob.n, B.A16,
                                           P.lda16, s));
        A16 = B.A16;
        lda16 = P.lda16;
      }
    }
    if (P.any_fp8)
      RSVD_HIP(rsvd::launch_cast_fp8(A, dt == RSVD_F64, lda, P.prob.m, P.prob.n, B.A8, P.lda8,
                                     B.A8T, P.ldat8, B.sA8, s));
    return RSVD_OK;
  }

  // Sparse A: check the arrays (flag on the device) and build the CSC copy
  // that applies A^T (stable sort of the nonzeros by column).
  rsvd_status bind_csr(const int32_t* rp, const int32_t* ci, const float* v) {
    rowptr = rp;
    colind = ci;
    values = v;
    const int64_t m = P.prob.m, n = P.prob.n, nnz = P.prob.nnz;
    RSVD_HIP(rsvd::launch_csr_check(rp, ci, m, n, nnz, B.status, s));
    size_t need = 0;
    if (P.head_k > 0) {
      const hipError_t eh = rsvd::launch_head_select(rp, ci, m, n, nnz, P.head_k, B.colcnt,
                                                     B.headof, B.headcol, B.rk0, B.rk1, B.rv0,
                                                     B.rv1, B.sort_temp, P.sort_temp, &need, s);
      if (eh == hipErrorOutOfMemory && need > P.sort_temp)
        return set_err(h, RSVD_E_BUDGET,
                       "the column ranking needs " + std::to_string(need) + " bytes of scratch, "
                       "the plan reserved " + std::to_string(P.sort_temp));
      RSVD_HIP(eh);
    }
    const hipError_t e = rsvd::launch_build_csc(rp, ci, v, m, n, nnz, P.csc_parts,
                                                P.head_k > 0 ? B.headof : nullptr, P.head_k,
                                                P.head_parts, B.keys0, B.keys1, B.pay0, B.pay1,
                                                B.sort_temp, P.sort_temp, B.colptr, B.rowind,
                                                B.cval, &need, s);
    if (e == hipErrorOutOfMemory && need > P.sort_temp)
      return set_err(h, RSVD_E_BUDGET,
                     "the CSC sort needs " + std::to_string(need) + " bytes of scratch, the plan "
                     "reserved " + std::to_string(P.sort_temp));
    RSVD_HIP(e);
    return RSVD_OK;
  }

  // COO input: order the entries by row into CSR arrays in the workspace
  // (stable: a row keeps its entries' input order), then continue as CSR.
  rsvd_status bind_coo(const void* ri, const void* ci, int bits, const float* v) {
    const int64_t m = P.prob.m, n = P.prob.n, nnz = P.prob.nnz;
    coo_bits = bits;
    size_t need = 0;
    const hipError_t e = rsvd::launch_coo_to_csr(ri, ci, bits, v, m, n, nnz, B.keys0, B.keys1,
                                                 B.pay0, B.pay1, B.sort_temp, P.sort_temp,
                                                 B.coo_ptr, B.coo_col, B.coo_val, B.status, &need,
                                                 s);
    if (e == hipErrorOutOfMemory && need > P.sort_temp)
      return set_err(h, RSVD_E_BUDGET,
                     "the COO sort needs " + std::to_string(need) + " bytes of scratch, the plan "
                     "reserved " + std::to_string(P.sort_temp));
    RSVD_HIP(e);
    return bind_csr(B.coo_ptr, B.coo_col, B.coo_val);
  }

  // Operand copies of an FP32 panel for a product in precision prec: n-side
  // panels (ld = ldn) go to Xop16 / Xop8, m-side ones (ld = ldm) to Mop16 / Mop8.
  rsvd_status prep(int32_t prec, const float* src, bool nside) {
    const int64_t ld = nside ? P.ldn : P.ldm, rows = nside ? P.prob.n : P.prob.m;
    if (prec == RSVD_BF16)
      RSVD_HIP(rsvd::launch_panel_to_bf16(src, nside ? B.Xop16 : B.Mop16, ld * P.lp, s));
    else if (prec == RSVD_FP8E4M3)
      RSVD_HIP(rsvd::launch_panel_to_fp8(src, ld, rows, P.lp, nside ? B.Xop8 : B.Mop8,
                                         nside ? B.sX8 : B.sM8, B.f8part, s));
    return RSVD_OK;
  }

  // out (m-side panel, ld = ldm) = A X with X the n-side operand (Xop and its
  // BF16 / FP8 copies), in precision prec
  // One pass over host-resident A, tile by tile.  Even passes (A X) visit the
  // tiles row-major, odd passes (A^T Q) column-major backwards, so every pass
  // begins with the tiles the previous one ended on (the visit order of
  // rsvd_visit_order).  Each tile writes its own rows of its partial panel,
  // so the result does not depend on the order.
  rsvd_status stream_pass(bool nn, int32_t prec, const float* op, float* out) {
    const int64_t m = P.prob.m, n = P.prob.n;
    const bool split = nn ? P.TJ > 1 : P.TI > 1;
    const int64_t stride = split ? (nn ? P.ldm : P.ldn) * P.lp : 0;
    float* dst = split ? B.part : out;
    const bool b16 = prec == RSVD_BF16;
    std::vector<int64_t> order;
    order.reserve((size_t)(P.TI * P.TJ));
    if (pass_no % 2 == 0) {
      for (int64_t I = 0; I < P.TI; ++I)
        for (int64_t J = 0; J < P.TJ; ++J) order.push_back(I * P.TJ + J);
    } else {
      for (int64_t J = P.TJ - 1; J >= 0; --J)
        for (int64_t I = P.TI - 1; I >= 0; --I) order.push_back(I * P.TJ + J);
    }
    ++pass_no;
    Streamer& St = *st8;
    RSVD_HIP(tick(nn, true));
    for (int64_t t : order) {
      const int64_t I = t / P.TJ, J = t % P.TJ;
      const int64_t r0 = I * P.tm, rows = std::min(m, r0 + P.tm) - r0;
      const int64_t c0 = J * P.tn, cols = std::min(n, c0 + P.tn) - c0;
      const int64_t tiles = P.TI * P.TJ;
      const int64_t owned = P.slots >= tiles ? tiles : P.slots - 2;   // tiles with a slot of their own
      int64_t j = -1;
      if (t < owned) {
        j = t;
      } else {
        for (int64_t x = owned; x < P.slots; ++x)
          if (St.tile[x] == t) j = x;
      }
      if (j < 0 || St.tile[j] != t) {   // load: own slot, or the older streaming slot
        if (j < 0) {
          j = owned;
          for (int64_t x = owned + 1; x < P.slots; ++x)
            if (St.last_use[x] < St.last_use[j]) j = x;
        }
        RSVD_HIP(hipStreamWaitEvent(St.copy, St.freed[j], 0));
        RSVD_HIP(hipMemcpy2DAsync(B.slots + j * P.slot_bytes, P.slot_ld * P.elem,
                                  Ahost + (r0 * ldh + c0) * P.elem, ldh * P.elem, cols * P.elem,
                                  rows, hipMemcpyHostToDevice, St.copy));
        RSVD_HIP(hipEventRecord(St.ready[j], St.copy));
        St.tile[j] = t;
        St.h2d_bytes += (double)rows * cols * P.elem;
        ++St.loads;
      }
      St.last_use[j] = ++St.clock;
      RSVD_HIP(hipStreamWaitEvent(s, St.ready[j], 0));
      const char* slot = B.slots + j * P.slot_bytes;
      if (nn) {
        float* o = dst + J * stride + r0;
        if (b16)
          RSVD_HIP(rsvd::launch_nn_bf16((const uint16_t*)slot, P.slot_ld, rows, cols, P.tn, 1,
                                        B.Xop16 + c0, P.ldn, P.lp, o, P.ldm, 0, s));
        else
          RSVD_HIP(rsvd::launch_nn_f32((const float*)slot, P.slot_ld, rows, cols, P.tn, 1, op + c0,
                                       P.ldn, P.lp, o, P.ldm, 0, s));
      } else {
        float* o = dst + I * stride + c0;
        if (b16)
          RSVD_HIP(rsvd::launch_tn_bf16((const uint16_t*)slot, P.slot_ld, rows, cols, P.tm, 1,
                                        B.Mop16 + r0, P.ldm, P.lp, o, P.ldn, 0, s));
        else
          RSVD_HIP(rsvd::launch_tn_f32((const float*)slot, P.slot_ld, rows, cols, P.tm, 1, op + r0,
                                       P.ldm, P.lp, o, P.ldn, 0, s));
      }
      RSVD_HIP(hipEventRecord(St.freed[j], s));
    }
    RSVD_HIP(tick(nn, false));
    if (split)
      RSVD_HIP(rsvd::launch_reduce_parts(B.part, stride, nn ? P.TJ : P.TI, out, stride, s));
    return RSVD_OK;
  }

  rsvd_status product_nn(int32_t prec, const float* X, float* out) {
    if (P.host) return stream_pass(true, prec, X, out);
    if (P.csr) {
      RSVD_HIP(tick(true, true));
      RSVD_HIP(rsvd::launch_spmm(rowptr, colind, values, P.prob.m, 1, P.prob.nnz, X, P.ldn,
                                 P.prob.n, P.lp, B.Xr, B.Yr, B.carry, B.first, out, P.ldm, s));
      RSVD_HIP(tick(true, false));
      return RSVD_OK;
    }
    const int64_t m = P.prob.m, n = P.prob.n;
    const bool split = P.TJ > 1;
    const int64_t stride = split ? P.ldm * P.lp : 0;
    float* dst = split ? B.part : out;
    RSVD_HIP(tick(true, true));
    if (prec == RSVD_BF16 && cast_src) {
      RSVD_HIP(rsvd::launch_nn_bf16_cast(cast_src, cast_lda, m, n, P.tn, P.TJ, B.A16, P.lda16,
                                         B.Xop16, P.ldn, P.lp, dst, P.ldm, stride, s));
      cast_src = nullptr;
    } else if (prec == RSVD_BF16)
      RSVD_HIP(rsvd::launch_nn_bf16(A16, lda16, m, n, P.tn, P.TJ, B.Xop16, P.ldn, P.lp, dst, P.ldm,
                                    stride, s));
    else if (prec == RSVD_FP8E4M3)
      RSVD_HIP(rsvd::launch_nn_fp8(B.A8, P.lda8, m, n, P.tn, P.TJ, B.sA8, rsvd::ceil_div(n, 64), 1,
                                   B.Xop8, P.ldn, B.sX8, P.lp, dst, P.ldm, stride, s));
    else
      RSVD_HIP(rsvd::launch_nn_f32(A32, lda32, m, n, P.tn, P.TJ, X, P.ldn, P.lp, dst, P.ldm,
                                   stride, s));
    RSVD_HIP(tick(true, false));
    if (split) RSVD_HIP(rsvd::launch_reduce_parts(B.part, stride, P.TJ, out, stride, s));
    return RSVD_OK;
  }

  // out (n-side panel) = A^T Q with Q the m-side operand (Mop and its copies)
  rsvd_status product_tn(int32_t prec, const float* Q, float* out) {
    if (P.host) return stream_pass(false, prec, Q, out);
    if (P.csr) {
      RSVD_HIP(tick(false, true));
      RSVD_HIP(rsvd::launch_spmm(B.colptr, B.rowind, B.cval, P.prob.n, P.csc_parts, P.prob.nnz,
                                 Q, P.ldm, P.prob.m, P.lp, B.Xr, B.Yr, B.carry, B.first, out,
                                 P.ldn, s, B.headcol, P.head_k, P.head_parts));
      RSVD_HIP(tick(false, false));
      return RSVD_OK;
    }
    const int64_t m = P.prob.m, n = P.prob.n;
    const bool split = P.TI > 1;
    const int64_t stride = split ? P.ldn * P.lp : 0;
    float* dst = split ? B.part : out;
    if (prec == RSVD_BF16)
      if (rsvd_status st = settle_cast()) return st;
    RSVD_HIP(tick(false, true));
    if (prec == RSVD_BF16)
      RSVD_HIP(rsvd::launch_tn_bf16(A16, lda16, m, n, P.tm, P.TI, B.Mop16, P.ldm, P.lp, dst, P.ldn,
                                    stride, s));
    else if (prec == RSVD_FP8E4M3)   // the same kernel on the transposed FP8 copy
      RSVD_HIP(rsvd::launch_nn_fp8(B.A8T, P.ldat8, n, m, P.tm, P.TI, B.sA8, 1, rsvd::ceil_div(n, 64),
                                   B.Mop8, P.ldm, B.sM8, P.lp, dst, P.ldn, stride, s));
    else
      RSVD_HIP(rsvd::launch_tn_f32(A32, lda32, m, n, P.tm, P.TI, Q, P.ldm, P.lp, dst, P.ldn,
                                   stride, s));
    RSVD_HIP(tick(false, false));
    if (split) RSVD_HIP(rsvd::launch_reduce_parts(B.part, stride, P.TI, out, stride, s));
    return RSVD_OK;
  }

  // BF16 copy of a finished FP32 panel for the next BF16 product.
  rsvd_status to_bf16(const float* src, uint16_t* dst, int64_t ld) {
    RSVD_HIP(rsvd::launch_panel_to_bf16(src, dst, ld * P.lp, s));
    return RSVD_OK;
  }

  rsvd_status gram(const float* Pn, int64_t rows, int64_t ld) {
    const int64_t chunks = rsvd::gram_chunks_for(P, rows);
    RSVD_HIP(rsvd::launch_gram(Pn, ld, rows, P.lp, P.gram_rows, chunks, B.gpart, B.G, s));
    return RSVD_OK;
  }

  // The main stream waits for the side stream's last deferred pass.
  rsvd_status join_side() {
    if (side_busy) {
      RSVD_HIP(hipStreamWaitEvent(s, side->join, 0));
      side_busy = false;
    }
    return RSVD_OK;
  }

  // One CholeskyQR pass: out = in R^-1 with R^T R = in^T in.  With pside >= 0
  // and a pending factor Wp on that side (in = A X1 with X = X1 Wp), the pass
  // is taken of in Wp: G = Wp^T (in^T in) Wp and out = in (Wp W1).
  rsvd_status cholqr_pass(const float* in, float* out, int64_t rows, int64_t ld, int pside = -1) {
    rsvd_status st = gram(in, rows, ld);
    if (st != RSVD_OK) return st;
    const float* Wuse = B.W;
    if (pside >= 0 && pend[pside]) {
      if ((st = join_side())) return st;
      RSVD_HIP(rsvd::launch_congruence(B.G, Wpend(pside), B.L, B.Tc, P.lp, s));
      RSVD_HIP(rsvd::launch_chol_inv(B.Tc, P.lp, P.l, B.W, B.status, kCholTau, B.L, s));
      RSVD_HIP(rsvd::launch_lp_product(Wpend(pside), B.W, B.Wc, P.lp, s));
      Wuse = B.Wc;
      pend[pside] = false;
    } else {
      RSVD_HIP(rsvd::launch_chol_inv(B.G, P.lp, P.l, B.W, B.status, kCholTau, B.L, s));
    }
    RSVD_HIP(rsvd::launch_apply(in, ld, rows, P.l, Wuse, P.lp, P.lp, P.lp, true, out, ld, ld, s));
    return RSVD_OK;
  }

  // Second pass of `q1` (side sd) on the side stream: its Gram and Cholesky
  // give the pending factor; nothing else reads q1's buffer until a later
  // pass of the same side, after the consumer has joined.
  rsvd_status defer_second(const float* q1, int64_t rows, int64_t ld, int sd) {
    RSVD_HIP(make_side(h->p, side));
    RSVD_HIP(hipEventRecord(side->fork, s));
    RSVD_HIP(hipStreamWaitEvent(side->s, side->fork, 0));
    const int64_t chunks = rsvd::gram_chunks_for(P, rows);
    RSVD_HIP(rsvd::launch_gram(q1, ld, rows, P.lp, P.gram_rows, chunks, B.gpart2, B.G2, side->s));
    RSVD_HIP(rsvd::launch_chol_inv(B.G2, P.lp, P.l, Wpend(sd), B.status, kCholTau, B.Ls2,
                                   side->s));
    RSVD_HIP(hipEventRecord(side->join, side->s));
    side_busy = true;
    pend[sd] = true;
    return RSVD_OK;
  }

  // Orthonormal basis of `in` (side sd: 0 m-side, 1 n-side) written to
  // `out`: CholeskyQR2, or one pass.  `in` is the product of A (or A^T) with
  // the other side's basis, whose pending factor the first pass folds in.
  // defer: the second pass runs on the side stream and leaves out = Q1 with
  // a pending factor; otherwise it runs here through `tmp`.
  rsvd_status orth(const float* in, float* out, float* tmp, int64_t rows, int64_t ld, bool twice,
                   int sd = -1, bool defer = false) {
    const int pside = sd < 0 ? -1 : 1 - sd;
    if (!twice) return cholqr_pass(in, out, rows, ld, pside);
    if (defer && allow_defer && sd >= 0) {
      rsvd_status st = cholqr_pass(in, out, rows, ld, pside);
      if (st != RSVD_OK) return st;
      return defer_second(out, rows, ld, sd);
    }
    rsvd_status st = cholqr_pass(in, tmp, rows, ld, pside);
    if (st != RSVD_OK) return st;
    return cholqr_pass(tmp, out, rows, ld);
  }

  // Steps 1-6 of the randomized SVD on the power matrix (Section 2.1 on
  // Section 2.2 Eq. (2)): leaves Q in Mop (FP32), B^T in N0, the first kout
  // singular values in S and the small factors W (U_B) and W2 (U_B S^-1).
  template <typename Mark>
  rsvd_status forward(Mark& mark, double* S, int64_t kout) {
    const int64_t m = P.prob.m, n = P.prob.n;
    const bool cq1 = (P.opt.flags & RSVD_FLAG_CHOLQR1) != 0;
    const int32_t ps = P.opt.prec_sketch, pw = P.opt.prec_power, pj = P.opt.prec_project;
    rsvd_status st;
    if (ck && ck->resume) return forward_resumed(mark, S, kout);
    RSVD_HIP(rsvd::launch_omega_panel(P.prob.seed, n, P.l, P.lp, B.Xop, P.ldn, s));   // step 1
    if ((st = prep(ps, B.Xop, true))) return st;
    RSVD_HIP(mark(1));
    if ((st = product_nn(ps, B.Xop, B.M0))) return st;                                 // step 2
    RSVD_HIP(mark(2));
    if ((st = orth(B.M0, B.Mop, B.M1, m, P.ldm, !cq1 || P.prob.q == 0, 0, true))) return st;   // 3-4
    if ((st = prep(P.prob.q > 0 ? pw : pj, B.Mop, false))) return st;
    RSVD_HIP(mark(3));
    if (ck && !P.auto_q && (st = ck_after(1))) return st;
    if (P.auto_q) {
      // Section 2.2, automatic iteration parameter: each product A^T Q_t is
      // the projection B^T the factorisation would use with q = t; its small
      // SVD gives the singular values for that q.  Stop at the first q whose
      // leading k values moved by at most q_tol from q - 1 (or at prob.q),
      // keeping that B^T and its small SVD.
      for (int64_t t = 0;; ++t) {
        if ((st = product_tn(pw, B.Mop, B.N0))) return st;
        if ((st = small_svd_eig(B.N0))) return st;
        if ((st = small_svd_solve(S, kout))) return st;
        RSVD_HIP(rsvd::launch_ritz_delta(S, kout, t == 0, B.prevS, s));
        double delta = 0.0;
        RSVD_HIP(hipMemcpyAsync(&delta, B.prevS + kout, sizeof delta, hipMemcpyDeviceToHost, s));
        RSVD_HIP(hipStreamSynchronize(s));
        q_used = t;
        q_delta = delta;
        if (t == P.prob.q || (t > 0 && delta <= P.q_tol)) break;
        if ((st = orth(B.N0, B.Xop, B.N1, n, P.ldn, !cq1, 1, true))) return st;
        if ((st = prep(pw, B.Xop, true))) return st;
        if ((st = product_nn(pw, B.Xop, B.M0))) return st;
        if ((st = orth(B.M0, B.Mop, B.M1, m, P.ldm, true, 0, true))) return st;
        if ((st = prep(pw, B.Mop, false))) return st;
      }
      for (int i = 4; i <= 7; ++i) RSVD_HIP(mark(i));
      return RSVD_OK;
    }
    return passes_from(mark, S, kout, 2);
  }

  // Passes t_from .. 2q + 2 over A, then the small SVD.  Pass 1 is the sketch;
  // passes 2t and 2t + 1 are power step t = 1..q (Eq. (2), right to left),
  // each product re-orthonormalised; pass 2q + 2 is the projection (step 5).
  template <typename Mark>
  rsvd_status passes_from(Mark& mark, double* S, int64_t kout, int64_t t_from) {
    const int64_t m = P.prob.m, n = P.prob.n;
    const bool cq1 = (P.opt.flags & RSVD_FLAG_CHOLQR1) != 0;
    const int32_t pw = P.opt.prec_power, pj = P.opt.prec_project;
    const int64_t npass = 2 * P.prob.q + 2;
    rsvd_status st;
    q_used = P.prob.q;
    for (int64_t t = t_from; t <= npass; ++t) {
      if (t == npass) {
        RSVD_HIP(mark(4));
        if ((st = product_tn(pj, B.Mop, B.N0))) return st;                             // step 5
        RSVD_HIP(mark(5));
      } else if (t % 2 == 0) {
        if ((st = product_tn(pw, B.Mop, B.N0))) return st;
        if ((st = orth(B.N0, B.Xop, B.N1, n, P.ldn, !cq1, 1, true))) return st;
        if ((st = prep(pw, B.Xop, true))) return st;
      } else {
        const bool last = t == npass - 1;
        if ((st = product_nn(pw, B.Xop, B.M0))) return st;
        if ((st = orth(B.M0, B.Mop, B.M1, m, P.ldm, !cq1 || last, 0, true))) return st;
        if ((st = prep(last ? pj : pw, B.Mop, false))) return st;
      }
      if (ck && (st = ck_after(t))) return st;
    }
    if (t_from > npass) {   // resumed after the projection
      RSVD_HIP(mark(4));
      RSVD_HIP(mark(5));
    }
    if ((st = small_svd_eig(B.N0))) return st;                                         // SVD0 prep
    RSVD_HIP(mark(6));
    if ((st = small_svd_solve(S, kout))) return st;                                    // step 6
    RSVD_HIP(mark(7));
    return RSVD_OK;
  }

  // ---- per-pass persistence ------------------------------------------------
  // The state after pass t: side 0 the m-side basis Q (Mop), side 1 the
  // n-side panel (Xop), side 2 after the projection Q and B^T (Mop over N0).
  struct PanelPart {
    float* dev;
    int64_t ld, rows, row0;
  };
  int parts_of(int side, PanelPart* pp) const {
    const int64_t m = P.prob.m, n = P.prob.n;
    if (side == 0) {
      pp[0] = {B.Mop, P.ldm, m, 0};
      return 1;
    }
    if (side == 1) {
      pp[0] = {B.Xop, P.ldn, n, 0};
      return 1;
    }
    pp[0] = {B.Mop, P.ldm, m, 0};
    pp[1] = {B.N0, P.ldn, n, m};
    return 2;
  }

  rsvd_status ck_after(int64_t t) {
    if (ck->out) {
      const int64_t npass = 2 * P.prob.q + 2;
      const int side = ckpt_side(t, npass);
      const int64_t rows = ckpt_rows(P, side), main_rows = rows - P.lp;
      const int pside = side == 1 ? 1 : 0;
      PanelPart pp[2];
      const int np = parts_of(side, pp);
      if (rsvd_status st = join_side()) return st;
      RSVD_HIP(hipStreamSynchronize(s));
      for (int i = 0; i < np; ++i)
        RSVD_HIP(hipMemcpy2DAsync(ck->out_panel + pp[i].row0, (size_t)rows * 4, pp[i].dev,
                                  (size_t)pp[i].ld * 4, (size_t)pp[i].rows * 4, (size_t)P.lp,
                                  hipMemcpyDeviceToHost, s));
      std::vector<float> wp((size_t)P.lp * P.lp, 0.f);
      if (pend[pside])
        RSVD_HIP(hipMemcpyAsync(wp.data(), Wpend(pside), wp.size() * 4, hipMemcpyDeviceToHost, s));
      int32_t stw[rsvd::kStatusWords];
      RSVD_HIP(hipMemcpyAsync(stw, B.status, sizeof stw, hipMemcpyDeviceToHost, s));
      RSVD_HIP(hipStreamSynchronize(s));
      for (int64_t c = 0; c < P.lp; ++c)
        for (int64_t a = 0; a < P.lp; ++a)
          ck->out_panel[c * rows + main_rows + a] = wp[(size_t)(a * P.lp + c)];
      rsvd_checkpoint c{};
      c.magic = RSVD_CKPT_MAGIC;
      c.version = 1;
      c.passes = (int32_t)t;
      c.m = P.prob.m;
      c.n = P.prob.n;
      c.k = P.prob.k;
      c.p = P.prob.p;
      c.q = P.prob.q;
      c.seed = P.prob.seed;
      c.prec_sketch = P.opt.prec_sketch;
      c.prec_power = P.opt.prec_power;
      c.prec_project = P.opt.prec_project;
      c.flags = P.opt.flags & RSVD_FLAG_CHOLQR1;
      c.rows = rows;
      c.cols = P.lp;
      c.side = side;
      c.dropped = stw[rsvd::kStDropped];
      c.nonfinite = stw[rsvd::kStNonFinite];
      c.pending = pend[pside] ? 1 : 0;
      c.panel_hash = ckpt_hash(ck->out_panel, (size_t)rows * (size_t)P.lp);
      *ck->out = c;
    }
    if (ck->stop_after == t) {
      // a deferred CholeskyQR pass may still run on the side stream: order it
      // before whatever the caller enqueues next on its stream
      if (rsvd_status st = join_side()) return st;
      return RSVD_STOPPED;
    }
    return RSVD_OK;
  }

  // Continue after the checkpointed pass: load its panel(s) and counters,
  // make the operand copy the next pass reads, then run the remaining passes.
  template <typename Mark>
  rsvd_status forward_resumed(Mark& mark, double* S, int64_t kout) {
    const int32_t pw = P.opt.prec_power, pj = P.opt.prec_project;
    const rsvd_checkpoint& c = *ck->resume;
    const int64_t npass = 2 * P.prob.q + 2, t0 = c.passes;
    PanelPart pp[2];
    const int np = parts_of(c.side, pp);
    for (int i = 0; i < np; ++i)
      RSVD_HIP(hipMemcpy2DAsync(pp[i].dev, (size_t)pp[i].ld * 4, ck->resume_panel + pp[i].row0,
                                (size_t)c.rows * 4, (size_t)pp[i].rows * 4, (size_t)P.lp,
                                hipMemcpyHostToDevice, s));
    const int32_t cnt[2] = {c.dropped, c.nonfinite};
    RSVD_HIP(hipMemcpyAsync(B.status + rsvd::kStDropped, &cnt[0], 4, hipMemcpyHostToDevice, s));
    RSVD_HIP(hipMemcpyAsync(B.status + rsvd::kStNonFinite, &cnt[1], 4, hipMemcpyHostToDevice, s));
    const int pside = c.side == 1 ? 1 : 0;
    std::vector<float> wp((size_t)P.lp * P.lp);
    if (c.pending) {
      const int64_t main_rows = c.rows - P.lp;
      for (int64_t cc = 0; cc < P.lp; ++cc)
        for (int64_t a = 0; a < P.lp; ++a)
          wp[(size_t)(a * P.lp + cc)] = ck->resume_panel[cc * c.rows + main_rows + a];
      RSVD_HIP(hipMemcpyAsync(Wpend(pside), wp.data(), wp.size() * 4, hipMemcpyHostToDevice, s));
      pend[pside] = true;
    }
    RSVD_HIP(hipStreamSynchronize(s));   // the host buffers above live on this stack frame
    pass_no = t0;
    rsvd_status st;
    if (c.side == 0) {
      if ((st = prep(t0 == npass - 1 ? pj : pw, B.Mop, false))) return st;
    } else if (c.side == 1) {
      if ((st = prep(pw, B.Xop, true))) return st;
    }
    for (int i = 1; i <= 3; ++i) RSVD_HIP(mark(i));
    return passes_from(mark, S, kout, t0 + 1);
  }

  // Small SVD of B from Bt (n-side panel): leaves sorted S (k), Wu, Wv.
  // B^T = Bt Wp when the m-side basis has a pending factor Wp: C = Wp^T
  // (Bt^T Bt) Wp here, and small_svd_solve folds Wp into the small factors.
  rsvd_status small_svd_eig(const float* Bt) {
    rsvd_status st = gram(Bt, P.prob.n, P.ldn);
    if (st != RSVD_OK) return st;
    gsmall = B.G;
    if (pend[0]) {
      if ((st = join_side())) return st;
      RSVD_HIP(rsvd::launch_congruence(B.G, B.Wpm, B.L, B.Tc, P.lp, s));
      gsmall = B.Tc;
    }
    return RSVD_OK;
  }
  rsvd_status small_svd_solve(double* S, int64_t kout) {
    // C = L L^T, then one-sided Jacobi on L (no drop: tau = 0 keeps every
    // positive pivot; exactly dependent directions give zero columns): in one
    // workgroup up to width 128, over many workgroups (block Jacobi) beyond
    // Widths <= 128: the tridiagonal eigensolver of C first; the Cholesky and
    // Jacobi kernels then return at once unless its checks failed (close or
    // repeated eigenvalues, non-finite input), all decided on the device.
    const int32_t* skip = nullptr;
    if (B.tri) {
      RSVD_HIP(rsvd::launch_tri_eig(gsmall, P.lp, P.l, B.lam, B.Ev, B.tri, B.status, s));
      skip = B.status + rsvd::kStTriOk;
    }
    RSVD_HIP(rsvd::launch_chol_factor(gsmall, P.lp, P.l, B.L, B.status, 0.0, s, skip));
    if (rsvd::small_svd_one_sided(P.lp))
      RSVD_HIP(rsvd::launch_ojacobi(B.L, P.lp, P.l, B.lam, B.Ev, B.status, kJacobiTol,
                                    rsvd::kJacobiMaxSweeps, s, skip));
    else
      RSVD_HIP(rsvd::launch_bjacobi(B.L, P.lp, P.l, B.Mj, B.bjctl, B.lam, B.Ev, B.status,
                                    kJacobiTol, s));
    RSVD_HIP(rsvd::launch_finish_small(B.lam, B.Ev, P.lp, P.l, kout, S, B.W, B.W2, B.order,
                                       B.status, s));
    if (pend[0]) {   // U = Q1 (Wp U_B), V = Bt (Wp U_B S^-1)
      RSVD_HIP(rsvd::launch_lp_product(B.Wpm, B.W, B.Wc, P.lp, s));
      RSVD_HIP(hipMemcpyAsync(B.W, B.Wc, (size_t)P.lp * P.lp * 4, hipMemcpyDeviceToDevice, s));
      RSVD_HIP(rsvd::launch_lp_product(B.Wpm, B.W2, B.Wc, P.lp, s));
      RSVD_HIP(hipMemcpyAsync(B.W2, B.Wc, (size_t)P.lp * P.lp * 4, hipMemcpyDeviceToDevice, s));
    }
    return RSVD_OK;
  }
};

// Static workspace of rsvd_factor_noalloc (one copy per device, held until
// the process ends).  Its device address per device, from
// hipGetSymbolAddress; kMaxDevices bounds the device ordinals served.
__device__ __align__(256) static char scratch[RSVD_NOALLOC_WS_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

rsvd_status scratch_ptr(rsvd_plan_t h, void** out) {
  int dev = -1;
  RSVD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return set_err(h, RSVD_E_UNSUPPORTED, "device ordinal " + std::to_string(dev) +
                                              " is beyond the static workspace table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    RSVD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || (((uintptr_t)p) & 255))
      return set_err(h, RSVD_E_HIP, "static workspace address is NULL or not 256-byte aligned");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return RSVD_OK;
}

rsvd_status check_plan(rsvd_plan_t h) {
  if (!h) return set_err(nullptr, RSVD_E_INVALID_ARG, "plan is NULL");
  return RSVD_OK;
}

rsvd_status check_A(rsvd_plan_t h, const void* A, int64_t lda) {
  const rsvd::Plan& P = h->p;
  if (!A) return set_err(h, RSVD_E_INVALID_ARG, "A is NULL");
  if (lda < P.prob.n) return set_err(h, RSVD_E_INVALID_ARG, "lda < n");
  if (P.host) {
    // the copies overlap the products only from page-locked memory
    hipPointerAttribute_t at;
    const hipError_t e = hipPointerGetAttributes(&at, A);
    (void)hipGetLastError();
    if (e != hipSuccess || at.type != hipMemoryTypeHost)
      return set_err(h, RSVD_E_INVALID_ARG, "host-resident A must be pinned (page-locked) memory");
  }
  if (P.prob.dtype == RSVD_F32 && (((uintptr_t)A) & 3) != 0)
    return set_err(h, RSVD_E_INVALID_ARG, "FP32 A must be 4-byte aligned");
  if (P.prob.dtype == RSVD_BF16 && ((lda % 8) != 0 || (((uintptr_t)A) & 15) != 0))
    return set_err(h, RSVD_E_INVALID_ARG, "BF16 A needs lda % 8 == 0 and a 16-byte aligned base");
  if (P.prob.dtype == RSVD_F64 && (((uintptr_t)A) & 7) != 0)
    return set_err(h, RSVD_E_INVALID_ARG, "FP64 A must be 8-byte aligned");
  return RSVD_OK;
}

rsvd_status check_ws(rsvd_plan_t h, void* ws) {
  if (!ws) return set_err(h, RSVD_E_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws) & 255) return set_err(h, RSVD_E_INVALID_ARG, "workspace must be 256-byte aligned");
  return RSVD_OK;
}


Events* plan_events(rsvd_plan_t h, rsvd_status& st) {
  st = RSVD_OK;
  if (!h->p.hip_events) {
    Events* e = new (std::nothrow) Events;
    if (!e) {
      st = set_err(h, RSVD_E_INVALID_ARG, "out of host memory");
      return nullptr;
    }
    h->p.hip_events = e;
  }
  Events* ev = static_cast<Events*>(h->p.hip_events);
  hipError_t err = make_events(*ev, (size_t)(2 * h->p.prob.q + 2));
  if (err != hipSuccess) {
    st = hip_err(h, err, "hipEventCreate");
    return nullptr;
  }
  return ev;
}

// Wait for the stream, fill the report from the events and status words and
// turn device-side outcomes into the status.
rsvd_status finish_report(rsvd_plan_t h, const Runner& R, Events* ev, rsvd_report* report) {
  const rsvd::Plan& P = h->p;
  const int64_t m = P.prob.m, n = P.prob.n;
  std::memset(report, 0, sizeof *report);
  RSVD_HIP(hipStreamSynchronize(R.s));
  float ms = 0.f;
  for (int i = 0; ev && i < 8; ++i) {
    RSVD_HIP(hipEventElapsedTime(&ms, ev->ev[i], ev->ev[i + 1]));
    report->stage_ms[i] = ms;
  }
  if (ev) {
    RSVD_HIP(hipEventElapsedTime(&ms, ev->ev[0], ev->ev[8]));
    report->total_ms = ms;
  }
  for (size_t x = 0; x < R.nn_idx.size(); ++x) {
    const int i = R.nn_idx[x];
    RSVD_HIP(hipEventElapsedTime(&ms, ev->kern[2 * i], ev->kern[2 * i + 1]));
    report->gemm_nn_ms += ms;
    if (x == 0) report->sketch_ms = ms;
  }
  for (int i : R.tn_idx) {
    RSVD_HIP(hipEventElapsedTime(&ms, ev->kern[2 * i], ev->kern[2 * i + 1]));
    report->gemm_tn_ms += ms;
  }
  report->gemm_nn_launches = (int32_t)R.nn_idx.size();
  report->gemm_tn_launches = (int32_t)R.tn_idx.size();
  int32_t stw[rsvd::kStatusWords];
  RSVD_HIP(hipMemcpyAsync(stw, R.B.status, sizeof stw, hipMemcpyDeviceToHost, R.s));
  RSVD_HIP(hipStreamSynchronize(R.s));
  const double passes = 2.0 * (double)P.prob.q + 2.0;
  report->flops_alg = passes * 2.0 * (double)m * (double)n * (double)P.l;
  auto pass_bytes = [&](int32_t prec) {
    const double e = prec == RSVD_BF16 ? 2.0 : prec == RSVD_FP8E4M3 ? 1.0 : 4.0;
    return (double)m * (double)n * e + ((double)m + (double)n) * P.l * e;
  };
  report->bytes_alg = pass_bytes(P.opt.prec_sketch) +
                      2.0 * (double)P.prob.q * pass_bytes(P.opt.prec_power) +
                      pass_bytes(P.opt.prec_project);
  report->ws_bytes = (int64_t)P.ws.total;
  {
    const int64_t eb = P.prob.dtype == RSVD_F64 ? 8 : P.prob.dtype == RSVD_BF16 ? 2 : 4;
    // caller arrays: CSR (rowptr, colind, values) or COO (two index arrays of
    // coo_bits, values); the CSR copy of COO input lives in the workspace
    const int64_t a_bytes = P.coo   ? P.prob.nnz * (2 * (R.coo_bits / 8) + 4)
                            : P.csr ? P.prob.nnz * 8 + (m + 1) * 4
                            : P.host ? 0 : m * n * eb;
    report->peak_hbm = (int64_t)P.ws.total + a_bytes + (m + n) * P.prob.k * 4 + P.prob.k * 8;
  }
  report->dropped = stw[rsvd::kStDropped];
  report->jacobi_sweeps = stw[rsvd::kStSweeps];
  report->nonfinite = stw[rsvd::kStNonFinite];
  report->q_used = (int32_t)R.q_used;
  report->q_delta = R.q_delta;
  if (P.host && R.st8) {
    report->slots = (int32_t)P.slots;
    report->h2d_bytes = R.st8->h2d_bytes;
    report->tile_loads = R.st8->loads;
  }
  if (P.csr) {
    report->flops_alg = passes * 2.0 * (double)P.prob.nnz * (double)P.l;
    report->bytes_alg = passes * ((double)P.prob.nnz * 8.0 + ((double)m + (double)n) * P.l * 4.0);
  }
  if (stw[rsvd::kStBadSparse] > 0)
    return set_err(h, RSVD_E_INVALID_ARG, "malformed CSR input (pointers or column indices)");
  if (stw[rsvd::kStNonFinite] > 0) return set_err(h, RSVD_E_NUMERIC, "NaN or Inf met on the device");
  if (stw[rsvd::kStTies] > 0) return RSVD_W_DEGENERATE;
  if (stw[rsvd::kStDropped] > 0 || stw[rsvd::kStRankSmall] > 0) return RSVD_W_RANK_DEFICIENT;
  return RSVD_OK;
}

}  // namespace

namespace {

// The whole path after A has been bound (dense or sparse).
template <typename Bind>
rsvd_status factor_common(rsvd_plan_t h, Bind bind, void* ws, float* U, int64_t ldu, double* S,
                          float* V, int64_t ldv, void* stream, rsvd_report* report,
                          const Runner::Ckpt* ck = nullptr, bool no_alloc = false) {
  const rsvd::Plan& P = h->p;
  const int64_t m = P.prob.m, n = P.prob.n, k = P.prob.k;
  if (!U || !S || !V) return set_err(h, RSVD_E_INVALID_ARG, "U, S and V must be non-NULL");
  if (ldu < m || ldv < n) return set_err(h, RSVD_E_INVALID_ARG, "ldu < m or ldv < n");

  hipStream_t s = (hipStream_t)stream;
  Runner R(h, ws, s);
  R.ck = ck;
  // no_alloc: nothing is created (no timing events, no side stream)
  R.allow_defer = !no_alloc;
  Events* ev = nullptr;
  if (report && !no_alloc) {
    rsvd_status est;
    if (!(ev = plan_events(h, est))) return est;
    R.ev = ev;
  }
  auto mark = [&](int i) -> hipError_t { return ev ? hipEventRecord(ev->ev[i], s) : hipSuccess; };
  rsvd_status st;

  RSVD_HIP(mark(0));
  RSVD_HIP(rsvd::launch_fill_i32(R.B.status, rsvd::kStatusWords, 0, s));
  if ((st = bind(R))) return st;
  if ((st = R.forward(mark, S, k))) return st;   // RSVD_STOPPED leaves U, S, V unwritten
  // step 7: U = Q E_k (W), V = B^T E_k S^-1 (W2)
  RSVD_HIP(rsvd::launch_apply(R.B.Mop, P.ldm, m, P.l, R.B.W, P.lp, P.lp, k, false, U, ldu, m, s));
  RSVD_HIP(rsvd::launch_apply(R.B.N0, P.ldn, n, P.l, R.B.W2, P.lp, P.lp, k, false, V, ldv, n, s));
  if (!(P.opt.flags & RSVD_FLAG_NO_SIGN_FIX))
    RSVD_HIP(rsvd::launch_sign_fix(U, ldu, m, V, ldv, n, k, R.B.signs, s));
  RSVD_HIP(mark(8));

  if (!report) return RSVD_OK;
  return finish_report(h, R, ev, report);
}

}  // namespace

extern "C" {

const char* rsvd_version(void) { return "rsvd-mi355x 0.1"; }

const char* rsvd_status_str(rsvd_status s) {
  switch (s) {
    case RSVD_OK: return "ok";
    case RSVD_W_RANK_DEFICIENT: return "warning: rank deficient sketch (directions dropped)";
    case RSVD_W_DEGENERATE: return "warning: degenerate singular values";
    case RSVD_STOPPED: return "stopped after the requested pass";
    case RSVD_E_INVALID_ARG: return "invalid argument";
    case RSVD_E_BUDGET: return "workspace exceeds the HBM budget";
    case RSVD_E_HIP: return "HIP runtime error";
    case RSVD_E_UNSUPPORTED: return "unsupported combination";
    case RSVD_E_NUMERIC: return "non-finite values met";
    default: return "unknown status";
  }
}

const char* rsvd_last_error(rsvd_plan_t plan) {
  return plan ? plan->p.last_error.c_str() : g_last_error.c_str();
}

rsvd_status rsvd_plan(const rsvd_problem* prob, const rsvd_options* opt, rsvd_plan_t* out,
                      size_t* device_ws_bytes) {
  if (!prob || !out || !device_ws_bytes)
    return set_err(nullptr, RSVD_E_INVALID_ARG, "prob, out and device_ws_bytes must be non-NULL");
  *out = nullptr;
  *device_ws_bytes = 0;
  rsvd_plan_s* h = new (std::nothrow) rsvd_plan_s;
  if (!h) return set_err(nullptr, RSVD_E_INVALID_ARG, "out of host memory");
  rsvd_status st = rsvd::make_plan(*prob, opt, h->p);
  if (st < 0) {
    g_last_error = h->p.last_error;
    delete h;
    return st;
  }
  *out = h;
  *device_ws_bytes = h->p.ws.total;
  return RSVD_OK;
}

rsvd_status rsvd_plan_set_streams(rsvd_plan_t h, void* copy_stream, void* side_stream) {
  if (rsvd_status st = check_plan(h)) return st;
  rsvd::Plan& P = h->p;
  // a stream already in use is released (or left to its owner) first
  destroy_streamer(static_cast<Streamer*>(P.streamer));
  P.streamer = nullptr;
  destroy_side(static_cast<Side*>(P.side));
  P.side = nullptr;
  P.user_copy = copy_stream;
  P.user_side = side_stream;
  return RSVD_OK;
}

void rsvd_plan_destroy(rsvd_plan_t plan) {
  if (!plan) return;
  destroy_events(static_cast<Events*>(plan->p.hip_events));
  destroy_streamer(static_cast<Streamer*>(plan->p.streamer));
  destroy_side(static_cast<Side*>(plan->p.side));
  delete plan;
}

rsvd_status rsvd_tile_map(rsvd_plan_t h, int64_t* out, size_t cap, size_t* n_out) {
  if (rsvd_status st = check_plan(h)) return st;
  if (!n_out || (!out && cap)) return set_err(h, RSVD_E_INVALID_ARG, "bad output arguments");
  const rsvd::Plan& P = h->p;
  const int64_t Pg = P.opt.grid_p, Qg = P.opt.grid_q;
  size_t w = 0;
  for (int64_t I = 0; I < P.TI; ++I) {
    const int64_t r0 = I * P.tm, r1 = std::min(P.prob.m, r0 + P.tm);
    for (int64_t J = 0; J < P.TJ; ++J) {
      const int64_t c0 = J * P.tn, c1 = std::min(P.prob.n, c0 + P.tn);
      const int64_t v[12] = {I,      J,      r0,     r1 - r0, c0, c1 - c0, I % Pg, J % Qg, I / Pg,
                             J / Qg, ((r0 / P.tm) / Pg) * P.tm + r0 % P.tm,
                             ((c0 / P.tn) / Qg) * P.tn + c0 % P.tn};
      for (int e = 0; e < 12; ++e, ++w)
        if (w < cap) out[w] = v[e];
    }
  }
  *n_out = w;
  return RSVD_OK;
}

rsvd_status rsvd_visit_order(rsvd_plan_t h, int64_t pass_index, int64_t* out, size_t cap,
                             size_t* n_out) {
  if (rsvd_status st = check_plan(h)) return st;
  if (!n_out || (!out && cap) || pass_index < 0)
    return set_err(h, RSVD_E_INVALID_ARG, "bad arguments");
  const rsvd::Plan& P = h->p;
  size_t w = 0;
  if (pass_index % 2 == 0) {
    for (int64_t I = 0; I < P.TI; ++I)
      for (int64_t J = 0; J < P.TJ; ++J, ++w)
        if (w < cap) out[w] = I * P.TJ + J;
  } else {
    for (int64_t J = P.TJ - 1; J >= 0; --J)
      for (int64_t I = P.TI - 1; I >= 0; --I, ++w)
        if (w < cap) out[w] = I * P.TJ + J;
  }
  *n_out = w;
  return RSVD_OK;
}

rsvd_status rsvd_philox_raw(uint64_t seed, uint32_t stream_id, int64_t row0, int64_t rows,
                            int64_t blocks, uint32_t* out, void* stream) {
  rsvd_plan_t h = nullptr;
  if (row0 < 0 || rows < 0 || blocks < 0 || (rows * blocks > 0 && !out))
    return set_err(nullptr, RSVD_E_INVALID_ARG, "bad philox arguments");
  if (blocks > 0xFFFFFFFFll) return set_err(nullptr, RSVD_E_INVALID_ARG, "too many column blocks");
  RSVD_HIP(rsvd::launch_philox_raw(seed, stream_id, row0, rows, blocks, out, (hipStream_t)stream));
  return RSVD_OK;
}

rsvd_status rsvd_omega(uint64_t seed, int64_t n, int64_t l, int64_t row0, int64_t rows,
                       int32_t dtype, void* out, int64_t ldo, void* stream) {
  rsvd_plan_t h = nullptr;
  if (n < 0 || l < 0 || row0 < 0 || rows < 0 || row0 + rows > n || ldo < l ||
      (rows > 0 && !out) || (dtype != RSVD_F64 && dtype != RSVD_F32) || l / 4 >= 65535)
    return set_err(nullptr, RSVD_E_INVALID_ARG, "bad omega arguments");
  RSVD_HIP(rsvd::launch_omega_rows(seed, l, row0, rows, dtype == RSVD_F64, out, ldo,
                                   (hipStream_t)stream));
  return RSVD_OK;
}

rsvd_status rsvd_factor(rsvd_plan_t h, const void* A, int64_t lda, void* ws, float* U, int64_t ldu,
                        double* S, float* V, int64_t ldv, void* stream, rsvd_report* report) {
  if (rsvd_status st = check_plan(h)) return st;
  if (h->p.csr) return set_err(h, RSVD_E_INVALID_ARG, "the plan is for CSR input: use rsvd_factor_csr");
  if (rsvd_status st = check_A(h, A, lda)) return st;
  if (rsvd_status st = check_ws(h, ws)) return st;
  return factor_common(h, [&](Runner& R) { return R.bind_A(A, lda); }, ws, U, ldu, S, V, ldv,
                       stream, report);
}

// rsvd_factor_noalloc: the workspace is the library's own device array
// `scratch` instead of a caller buffer.  Host code never passes the array's
// name to a kernel (that is a host-side stand-in); the device address comes
// from hipGetSymbolAddress, taken once per device with that device current
// and kept per device.  Every call on a device shares its array.
rsvd_status rsvd_factor_noalloc(rsvd_plan_t h, const void* A, int64_t lda, float* U, int64_t ldu,
                                double* S, float* V, int64_t ldv, void* stream) {
  if (rsvd_status st = check_plan(h)) return st;
  const rsvd::Plan& P = h->p;
  if (P.csr) return set_err(h, RSVD_E_UNSUPPORTED, "rsvd_factor_noalloc takes dense A only");
  if (P.host)
    return set_err(h, RSVD_E_UNSUPPORTED, "rsvd_factor_noalloc needs A in device memory");
  if (P.ws.total > RSVD_NOALLOC_WS_BYTES)
    return set_err(h, RSVD_E_BUDGET,
                   "the plan needs " + std::to_string(P.ws.total) +
                       " bytes of workspace; the static workspace of rsvd_factor_noalloc holds " +
                       std::to_string((unsigned long long)RSVD_NOALLOC_WS_BYTES));
  if (rsvd_status st = check_A(h, A, lda)) return st;
  void* ws = nullptr;
  if (rsvd_status st = scratch_ptr(h, &ws)) return st;
  return factor_common(h, [&](Runner& R) { return R.bind_A(A, lda); }, ws, U, ldu, S, V, ldv,
                       stream, nullptr, nullptr, /*no_alloc=*/true);
}

rsvd_status rsvd_factor_csr(rsvd_plan_t h, const int32_t* rowptr, const int32_t* colind,
                            const float* values, void* ws, float* U, int64_t ldu, double* S,
                            float* V, int64_t ldv, void* stream, rsvd_report* report) {
  if (rsvd_status st = check_plan(h)) return st;
  if (!h->p.csr) return set_err(h, RSVD_E_INVALID_ARG, "the plan is for dense input: use rsvd_factor");
  if (h->p.coo) return set_err(h, RSVD_E_INVALID_ARG, "the plan is for COO input: use rsvd_factor_coo");
  if (!rowptr || (h->p.prob.nnz > 0 && (!colind || !values)))
    return set_err(h, RSVD_E_INVALID_ARG, "CSR arrays must be non-NULL");
  if (rsvd_status st = check_ws(h, ws)) return st;
  return factor_common(h, [&](Runner& R) { return R.bind_csr(rowptr, colind, values); }, ws, U, ldu,
                       S, V, ldv, stream, report);
}

rsvd_status rsvd_factor_coo(rsvd_plan_t h, const void* rowind, const void* colind,
                            int32_t index_bits, const float* values, void* ws, float* U,
                            int64_t ldu, double* S, float* V, int64_t ldv, void* stream,
                            rsvd_report* report) {
  if (rsvd_status st = check_plan(h)) return st;
  if (!h->p.coo) return set_err(h, RSVD_E_INVALID_ARG, "the plan is not for COO input");
  if (index_bits != 32 && index_bits != 64)
    return set_err(h, RSVD_E_INVALID_ARG, "index_bits must be 32 or 64");
  if (h->p.prob.nnz > 0 && (!rowind || !colind || !values))
    return set_err(h, RSVD_E_INVALID_ARG, "COO arrays must be non-NULL");
  if (rsvd_status st = check_ws(h, ws)) return st;
  return factor_common(h, [&](Runner& R) { return R.bind_coo(rowind, colind, index_bits, values); },
                       ws, U, ldu, S, V, ldv, stream, report);
}

rsvd_status rsvd_checkpoint_bytes(rsvd_plan_t h, size_t* panel_bytes) {
  if (rsvd_status st = check_plan(h)) return st;
  if (!panel_bytes) return set_err(h, RSVD_E_INVALID_ARG, "panel_bytes is NULL");
  const rsvd::Plan& P = h->p;
  *panel_bytes = (size_t)(P.prob.m + P.prob.n + P.lp) * (size_t)P.lp * 4;
  return RSVD_OK;
}

rsvd_status rsvd_factor_resumable(rsvd_plan_t h, const void* A, int64_t lda, void* ws, float* U,
                                  int64_t ldu, double* S, float* V, int64_t ldv, void* stream,
                                  rsvd_report* report, const rsvd_checkpoint* resume,
                                  const float* resume_panel, int32_t stop_after,
                                  rsvd_checkpoint* ckpt, float* ckpt_panel) {
  if (rsvd_status st = check_plan(h)) return st;
  const rsvd::Plan& P = h->p;
  if (P.csr) return set_err(h, RSVD_E_UNSUPPORTED, "checkpoints are implemented for dense A");
  if (P.auto_q)
    return set_err(h, RSVD_E_UNSUPPORTED, "checkpoints are implemented for a fixed q (no AUTO_Q)");
  const int64_t npass = 2 * P.prob.q + 2;
  if (stop_after < 0 || stop_after > npass)
    return set_err(h, RSVD_E_INVALID_ARG, "stop_after must lie in [0, 2q + 2]");
  if (ckpt && !ckpt_panel) return set_err(h, RSVD_E_INVALID_ARG, "ckpt needs ckpt_panel");
  if (resume) {
    const rsvd_checkpoint& c = *resume;
    if (!resume_panel) return set_err(h, RSVD_E_INVALID_ARG, "resume needs resume_panel");
    if (c.magic != RSVD_CKPT_MAGIC || c.version != 1)
      return set_err(h, RSVD_E_INVALID_ARG, "not a version-1 checkpoint");
    if (c.m != P.prob.m || c.n != P.prob.n || c.k != P.prob.k || c.p != P.prob.p ||
        c.q != P.prob.q || c.seed != P.prob.seed || c.prec_sketch != P.opt.prec_sketch ||
        c.prec_power != P.opt.prec_power || c.prec_project != P.opt.prec_project ||
        c.flags != (P.opt.flags & RSVD_FLAG_CHOLQR1))
      return set_err(h, RSVD_E_INVALID_ARG, "the checkpoint belongs to another problem or plan");
    if (c.passes < 1 || c.passes > npass)
      return set_err(h, RSVD_E_INVALID_ARG, "checkpoint pass out of range");
    const int side = ckpt_side(c.passes, npass);
    if (c.side != side || c.rows != ckpt_rows(P, side) || c.cols != P.lp ||
        (c.pending != 0 && c.pending != 1))
      return set_err(h, RSVD_E_INVALID_ARG, "checkpoint shape does not match its pass");
    if (ckpt_hash(resume_panel, (size_t)c.rows * (size_t)c.cols) != c.panel_hash)
      return set_err(h, RSVD_E_INVALID_ARG, "checkpoint panel does not match its hash");
    if (stop_after != 0 && stop_after <= c.passes)
      return set_err(h, RSVD_E_INVALID_ARG, "stop_after must lie after the resumed pass");
  }
  if (rsvd_status st = check_A(h, A, lda)) return st;
  if (rsvd_status st = check_ws(h, ws)) return st;
  const Runner::Ckpt ck{resume, resume_panel, stop_after, ckpt, ckpt_panel};
  return factor_common(h, [&](Runner& R) { return R.bind_A(A, lda); }, ws, U, ldu, S, V, ldv,
                       stream, report, &ck);
}

rsvd_status rsvd_step_spmm(rsvd_plan_t h, int32_t op, const int32_t* rowptr, const int32_t* colind,
                           const float* values, const float* X, int64_t ldx, float* out,
                           int64_t ldo, void* ws, void* stream) {
  if (rsvd_status st = check_plan(h)) return st;
  if (!h->p.csr) return set_err(h, RSVD_E_INVALID_ARG, "the plan is for dense input");
  if (rsvd_status st = check_ws(h, ws)) return st;
  const rsvd::Plan& P = h->p;
  const int64_t m = P.prob.m, n = P.prob.n;
  if (op != 0 && op != 1) return set_err(h, RSVD_E_INVALID_ARG, "op must be 0 or 1");
  const int64_t in_rows = op == 0 ? n : m, out_rows = op == 0 ? m : n;
  if (!rowptr || !X || !out || ldx < in_rows || ldo < out_rows ||
      (P.prob.nnz > 0 && (!colind || !values)))
    return set_err(h, RSVD_E_INVALID_ARG, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  Runner R(h, ws, s);
  rsvd_status st;
  RSVD_HIP(rsvd::launch_fill_i32(R.B.status, rsvd::kStatusWords, 0, s));
  if ((st = R.bind_csr(rowptr, colind, values))) return st;
  if (op == 0) {
    RSVD_HIP(rsvd::launch_panel_copy(X, ldx, n, P.l, R.B.Xop, P.ldn, P.ldn, P.lp, s));
    if ((st = R.product_nn(RSVD_F32, R.B.Xop, R.B.M0))) return st;
    RSVD_HIP(rsvd::launch_panel_copy(R.B.M0, P.ldm, m, P.l, out, ldo, m, P.l, s));
  } else {
    RSVD_HIP(rsvd::launch_panel_copy(X, ldx, m, P.l, R.B.Mop, P.ldm, P.ldm, P.lp, s));
    if ((st = R.product_tn(RSVD_F32, R.B.Mop, R.B.N0))) return st;
    RSVD_HIP(rsvd::launch_panel_copy(R.B.N0, P.ldn, n, P.l, out, ldo, n, P.l, s));
  }
  int32_t bad = 0;
  RSVD_HIP(hipMemcpyAsync(&bad, R.B.status + rsvd::kStBadSparse, 4, hipMemcpyDeviceToHost, s));
  RSVD_HIP(hipStreamSynchronize(s));
  if (bad) return set_err(h, RSVD_E_INVALID_ARG, "malformed CSR input (pointers or column indices)");
  return RSVD_OK;
}

rsvd_status rsvd_step_product(rsvd_plan_t h, int32_t op, const void* A, int64_t lda, const float* X,
                              int64_t ldx, float* out, int64_t ldo, void* ws, void* stream) {
  if (rsvd_status st = check_plan(h)) return st;
  if (h->p.csr) return set_err(h, RSVD_E_INVALID_ARG, "this call needs dense A (plan is for CSR)");
  if (h->p.host)
    return set_err(h, RSVD_E_UNSUPPORTED, "this call needs A in device memory (plan is host-resident)");
  if (rsvd_status st = check_A(h, A, lda)) return st;
  if (rsvd_status st = check_ws(h, ws)) return st;
  const rsvd::Plan& P = h->p;
  const int64_t m = P.prob.m, n = P.prob.n;
  if (op != 0 && op != 1) return set_err(h, RSVD_E_INVALID_ARG, "op must be 0 or 1");
  const int64_t in_rows = op == 0 ? n : m, out_rows = op == 0 ? m : n;
  if (!X || !out || ldx < in_rows || ldo < out_rows)
    return set_err(h, RSVD_E_INVALID_ARG, "bad panel arguments");
  hipStream_t s = (hipStream_t)stream;
  Runner R(h, ws, s);
  rsvd_status st;
  if ((st = R.bind_A(A, lda))) return st;
  if (op == 0) {
    RSVD_HIP(rsvd::launch_panel_copy(X, ldx, n, P.l, R.B.Xop, P.ldn, P.ldn, P.lp, s));
    if ((st = R.prep(P.opt.prec_sketch, R.B.Xop, true))) return st;
    if ((st = R.product_nn(P.opt.prec_sketch, R.B.Xop, R.B.M0))) return st;
    RSVD_HIP(rsvd::launch_panel_copy(R.B.M0, P.ldm, m, P.l, out, ldo, m, P.l, s));
  } else {
    RSVD_HIP(rsvd::launch_panel_copy(X, ldx, m, P.l, R.B.Mop, P.ldm, P.ldm, P.lp, s));
    if ((st = R.prep(P.opt.prec_project, R.B.Mop, false))) return st;
    if ((st = R.product_tn(P.opt.prec_project, R.B.Mop, R.B.N0))) return st;
    RSVD_HIP(rsvd::launch_panel_copy(R.B.N0, P.ldn, n, P.l, out, ldo, n, P.l, s));
  }
  return RSVD_OK;
}

rsvd_status rsvd_step_orth(rsvd_plan_t h, int32_t side, const float* Y, int64_t ldy, float* Q,
                           int64_t ldq, void* ws, void* stream) {
  if (rsvd_status st = check_plan(h)) return st;
  if (rsvd_status st = check_ws(h, ws)) return st;
  const rsvd::Plan& P = h->p;
  if (side != 0 && side != 1) return set_err(h, RSVD_E_INVALID_ARG, "side must be 0 or 1");
  const int64_t rows = side == 0 ? P.prob.m : P.prob.n;
  const int64_t ld = side == 0 ? P.ldm : P.ldn;
  if (!Y || !Q || ldy < rows || ldq < rows) return set_err(h, RSVD_E_INVALID_ARG, "bad panel arguments");
  hipStream_t s = (hipStream_t)stream;
  Runner R(h, ws, s);
  float* a = side == 0 ? R.B.M0 : R.B.N0;
  float* b = side == 0 ? R.B.M1 : R.B.N1;
  float* c = side == 0 ? R.B.Mop : R.B.Xop;
  RSVD_HIP(rsvd::launch_fill_i32(R.B.status, rsvd::kStatusWords, 0, s));
  RSVD_HIP(rsvd::launch_panel_copy(Y, ldy, rows, P.l, a, ld, ld, P.lp, s));
  rsvd_status st;
  if ((st = R.orth(a, c, b, rows, ld, true))) return st;
  RSVD_HIP(rsvd::launch_panel_copy(c, ld, rows, P.l, Q, ldq, rows, P.l, s));
  return RSVD_OK;
}

rsvd_status rsvd_step_gram(rsvd_plan_t h, int32_t side, const float* Y, int64_t ldy, double* G,
                           void* ws, void* stream) {
  if (rsvd_status st = check_plan(h)) return st;
  if (rsvd_status st = check_ws(h, ws)) return st;
  const rsvd::Plan& P = h->p;
  if (side != 0 && side != 1) return set_err(h, RSVD_E_INVALID_ARG, "side must be 0 or 1");
  const int64_t rows = side == 0 ? P.prob.m : P.prob.n;
  const int64_t ld = side == 0 ? P.ldm : P.ldn;
  if (!Y || !G || ldy < rows) return set_err(h, RSVD_E_INVALID_ARG, "bad panel arguments");
  hipStream_t s = (hipStream_t)stream;
  Runner R(h, ws, s);
  float* a = side == 0 ? R.B.M0 : R.B.N0;
  RSVD_HIP(rsvd::launch_panel_copy(Y, ldy, rows, P.l, a, ld, ld, P.lp, s));
  rsvd_status st;
  if ((st = R.gram(a, rows, ld))) return st;
  RSVD_HIP(hipMemcpy2DAsync(G, P.l * sizeof(double), R.B.G, P.lp * sizeof(double),
                            P.l * sizeof(double), P.l, hipMemcpyDeviceToDevice, s));
  return RSVD_OK;
}

rsvd_status rsvd_step_small_svd(rsvd_plan_t h, const float* Bt, int64_t ldb, double* sig,
                                double* ub, void* ws, void* stream) {
  if (rsvd_status st = check_plan(h)) return st;
  if (rsvd_status st = check_ws(h, ws)) return st;
  const rsvd::Plan& P = h->p;
  if (!Bt || !sig || !ub || ldb < P.prob.n) return set_err(h, RSVD_E_INVALID_ARG, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  Runner R(h, ws, s);
  RSVD_HIP(rsvd::launch_fill_i32(R.B.status, rsvd::kStatusWords, 0, s));
  RSVD_HIP(rsvd::launch_panel_copy(Bt, ldb, P.prob.n, P.l, R.B.N0, P.ldn, P.ldn, P.lp, s));
  rsvd_status st;
  if ((st = R.small_svd_eig(R.B.N0))) return st;
  if ((st = R.small_svd_solve(sig, P.l))) return st;
  // U_B(a, c) = Ev(a, order c) in FP64
  RSVD_HIP(rsvd::launch_gather_cols(R.B.Ev, P.lp, P.l, R.B.order, ub, s));
  return RSVD_OK;
}

rsvd_status rsvd_backward(rsvd_plan_t h, const void* A, int64_t lda, const float* gU,
                          int64_t ldgu, const double* gS, const float* gV, int64_t ldgv,
                          float* gA, int64_t ldga, void* ws, void* stream, rsvd_report* report) {
  if (rsvd_status st = check_plan(h)) return st;
  if (h->p.csr) return set_err(h, RSVD_E_INVALID_ARG, "this call needs dense A (plan is for CSR)");
  if (h->p.host)
    return set_err(h, RSVD_E_UNSUPPORTED, "this call needs A in device memory (plan is host-resident)");
  if (rsvd_status st = check_A(h, A, lda)) return st;
  if (rsvd_status st = check_ws(h, ws)) return st;
  const rsvd::Plan& P = h->p;
  const int64_t m = P.prob.m, n = P.prob.n, k = P.prob.k, l = P.l, lp = P.lp, kp = P.kp;
  if (!P.backward) return set_err(h, RSVD_E_INVALID_ARG, "plan was made without RSVD_FLAG_BACKWARD");
  if (!gA || ldga < n) return set_err(h, RSVD_E_INVALID_ARG, "gA is NULL or ldga < n");
  if ((gU && ldgu < m) || (gV && ldgv < n))
    return set_err(h, RSVD_E_INVALID_ARG, "ldgu < m or ldgv < n");
  hipStream_t s = (hipStream_t)stream;
  Runner R(h, ws, s);
  Events* ev = nullptr;
  if (report) {
    rsvd_status est;
    if (!(ev = plan_events(h, est))) return est;
    R.ev = ev;
  }
  auto mark = [&](int i) -> hipError_t { return ev ? hipEventRecord(ev->ev[i], s) : hipSuccess; };
  const Buffers& B = R.B;
  rsvd_status st;
  RSVD_HIP(mark(0));
  RSVD_HIP(rsvd::launch_fill_i32(B.status, rsvd::kStatusWords, 0, s));
  if ((st = R.bind_A(A, lda))) return st;
  // the l Ritz triplets, recomputed from the seed (no stored sketch)
  if ((st = R.forward(mark, B.Sl, l))) return st;
  float* Ul = B.Pcat;                          // first lp columns of P
  float* Vl = B.N1;
  RSVD_HIP(rsvd::launch_apply(B.Mop, P.ldm, m, l, B.W, lp, lp, lp, false, Ul, P.ldm, P.ldm, s));
  RSVD_HIP(rsvd::launch_apply(B.N0, P.ldn, n, l, B.W2, lp, lp, lp, false, Vl, P.ldn, P.ldn, s));
  if (!(P.opt.flags & RSVD_FLAG_NO_SIGN_FIX))
    RSVD_HIP(rsvd::launch_sign_fix(Ul, P.ldm, m, Vl, P.ldn, n, k, B.signs, s));
  // cotangents, zero-padded to kp columns
  if (gU)
    RSVD_HIP(rsvd::launch_panel_copy(gU, ldgu, m, k, B.gUp, P.ldm, P.ldm, kp, s));
  else
    RSVD_HIP(rsvd::launch_colscale(nullptr, 0, nullptr, 0, nullptr, m, kp, B.gUp, P.ldm, P.ldm, s));
  if (gV)
    RSVD_HIP(rsvd::launch_panel_copy(gV, ldgv, n, k, B.gVp, P.ldn, P.ldn, kp, s));
  else
    RSVD_HIP(rsvd::launch_colscale(nullptr, 0, nullptr, 0, nullptr, n, kp, B.gVp, P.ldn, P.ldn, s));
  // J_u = U_l^T gU, J_v = V_l^T gV (FP64)
  RSVD_HIP(rsvd::launch_xgram(Ul, P.ldm, lp, B.gUp, P.ldm, kp, m, P.gram_rows,
                              rsvd::gram_chunks_for(P, m), B.gpart, B.Ju, s));
  RSVD_HIP(rsvd::launch_xgram(Vl, P.ldn, lp, B.gVp, P.ldn, kp, n, P.gram_rows,
                              rsvd::gram_chunks_for(P, n), B.gpart, B.Jv, s));
  RSVD_HIP(rsvd::launch_adj_core(B.Sl, lp, l, k, kp, B.Ju, B.Jv, gS, B.coreT, B.JuW, B.JvW,
                                 B.sinv, B.status, s));
  float* R1 = B.Rcat;
  float* Vk = B.Rcat + lp * P.ldn;
  float* R3 = B.Rcat + (lp + kp) * P.ldn;
  float* P2 = B.Pcat + lp * P.ldm;
  float* P3 = B.Pcat + (lp + kp) * P.ldm;
  // R1 = V_l core^T
  RSVD_HIP(rsvd::launch_apply(Vl, P.ldn, n, l, B.coreT, lp, lp, lp, false, R1, P.ldn, P.ldn, s));
  // P2 = (gU - U_l J_u) S_k^-1, P3 = U_k S_k^-1
  RSVD_HIP(rsvd::launch_apply(Ul, P.ldm, m, l, B.JuW, kp, kp, kp, false, B.M1, P.ldm, P.ldm, s));
  RSVD_HIP(rsvd::launch_colscale(B.gUp, P.ldm, B.M1, P.ldm, B.sinv, m, kp, P2, P.ldm, P.ldm, s));
  RSVD_HIP(rsvd::launch_colscale(Ul, P.ldm, nullptr, 0, B.sinv, m, kp, P3, P.ldm, P.ldm, s));
  // R3 = gV - V_l J_v, V_k
  RSVD_HIP(rsvd::launch_apply(Vl, P.ldn, n, l, B.JvW, kp, kp, kp, false, B.N0, P.ldn, P.ldn, s));
  RSVD_HIP(rsvd::launch_colscale(B.gVp, P.ldn, B.N0, P.ldn, nullptr, n, kp, R3, P.ldn, P.ldn, s));
  RSVD_HIP(rsvd::launch_colscale(Vl, P.ldn, nullptr, 0, nullptr, n, kp, Vk, P.ldn, P.ldn, s));
  // gA = [U_l | P2 | P3] [R1 | V_k | R3]^T
  RSVD_HIP(rsvd::launch_outer(B.Pcat, P.ldm, B.Rcat, P.ldn, P.rcat, m, n, gA, ldga, s));
  RSVD_HIP(mark(8));
  if (!report) return RSVD_OK;
  return finish_report(h, R, ev, report);
}

rsvd_status rsvd_residual(rsvd_plan_t h, const void* A, int64_t lda, const float* U, int64_t ldu,
                          const double* S, const float* V, int64_t ldv, double* out, void* ws,
                          void* stream) {
  if (rsvd_status st = check_plan(h)) return st;
  if (h->p.csr) return set_err(h, RSVD_E_INVALID_ARG, "this call needs dense A (plan is for CSR)");
  if (h->p.host)
    return set_err(h, RSVD_E_UNSUPPORTED, "this call needs A in device memory (plan is host-resident)");
  if (rsvd_status st = check_A(h, A, lda)) return st;
  if (rsvd_status st = check_ws(h, ws)) return st;
  const rsvd::Plan& P = h->p;
  if (!U || !S || !V || !out || ldu < P.prob.m || ldv < P.prob.n)
    return set_err(h, RSVD_E_INVALID_ARG, "bad residual arguments");
  if (P.prob.dtype == RSVD_BF16)
    return set_err(h, RSVD_E_UNSUPPORTED, "residual of a BF16 A is not implemented");
  hipStream_t s = (hipStream_t)stream;
  Buffers B = carve(P, ws);
  RSVD_HIP(rsvd::launch_residual(A, P.prob.dtype == RSVD_F64, lda, P.prob.m, P.prob.n, U, ldu, S, V,
                                 ldv, P.prob.k, B.gpart, out, s));
  return RSVD_OK;
}

}  // extern "C"
