"""Randomized SVD with power iteration, plain FP64 (Sections 2.1 and 2.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The oracle computes, in FP64 and without any blocking, the randomized SVD of
Section 2.1 (steps 1-7) applied to the power matrix A_q = (A A^T)^q A of
Section 2.2, Eq. (1), evaluated right to left as Eq. (2) prescribes (start
with A O, never form A A^T).  Readings taken where the paper is silent:

* Oversampling: the sketch has l = k + p columns and the result keeps k
  (p = 0 is the paper's algorithm with r = k).
* Orthonormalisation inside the power iteration: Eq. (2) applies the power
  matrix to O as written; in floating point the columns of (A A^T)^q A O
  collapse onto the top singular vector, so the default schedule ("each")
  re-orthonormalises after every product with A or A^T (the subspace
  iteration of Halko, Martinsson & Tropp, Alg. 4.4).  In exact arithmetic
  every schedule spans the same subspace, so the results coincide; the
  paper's schedule is available as ortho="final_only" for checking that.
* Step 6 is computed from B^T = A^T Q (the paper also forms A^T Q_r and
  transposes, Section 4.1 stage list): QR of B^T, then a one-sided Jacobi SVD
  of the small triangular factor.
* Signs: for each i, the entry of largest magnitude of V[:, i] (lowest row
  index on ties) is made positive, negating U[:, i] with it.

Parity pins (tests/test_oracle_rsvd.py): exact recovery of rank <= l inputs
(sigma to 1e-12 relative, A V = U S), l = min(m, n) reproduces the full SVD
(LAPACK and brute-force Jacobi), interlacing sigma_i(Q^T A) <= sigma_i(A),
U^T A = S V^T to 1e-13, Eckart-Young, the power-matrix identity
sigma(A_q) = sigma(A)^(2q+1) with the same singular vectors (Section 2.2), and
agreement of the "each" and "final_only" schedules on well-conditioned cases.
"""

import time

import numpy as np

from . import philox
from .householder import householder_qr
from .jacobi import one_sided_jacobi, sort_desc


def _check(m, n, k, p, q):
    if k < 1 or p < 0 or q < 0:
        raise ValueError("need k >= 1, p >= 0, q >= 0")
    if k + p > min(m, n):
        raise ValueError("need k + p <= min(m, n)")


def _orth(Y):
    Q, _ = householder_qr(Y)
    return Q


class _Clock:
    """Wall time per stage, recorded into `times` (a dict) when one is given;
    it only reads the clock between the steps."""

    def __init__(self, times):
        self.times = times
        self.t = time.perf_counter()

    def lap(self, name):
        if self.times is None:
            return
        now = time.perf_counter()
        self.times[name] = self.times.get(name, 0.0) + (now - self.t)
        self.t = now


def range_finder(A, l, q, seed, ortho="each", times=None):
    """Orthonormal basis Q (m x l) of the range of (A A^T)^q A O.

    Section 2.1 steps 1-4 on the power matrix of Section 2.2 Eq. (2).
    A may be a dense FP64 array or any object with @ and .T (scipy sparse).
    times: optional dict receiving the wall time of the stages (omega,
    sketch, orth, power).
    """
    m, n = A.shape
    clk = _Clock(times)
    O = philox.omega(seed, n, l)                 # step 1
    clk.lap("omega")
    Y = np.asarray(A @ O, dtype=np.float64)      # step 2 (right-most product)
    clk.lap("sketch")
    if ortho == "each":
        Q = _orth(Y)                             # steps 3-4
        clk.lap("orth")
        for _ in range(q):                       # Eq. (2), right to left
            W = np.asarray(A.T @ Q, dtype=np.float64)
            Qw = _orth(W)
            Y = np.asarray(A @ Qw, dtype=np.float64)
            Q = _orth(Y)
        clk.lap("power")
    elif ortho == "final_only":
        for _ in range(q):
            Y = np.asarray(A @ np.asarray(A.T @ Y, dtype=np.float64), dtype=np.float64)
        clk.lap("power")
        Q = _orth(Y)
        clk.lap("orth")
    else:
        raise ValueError("ortho must be 'each' or 'final_only'")
    return Q


def small_svd(Bt):
    """SVD of B = Bt^T (l x n) from Bt (n x l): returns (Ub, s, Vfull),
    B = Ub diag(s) Vfull^T, sorted descending (Section 2.1, step 6)."""
    Qb, Rb = householder_qr(Bt)                  # Bt = Qb Rb, so B = Rb^T Qb^T
    Ut, s, X, _ = one_sided_jacobi(Rb.T)         # Rb^T = Ut diag(s) X^T
    order = sort_desc(s)
    Ut, s, X = Ut[:, order], s[order], X[:, order]
    return Ut, s, Qb @ X


def sign_fix(U, V):
    """Make the largest-magnitude entry of each V column positive (lowest
    index on ties), flipping the matching U column."""
    U = U.copy()
    V = V.copy()
    for i in range(V.shape[1]):
        j = int(np.argmax(np.abs(V[:, i])))      # argmax returns the lowest index
        if V[j, i] < 0.0:
            U[:, i] = -U[:, i]
            V[:, i] = -V[:, i]
    return U, V


def rsvd(A, k, p, q, seed=0, ortho="each", signs=True, full=False, times=None):
    """Rank-k randomized SVD of A with oversampling p and q power steps.

    Returns dict with U (m x k), S (k,), V (n x k); with full=True also the
    range basis Q (m x l), B^T (n x l) and all l Ritz triplets
    (Ul, Sl, Vl).  times: optional dict that receives the wall time of each
    stage (omega, sketch, orth, power, projection, svd0, post), in seconds.
    """
    m, n = A.shape
    _check(m, n, k, p, q)
    l = k + p
    Q = range_finder(A, l, q, seed, ortho=ortho, times=times)
    clk = _Clock(times)
    Bt = np.asarray(A.T @ Q, dtype=np.float64)   # step 5 as B^T = A^T Q
    clk.lap("projection")
    Ub, s, Vf = small_svd(Bt)                    # step 6
    clk.lap("svd0")
    Ul = Q @ Ub                                  # step 7
    if signs:
        Ul, Vf = sign_fix(Ul, Vf)
    clk.lap("post")
    out = {"U": Ul[:, :k].copy(), "S": s[:k].copy(), "V": Vf[:, :k].copy()}
    if full:
        out.update({"Q": Q, "Bt": Bt, "Ul": Ul, "Sl": s, "Vl": Vf})
    return out


def rsvd_auto_q(A, k, p, q_max, tol=1e-4, seed=0):
    """Randomized SVD with the iteration parameter chosen automatically
    (Section 2.2: the decay of the singular values is measured for increasing
    q and q stops growing once accuracy no longer improves).

    Reading taken: after t power steps the projection B_t^T = A^T Q_t gives
    the singular values s^(t) the factorisation returns with q = t; the first
    t >= 1 with max_{i<k} |s_i^(t) - s_i^(t-1)| / s_i^(t) <= tol is chosen
    (q_max if none).  Returns the rsvd() dict for that q plus "q_used" and
    "deltas" (the relative changes, one per t >= 1).
    """
    m, n = A.shape
    _check(m, n, k, p, q_max)
    l = k + p
    O = philox.omega(seed, n, l)
    Q = _orth(np.asarray(A @ O, dtype=np.float64))
    prev, deltas = None, []
    t = 0
    while True:
        Bt = np.asarray(A.T @ Q, dtype=np.float64)
        Ub, s, Vf = small_svd(Bt)
        if prev is not None:
            sk, pk = s[:k], prev[:k]
            rel = np.where(sk > 0, np.abs(sk - pk) / np.where(sk > 0, sk, 1.0),
                           np.where(pk != 0, 1.0, 0.0))
            deltas.append(float(np.max(rel)))
        if t == q_max or (deltas and deltas[-1] <= tol):
            break
        prev = s
        Qw = _orth(Bt)
        Q = _orth(np.asarray(A @ Qw, dtype=np.float64))
        t += 1
    Ul, Vf = sign_fix(Q @ Ub, Vf)
    return {"U": Ul[:, :k].copy(), "S": s[:k].copy(), "V": Vf[:, :k].copy(), "q_used": t,
            "deltas": deltas}
