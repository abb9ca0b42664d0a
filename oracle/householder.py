"""Thin QR by Householder reflections, FP64 (Section 2.1, steps 3-4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps 3-4 of the randomized SVD take a QR decomposition Y = QR of the m x r
sketch and keep the first r columns of Q.  (The printed sizes of Q and R are
garbled; the thin factorisation Q: m x r with orthonormal columns, R: r x r
upper triangular, is what the steps use.)  This module computes it the
textbook way (Golub & Van Loan, Householder QR): column by column, reflect the
trailing part of the column onto a multiple of e_1, then form the thin Q by
applying the reflectors to the first r columns of the identity in reverse.

Parity pins (tests/test_oracle_linalg.py): Q^T Q = I and Q R = Y to 1e-14,
R upper triangular, |diag R| and Q (up to column signs) equal LAPACK's
(numpy.linalg.qr), and exact results on matrices whose QR is known in closed
form (orthonormal columns times a triangular factor).
"""

import numpy as np


def householder_qr(Y):
    """Thin QR of an m x r FP64 matrix (m >= r).  Returns (Q, R)."""
    A = np.array(Y, dtype=np.float64, copy=True)
    m, r = A.shape
    if m < r:
        raise ValueError("householder_qr needs m >= r")
    vs = []
    for k in range(r):
        x = A[k:, k]
        alpha = np.linalg.norm(x)
        v = x.copy()
        if alpha == 0.0:
            vs.append(None)      # column already zero below the diagonal
            continue
        # v = x + sign(x_0) * ||x|| e_1 avoids cancellation
        s = 1.0 if x[0] >= 0.0 else -1.0
        v[0] += s * alpha
        vnorm2 = v @ v
        # apply H = I - 2 v v^T / (v^T v) to the trailing columns
        A[k:, k:] -= np.outer(v, (2.0 / vnorm2) * (v @ A[k:, k:]))
        vs.append((v, vnorm2))
    R = np.triu(A[:r, :r])
    Q = np.zeros((m, r), dtype=np.float64)
    Q[np.arange(r), np.arange(r)] = 1.0
    for k in range(r - 1, -1, -1):
        if vs[k] is None:
            continue
        v, vnorm2 = vs[k]
        Q[k:, :] -= np.outer(v, (2.0 / vnorm2) * (v @ Q[k:, :]))
    return Q, R
