"""Accuracy measures used to compare a computed SVD with the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* sigma_err: max_i<=k |s_hat_i - s_i| / max(s_i, floor * s_1).
* sin_theta: largest principal angle sine between two bases,
  ||(I - U U^T) U_hat||_2, from the smallest singular value of U^T U_hat.
* residual_fro: ||A - U diag(S) V^T||_F accumulated in FP64 over row blocks
  (direct, no ||A||^2 - sum s^2 cancellation).
"""

import numpy as np


def sigma_err(s_hat, s_ref, k=None, floor=1e-6):
    s_hat = np.asarray(s_hat, dtype=np.float64)
    s_ref = np.asarray(s_ref, dtype=np.float64)
    if k is None:
        k = min(len(s_hat), len(s_ref))
    s_hat, s_ref = s_hat[:k], s_ref[:k]
    den = np.maximum(np.abs(s_ref), floor * np.abs(s_ref).max())
    return float(np.max(np.abs(s_hat - s_ref) / den))


def _orthonormalize(U):
    q, _ = np.linalg.qr(np.asarray(U, dtype=np.float64))
    return q


def sin_theta(U_ref, U_hat):
    """sin of the largest principal angle between span(U_ref) and
    span(U_hat): the 2-norm of the part of U_hat outside span(U_ref)
    (computed directly, not as sqrt(1 - cos^2), which cancels)."""
    a = _orthonormalize(U_ref)
    b = _orthonormalize(U_hat)
    resid = b - a @ (a.T @ b)
    if resid.size == 0:
        return 0.0
    return float(min(1.0, np.linalg.norm(resid, 2)))


def residual_fro(A, U, S, V, block=4096):
    U = np.asarray(U, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    m = A.shape[0]
    tot = 0.0
    for i0 in range(0, m, block):
        i1 = min(m, i0 + block)
        Ablk = A[i0:i1]
        if hasattr(Ablk, "toarray"):
            Ablk = Ablk.toarray()
        R = np.asarray(Ablk, dtype=np.float64) - (U[i0:i1] * S) @ V.T
        tot += float(np.einsum("ij,ij->", R, R))
    return float(np.sqrt(tot))


def orth_err(U):
    U = np.asarray(U, dtype=np.float64)
    return float(np.max(np.abs(U.T @ U - np.eye(U.shape[1]))))


def align_signs(U_ref, U_hat, *others):
    """Flip columns of U_hat (and of each matrix in others) to match the
    sign of U_ref column-wise (by the sign of the column dot product)."""
    d = np.sign(np.einsum("ij,ij->j", np.asarray(U_ref, np.float64),
                          np.asarray(U_hat, np.float64)))
    d[d == 0] = 1.0
    return (np.asarray(U_hat) * d,) + tuple(np.asarray(o) * d for o in others)
