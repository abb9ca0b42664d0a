"""One-sided (Hestenes) Jacobi SVD in FP64 (Section 2.1, step 6).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Step 6 needs an SVD of the small matrix B.  The paper uses the QR-based SVD of
Golub & Van Loan; any correct SVD computes the same factors up to signs and the
basis inside repeated singular values, so the oracle takes the plainest
algorithm that is accurate to the last bits: one-sided Jacobi.  Columns i < j
of the working matrix W are rotated in the (i, j) plane so that they become
orthogonal; the rotation is the Jacobi rotation that diagonalises the 2 x 2
Gram matrix [[a, g], [g, b]] of the pair (a = |w_i|^2, b = |w_j|^2,
g = w_i . w_j); sweeps repeat until every pair satisfies |g| <= tol*sqrt(a b).
The accumulated rotations X give W = M X with orthogonal columns, so
M = U diag(s) X^T with s_i = |W_i| and U_i = W_i / s_i.

Parity pins (tests/test_oracle_linalg.py): singular values against LAPACK
(numpy.linalg.svd) on random matrices of sizes 1..64, the closed form of 2 x 2
matrices, exact values for diagonal and signed-permutation matrices,
orthogonality of U and X, and M = U diag(s) X^T.
"""

import numpy as np


def one_sided_jacobi(M, tol=1e-15, max_sweeps=60):
    """SVD of an r x c FP64 matrix with r >= c by one-sided Jacobi.

    Returns (U, s, X, sweeps): U r x c, s (c,) unsorted, X c x c orthogonal,
    M = U diag(s) X^T.  Columns with s = 0 give a zero column in U.
    """
    W = np.array(M, dtype=np.float64, copy=True)
    r, c = W.shape
    if r < c:
        raise ValueError("one_sided_jacobi needs rows >= cols")
    X = np.eye(c)
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        rotated = False
        for i in range(c - 1):
            for j in range(i + 1, c):
                a = W[:, i] @ W[:, i]
                b = W[:, j] @ W[:, j]
                g = W[:, i] @ W[:, j]
                if g == 0.0 or abs(g) <= tol * np.sqrt(a * b):
                    continue
                rotated = True
                zeta = (b - a) / (2.0 * g)
                t = (1.0 if zeta >= 0.0 else -1.0) / (abs(zeta) + np.sqrt(1.0 + zeta * zeta))
                cs = 1.0 / np.sqrt(1.0 + t * t)
                sn = cs * t
                wi = W[:, i].copy()
                W[:, i] = cs * wi - sn * W[:, j]
                W[:, j] = sn * wi + cs * W[:, j]
                xi = X[:, i].copy()
                X[:, i] = cs * xi - sn * X[:, j]
                X[:, j] = sn * xi + cs * X[:, j]
        if not rotated:
            break
    s = np.sqrt(np.einsum("ij,ij->j", W, W))
    U = np.zeros_like(W)
    nz = s > 0.0
    U[:, nz] = W[:, nz] / s[nz]
    return U, s, X, sweeps


def sort_desc(s):
    """Indices that sort s descending, ties kept in index order (stable)."""
    return np.argsort(-np.asarray(s), kind="stable")


def jacobi_svd(M, tol=1e-15):
    """Thin SVD of any FP64 matrix by one-sided Jacobi, sorted descending.

    Returns (U, s, V) with M = U diag(s) V^T, U: r x p, V: c x p,
    p = min(r, c).
    """
    M = np.asarray(M, dtype=np.float64)
    if M.shape[0] >= M.shape[1]:
        U, s, V, _ = one_sided_jacobi(M, tol=tol)
    else:
        V, s, U, _ = one_sided_jacobi(M.T, tol=tol)
    order = sort_desc(s)
    return U[:, order], s[order], V[:, order]
