"""Pins of the oracle's Householder QR (Section 2.1, steps 3-4) and one-sided
Jacobi SVD (Section 2.1, step 6) against LAPACK and closed forms."""
import numpy as np
import pytest

from oracle.householder import householder_qr
from oracle.jacobi import jacobi_svd, one_sided_jacobi, sort_desc


@pytest.mark.parametrize("m,r", [(1, 1), (5, 3), (40, 40), (200, 17), (513, 64)])
def test_householder_against_lapack(m, r):
    rng = np.random.default_rng(m * 100 + r)
    Y = rng.standard_normal((m, r))
    Q, R = householder_qr(Y)
    assert Q.shape == (m, r) and R.shape == (r, r)
    assert np.allclose(np.tril(R, -1), 0.0)
    assert np.max(np.abs(Q.T @ Q - np.eye(r))) < 1e-14 * max(1, r)
    assert np.max(np.abs(Q @ R - Y)) < 1e-14 * np.abs(Y).max() * r
    Ql, Rl = np.linalg.qr(Y)
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rl)), rtol=1e-12)
    d = np.sign(np.diag(R)) * np.sign(np.diag(Rl))
    assert np.allclose(Q * d, Ql, atol=1e-12)


def test_householder_known_factorisation():
    # Y = Q0 R0 with Q0 orthonormal columns and R0 upper triangular, positive diagonal
    rng = np.random.default_rng(1)
    Q0, _ = np.linalg.qr(rng.standard_normal((30, 6)))
    R0 = np.triu(rng.uniform(0.5, 2.0, (6, 6)))
    Q, R = householder_qr(Q0 @ R0)
    d = np.sign(np.diag(R))
    assert np.allclose(d[:, None] * R, R0, atol=1e-13)
    assert np.allclose(Q * d, Q0, atol=1e-13)


def test_householder_rank_deficient_still_orthonormal():
    rng = np.random.default_rng(2)
    B = rng.standard_normal((50, 3))
    Y = B @ rng.standard_normal((3, 8))       # rank 3, 8 columns
    Q, R = householder_qr(Y)
    assert np.max(np.abs(Q.T @ Q - np.eye(8))) < 1e-13
    assert np.max(np.abs(Q @ R - Y)) < 1e-12


@pytest.mark.parametrize("r,c", [(1, 1), (2, 2), (7, 3), (16, 16), (64, 40), (64, 64)])
def test_jacobi_against_lapack(r, c):
    rng = np.random.default_rng(r * 7 + c)
    M = rng.standard_normal((r, c))
    U, s, V = jacobi_svd(M)
    sl = np.linalg.svd(M, compute_uv=False)
    assert np.allclose(s, sl, rtol=1e-13, atol=1e-14 * sl[0])
    assert np.max(np.abs(U.T @ U - np.eye(c))) < 1e-13
    assert np.max(np.abs(V.T @ V - np.eye(c))) < 1e-13
    assert np.max(np.abs((U * s) @ V.T - M)) < 1e-13 * max(1.0, sl[0])


def test_jacobi_wide_matrix():
    rng = np.random.default_rng(5)
    M = rng.standard_normal((4, 9))
    U, s, V = jacobi_svd(M)
    assert np.allclose(s, np.linalg.svd(M, compute_uv=False), rtol=1e-13)
    assert np.max(np.abs((U * s) @ V.T - M)) < 1e-13


def test_jacobi_2x2_closed_form():
    # singular values of [[a, b], [0, d]]: s1*s2 = |a d|, s1^2 + s2^2 = a^2 + b^2 + d^2
    for a, b, d in [(3.0, 4.0, 5.0), (1.0, 1e-8, 1.0), (2.0, -7.0, 0.5)]:
        _, s, _ = jacobi_svd(np.array([[a, b], [0.0, d]]))
        t = a * a + b * b + d * d
        disc = np.sqrt(t * t - 4.0 * (a * d) ** 2)
        ref = np.sqrt(np.array([(t + disc) / 2.0, (t - disc) / 2.0]))
        assert np.allclose(s, ref, rtol=1e-14)


def test_jacobi_diagonal_and_signed_permutation():
    D = np.diag([3.0, -1.0, 7.0, 0.5])
    P = np.eye(4)[[2, 0, 3, 1]]
    for M in (D, P @ D, D @ P.T, P @ D @ P.T):
        _, s, _ = jacobi_svd(M)
        assert np.array_equal(s, np.array([7.0, 3.0, 1.0, 0.5]))


def test_jacobi_zero_column_and_ties():
    M = np.zeros((5, 3))
    M[0, 0] = 2.0
    M[1, 2] = 2.0
    U, s, X, _ = one_sided_jacobi(M)
    assert np.array_equal(np.sort(s)[::-1], np.array([2.0, 2.0, 0.0]))
    order = sort_desc(s)
    assert list(order) == [0, 2, 1]      # stable on the tie 2.0 = 2.0
