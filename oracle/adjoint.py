"""Adjoint (reverse-mode derivative) of the truncated SVD, plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no derivative; this is the backward pass of the randomized SVD
treated as if its l Ritz triplets (U_l, S_l, V_l) were exact singular
triplets of A.  With cotangents gU (m x k), gS (k), gV (n x k) zero-padded to
l columns, skew(X) = X - X^T and F_ij = 1 / (s_j^2 - s_i^2) (i != j),
F_ii = 0:

  gA = U_l [ (F o skew(U_l^T gU)) S_l + S_l (F o skew(V_l^T gV)) + diag(gS) ] V_l^T
       + (I - U_l U_l^T) gU S_k^-1 V_k^T
       + U_k S_k^-1 gV^T (I - V_l V_l^T)

the standard real-SVD adjoint (Townsend 2016; Ionescu et al. 2015), written
here from its derivation.  Ties: F_ij = 0 when |s_i^2 - s_j^2| <= 1e-12 s_1^2;
1/s_i = 0 when s_i <= 1e-12 s_1.

When l = min(m, n), or rank A <= l, the Ritz triplets are the exact SVD and
this is the exact derivative.

Parity pins (tests/test_oracle_adjoint.py): central finite differences of the
oracle's forward pass on instances with l = n (where the forward pass is the
exact truncated SVD), and the closed form gA = U diag(w) V^T + 2 (A - A_k) of
the loss sum w_i s_i + ||A - U S V^T||_F^2.
"""

import numpy as np

TIE_REL = 1e-12


def svd_adjoint(Ul, Sl, Vl, k, gU=None, gS=None, gV=None):
    Ul = np.asarray(Ul, np.float64)
    Vl = np.asarray(Vl, np.float64)
    Sl = np.asarray(Sl, np.float64)
    m, l = Ul.shape
    n = Vl.shape[0]
    gUp = np.zeros((m, l))
    gVp = np.zeros((n, l))
    gSp = np.zeros(l)
    if gU is not None:
        gUp[:, :k] = gU
    if gS is not None:
        gSp[:k] = gS
    if gV is not None:
        gVp[:, :k] = gV
    s2 = Sl * Sl
    diff = s2[None, :] - s2[:, None]                      # s_j^2 - s_i^2
    tie = np.abs(diff) <= TIE_REL * s2.max()
    F = np.zeros((l, l))
    F[~tie] = 1.0 / diff[~tie]
    np.fill_diagonal(F, 0.0)
    sinv = np.zeros(l)
    big = Sl > TIE_REL * Sl.max()
    sinv[big] = 1.0 / Sl[big]
    Ju = Ul.T @ gUp
    Jv = Vl.T @ gVp
    core = (F * (Ju - Ju.T)) * Sl[None, :] + Sl[:, None] * (F * (Jv - Jv.T)) + np.diag(gSp)
    gA = Ul @ core @ Vl.T
    gA += (gUp - Ul @ (Ul.T @ gUp)) * sinv[None, :] @ Vl.T
    gA += (Ul * sinv[None, :]) @ (gVp.T - (gVp.T @ Vl) @ Vl.T)
    return gA
