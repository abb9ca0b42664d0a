"""Pins of the oracle SVD adjoint: finite differences of the oracle forward
pass, torch's independent FP64 SVD autograd, and the closed form of the
sum(w * sigma) + ||A - U S V^T||_F^2 loss."""
import numpy as np
import pytest
import torch

from oracle.adjoint import svd_adjoint
from oracle.rsvd import rsvd


def loss_parts(A, k, p, q, a, b, c, d, w):
    out = rsvd(A, k, p, q, seed=0, full=True)
    U, S, V = out["U"], out["S"], out["V"]
    L = np.sum(c * (a @ U) ** 2) + np.sum(d * (b @ V) ** 2) + np.sum(w * S)
    gU = 2.0 * np.outer(a, c * (a @ U))
    gV = 2.0 * np.outer(b, d * (b @ V))
    return L, out, gU, w.copy(), gV


def test_adjoint_matches_finite_differences():
    rng = np.random.default_rng(100)
    m, n, k = 40, 24, 5
    U0, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V0, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (U0 * np.arange(1, n + 1) ** -0.5) @ V0.T + 1e-4 * rng.standard_normal((m, n))
    a, b = rng.standard_normal(m), rng.standard_normal(n)
    c, d, w = rng.uniform(0.5, 1.5, k), rng.uniform(0.5, 1.5, k), rng.uniform(0, 1, k)
    p = n - k                          # l = n: the forward pass is the exact SVD
    L, out, gU, gS, gV = loss_parts(A, k, p, 2, a, b, c, d, w)
    gA = svd_adjoint(out["Ul"], out["Sl"], out["Vl"], k, gU, gS, gV)
    h = 1e-6 * np.linalg.norm(A)
    for _ in range(6):
        E = rng.standard_normal((m, n))
        Lp = loss_parts(A + h * E, k, p, 2, a, b, c, d, w)[0]
        Lm = loss_parts(A - h * E, k, p, 2, a, b, c, d, w)[0]
        fd = (Lp - Lm) / (2 * h)
        an = float(np.sum(gA * E))
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an))


def test_adjoint_matches_torch_full_svd_autograd():
    rng = np.random.default_rng(3)
    m, n, k = 30, 12, 4
    A = rng.standard_normal((m, n))
    a, b = rng.standard_normal(m), rng.standard_normal(n)
    c, d, w = rng.uniform(0.5, 1.5, k), rng.uniform(0.5, 1.5, k), rng.uniform(0, 1, k)
    At = torch.tensor(A, requires_grad=True)
    U, S, Vh = torch.linalg.svd(At, full_matrices=False)
    Uk, Sk, Vk = U[:, :k], S[:k], Vh[:k].T
    L = (torch.tensor(c) * (torch.tensor(a) @ Uk) ** 2).sum() \
        + (torch.tensor(d) * (torch.tensor(b) @ Vk) ** 2).sum() + (torch.tensor(w) * Sk).sum()
    L.backward()
    _, out, gU, gS, gV = loss_parts(A, k, n - k, 1, a, b, c, d, w)
    gA = svd_adjoint(out["Ul"], out["Sl"], out["Vl"], k, gU, gS, gV)
    assert np.allclose(gA, At.grad.numpy(), rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("p", [4, 20])
def test_closed_form_of_sigma_plus_residual_loss(p):
    # L = sum w_i s_i + ||A - U S V^T||_F^2 composed with the rSVD outputs has
    # gradient U diag(w) V^T + 2 A (I - V V^T) (uses U^T A = S V^T)
    rng = np.random.default_rng(p)
    m, n, k = 50, 30, 6
    A = rng.standard_normal((m, n)) * (np.arange(1, n + 1) ** -0.5)
    w = rng.uniform(0, 1, k)
    out = rsvd(A, k, p, 2, seed=1, full=True)
    U, S, V = out["U"], out["S"], out["V"]
    R = A - (U * S) @ V.T
    gU = -2.0 * R @ V * S
    gS = w - 2.0 * np.einsum("ij,ij->j", U, R @ V)
    gV = -2.0 * R.T @ U * S
    gA = svd_adjoint(out["Ul"], out["Sl"], out["Vl"], k, gU, gS, gV) + 2.0 * R
    ref = (U * w) @ V.T + 2.0 * A @ (np.eye(n) - V @ V.T)
    assert np.allclose(gA, ref, rtol=1e-10, atol=1e-11)
