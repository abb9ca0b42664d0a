"""Adjoint (rsvd_backward) against the FP64 oracle adjoint (itself pinned by
finite differences on the CPU), torch's FP64 SVD autograd, and the closed form
of sum(w s) + ||A - U S V^T||^2; relative error target 1e-4."""
import numpy as np
import pytest
import torch

import workloads
from oracle import metrics
from oracle.adjoint import svd_adjoint
from oracle.rsvd import rsvd as oracle_rsvd
from paper_1907_06470_amd import RSVD, Plan
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def loss_cotangents(U, S, V, a, b, c, d, w):
    """Cotangents of L = sum c_i (a.u_i)^2 + sum d_i (b.v_i)^2 + sum w_i s_i."""
    gU = 2.0 * np.outer(a, c * (a @ U))
    gV = 2.0 * np.outer(b, d * (b @ V))
    return gU, w.copy(), gV


@pytest.mark.parametrize("seed", [100, 101, 102])
def test_backward_matches_oracle_adjoint_on_exact_svd_instances(seed):
    # 256 x 128, sigma_i = i^-1/2 + 1e-4 noise, k = 16, l = n = 128, q = 3:
    # the forward pass is the exact truncated SVD
    dev = need_gpu()
    A = workloads.fd_instance(seed).numpy()
    m, n, k, p, q = 256, 128, 16, 112, 3
    rng = np.random.default_rng(seed)
    a, b = rng.standard_normal(m), rng.standard_normal(n)
    c, d, w = rng.uniform(0.5, 1.5, k), rng.uniform(0.5, 1.5, k), rng.uniform(0, 1, k)
    A32 = A.astype(np.float32)
    ref = oracle_rsvd(A32.astype(np.float64), k, p, q, seed=0, full=True)
    gU, gS, gV = loss_cotangents(ref["U"], ref["S"], ref["V"], a, b, c, d, w)
    gA_ref = svd_adjoint(ref["Ul"], ref["Sl"], ref["Vl"], k, gU, gS, gV)
    plan = Plan(m, n, k, p, q, backward=True)
    Ad = torch.as_tensor(A32, device=dev)
    gA, info = plan.backward(Ad, torch.as_tensor(gU, device=dev), torch.as_tensor(gS, device=dev),
                             torch.as_tensor(gV, device=dev))
    err = rel(gA.cpu().double().numpy(), gA_ref)
    say(f"adjoint seed {seed}: rel err {err:.2e}, status {info['status']}")
    assert err <= GRAD_TOL


def test_backward_partial_cotangents():
    dev = need_gpu()
    A = workloads.fd_instance(103).numpy().astype(np.float32)
    m, n, k, p, q = 256, 128, 16, 112, 3
    ref = oracle_rsvd(A.astype(np.float64), k, p, q, seed=0, full=True)
    w = np.linspace(0.1, 1.0, k)
    gA_ref = svd_adjoint(ref["Ul"], ref["Sl"], ref["Vl"], k, None, w, None)
    plan = Plan(m, n, k, p, q, backward=True)
    gA, _ = plan.backward(torch.as_tensor(A, device=dev), None, torch.as_tensor(w, device=dev), None)
    assert rel(gA.cpu().double().numpy(), gA_ref) <= GRAD_TOL
    # the sigma-only gradient is U diag(w) V^T exactly
    assert rel(gA.cpu().double().numpy(), (ref["U"] * w) @ ref["V"].T) <= GRAD_TOL


def test_backward_matches_torch_full_svd_autograd():
    dev = need_gpu()
    rng = np.random.default_rng(7)
    m, n, k = 90, 40, 6
    A = (rng.standard_normal((m, n)) * np.arange(1, n + 1) ** -0.5).astype(np.float32)
    a, b = rng.standard_normal(m), rng.standard_normal(n)
    c, d, w = rng.uniform(0.5, 1.5, k), rng.uniform(0.5, 1.5, k), rng.uniform(0, 1, k)
    At = torch.tensor(A.astype(np.float64), requires_grad=True)
    Ut, St, Vht = torch.linalg.svd(At, full_matrices=False)
    Uk, Sk, Vk = Ut[:, :k], St[:k], Vht[:k].T
    L = (torch.tensor(c) * (torch.tensor(a) @ Uk) ** 2).sum() \
        + (torch.tensor(d) * (torch.tensor(b) @ Vk) ** 2).sum() + (torch.tensor(w) * Sk).sum()
    L.backward()
    ref_grad = At.grad.numpy()
    # the loss is invariant to the sign of each singular pair, but its cotangents
    # are not: take them from the factors this plan returns
    plan = Plan(m, n, k, n - k, 2, backward=True)
    Ad = torch.as_tensor(A, device=dev)
    U, S, V, _ = plan.factor(Ad)
    Un, Vn = U.cpu().double().numpy(), V.cpu().double().numpy()
    assert np.allclose(np.abs(Un.T @ Uk.detach().numpy()), np.eye(k), atol=1e-4)
    gU, gS, gV = loss_cotangents(Un, S.cpu().numpy(), Vn, a, b, c, d, w)
    gA, _ = plan.backward(Ad, torch.as_tensor(gU, device=dev), torch.as_tensor(gS, device=dev),
                          torch.as_tensor(gV, device=dev))
    assert rel(gA.cpu().double().numpy(), ref_grad) <= GRAD_TOL


@pytest.mark.parametrize("m,n,k,p,q", [(4096, 2048, 64, 16, 3), (3000, 1200, 40, 24, 2),
                                       (140000, 256, 32, 16, 1)])   # tall: staged m-side products
def test_autograd_function_closed_form_of_sigma_plus_residual_loss(m, n, k, p, q):
    # L = sum w_i s_i + ||A - U S V^T||_F^2 through torch autograd; because
    # U^T A = S V^T, dL/dA = U diag(w) V^T + 2 A (I - V V^T)
    dev = need_gpu()
    sigma = workloads.spectrum_pow(min(m, n), 0.5)
    A0 = workloads.dense_lowrank(m, n, sigma, 1e-4, seed=5, out_dtype=torch.float32)
    w = torch.as_tensor(np.random.default_rng(7).uniform(0, 1, k), device=dev)
    A = A0.to(dev).requires_grad_(True)
    U, S, V = RSVD.apply(A, k, p, q, 0, "fp32")
    R = A - (U * S.float()) @ V.T
    L = (w * S).sum() + (R.double() ** 2).sum()
    L.backward()
    Un, Vn, An = U.detach().double().cpu().numpy(), V.detach().double().cpu().numpy(), A0.double().numpy()
    ref = (Un * w.cpu().numpy()) @ Vn.T + 2.0 * (An - (An @ Vn) @ Vn.T)
    err = rel(A.grad.double().cpu().numpy(), ref)
    say(f"closed form {m}x{n}: rel err {err:.2e}")
    assert err <= GRAD_TOL


def test_backward_rejects_plan_without_backward_flag():
    dev = need_gpu()
    from paper_1907_06470_amd import _lib as L
    plan = Plan(200, 100, 5, 5, 1)
    with pytest.raises(L.RsvdError) as e:
        plan.backward(torch.randn(200, 100, device=dev), None, None, None)
    assert e.value.status == L.E_INVALID_ARG


def test_residual_matches_direct_fp64():
    dev = need_gpu()
    A, meta = workloads.make("plain_gpu", scale=0.1)
    plan = Plan(A.shape[0], A.shape[1], 50, 10, 2)
    Ad = A.to(dev)
    U, S, V, _ = plan.factor(Ad)
    r = plan.residual(Ad, U, S, V).item()
    ref = metrics.residual_fro(A.double().numpy(), U.cpu().double().numpy(), S.cpu().numpy(),
                               V.cpu().double().numpy())
    assert abs(r - ref) <= 1e-5 * ref


@pytest.mark.parametrize("precision,m,n,k,p,q", [
    ("fp32", 8192, 4096, 128, 32, 3),   # widths of the mixed-precision workload (l = 160)
    ("bf16", 8192, 4096, 128, 32, 3),
    ("fp8", 8192, 4096, 128, 32, 3),
    ("fp32", 3000, 2000, 200, 30, 2),   # wide sketch, l = 230
])
def test_closed_form_after_each_forward_form(precision, m, n, k, p, q):
    """The closed form of sum(w s) + ||A - U S V^T||^2 holds exactly when
    U^T A = S V^T.  The FP32 form meets that to rounding; the BF16 and FP8
    forms only to their operand rounding (their Ritz triplets are those of
    the rounded projection).  So the gradient is held to 1e-4 plus twice the
    measured relative departure of U^T A from S V^T."""
    dev = need_gpu()
    sigma = workloads.spectrum_pow(min(m, n), 0.5)
    A0 = workloads.dense_lowrank(m, n, sigma, 1e-4, seed=5, out_dtype=torch.float32)
    w = torch.as_tensor(np.random.default_rng(7).uniform(0, 1, k), device=dev)
    A = A0.to(dev).requires_grad_(True)
    U, S, V = RSVD.apply(A, k, p, q, 0, precision)
    R = A - (U * S.float()) @ V.T
    L = (w * S).sum() + (R.double() ** 2).sum()
    L.backward()
    Un, Vn, An = U.detach().double().cpu().numpy(), V.detach().double().cpu().numpy(), A0.double().numpy()
    Sn = S.detach().cpu().numpy()
    ref = (Un * w.cpu().numpy()) @ Vn.T + 2.0 * (An - (An @ Vn) @ Vn.T)
    err = rel(A.grad.double().cpu().numpy(), ref)
    dep = float(np.linalg.norm(Un.T @ An - Sn[:, None] * Vn.T) / np.linalg.norm(Sn))
    say(f"closed form {precision} {m}x{n} l={k + p}: rel err {err:.2e}, |U^T A - S V^T| / |S| {dep:.1e}")
    assert err <= GRAD_TOL + 2.0 * dep
    if precision == "fp32":
        assert err <= GRAD_TOL
