"""BF16 form: products with A and the panel rounded to BF16 (nearest even) and
accumulated in FP32, checked against the FP64 product of the same rounded
operands; end to end against the FP64 oracle at the stated BF16 target
(sigma relative error <= 1e-3)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import metrics
from oracle.rsvd import rsvd as oracle_rsvd
from paper_1907_06470_amd import Plan
from tests.gpu_util import col_major_from_numpy, gamma_bound, need_gpu, rand_panel, say

pytestmark = pytest.mark.gpu

SIGMA_TOL_BF16 = 1e-3


def bf16_round(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("m,n,l,tile", [
    (1000, 700, 20, (256, 192)),
    (777, 1234, 70, (0, 0)),
    (300, 260, 190, (96, 64)),
    (513, 2049, 128, (512, 1024)),
    (1000, 1024, 120, (256, 320)),
    (520, 2080, 128, (224, 416)),
    (33, 5000, 3, (32, 4096)),
    (700, 800, 230, (256, 256)),    # lp = 256: two slices of the direct-to-LDS width 128
    (500, 640, 330, (0, 0)),        # lp = 352
])
def test_bf16_products_within_rounding_bound(m, n, l, tile):
    dev = need_gpu()
    say("bf16 product", m, n, l, tile)
    k = max(1, l // 2)
    plan = Plan(m, n, k, l - k, 1, precision="bf16", tile=tile)
    rng = np.random.default_rng(m * 3 + n + l)
    A = rng.standard_normal((m, n)).astype(np.float32)
    Ad = torch.as_tensor(A, device=dev)
    Ab = bf16_round(A)
    X = rand_panel(n, l, 1)
    Y = plan.step_product(0, Ad, col_major_from_numpy(X, dev)).cpu().numpy()
    Xb = bf16_round(X)
    ref = Ab @ Xb
    assert np.all(np.abs(Y - ref) <= gamma_bound(n, np.abs(Ab) @ np.abs(Xb)) + 1e-30)
    Qp = rand_panel(m, l, 2)
    Z = plan.step_product(1, Ad, col_major_from_numpy(Qp, dev)).cpu().numpy()
    Qb = bf16_round(Qp)
    ref = Ab.T @ Qb
    assert np.all(np.abs(Z - ref) <= gamma_bound(m, np.abs(Ab).T @ np.abs(Qb)) + 1e-30)


def test_bf16_product_from_bf16_storage():
    dev = need_gpu()
    m, n, l = 600, 512, 40
    A = np.random.default_rng(5).standard_normal((m, n)).astype(np.float32)
    A16 = torch.as_tensor(A).to(torch.bfloat16).to(dev)
    plan = Plan(m, n, 20, 20, 1, dtype=torch.bfloat16, precision="bf16", tile=(128, 128))
    X = rand_panel(n, l, 3)
    Y = plan.step_product(0, A16, col_major_from_numpy(X, dev)).cpu().numpy()
    Ab, Xb = bf16_round(A), bf16_round(X)
    assert np.all(np.abs(Y - Ab @ Xb) <= gamma_bound(n, np.abs(Ab) @ np.abs(Xb)) + 1e-30)


@pytest.mark.parametrize("m,n,l,tile", [
    (1000, 1024, 120, (256, 320)),   # ragged row block of A X; partial last slab of each Aᵀ Q tile
    (520, 2080, 128, (224, 416)),    # Aᵀ Q column block of 32; A X tiles end in a partial slab
    (257, 4096, 100, (0, 0)),        # one row past a block; m not a multiple of 8 (Aᵀ Q other form)
    (128, 160, 128, (32, 32)),       # tiles shallower than one slab
    (136, 224, 120, (64, 96)),       # one partial row block; a whole slab plus a tail per tile
    # width 160 (three-stage ring, six-step loop and its remainders)
    (1000, 1024, 150, (256, 320)),
    (520, 2080, 160, (224, 416)),
    (257, 4096, 140, (0, 0)),
    (160, 192, 160, (32, 32)),
    (176, 224, 150, (64, 96)),
    (640, 3000, 160, (384, 1472)),   # 23 whole slabs per A X tile, 6 per Aᵀ Q tile
])
def test_bf16_products_from_bf16_storage_direct_widths(m, n, l, tile):
    """Panel widths 128 and 160 with BF16-stored A (the direct-to-LDS product
    kernels) against the FP64 product of the same operands, within the FP32
    summation bound."""
    dev = need_gpu()
    say("bf16 width-128 products", m, n, l, tile)
    k = max(1, l - 20)
    rng = np.random.default_rng(m + 7 * n + l)
    A = rng.standard_normal((m, n)).astype(np.float32)
    A16 = torch.as_tensor(A).to(torch.bfloat16).to(dev)
    plan = Plan(m, n, k, l - k, 1, dtype=torch.bfloat16, precision="bf16", tile=tile)
    Ab = bf16_round(A)
    X = rand_panel(n, l, 4)
    Y = plan.step_product(0, A16, col_major_from_numpy(X, dev)).cpu().numpy()
    Xb = bf16_round(X)
    assert np.all(np.abs(Y - Ab @ Xb) <= gamma_bound(n, np.abs(Ab) @ np.abs(Xb)) + 1e-30)
    Qp = rand_panel(m, l, 5)
    Z = plan.step_product(1, A16, col_major_from_numpy(Qp, dev)).cpu().numpy()
    Qb = bf16_round(Qp)
    assert np.all(np.abs(Z - Ab.T @ Qb) <= gamma_bound(m, np.abs(Ab).T @ np.abs(Qb)) + 1e-30)


def factor_vs_oracle(A_host, k, p, q, tile=None, dtype=torch.float32, precision="bf16"):
    dev = need_gpu()
    m, n = A_host.shape
    A = torch.as_tensor(A_host, dtype=dtype).to(dev)
    plan = Plan(m, n, k, p, q, dtype=dtype, precision=precision, tile=tile)
    U, S, V, info = plan.factor(A)
    S, U, V = S.cpu().numpy(), U.cpu().double().numpy(), V.cpu().double().numpy()
    Aref = A.cpu().double().numpy()
    ref = oracle_rsvd(Aref, k, p, q, seed=0)
    err = metrics.sigma_err(S, ref["S"])
    say(f"bf16 m={m} n={n} k={k}: sigma err {err:.2e}, sin U {metrics.sin_theta(ref['U'], U):.1e}, "
        f"{info['total_ms']:.2f} ms")
    assert err <= SIGMA_TOL_BF16
    assert metrics.orth_err(U) < 1e-5
    return err


def test_bf16_plain_small_workload():
    A, meta = workloads.make("plain_small", out_dtype=torch.float32)
    factor_vs_oracle(A.numpy(), meta["k"], meta["p"], meta["q"])


def test_bf16_scaled_plain_gpu_workload():
    A, meta = workloads.make("plain_gpu", scale=0.2)
    factor_vs_oracle(A.numpy(), meta["k"], meta["p"], meta["q"], tile=(1024, 1024))


def test_bf16_from_fp64_input_and_ragged_tiles():
    sigma = workloads.spectrum_pow(600, 1.0)
    A = workloads.dense_lowrank(1500, 900, sigma, 1e-4, seed=21, out_dtype=torch.float64).numpy()
    factor_vs_oracle(A, 15, 10, 2, tile=(256, 160), dtype=torch.float64)


def test_mixed_precision_per_pass():
    # BF16 sketch and power steps, FP32 projection
    dev = need_gpu()
    A, meta = workloads.make("plain_gpu", scale=0.1)
    m, n = A.shape
    from paper_1907_06470_amd import _lib as L
    import ctypes
    prob = L.Problem(m=m, n=n, k=50, p=10, q=2, format=L.DENSE, dtype=L.F32, loc=L.LOC_DEVICE, seed=0)
    opt = L.Options(prec_sketch=L.BF16, prec_power=L.BF16, prec_project=L.F32, ortho=0,
                    tile_m=512, tile_n=512, grid_p=1, grid_q=1)
    h, ws = ctypes.c_void_p(), ctypes.c_size_t()
    assert L.lib().rsvd_plan(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(h), ctypes.byref(ws)) == 0
    Ad = A.to(dev)
    wsb = torch.empty(ws.value, dtype=torch.uint8, device=dev)
    U = torch.empty(50, m, device=dev)
    S = torch.empty(50, dtype=torch.float64, device=dev)
    V = torch.empty(50, n, device=dev)
    rep = L.Report()
    st = L.lib().rsvd_factor(h, ctypes.c_void_p(Ad.data_ptr()), n, ctypes.c_void_p(wsb.data_ptr()),
                             ctypes.c_void_p(U.data_ptr()), m, ctypes.c_void_p(S.data_ptr()),
                             ctypes.c_void_p(V.data_ptr()), n, None, ctypes.byref(rep))
    L.lib().rsvd_plan_destroy(h)
    assert st >= 0
    ref = oracle_rsvd(A.double().numpy(), 50, 10, 2, seed=0)
    assert metrics.sigma_err(S.cpu().numpy(), ref["S"]) <= SIGMA_TOL_BF16
