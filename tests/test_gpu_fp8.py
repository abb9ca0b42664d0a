"""FP8 (e4m3) form: A quantised once with one power-of-two scale per 64 x 64
block, panels with one per column, products on the FP8 matrix cores with FP32
accumulation.  Products are checked against the FP64 product of the same
quantised operands (quantisation by the CPU reference encoder); the matrix
cores sum each 64-term slab with reduced internal precision, so the bound is
2^-8 of the product of absolute values.  End to end the FP8 form has no
accuracy target: its singular values are held to the accuracy the FP64 oracle
reaches against the exact ones."""
import numpy as np
import pytest
import torch

import workloads
from oracle import metrics
from oracle.rsvd import rsvd as oracle_rsvd
from paper_1907_06470_amd import Plan
from tests import fp8_format as f8
from tests.gpu_util import col_major_from_numpy, need_gpu, rand_panel, say

pytestmark = pytest.mark.gpu

SLAB_REL = 2.0 ** -8


@pytest.mark.parametrize("m,n,l,tile", [
    (1000, 700, 20, (256, 192)),
    (777, 1234, 70, (0, 0)),
    (300, 260, 128, (128, 64)),
    (513, 2049, 100, (512, 1024)),
    (65, 5000, 3, (64, 4096)),
    (136, 224, 120, (64, 128)),
    (640, 768, 230, (256, 256)),
    (512, 448, 330, (0, 0)),
    (1000, 700, 150, (256, 192)),     # width 160: direct-to-LDS, three-stage ring
    (640, 1536, 160, (128, 1408)),    # 11 whole slabs per A X tile (six-step loop + 5)
])
def test_fp8_products_match_quantised_operands(m, n, l, tile):
    dev = need_gpu()
    say("fp8 product", m, n, l, tile)
    k = max(1, l // 2)
    plan = Plan(m, n, k, l - k, 1, precision="fp8", tile=tile)
    rng = np.random.default_rng(m + 7 * n + l)
    A = (rng.standard_normal((m, n)) * np.exp2(rng.integers(-3, 4, (m, 1)))).astype(np.float32)
    Aq, _ = f8.quantize_blocks(A)
    Ad = torch.as_tensor(A, device=dev)
    X = rand_panel(n, l, 1)
    Y = plan.step_product(0, Ad, col_major_from_numpy(X, dev)).cpu().numpy().astype(np.float64)
    Xq, _ = f8.quantize_columns(X)
    ref = Aq @ Xq
    bound = SLAB_REL * (np.abs(Aq) @ np.abs(Xq)) + 1e-30
    assert np.all(np.abs(Y - ref) <= bound), np.max(np.abs(Y - ref) / bound)
    Qp = rand_panel(m, l, 2)
    Z = plan.step_product(1, Ad, col_major_from_numpy(Qp, dev)).cpu().numpy().astype(np.float64)
    Qq, _ = f8.quantize_columns(Qp)
    ref = Aq.T @ Qq
    bound = SLAB_REL * (np.abs(Aq).T @ np.abs(Qq)) + 1e-30
    assert np.all(np.abs(Z - ref) <= bound), np.max(np.abs(Z - ref) / bound)


def test_fp8_quantisation_error_is_the_format_error():
    # the products differ from the FP32 products by the e4m3 rounding only:
    # relative error of one value <= 2^-4, so a product with positive
    # operands is within 2 * 2^-4 (+ slab rounding) of the exact one
    dev = need_gpu()
    m, n, l = 512, 768, 32
    rng = np.random.default_rng(3)
    A = rng.uniform(0.5, 2.0, (m, n)).astype(np.float32)
    X = rng.uniform(0.5, 2.0, (n, l)).astype(np.float32)
    plan = Plan(m, n, 16, 16, 1, precision="fp8", tile=(256, 256))
    Y = plan.step_product(0, torch.as_tensor(A, device=dev), col_major_from_numpy(X, dev)).cpu().numpy()
    exact = A.astype(np.float64) @ X.astype(np.float64)
    assert np.max(np.abs(Y / exact - 1.0)) <= 2 * 2.0 ** -4 + SLAB_REL


# The FP8 forms have no accuracy target.  Rounding the sketch operands to e4m3
# (3 mantissa bits) perturbs the random start, and on a spectrum that decays
# slowly two power steps do not erase the start: the result differs from the
# oracle's with the same seed by ~5e-3 (CPU emulation of the same rounding
# gives the same figures), while the oracle's results for other seeds differ
# from it by 1e-2 to 3e-2.  What is asserted is accuracy against the exact
# singular values (LAPACK, FP64): no worse than the oracle's own, within 2e-3,
# for every split of the passes over the FP8 form.
@pytest.mark.parametrize("mix", [("fp8", "fp8", "fp8"), ("fp8", "fp8", "bf16"),
                                 ("fp8", "bf16", "fp32")])
def test_fp8_factor_end_to_end(mix):
    dev = need_gpu()
    A, meta = workloads.make("plain_gpu", scale=0.1)
    m, n = A.shape
    k, p, q = 50, 10, 2
    say("fp8 end to end", m, n, mix)
    plan = Plan(m, n, k, p, q, precision=mix)
    U, S, V, info = plan.factor(A.to(dev))
    Ad = A.double().numpy()
    ref = oracle_rsvd(Ad, k, p, q, seed=0)
    exact = np.linalg.svd(Ad, compute_uv=False)[:k]
    err = metrics.sigma_err(S.cpu().numpy(), exact)
    err_oracle = metrics.sigma_err(ref["S"], exact)
    spread = metrics.sigma_err(S.cpu().numpy(), ref["S"])
    say(f"fp8 form {mix}: sigma err vs exact {err:.3e} (oracle {err_oracle:.3e}), "
        f"vs oracle {spread:.3e}")
    assert err <= err_oracle + 2e-3
    assert spread <= 1e-2
    Un, Vn = U.cpu().double().numpy(), V.cpu().double().numpy()
    assert metrics.orth_err(Un) <= 1e-5 and metrics.orth_err(Vn) <= 1e-5
    assert info["status"] == 0


def test_fp8_rejects_tiles_not_multiple_of_64():
    need_gpu()
    from paper_1907_06470_amd import _lib as L
    with pytest.raises(L.RsvdError):
        Plan(500, 400, 10, 5, 1, precision="fp8", tile=(96, 64))
