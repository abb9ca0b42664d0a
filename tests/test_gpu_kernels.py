"""Step-level parity of the HIP kernels against the oracle, through the C ABI:
Philox words (bitwise), Gaussian test matrix (ulps), block-wise products
(componentwise rounding bound), CholeskyQR2 and the small SVD."""
import numpy as np
import pytest
import torch

from oracle import metrics, philox
from oracle.householder import householder_qr
from oracle.rsvd import small_svd
from paper_1907_06470_amd import Plan, omega, philox_raw
from tests.gpu_util import col_major_from_numpy, gamma_bound, need_gpu, rand_panel, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,row0,rows,blocks", [
    (0, 0, 257, 7), (1, 5, 100, 1), (2**32 + 7, 123456, 64, 33), (2**64 - 1, 2**32 - 3, 9, 4)])
def test_philox_words_bitwise(seed, row0, rows, blocks):
    dev = need_gpu()
    say("philox", seed, row0, rows, blocks)
    got = philox_raw(seed, 0, row0, rows, blocks, device=dev).cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    ref = philox.raw_words(seed, rows, blocks, row0=row0).astype(np.int64)
    assert np.array_equal(got, ref)


def test_philox_other_stream_bitwise():
    dev = need_gpu()
    got = philox_raw(99, 3, 0, 50, 5, device=dev).cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    ref = philox.raw_words(99, 50, 5, row0=0, stream=3).astype(np.int64)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("seed,n,l,row0,rows", [(0, 5000, 37, 0, 5000), (7, 100000, 120, 99000, 1000)])
def test_omega_fp64_within_4_ulp(seed, n, l, row0, rows):
    dev = need_gpu()
    say("omega f64", seed, n, l)
    got = omega(seed, n, l, row0, rows, dtype=torch.float64, device=dev).cpu().numpy()
    ref = philox.omega(seed, n, l, row0=row0, rows=rows)
    ulp = np.spacing(np.abs(ref))
    assert np.all(np.abs(got - ref) <= 4 * ulp)


def test_omega_fp32_is_the_rounded_fp64():
    dev = need_gpu()
    got = omega(3, 20000, 64, dtype=torch.float32, device=dev).cpu().numpy()
    ref = philox.omega(3, 20000, 64)
    r32 = ref.astype(np.float32)
    same = got == r32
    assert same.mean() > 0.9999
    assert np.all(np.abs(got[~same].astype(np.float64) - r32[~same]) <= np.spacing(np.abs(r32[~same])))


PRODUCT_CASES = [
    (1000, 700, 20, (256, 192)),     # several tiles, ragged tails, lp = 32
    (777, 1234, 70, (0, 0)),         # automatic tiles, lp = 96
    (300, 260, 190, (96, 64)),       # widest sketch, lp = 192
    (128, 64, 32, (128, 64)),        # one tile
    (33, 5000, 3, (32, 4096)),       # short and wide
    (600, 450, 230, (256, 160)),     # wide sketch, lp = 256: two 128-column slices
    (420, 700, 330, (0, 0)),         # lp = 352: slices of 192 and 160
    (530, 512, 500, (256, 256)),     # widest sketch, lp = 512
]


@pytest.mark.parametrize("m,n,l,tile", PRODUCT_CASES)
def test_blockwise_products_within_rounding_bound(m, n, l, tile):
    dev = need_gpu()
    say("product", m, n, l, tile)
    k = max(1, l // 2)
    plan = Plan(m, n, k, l - k, 1, tile=tile)
    rng = np.random.default_rng(m + n + l)
    A = rng.standard_normal((m, n)).astype(np.float32)
    Ad = torch.as_tensor(A, device=dev)
    X = rand_panel(n, l, 1)
    Y = plan.step_product(0, Ad, col_major_from_numpy(X, dev)).cpu().numpy()
    ref = A.astype(np.float64) @ X.astype(np.float64)
    bound = gamma_bound(n, np.abs(A.astype(np.float64)) @ np.abs(X.astype(np.float64)))
    assert np.all(np.abs(Y - ref) <= bound + 1e-30)
    Qp = rand_panel(m, l, 2)
    Z = plan.step_product(1, Ad, col_major_from_numpy(Qp, dev)).cpu().numpy()
    ref = A.astype(np.float64).T @ Qp.astype(np.float64)
    bound = gamma_bound(m, np.abs(A.astype(np.float64)).T @ np.abs(Qp.astype(np.float64)))
    assert np.all(np.abs(Z - ref) <= bound + 1e-30)


def test_products_with_fp64_input_use_the_fp32_rounding():
    dev = need_gpu()
    m, n, l = 500, 300, 24
    plan = Plan(m, n, 12, 12, 1, dtype=torch.float64, tile=(128, 96))
    A = np.random.default_rng(0).standard_normal((m, n))
    X = rand_panel(n, l, 3)
    Y = plan.step_product(0, torch.as_tensor(A, device=dev), col_major_from_numpy(X, dev)).cpu().numpy()
    A32 = A.astype(np.float32).astype(np.float64)
    ref = A32 @ X.astype(np.float64)
    assert np.all(np.abs(Y - ref) <= gamma_bound(n, np.abs(A32) @ np.abs(X.astype(np.float64))))


@pytest.mark.parametrize("rows,l,side", [(3000, 40, 0), (2500, 120, 1), (777, 190, 0), (100, 1, 0),
                                         (70000, 64, 0), (20000, 150, 1), (70001, 190, 0),
                                         (5000, 230, 1), (9001, 330, 0), (2000, 500, 0)])
def test_gram_is_the_fp64_product(rows, l, side):
    dev = need_gpu()
    say("gram", rows, l)
    m, n = (rows, max(l, 64)) if side == 0 else (max(l, 64), rows)
    k = max(1, l // 2)
    plan = Plan(m, n, k, l - k, 1)
    Y = rand_panel(rows, l, 6)
    G = plan.step_gram(side, col_major_from_numpy(Y, dev)).cpu().numpy()
    Y64 = Y.astype(np.float64)
    ref = Y64.T @ Y64
    # FP32 x FP32 products are exact in FP64; only the FP64 sums round
    bound = gamma_bound(rows, np.abs(Y64).T @ np.abs(Y64), u=2.0 ** -53)
    assert np.all(np.abs(G - ref) <= bound)
    assert np.array_equal(G, G.T)


@pytest.mark.parametrize("rows,l,cond,side", [(3000, 40, 10.0, 0), (2500, 120, 1e4, 1), (777, 190, 1e3, 0),
                                              (64, 64, 1.0, 0), (3000, 150, 1e3, 1), (5000, 176, 1e5, 0),
                                              (140001, 190, 1e3, 0), (133000, 96, 10.0, 1),
                                              (6000, 230, 1e4, 1), (8000, 330, 1e3, 0),
                                              (150001, 330, 1e2, 0), (3000, 500, 1e2, 0)])
def test_cholqr2_orthonormal_basis_of_the_span(rows, l, cond, side):
    dev = need_gpu()
    say("orth", rows, l, cond)
    m, n = (rows, max(l, 64)) if side == 0 else (max(l, 64), rows)
    k = max(1, l // 2)
    plan = Plan(m, n, k, l - k, 1)
    scale = np.logspace(0, -np.log10(cond), l)
    Y = rand_panel(rows, l, 5, scale)
    Q = plan.step_orth(side, col_major_from_numpy(Y, dev)).cpu().numpy().astype(np.float64)
    say(f"orth err {metrics.orth_err(Q):.3e}")
    assert metrics.orth_err(Q) < 2e-6 * max(1.0, l / 32)
    Qref, _ = householder_qr(Y.astype(np.float64))
    assert metrics.sin_theta(Qref, Q) < 1e-6 * cond * 10


@pytest.mark.parametrize("rows,l,r", [(2000, 24, 9), (3000, 170, 40), (4000, 330, 70)])
def test_cholqr2_drops_dependent_directions(rows, l, r):
    dev = need_gpu()
    say("orth drop", rows, l, r)
    plan = Plan(rows, max(100, l), l // 2, l - l // 2, 1)
    rng = np.random.default_rng(1)
    Y = (rng.standard_normal((rows, r)) @ rng.standard_normal((r, l))).astype(np.float32)
    Q = plan.step_orth(0, col_major_from_numpy(Y, dev)).cpu().numpy().astype(np.float64)
    norms = np.linalg.norm(Q, axis=0)
    live = norms > 0.5
    oe = metrics.orth_err(Q[:, live])
    say(f"orth drop: live {live.sum()}, orth err {oe:.3e}")
    assert live.sum() == r
    assert np.all(norms[~live] == 0.0)
    assert oe < 1e-5
    # Q = Y W is formed in FP32: its columns leave span(Y) by the rounding of
    # the product, about u32 * cond(Y_kept) relative (u32 = 2^-24)
    kappa = np.linalg.cond(Y[:, live].astype(np.float64))
    assert metrics.sin_theta(Y.astype(np.float64), Q[:, live]) < 4 * 2.0 ** -24 * max(kappa, 10.0)


@pytest.mark.parametrize("n,l,decay", [(5000, 30, 1.0), (20000, 120, 2.0), (700, 190, 0.5), (64, 1, 0.0),
                                        (5000, 230, 1.0), (3000, 330, 0.5), (2000, 500, 1.0),
                                        (900, 17, 0.5)])
def test_small_svd_matches_oracle(n, l, decay):
    dev = need_gpu()
    say("small svd", n, l)
    k = max(1, l // 2)
    plan = Plan(max(n, l), n, k, l - k, 1)
    scale = np.arange(1, l + 1, dtype=np.float64) ** -decay
    Bt = rand_panel(n, l, 9, scale)
    sig, ub = plan.step_small_svd(col_major_from_numpy(Bt, dev))
    sig, ub = sig.cpu().numpy(), ub.cpu().numpy()
    Ub_ref, s_ref, _ = small_svd(Bt.astype(np.float64))
    assert np.all(np.abs(sig - s_ref) <= 1e-10 * s_ref[0])
    gaps = np.minimum(np.abs(np.diff(s_ref, prepend=np.inf)), np.abs(np.diff(s_ref, append=-np.inf))) / s_ref[0]
    ok = gaps > 1e-4
    dots = np.abs(np.einsum("ij,ij->j", ub, Ub_ref))
    assert np.all(dots[ok] > 1 - 1e-8)
    assert metrics.orth_err(ub) < 1e-12
