"""Sparse A (CSR): products against scipy's CSR x dense in FP64 within the
FP32 summation bound, bitwise reproducibility (the work split by nonzero
chunks with ordered carries does not depend on scheduling), empty rows and
columns, malformed arrays reported without faults, and the whole factorisation
against the FP64 oracle run on the same scipy matrix."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads
from oracle import metrics
from oracle.rsvd import rsvd as oracle_rsvd
from paper_1907_06470_amd import Plan, factor
from paper_1907_06470_amd import _lib as L
from tests.gpu_util import col_major_from_numpy, gamma_bound, need_gpu, rand_panel, say

pytestmark = pytest.mark.gpu


def _csr(m, n, per_row, seed, drop_rows=0):
    rp, ci, v = workloads.zipf_csr(m, n, per_row, seed=seed)
    if drop_rows:   # empty every drop_rows-th row
        M = sp.csr_matrix((v.numpy(), ci.numpy(), rp.numpy()), shape=(m, n))
        keep = np.ones(m, bool)
        keep[::drop_rows] = False
        M = sp.diags(keep.astype(np.float32)) @ M
        M = sp.csr_matrix(M)
        M.eliminate_zeros()
        M.sort_indices()
        rp = torch.as_tensor(M.indptr.astype(np.int32))
        ci = torch.as_tensor(M.indices.astype(np.int32))
        v = torch.as_tensor(M.data.astype(np.float32))
    M = sp.csr_matrix((v.numpy().astype(np.float64), ci.numpy(), rp.numpy()), shape=(m, n))
    return rp, ci, v, M


@pytest.mark.parametrize("m,n,per_row,l,drop", [
    (20000, 5000, 20, 64, 0),      # hot columns span many nonzero chunks of A^T
    (7000, 9000, 13, 100, 3),      # empty rows, unused columns, wide panel
    (300, 200, 1, 20, 0),          # fewer nonzeros than one chunk
    (5000, 3000, 37, 190, 7),      # widest panel (three columns per lane)
    (200000, 3000, 3, 190, 5),     # tall, 391 head blocks of 512 rows
    (1200000, 3000, 2, 230, 5),    # taller: the CSC copy is split into two row blocks
    (20000, 6000, 25, 330, 0),     # wide sketch: two column slices of 192 and 138
])
def test_sparse_products_match_scipy(m, n, per_row, l, drop):
    dev = need_gpu()
    say("spmm", m, n, per_row, l, drop)
    rp, ci, v, M = _csr(m, n, per_row, seed=m + n, drop_rows=drop)
    k = max(1, l // 2)
    plan = Plan(m, n, k, l - k, 1, nnz=int(ci.numel()))
    args = (rp.to(dev), ci.to(dev), v.to(dev))
    X = rand_panel(n, l, 1)
    Y = plan.step_spmm(0, *args, col_major_from_numpy(X, dev)).cpu().numpy().astype(np.float64)
    absM = abs(M)
    ref = M @ X.astype(np.float64)
    assert np.all(np.abs(Y - ref) <= gamma_bound(per_row + 2, absM @ np.abs(X)) + 1e-30)
    Q = rand_panel(m, l, 2)
    Z = plan.step_spmm(1, *args, col_major_from_numpy(Q, dev)).cpu().numpy().astype(np.float64)
    ref = M.T @ Q.astype(np.float64)
    # a column sums per row block of A (at most 16), then the blocks in order
    K = int(np.max(np.diff(M.tocsc().indptr))) + 2 + 16
    assert np.all(np.abs(Z - ref) <= gamma_bound(K, absM.T @ np.abs(Q)) + 1e-30)
    Z2 = plan.step_spmm(1, *args, col_major_from_numpy(Q, dev)).cpu().numpy().astype(np.float64)
    assert np.array_equal(Z, Z2)


def test_sparse_head_block_edges():
    """A^T Q through the head columns' LDS blocks of 512 rows: a last block of
    one row, a column with an entry in every row, empty columns and a column
    whose only entry is in the last row, next to Zipf columns."""
    dev = need_gpu()
    m, n, l = 3 * 512 + 1, 700, 96
    say("spmm head edges", m, n, l)
    rp, ci, v, Z0 = _csr(m, n, 9, seed=11)
    M = sp.lil_matrix(Z0)
    M[:, 0:4] = 0.0                                   # empty columns
    M[:, 5] = np.linspace(0.5, 1.5, m)[:, None]       # an entry in every row
    M[:, 10] = 0.0
    M[m - 1, 10] = 3.0                                # only in the last row
    M = sp.csr_matrix(M)
    M.eliminate_zeros()
    M.sort_indices()
    rp = torch.as_tensor(M.indptr.astype(np.int32))
    ci = torch.as_tensor(M.indices.astype(np.int32))
    v = torch.as_tensor(M.data.astype(np.float32))
    M = sp.csr_matrix((v.numpy().astype(np.float64), ci.numpy(), rp.numpy()), shape=(m, n))
    k = l // 2
    plan = Plan(m, n, k, l - k, 1, nnz=int(ci.numel()))
    args = (rp.to(dev), ci.to(dev), v.to(dev))
    Q = rand_panel(m, l, 5)
    Z = plan.step_spmm(1, *args, col_major_from_numpy(Q, dev)).cpu().numpy().astype(np.float64)
    ref = M.T @ Q.astype(np.float64)
    K = int(np.max(np.diff(M.tocsc().indptr))) + 2 + 16
    assert np.all(np.abs(Z - ref) <= gamma_bound(K, abs(M).T @ np.abs(Q)) + 1e-30)
    # one entry: one rounded product, then sums of exact zeros
    assert not np.any(Z[0:4]) and np.array_equal(Z[10], (np.float32(3.0) * Q[m - 1]).astype(np.float64))
    Z2 = plan.step_spmm(1, *args, col_major_from_numpy(Q, dev)).cpu().numpy().astype(np.float64)
    assert np.array_equal(Z, Z2)


def test_empty_sparse_matrix():
    """No entries: the products are zero (the head columns' output rows are
    cleared without a product), every sketch direction is dropped and
    S = 0 with finite U, V."""
    dev = need_gpu()
    m, n = 3000, 800
    say("empty sparse", m, n)
    rp = torch.zeros(m + 1, dtype=torch.int32, device=dev)
    ci = torch.zeros(0, dtype=torch.int32, device=dev)
    v = torch.zeros(0, dtype=torch.float32, device=dev)
    plan = Plan(m, n, 5, 5, 1, nnz=0)
    Q = rand_panel(m, 10, 3)
    Z = plan.step_spmm(1, rp, ci, v, col_major_from_numpy(Q, dev))
    X = rand_panel(n, 10, 4)
    Y = plan.step_spmm(0, rp, ci, v, col_major_from_numpy(X, dev))
    assert not bool(torch.any(Z != 0)) and not bool(torch.any(Y != 0))
    U, S, V, info = plan.factor_csr(rp, ci, v)
    torch.cuda.synchronize()
    assert torch.all(S == 0)
    assert bool(torch.isfinite(U).all()) and bool(torch.isfinite(V).all())
    assert info["status"] in (L.OK, L.W_RANK_DEFICIENT)


def test_sparse_factor_matches_oracle_and_is_reproducible():
    dev = need_gpu()
    m, n, per_row = 12000, 4000, 30
    rp, ci, v, M = _csr(m, n, per_row, seed=4)
    k, p, q = 40, 20, 3
    plan = Plan(m, n, k, p, q, nnz=int(ci.numel()))
    args = (rp.to(dev), ci.to(dev), v.to(dev))
    U, S, V, info = plan.factor_csr(*args)
    U2, S2, V2, _ = plan.factor_csr(*args)
    assert torch.equal(S, S2) and torch.equal(U, U2) and torch.equal(V, V2)
    ref = oracle_rsvd(M, k, p, q, seed=0)
    err = metrics.sigma_err(S.cpu().numpy(), ref["S"])
    say(f"sparse sigma err {err:.3e}")
    assert err <= 1e-5
    Un = U.cpu().double().numpy()
    assert metrics.orth_err(Un) <= 1e-5
    # U^T A = S V^T holds for the randomized SVD (B = Q^T A)
    lhs = (M.T @ Un).T
    rhs = S.cpu().numpy()[:, None] * V.cpu().double().numpy().T
    assert np.max(np.abs(lhs - rhs)) <= 1e-4 * S[0].item()


def test_torch_sparse_csr_tensor_through_factor():
    dev = need_gpu()
    m, n = 3000, 2000
    rp, ci, v, M = _csr(m, n, 15, seed=9)
    A = torch.sparse_csr_tensor(rp.long(), ci.long(), v, size=(m, n)).to(dev)
    U, S, V, info = factor(A, 10, 10, 2)
    ref = oracle_rsvd(M, 10, 10, 2, seed=0)
    assert metrics.sigma_err(S.cpu().numpy(), ref["S"]) <= 1e-5


@pytest.mark.parametrize("breakage", ["column_out_of_range", "decreasing_pointer", "wrong_total"])
def test_malformed_csr_is_reported(breakage):
    dev = need_gpu()
    m, n = 2000, 1000
    rp, ci, v, M = _csr(m, n, 10, seed=5)
    rp, ci = rp.clone(), ci.clone()
    if breakage == "column_out_of_range":
        ci[777] = n + 5
    elif breakage == "decreasing_pointer":
        rp[500] = rp[499] - 3
    else:
        rp[-1] = rp[-1] - 1
    plan = Plan(m, n, 8, 8, 1, nnz=int(ci.numel()))
    with pytest.raises(L.RsvdError) as e:
        plan.factor_csr(rp.to(dev), ci.to(dev), v.to(dev))
    assert e.value.status == L.E_INVALID_ARG
    with pytest.raises(L.RsvdError):
        plan.step_spmm(0, rp.to(dev), ci.to(dev), v.to(dev),
                       col_major_from_numpy(rand_panel(n, 16, 3), dev))
