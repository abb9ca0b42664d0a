"""Sparse A in COO form (Section 3.3: coordinates with 32- or 64-bit
indices).  A row-sorted COO gives exactly the CSR path's result (the stable
row sort keeps the order within a row); unsorted entries with repeated
coordinates match the FP64 oracle on the summed scipy matrix; indices out of
range are reported without faults."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads
from oracle import metrics
from oracle.rsvd import rsvd as oracle_rsvd
from paper_1907_06470_amd import Plan
from paper_1907_06470_amd import _lib as L
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("itype", [torch.int32, torch.int64])
def test_row_sorted_coo_equals_csr_bitwise(itype):
    dev = need_gpu()
    m, n, per_row = 9000, 4000, 17
    say("coo-vs-csr", itype)
    rp, ci, v = workloads.zipf_csr(m, n, per_row, seed=31)
    nnz = int(ci.numel())
    rows = torch.repeat_interleave(torch.arange(m, dtype=torch.int64), rp.diff().to(torch.int64))
    k, p, q = 30, 18, 2
    U0, S0, V0, _ = Plan(m, n, k, p, q, nnz=nnz).factor_csr(rp.to(dev), ci.to(dev), v.to(dev))
    plan = Plan(m, n, k, p, q, nnz=nnz, coo=True)
    U1, S1, V1, info = plan.factor_coo(rows.to(itype).to(dev), ci.to(itype).to(dev), v.to(dev))
    assert info["status"] == L.OK
    assert torch.equal(S0, S1) and torch.equal(U0, U1) and torch.equal(V0, V1)


def test_unsorted_coo_with_repeats_matches_oracle():
    dev = need_gpu()
    n, nnz = 6000, 30000
    say("coo-banded", n, nnz)
    r, c, v = workloads.banded_random_coo(n, nnz, 2, seed=8)
    perm = torch.randperm(nnz, generator=torch.Generator().manual_seed(3))
    r, c, v = r[perm], c[perm], v[perm]
    # repeat a few coordinates with their own values (they add up)
    r = torch.cat([r, r[:500]])
    c = torch.cat([c, c[:500]])
    v = torch.cat([v, 0.5 * v[:500]])
    M = sp.coo_matrix((v.numpy().astype(np.float64), (r.numpy(), c.numpy())), shape=(n, n)).tocsr()
    k, p, q = 24, 16, 2
    plan = Plan(n, n, k, p, q, nnz=int(r.numel()), coo=True)
    U, S, V, info = plan.factor_coo(r.to(dev), c.to(dev), v.to(dev))
    ref = oracle_rsvd(M, k, p, q, seed=0)
    err = metrics.sigma_err(S.cpu().numpy(), ref["S"])
    say(f"coo sigma err {err:.3e}")
    assert err <= 1e-5
    assert metrics.orth_err(U.cpu().double().numpy()) <= 1e-5
    assert metrics.orth_err(V.cpu().double().numpy()) <= 1e-5
    U2, S2, V2, _ = plan.factor_coo(r.to(dev), c.to(dev), v.to(dev))
    assert torch.equal(S, S2) and torch.equal(U, U2) and torch.equal(V, V2)


def test_coo_index_out_of_range_is_reported():
    dev = need_gpu()
    n, nnz = 500, 2000
    r, c, v = workloads.banded_random_coo(n, nnz, 1, seed=9)
    c = c.clone()
    c[17] = n + 5                       # clamped in the kernels, flagged in the status
    plan = Plan(n, n, 5, 5, 1, nnz=nnz, coo=True)
    with pytest.raises(L.RsvdError) as e:
        plan.factor_coo(r.to(dev), c.to(dev), v.to(dev))
    assert e.value.status == L.E_INVALID_ARG
