"""Wide sketches (padded width above 192, up to 512): column-sliced products,
the global-memory Cholesky and the block one-sided Jacobi, end to end against
the FP64 oracle on the same input and Gaussian test matrix.  The widths are
those of the out-of-core configuration (k = 200, p = 30, l = 230) and the
sparse one (k = 300, p = 30, l = 330), on shapes the oracle finishes in
seconds; sigma is held to the form's target (FP32 1e-5, BF16 1e-3)."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads
from oracle import metrics
from oracle.rsvd import rsvd as oracle_rsvd
from paper_1907_06470_amd import Plan
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu

BJ_MAX_SWEEPS = 20   # sweeps the block Jacobi enqueues (plan.h)


def _check(A64, U, S, V, info, ref, tol, label):
    U, S, V = U.cpu().double().numpy(), S.cpu().numpy(), V.cpu().double().numpy()
    err = metrics.sigma_err(S, ref["S"])
    su, sv = metrics.sin_theta(ref["U"], U), metrics.sin_theta(ref["V"], V)
    say(f"{label}: sigma err {err:.2e}, sin U {su:.1e}, sin V {sv:.1e}, status {info['status']}, "
        f"sweeps {info.get('jacobi_sweeps')}, {info.get('total_ms', 0.0):.2f} ms")
    assert err <= tol
    assert metrics.orth_err(U) < 1e-5 and metrics.orth_err(V) < 1e-4
    assert 0 < info["jacobi_sweeps"] < BJ_MAX_SWEEPS
    lhs = (A64.T @ U).T if sp.issparse(A64) else U.T @ A64
    assert np.max(np.abs(lhs - S[:, None] * V.T)) <= 1e-4 * S[0]
    return err, su, sv


def test_dense_fp32_width_230():
    dev = need_gpu()
    m, n, k, p, q = 6000, 2500, 200, 30, 2
    A = workloads.dense_lowrank(m, n, workloads.spectrum_pow(n, 0.8), 1e-5, seed=21,
                                out_dtype=torch.float32)
    plan = Plan(m, n, k, p, q, seed=0, tile=(2048, 1024))
    U, S, V, info = plan.factor(A.to(dev))
    torch.cuda.synchronize()
    A64 = A.double().numpy()
    _check(A64, U, S, V, info, oracle_rsvd(A64, k, p, q, seed=0), 1e-5, "dense fp32 l=230")


def test_dense_bf16_width_330():
    dev = need_gpu()
    m, n, k, p, q = 4000, 2000, 300, 30, 3
    A = workloads.dense_lowrank(m, n, workloads.spectrum_pow(n, 0.5), 1e-4, seed=22,
                                out_dtype=torch.float32)
    plan = Plan(m, n, k, p, q, seed=0, precision="bf16")
    U, S, V, info = plan.factor(A.to(dev))
    torch.cuda.synchronize()
    A64 = A.double().numpy()
    ref = oracle_rsvd(A64, k, p, q, seed=0)
    Un, Sn = U.cpu().double().numpy(), S.cpu().numpy()
    err = metrics.sigma_err(Sn, ref["S"])
    say(f"dense bf16 l=330: sigma err {err:.2e}, sweeps {info['jacobi_sweeps']}")
    assert err <= 1e-3
    assert metrics.orth_err(Un) < 1e-5
    assert 0 < info["jacobi_sweeps"] < BJ_MAX_SWEEPS


def test_sparse_width_330():
    dev = need_gpu()
    m, n, per_row, k, p, q = 30000, 8000, 30, 300, 30, 3
    rp, ci, v = workloads.zipf_csr(m, n, per_row, seed=23)
    M = sp.csr_matrix((v.numpy().astype(np.float64), ci.numpy(), rp.numpy()), shape=(m, n))
    plan = Plan(m, n, k, p, q, nnz=int(ci.numel()))
    args = (rp.to(dev), ci.to(dev), v.to(dev))
    U, S, V, info = plan.factor_csr(*args)
    U2, S2, V2, _ = plan.factor_csr(*args)
    assert torch.equal(S, S2) and torch.equal(U, U2) and torch.equal(V, V2)
    _check(M, U, S, V, info, oracle_rsvd(M, k, p, q, seed=0), 1e-5, "sparse l=330")


def test_host_resident_width_230_equals_device_resident():
    dev = need_gpu()
    m, n, k, p, q, tile = 3000, 2400, 200, 30, 1, (1024, 1024)
    A = workloads.dense_lowrank(m, n, workloads.spectrum_pow(n, 0.8), 1e-5, seed=24,
                                out_dtype=torch.float32)
    Ud, Sd, Vd, _ = Plan(m, n, k, p, q, tile=tile).factor(A.to(dev))
    Uh, Sh, Vh, info = Plan(m, n, k, p, q, tile=tile, host=True,
                            hbm_budget=256 << 20).factor(A.pin_memory())
    say(f"host l=230: slots {info['slots']}, loads {info['tile_loads']}")
    assert torch.equal(Sd, Sh) and torch.equal(Ud, Uh) and torch.equal(Vd, Vh)
    A64 = A.double().numpy()
    _check(A64, Uh, Sh, Vh, info, oracle_rsvd(A64, k, p, q, seed=0), 1e-5, "host l=230")


def test_widest_sketch_512_exact_on_low_rank():
    """l = 500 on a matrix of rank 450 (noise-free): the sketch spans the
    range, so sigma is exact and the 50 extra directions are dropped or
    come out at rounding level."""
    dev = need_gpu()
    m, n, r = 3000, 1500, 450
    sigma = np.zeros(n)
    sigma[:r] = workloads.spectrum_pow(r, 0.5)
    A = workloads.dense_lowrank(m, n, sigma, 0.0, seed=25, out_dtype=torch.float32)
    k, p, q = 400, 100, 1
    plan = Plan(m, n, k, p, q)
    U, S, V, info = plan.factor(A.to(dev))
    torch.cuda.synchronize()
    A64 = A.double().numpy()
    s_true = np.linalg.svd(A64, compute_uv=False)[:k]
    err = metrics.sigma_err(S.cpu().numpy(), s_true)
    say(f"l=500 rank 450: sigma err {err:.2e}, status {info['status']}, dropped {info['dropped']}")
    assert err <= 1e-5
