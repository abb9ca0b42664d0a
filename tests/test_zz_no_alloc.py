"""rsvd_factor_noalloc (the entry point for callers that cannot allocate)
against rsvd_factor on the same inputs, through the C ABI: two calls in a
row on the library's static workspace, the second with a smaller problem,
each checked against rsvd_factor and the FP64 oracle.  The no-allocation
path runs both CholeskyQR passes of every basis on the caller's stream, so
it agrees with rsvd_factor to rounding (FP32 form: sigma within 1e-5
relative, the FP32 target, subspaces within 1e-4; BF16 form: sigma within
1e-3, the BF16 target), not bit for bit."""
import numpy as np
import pytest
import torch

import workloads
from oracle import metrics
from oracle.rsvd import rsvd as oracle_rsvd
from paper_1907_06470_amd import Plan
from paper_1907_06470_amd import _lib as L
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _case(A_host, k, p, q, precision="fp32", sigma_tol=1e-5, angle_tol=1e-4):
    dev = need_gpu()
    m, n = A_host.shape
    A = torch.as_tensor(A_host, dtype=torch.float32).to(dev)
    plan = Plan(m, n, k, p, q, seed=0, precision=precision)
    assert plan.ws_bytes <= L.NOALLOC_WS_BYTES
    U0, S0, V0, _ = plan.factor(A)
    U1, S1, V1, st = plan.factor_noalloc(A)
    torch.cuda.synchronize()
    U0, S0, V0 = U0.cpu().double().numpy(), S0.cpu().numpy(), V0.cpu().double().numpy()
    U1, S1, V1 = U1.cpu().double().numpy(), S1.cpu().numpy(), V1.cpu().double().numpy()
    ref = oracle_rsvd(A.cpu().double().numpy(), k, p, q, seed=0)
    e01 = metrics.sigma_err(S1, S0)
    e1r = metrics.sigma_err(S1, ref["S"])
    su, sv = metrics.sin_theta(U0, U1), metrics.sin_theta(V0, V1)
    say(f"noalloc {m}x{n} k={k} p={p} q={q} {precision}: status {st}, sigma vs factor {e01:.2e}, "
        f"vs oracle {e1r:.2e}, sin U {su:.1e}, sin V {sv:.1e}")
    assert st == L.OK
    assert e01 <= sigma_tol and e1r <= sigma_tol
    assert su <= angle_tol and sv <= angle_tol
    assert metrics.orth_err(U1) < 1e-5 and metrics.orth_err(V1) < 1e-4


def test_noalloc_two_calls_second_smaller():
    A, meta = workloads.make("plain_small", out_dtype=torch.float32)
    _case(A.numpy(), meta["k"], meta["p"], meta["q"])
    sigma = workloads.spectrum_pow(300, 1.0)
    B = workloads.dense_lowrank(600, 300, sigma, 1e-4, seed=7, device="cpu", out_dtype=torch.float32)
    _case(B.numpy(), 12, 8, 1)


def test_noalloc_bf16_form():
    sigma = workloads.spectrum_pow(700, 1.0)
    A = workloads.dense_lowrank(1400, 700, sigma, 1e-4, seed=11, device="cpu", out_dtype=torch.float32)
    _case(A.numpy(), 24, 8, 2, precision="bf16", sigma_tol=1e-3, angle_tol=1e-2)
