"""Automatic iteration parameter (Section 2.2): the GPU chooses the same q as
the FP64 oracle's rule when the tolerance sits in a clear gap between
successive relative changes, and its result is bitwise the fixed-q result at
that q."""
import numpy as np
import pytest
import torch

import workloads
from oracle import metrics
from oracle.rsvd import rsvd as oracle_rsvd
from oracle.rsvd import rsvd_auto_q
from paper_1907_06470_amd import Plan
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def _gap_tolerance(deltas, lo=1e-4, ratio=2.5):
    """A tolerance between two successive changes that differ by >= ratio
    (both well above FP32 noise: the GPU's changes agree with the oracle's to
    about 1%), taken as late as possible, and the q the rule then picks."""
    for j in range(len(deltas) - 2, 0, -1):   # q below the maximum
        if deltas[j] >= lo and deltas[j - 1] >= ratio * deltas[j]:
            return float(np.sqrt(deltas[j - 1] * deltas[j])), j + 1
    return None, None


@pytest.mark.parametrize("power,k,p", [(0.6, 20, 10), (1.0, 30, 10), (0.35, 16, 16)])
def test_auto_q_matches_oracle_choice_and_fixed_q(power, k, p):
    dev = need_gpu()
    m, n, qmax = 3000, 1500, 6
    A = workloads.dense_lowrank(m, n, workloads.spectrum_pow(min(m, n), power), 1e-5, seed=21,
                                out_dtype=torch.float32)
    Ah = A.double().numpy()
    probe = rsvd_auto_q(Ah, k, p, qmax, tol=0.0)
    tol, q_expect = _gap_tolerance(probe["deltas"])
    say("auto q", power, k, p, "deltas", [f"{d:.2e}" for d in probe["deltas"]], "tol", tol)
    if tol is None:
        pytest.skip("no clear gap between successive changes for this spectrum")
    ref = rsvd_auto_q(Ah, k, p, qmax, tol=tol)
    assert ref["q_used"] == q_expect
    Ad = A.to(dev)
    U, S, V, info = Plan(m, n, k, p, qmax, auto_q=True, q_tol=tol).factor(Ad)
    assert info["q_used"] == q_expect
    U2, S2, V2, info2 = Plan(m, n, k, p, q_expect).factor(Ad)
    assert info2["q_used"] == q_expect
    assert torch.equal(S, S2) and torch.equal(U, U2) and torch.equal(V, V2)
    assert metrics.sigma_err(S.cpu().numpy(), ref["S"]) <= 1e-5


def test_auto_q_zero_tolerance_and_bf16():
    dev = need_gpu()
    m, n = 2000, 1000
    A = workloads.dense_lowrank(m, n, workloads.spectrum_pow(min(m, n), 0.5), 1e-5, seed=22,
                                out_dtype=torch.float32).to(dev)
    _, S, _, info = Plan(m, n, 10, 10, 3, auto_q=True, q_tol=1e-300).factor(A)
    assert info["q_used"] == 3                     # never that small: runs to the maximum
    _, S3, _, _ = Plan(m, n, 10, 10, 3).factor(A)
    assert torch.equal(S, S3)
    _, Sb, _, infob = Plan(m, n, 10, 10, 5, precision="bf16", auto_q=True, q_tol=1e-2).factor(A)
    assert 1 <= infob["q_used"] <= 5 and infob["q_delta"] <= 1e-2
