"""Boundary checks of the C ABI on the device: the workspace size predicted
by rsvd_plan before anything runs (Section 3.4) is exactly what the calls
use (nothing is written past it), the report's device-memory figure, and
caller-owned copy and side streams."""
import numpy as np
import pytest
import torch

import workloads
from paper_1907_06470_amd import Plan
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu

SENTINEL = 0xA5
TAIL = 1 << 20


def _guarded_ws(plan, dev):
    buf = torch.full((plan.ws_bytes + TAIL,), SENTINEL, dtype=torch.uint8, device=dev)
    return buf, buf[:plan.ws_bytes]


def _tail_intact(buf, plan):
    return bool((buf[plan.ws_bytes:] == SENTINEL).all().item())


@pytest.mark.parametrize("kw", [dict(precision="fp32"), dict(precision="bf16"),
                                dict(precision="fp8"), dict(precision="fp32", backward=True),
                                dict(precision="fp32", k=200, p=30)])
def test_dense_calls_stay_inside_the_predicted_workspace(kw):
    dev = need_gpu()
    kw = dict(kw)
    k, p = kw.pop("k", 40), kw.pop("p", 24)
    m, n = 3000, 2048
    A = workloads.dense_lowrank(m, n, workloads.spectrum_pow(n, 1.0), 1e-4, seed=31,
                                out_dtype=torch.float32).to(dev)
    plan = Plan(m, n, k, p, 2, tile=(1024, 1024), **kw)
    buf, ws = _guarded_ws(plan, dev)
    U, S, V, info = plan.factor(A, ws=ws)
    if kw.get("backward"):
        plan.backward(A, None, torch.ones(k, dtype=torch.float64, device=dev), None, ws=ws)
    torch.cuda.synchronize()
    say(f"ws {plan.ws_bytes} bytes, peak_hbm {info['peak_hbm']}")
    assert _tail_intact(buf, plan)
    assert info["ws_bytes"] == plan.ws_bytes
    assert info["peak_hbm"] == plan.ws_bytes + m * n * 4 + (m + n) * k * 4 + k * 8


def test_sparse_and_host_calls_stay_inside_the_predicted_workspace():
    dev = need_gpu()
    m, n = 20000, 6000
    rp, ci, v = workloads.zipf_csr(m, n, 20, seed=32)
    plan = Plan(m, n, 40, 20, 2, nnz=int(ci.numel()))
    buf, ws = _guarded_ws(plan, dev)
    _, _, _, info = plan.factor_csr(rp.to(dev), ci.to(dev), v.to(dev), ws=ws)
    torch.cuda.synchronize()
    assert _tail_intact(buf, plan)
    nnz, k = int(ci.numel()), 40
    assert info["peak_hbm"] == plan.ws_bytes + 8 * nnz + 4 * (m + 1) + 4 * (m + n) * k + 8 * k
    # COO with 64-bit indices: the CSR copy is part of the workspace
    cplan = Plan(m, n, 40, 20, 2, nnz=nnz, coo=True)
    rows = torch.repeat_interleave(torch.arange(m, dtype=torch.int64), (rp[1:] - rp[:-1]).long())
    cbuf, cws = _guarded_ws(cplan, dev)
    _, _, _, cinfo = cplan.factor_coo(rows.to(dev), ci.long().to(dev), v.to(dev), ws=cws)
    torch.cuda.synchronize()
    assert _tail_intact(cbuf, cplan)
    assert cinfo["peak_hbm"] == cplan.ws_bytes + 20 * nnz + 4 * (m + n) * k + 8 * k
    A = workloads.dense_lowrank(2600, 1800, workloads.spectrum_pow(1800, 0.8), 1e-5, seed=33,
                                out_dtype=torch.float32)
    hplan = Plan(2600, 1800, 24, 8, 1, tile=(512, 512), host=True, hbm_budget=64 << 20)
    buf, ws = _guarded_ws(hplan, dev)
    _, _, _, info = hplan.factor(A.pin_memory(), ws=ws)
    torch.cuda.synchronize()
    assert _tail_intact(buf, hplan)
    assert info["ws_bytes"] <= 64 << 20


def test_caller_streams_give_the_same_result():
    dev = need_gpu()
    m, n = 2600, 1800
    A = workloads.dense_lowrank(m, n, workloads.spectrum_pow(n, 0.8), 1e-5, seed=34,
                                out_dtype=torch.float32)
    ref = Plan(m, n, 24, 8, 2, tile=(512, 512), host=True).factor(A.pin_memory())
    plan = Plan(m, n, 24, 8, 2, tile=(512, 512), host=True)
    copy_s, side_s = torch.cuda.Stream(), torch.cuda.Stream()
    plan.set_streams(copy_s, side_s)
    got = plan.factor(A.pin_memory())
    torch.cuda.synchronize()
    for a, b in zip(ref[:3], got[:3]):
        assert torch.equal(a, b)
    plan.set_streams(None, None)       # back to streams of the plan's own
    again = plan.factor(A.pin_memory())
    torch.cuda.synchronize()
    assert torch.equal(ref[1], again[1])
