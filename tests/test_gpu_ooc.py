"""Host-resident A (out of core, Section 3.5): tiles stream from pinned host
memory through HBM slots on a copy stream.  Each tile writes its own rows of
its partial panel with the same kernels as the device-resident path, so the
result is bitwise equal to it whatever the slot count; the copies are
accounted in the report."""
import ctypes

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


def _workload(m, n, seed=11):
    sigma = workloads.spectrum_pow(min(m, n), 0.8)
    return workloads.dense_lowrank(m, n, sigma, 1e-5, seed=seed, out_dtype=torch.float32)


@pytest.mark.parametrize("m,n,tile,q", [(3000, 2000, (1024, 1024), 2), (2600, 3100, (512, 768), 1)])
def test_host_resident_equals_device_resident_bitwise(m, n, tile, q):
    dev = need_gpu()
    say("ooc", m, n, tile, q)
    A = _workload(m, n)
    k, p = 24, 8
    Ud, Sd, Vd, _ = Plan(m, n, k, p, q, tile=tile).factor(A.to(dev))
    hp = Plan(m, n, k, p, q, tile=tile, host=True)
    Uh, Sh, Vh, info = hp.factor(A.pin_memory())
    assert torch.equal(Sd, Sh) and torch.equal(Ud, Uh) and torch.equal(Vd, Vh)
    tiles = -(-m // tile[0]) * -(-n // tile[1])
    # four slots by default: never fewer loads than tiles, never more than passes x tiles
    passes = 2 * q + 2
    assert tiles <= info["tile_loads"] <= passes * tiles
    assert info["h2d_bytes"] >= m * n * 4


def test_slot_count_changes_traffic_not_results():
    dev = need_gpu()
    m, n, tile, q = 3000, 2000, (1024, 1024), 2
    A = _workload(m, n, seed=12).pin_memory()
    k, p = 20, 12
    base = Plan(m, n, k, p, q, tile=tile, host=True)
    slot = 1024 * 1024 * 4
    few = Plan(m, n, k, p, q, tile=tile, host=True, hbm_budget=base.ws_bytes - 2 * slot)
    many = Plan(m, n, k, p, q, tile=tile, host=True, hbm_budget=base.ws_bytes + 10 * slot)
    mid = Plan(m, n, k, p, q, tile=tile, host=True, hbm_budget=base.ws_bytes)   # 4 slots
    r_few = few.factor(A)
    r_many = many.factor(A)
    r_mid = mid.factor(A)
    for x, y, z in zip(r_few[:3], r_many[:3], r_mid[:3]):
        assert torch.equal(x, y) and torch.equal(x, z)
    # 4 slots for 6 tiles: tiles 0 and 1 stay resident, the other four stream
    # through two slots, and each later pass reuses the tile the last one ended on
    assert r_mid[3]["slots"] == 4
    assert r_mid[3]["tile_loads"] == 6 + (2 * q + 1) * (6 - 2 - 1)
    passes, tiles = 2 * q + 2, 6
    say("loads", r_few[3]["tile_loads"], r_many[3]["tile_loads"], r_few[3]["slots"], r_many[3]["slots"])
    assert r_few[3]["slots"] == 2 and r_many[3]["slots"] == tiles
    assert r_many[3]["tile_loads"] == tiles                      # every tile stays resident
    assert r_many[3]["h2d_bytes"] == m * n * 4
    # two slots: each pass after the first reuses the tile the previous one ended on
    assert r_few[3]["tile_loads"] == passes * tiles - (passes - 1)
    ref = oracle_rsvd(A.double().numpy(), k, p, q, seed=0)
    assert metrics.sigma_err(r_few[1].cpu().numpy(), ref["S"]) <= 1e-5


def test_per_matrix_limit_keeps_a_in_core():
    """Section 3.5's per-matrix limit: with room for every tile of A, A is
    copied once per call and the later passes read it from HBM; a smaller
    limit streams it through fewer slots.  The results do not change."""
    dev = need_gpu()
    m, n, tile, q = 3000, 2000, (1024, 1024), 2
    A = _workload(m, n, seed=13).pin_memory()
    k, p = 20, 12
    slot = 1024 * 1024 * 4
    ref = Plan(m, n, k, p, q, tile=tile, host=True).factor(A)
    keep = Plan(m, n, k, p, q, tile=tile, host=True, a_budget=6 * slot).factor(A)
    three = Plan(m, n, k, p, q, tile=tile, host=True, a_budget=3 * slot + 100).factor(A)
    say("per-matrix limit", keep[3]["slots"], keep[3]["tile_loads"], three[3]["slots"],
        three[3]["tile_loads"])
    assert keep[3]["slots"] == 6 and keep[3]["tile_loads"] == 6
    assert keep[3]["h2d_bytes"] == m * n * 4
    assert three[3]["slots"] == 3 and three[3]["tile_loads"] > 6
    for x, y, z in zip(ref[:3], keep[:3], three[:3]):
        assert torch.equal(x, y) and torch.equal(x, z)


def test_host_resident_bf16_storage():
    dev = need_gpu()
    m, n, tile = 2048, 1536, (512, 512)
    A = _workload(m, n, seed=13)
    A16 = A.to(torch.bfloat16)
    Ud, Sd, Vd, _ = Plan(m, n, 16, 16, 1, dtype=torch.bfloat16, precision="bf16",
                         tile=tile).factor(A16.to(dev))
    Uh, Sh, Vh, info = Plan(m, n, 16, 16, 1, dtype=torch.bfloat16, precision="bf16", tile=tile,
                            host=True).factor(A16.pin_memory())
    assert torch.equal(Sd, Sh) and torch.equal(Ud, Uh) and torch.equal(Vd, Vh)
    assert info["h2d_bytes"] >= m * n * 2


def test_host_resident_bf16_panel_width_128():
    """Width-128 panels take the direct-to-LDS product kernels, launched per
    tile slot here and over the whole matrix in HBM: bitwise the same."""
    dev = need_gpu()
    m, n, tile = 2048, 1536, (512, 512)
    A = _workload(m, n, seed=15)
    A16 = A.to(torch.bfloat16)
    Ud, Sd, Vd, _ = Plan(m, n, 100, 20, 1, dtype=torch.bfloat16, precision="bf16",
                         tile=tile).factor(A16.to(dev))
    Uh, Sh, Vh, info = Plan(m, n, 100, 20, 1, dtype=torch.bfloat16, precision="bf16", tile=tile,
                            host=True).factor(A16.pin_memory())
    assert torch.equal(Sd, Sh) and torch.equal(Ud, Uh) and torch.equal(Vd, Vh)


def test_pageable_host_memory_is_rejected():
    need_gpu()
    m, n = 1024, 768
    A = _workload(m, n, seed=14)                 # ordinary (pageable) CPU tensor
    plan = Plan(m, n, 8, 8, 1, host=True)
    with pytest.raises(L.RsvdError) as e:
        plan.factor(A)
    assert e.value.status == L.E_INVALID_ARG


def test_device_only_calls_refuse_host_plans():
    dev = need_gpu()
    m, n = 1024, 768
    A = _workload(m, n, seed=15).pin_memory()
    plan = Plan(m, n, 8, 8, 1, host=True)
    U, S, V, _ = plan.factor(A)
    ws = plan.workspace(dev)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    st = L.lib().rsvd_residual(plan.handle, ctypes.c_void_p(A.data_ptr()), n,
                               ctypes.c_void_p(U.data_ptr()), m, ctypes.c_void_p(S.data_ptr()),
                               ctypes.c_void_p(V.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                               ctypes.c_void_p(ws.data_ptr()), None)
    assert st == L.E_UNSUPPORTED
