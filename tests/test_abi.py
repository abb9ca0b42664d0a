"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/rsvd.h declares; rsvd_plan validates its
arguments; tile maps and visit orders equal the oracle's bit for bit."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from oracle import tilemap
from paper_1907_06470_amd import _lib as L
from paper_1907_06470_amd.api import Plan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsvd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsvd_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.exported_symbols())


def test_version_and_status_strings():
    lib = L.lib()
    assert lib.rsvd_version().decode().startswith("rsvd-mi355x")
    for s in (0, 1, 2, -1, -2, -3, -4, -5):
        assert lib.rsvd_status_str(s)
    assert lib.rsvd_status_str(99) == b"unknown status"


def make(m=100, n=80, k=5, p=5, q=1, **kw):
    return Plan(m, n, k, p, q, **kw)


@pytest.mark.parametrize("args,status", [
    (dict(k=0), L.E_INVALID_ARG),
    (dict(p=-1), L.E_INVALID_ARG),
    (dict(q=-1), L.E_INVALID_ARG),
    (dict(k=50, p=40), L.E_INVALID_ARG),          # k + p > min(m, n)
    (dict(tile=(100, 64)), L.E_INVALID_ARG),      # not a multiple of 32
    (dict(precision="fp16"), L.E_INVALID_ARG),
    (dict(precision="fp8", tile=(96, 64)), L.E_INVALID_ARG),   # FP8 blocks are 64 x 64
    (dict(precision=("fp8", "bf16", "fp4")), L.E_INVALID_ARG),
])
def test_plan_rejects_bad_arguments(args, status):
    with pytest.raises(L.RsvdError) as e:
        make(**args)
    assert e.value.status == status
    assert L.lib().rsvd_last_error(None)


def test_plan_budget_error_names_the_bytes():
    with pytest.raises(L.RsvdError) as e:
        make(hbm_budget=1024)
    assert e.value.status == L.E_BUDGET
    assert "bytes" in str(e.value)
    p = make()
    ok = make(hbm_budget=p.ws_bytes)
    assert ok.ws_bytes == p.ws_bytes


def test_plan_unsupported_combinations():
    prob = L.Problem(m=100, n=80, k=5, p=5, q=1, format=L.CSR, dtype=L.F64, loc=L.LOC_DEVICE,
                     seed=0, nnz=400)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    assert L.lib().rsvd_plan(ctypes.byref(prob), None, ctypes.byref(h), ctypes.byref(ws)) == L.E_UNSUPPORTED
    prob.dtype = L.F32
    prob.loc = L.LOC_HOST_PINNED          # sparse input lives on the device
    assert L.lib().rsvd_plan(ctypes.byref(prob), None, ctypes.byref(h), ctypes.byref(ws)) == L.E_UNSUPPORTED
    prob.loc = L.LOC_DEVICE
    prob.nnz = -1
    assert L.lib().rsvd_plan(ctypes.byref(prob), None, ctypes.byref(h), ctypes.byref(ws)) == L.E_INVALID_ARG
    prob.nnz = 1 << 31                     # int32 indices
    assert L.lib().rsvd_plan(ctypes.byref(prob), None, ctypes.byref(h), ctypes.byref(ws)) == L.E_INVALID_ARG
    prob.nnz = 400
    assert L.lib().rsvd_plan(ctypes.byref(prob), None, ctypes.byref(h), ctypes.byref(ws)) == L.OK
    L.lib().rsvd_plan_destroy(h)
    prob.format = L.DENSE
    prob.loc = L.LOC_HOST_PINNED
    prob.dtype = L.F64            # streamed tiles are FP32 or BF16
    assert L.lib().rsvd_plan(ctypes.byref(prob), None, ctypes.byref(h), ctypes.byref(ws)) == L.E_UNSUPPORTED
    prob.dtype = L.F32
    prob.loc = 7
    assert L.lib().rsvd_plan(ctypes.byref(prob), None, ctypes.byref(h), ctypes.byref(ws)) == L.E_INVALID_ARG
    assert L.lib().rsvd_plan(None, None, ctypes.byref(h), ctypes.byref(ws)) == L.E_INVALID_ARG


def test_plan_with_null_options_uses_defaults():
    prob = L.Problem(m=300, n=200, k=10, p=5, q=2, format=L.DENSE, dtype=L.F32,
                     loc=L.LOC_DEVICE, seed=3)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    assert L.lib().rsvd_plan(ctypes.byref(prob), None, ctypes.byref(h), ctypes.byref(ws)) == L.OK
    assert ws.value > 0 and ws.value % 256 == 0
    L.lib().rsvd_plan_destroy(h)
    L.lib().rsvd_plan_destroy(None)


@pytest.mark.parametrize("m,n,tile,grid", [
    (50000, 20000, (4096, 4096), (1, 1)),
    (200000, 100000, (8192, 8192), (1, 1)),
    (1000, 700, (256, 192), (1, 1)),
    (1000, 700, (256, 192), (3, 2)),
    (97, 65, (32, 64), (2, 5)),
])
def test_tile_map_matches_oracle(m, n, tile, grid):
    p = Plan(m, n, 10, 5, 1, tile=tile, grid=grid)
    got = p.tile_map().numpy()
    ref = tilemap.tile_descriptors(m, n, tile[0], tile[1], grid[0], grid[1])
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)
    TI, TJ = tilemap.num_tiles(m, tile[0]), tilemap.num_tiles(n, tile[1])
    for t in range(2 * 1 + 2):
        assert np.array_equal(p.visit_order(t).numpy(), tilemap.visit_order(TI, TJ, t))


def test_auto_tiles_cover_the_matrix():
    p = Plan(50000, 20000, 100, 20, 2)
    d = p.tile_map().numpy()
    assert d[:, 3].sum() == 50000 * len(np.unique(d[:, 1]))
    assert d[:, 5].sum() == 20000 * len(np.unique(d[:, 0]))


def test_workspace_prediction_is_deterministic_and_monotone():
    a = Plan(1000, 500, 10, 10, 1).ws_bytes
    b = Plan(1000, 500, 10, 10, 1).ws_bytes
    c = Plan(2000, 500, 10, 10, 1).ws_bytes
    assert a == b and c > a


def test_missing_library_fails_loudly():
    code = ("import paper_1907_06470_amd._lib as L; L.LIB_PATH = '/nonexistent/librsvd.so'; "
            "L._lib = None\ntry:\n    L.lib()\nexcept RuntimeError as e:\n    print('LOUD', e)")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT)
    assert "LOUD" in out.stdout


def _host_plan_ws(budget, flags=0, prec=None, m=4096, n=3072, tile=(1024, 1024), a_budget=0,
                  new_budget=0, host=True):
    prob = L.Problem(m=m, n=n, k=20, p=12, q=1, format=L.DENSE, dtype=L.F32,
                     loc=L.LOC_HOST_PINNED if host else L.LOC_DEVICE, seed=0)
    pr = L.F32 if prec is None else prec
    opt = L.Options(prec_sketch=pr, prec_power=pr, prec_project=pr, ortho=0, tile_m=tile[0],
                    tile_n=tile[1], grid_p=1, grid_q=1, hbm_budget_bytes=budget, flags=flags,
                    a_budget_bytes=a_budget, new_budget_bytes=new_budget)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    st = L.lib().rsvd_plan(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(h), ctypes.byref(ws))
    if st == L.OK:
        L.lib().rsvd_plan_destroy(h)
    return st, ws.value


def test_host_resident_plans_size_their_tile_slots_from_the_budget():
    slot = 1024 * 1024 * 4
    st, ws_free = _host_plan_ws(0)              # no budget: four slots
    assert st == L.OK
    st, ws2 = _host_plan_ws(ws_free)            # the same bytes as a budget: same plan
    assert st == L.OK and ws2 == ws_free
    base = ws_free - 4 * slot
    st, ws_min = _host_plan_ws(base + 2 * slot)   # exactly two slots fit
    assert st == L.OK and ws_min == base + 2 * slot
    st, _ = _host_plan_ws(base + 2 * slot - 1)    # fewer than two: refused with the bytes
    assert st == L.E_BUDGET
    assert b"bytes" in L.lib().rsvd_last_error(None)
    st, ws_all = _host_plan_ws(base + 100 * slot)  # never more slots than tiles (4 x 3)
    assert st == L.OK and ws_all == base + 12 * slot


def test_per_operand_limits_follow_the_three_limit_chain():
    """Section 3.5: a limit for the tiles of A, one for the matrices the plan
    builds, one global; an unset limit takes the next one's value."""
    slot = 1024 * 1024 * 4
    _, ws_free = _host_plan_ws(0)
    own = ws_free - 4 * slot                        # everything but the four default slots
    # the limit on A alone sets the slots: 7 of the 12 tiles, all 12, at least 2
    assert _host_plan_ws(0, a_budget=7 * slot + 5) == (L.OK, own + 7 * slot)
    assert _host_plan_ws(0, a_budget=100 * slot) == (L.OK, own + 12 * slot)
    st, _ = _host_plan_ws(0, a_budget=2 * slot - 1)
    assert st == L.E_BUDGET and b"slots" in L.lib().rsvd_last_error(None)
    # the new-matrix limit bounds the plan's own matrices ...
    st, _ = _host_plan_ws(0, a_budget=4 * slot, new_budget=own - 1)
    assert st == L.E_BUDGET and b"own matrices" in L.lib().rsvd_last_error(None)
    assert _host_plan_ws(0, a_budget=4 * slot, new_budget=own) == (L.OK, own + 4 * slot)
    # ... and stands in for the limit on A when that one is unset (A then has
    # an allowance of its own, the same size)
    nb = own + 3 * slot
    assert _host_plan_ws(0, new_budget=nb) == (L.OK, own + (nb // slot) * slot)
    assert _host_plan_ws(0, new_budget=own + 20 * slot) == (L.OK, own + 12 * slot)
    # the global limit still caps the sum
    st, _ = _host_plan_ws(own + 5 * slot, a_budget=6 * slot)
    assert st == L.E_BUDGET
    assert _host_plan_ws(own + 6 * slot, a_budget=6 * slot) == (L.OK, own + 6 * slot)
    # a device-resident A above its limit is refused (plan it host-resident)
    m, n = 4096, 3072
    st, _ = _host_plan_ws(0, a_budget=m * n * 4 - 1, host=False)
    assert st == L.E_BUDGET and b"host-resident" in L.lib().rsvd_last_error(None)
    assert _host_plan_ws(0, a_budget=m * n * 4, host=False)[0] == L.OK


def test_host_resident_plans_reject_other_precisions_and_the_adjoint():
    assert _host_plan_ws(0, prec=L.BF16)[0] == L.E_UNSUPPORTED
    assert _host_plan_ws(0, flags=L.FLAG_BACKWARD)[0] == L.E_UNSUPPORTED


def test_noalloc_entry_point_refuses_plans_beyond_its_static_workspace():
    # checked on the host before any device call: stand-in pointers are never touched
    plan = Plan(50000, 20000, 100, 20, 2)
    assert plan.ws_bytes > L.NOALLOC_WS_BYTES
    fake = ctypes.c_void_p(256)
    st = L.lib().rsvd_factor_noalloc(plan.handle, fake, 20000, fake, 50000, fake, fake, 20000, None)
    assert st == L.E_BUDGET
    msg = L.lib().rsvd_last_error(plan.handle).decode()
    assert str(plan.ws_bytes) in msg and str(L.NOALLOC_WS_BYTES) in msg
    sparse = Plan(1000, 800, 10, 6, 1, nnz=5000)
    st = L.lib().rsvd_factor_noalloc(sparse.handle, fake, 800, fake, 1000, fake, fake, 800, None)
    assert st == L.E_UNSUPPORTED
