"""Per-pass persistence (Section 3.8), host side: the checkpoint header's
layout, the file round trip, and the checks rsvd_factor_resumable makes
before anything runs (a checkpoint of another problem, a pass out of range,
a wrong shape, a panel that does not match its hash)."""
import ctypes

import numpy as np
import pytest

from paper_1907_06470_amd import Checkpoint, Plan
from paper_1907_06470_amd import _lib as L


def _fnv1a_words(panel):
    h = 0xcbf29ce484222325
    for w in np.ascontiguousarray(panel, dtype=np.float32).view(np.uint32).ravel():
        h ^= int(w)
        h = (h * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_header_layout_matches_the_c_struct():
    # u64, 2 x i32, 5 x i64, u64, 4 x i32, 2 x i64, 4 x i32, u64 with natural alignment
    assert ctypes.sizeof(L.Checkpoint) == 120
    assert L.Checkpoint.passes.offset == 12
    assert L.Checkpoint.seed.offset == 56
    assert L.Checkpoint.rows.offset == 80
    assert L.Checkpoint.side.offset == 96
    assert L.Checkpoint.pending.offset == 108
    assert L.Checkpoint.panel_hash.offset == 112
    assert bytes.fromhex("%016x" % L.CKPT_MAGIC)[::-1] == b"RSVDCKP1"


def _header(plan, passes, side, rows, panel):
    # rows: the state rows; the panel also carries lp rows of a pending factor
    h = L.Checkpoint()
    h.magic, h.version, h.passes = L.CKPT_MAGIC, 1, passes
    h.m, h.n, h.k, h.p, h.q, h.seed = plan.m, plan.n, plan.k, plan.p, plan.q, plan.seed
    h.prec_sketch = h.prec_power = h.prec_project = L.F32
    h.flags = 0
    h.rows, h.cols, h.side = rows + panel.shape[0], panel.shape[0], side
    h.panel_hash = _fnv1a_words(panel)
    return h


def test_file_round_trip(tmp_path):
    plan = Plan(60, 40, 5, 3, 1, seed=7)
    rng = np.random.default_rng(0)
    panel = rng.standard_normal((32, 60 + 32)).astype(np.float32)
    ck = Checkpoint(_header(plan, 1, 0, 60, panel), panel)
    path = tmp_path / "state.ckpt"
    ck.save(path)
    back = Checkpoint.load(path)
    assert bytes(back.header) == bytes(ck.header)
    assert np.array_equal(back.panel, panel)
    with open(path, "r+b") as f:       # truncate the panel
        f.truncate(ctypes.sizeof(L.Checkpoint) + 100)
    with pytest.raises(ValueError):
        Checkpoint.load(path)


def _call(plan, hdr, panel, stop_after=0):
    # dummy device pointers: only calls that fail a host-side check before any
    # HIP call may be made with them
    dummy = ctypes.c_void_p(256)
    return L.lib().rsvd_factor_resumable(
        plan.handle, dummy, plan.n, dummy, dummy, plan.m, dummy, dummy, plan.n, None, None,
        ctypes.byref(hdr) if hdr is not None else None,
        ctypes.c_void_p(panel.ctypes.data) if panel is not None else None, stop_after, None, None)


def test_resume_checks_reject_before_running():
    plan = Plan(60, 40, 5, 3, 1, seed=7)        # lp = 32, q = 1: passes 1..4
    rng = np.random.default_rng(1)
    good = np.ascontiguousarray(rng.standard_normal((32, 40 + 32)).astype(np.float32))
    hdr = _header(plan, 2, 1, 40, good)          # pass 2: the n-side panel
    bad = []
    h = _header(plan, 2, 1, 40, good); h.magic ^= 1; bad.append((h, good, "not a version-1"))
    h = _header(plan, 2, 1, 40, good); h.seed += 1; bad.append((h, good, "another problem"))
    h = _header(plan, 2, 1, 40, good); h.prec_power = L.BF16; bad.append((h, good, "another problem"))
    h = _header(plan, 5, 1, 40, good); bad.append((h, good, "out of range"))
    h = _header(plan, 3, 1, 40, good); bad.append((h, good, "shape"))           # pass 3 is m-side
    h = _header(plan, 2, 0, 40, good); bad.append((h, good, "shape"))
    tampered = good.copy(); tampered[3, 7] += 1.0
    bad.append((hdr, tampered, "hash"))
    for h, panel, words in bad:
        st = _call(plan, h, panel)
        assert st == L.E_INVALID_ARG
        assert words in L.lib().rsvd_last_error(plan.handle).decode()
    # stop_after out of range, or not after the resumed pass
    assert _call(plan, None, None, stop_after=5) == L.E_INVALID_ARG
    assert _call(plan, hdr, good, stop_after=2) == L.E_INVALID_ARG


def test_resume_unsupported_combinations():
    auto = Plan(60, 40, 5, 3, 1, auto_q=True)
    st = _call(auto, None, None)
    assert st == L.E_UNSUPPORTED
    n = ctypes.c_size_t()
    plan = Plan(60, 40, 5, 3, 1)
    assert L.lib().rsvd_checkpoint_bytes(plan.handle, ctypes.byref(n)) == L.OK
    assert n.value == (60 + 40 + 32) * 32 * 4
