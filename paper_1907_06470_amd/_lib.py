"""ctypes view of librsvd.so (the C ABI declared in include/rsvd.h).

Loading fails loudly: there is no fallback path.  Build the library first with
``python -c "import __graft_entry__ as g; g.build()"`` (or
``python paper_1907_06470_amd/csrc/build.py``).
"""

import ctypes
import os
import threading

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librsvd.so")

# status codes
OK = 0
W_RANK_DEFICIENT = 1
W_DEGENERATE = 2
STOPPED = 3
E_INVALID_ARG = -1
E_BUDGET = -2
E_HIP = -3
E_UNSUPPORTED = -4
E_NUMERIC = -5

DENSE, CSR, COO = 0, 1, 2
F64, F32, BF16, FP8E4M3 = 0, 1, 2, 3
LOC_DEVICE, LOC_HOST_PINNED = 0, 1
ORTHO_EACH, ORTHO_FINAL_ONLY = 0, 2
FLAG_NO_SIGN_FIX, FLAG_CHOLQR1, FLAG_BACKWARD, FLAG_AUTO_Q, FLAG_JACOBI_ONLY = 1, 2, 4, 8, 16

c_i32, c_i64, c_u32, c_u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
c_vp, c_sz = ctypes.c_void_p, ctypes.c_size_t


class Problem(ctypes.Structure):
    _fields_ = [("m", c_i64), ("n", c_i64), ("k", c_i64), ("p", c_i64), ("q", c_i64),
                ("format", c_i32), ("dtype", c_i32), ("loc", c_i32), ("reserved", c_i32),
                ("seed", c_u64), ("nnz", c_i64)]


class Options(ctypes.Structure):
    _fields_ = [("prec_sketch", c_i32), ("prec_power", c_i32), ("prec_project", c_i32),
                ("ortho", c_i32), ("tile_m", c_i64), ("tile_n", c_i64), ("grid_p", c_i64),
                ("grid_q", c_i64), ("hbm_budget_bytes", c_u64), ("flags", c_i32),
                ("reserved", c_i32), ("q_tol", ctypes.c_double), ("a_budget_bytes", c_u64),
                ("new_budget_bytes", c_u64)]


class Report(ctypes.Structure):
    _fields_ = [("stage_ms", ctypes.c_double * 8), ("total_ms", ctypes.c_double),
                ("flops_alg", ctypes.c_double), ("bytes_alg", ctypes.c_double),
                ("gemm_nn_ms", ctypes.c_double), ("gemm_tn_ms", ctypes.c_double),
                ("ws_bytes", c_i64), ("gemm_nn_launches", c_i32), ("gemm_tn_launches", c_i32),
                ("dropped", c_i32), ("jacobi_sweeps", c_i32), ("nonfinite", c_i32),
                ("slots", c_i32), ("h2d_bytes", ctypes.c_double), ("tile_loads", c_i64),
                ("q_used", c_i32), ("reserved2", c_i32), ("q_delta", ctypes.c_double),
                ("sketch_ms", ctypes.c_double), ("peak_hbm", c_i64)]


CKPT_MAGIC = 0x31504B4344565352   # "RSVDCKP1" little-endian
NOALLOC_WS_BYTES = 64 << 20      # static workspace of rsvd_factor_noalloc (rsvd.h)


class Checkpoint(ctypes.Structure):
    _fields_ = [("magic", c_u64), ("version", c_i32), ("passes", c_i32), ("m", c_i64),
                ("n", c_i64), ("k", c_i64), ("p", c_i64), ("q", c_i64), ("seed", c_u64),
                ("prec_sketch", c_i32), ("prec_power", c_i32), ("prec_project", c_i32),
                ("flags", c_i32), ("rows", c_i64), ("cols", c_i64), ("side", c_i32),
                ("dropped", c_i32), ("nonfinite", c_i32), ("pending", c_i32),
                ("panel_hash", c_u64)]


_P = ctypes.POINTER
_SIGS = {
    "rsvd_plan": (c_i32, [_P(Problem), _P(Options), _P(c_vp), _P(c_sz)]),
    "rsvd_factor": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp, c_i64, c_vp, c_vp, c_i64, c_vp,
                            _P(Report)]),
    "rsvd_factor_noalloc": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp, c_i64, c_vp]),
    "rsvd_backward": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp, c_i64, c_vp, c_i64,
                              c_vp, c_vp, _P(Report)]),
    "rsvd_factor_csr": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp, c_i64, c_vp,
                                _P(Report)]),
    "rsvd_factor_coo": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp,
                                c_i64, c_vp, _P(Report)]),
    "rsvd_checkpoint_bytes": (c_i32, [c_vp, _P(c_sz)]),
    "rsvd_factor_resumable": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp, c_i64, c_vp, c_vp, c_i64,
                                      c_vp, _P(Report), _P(Checkpoint), c_vp, c_i32,
                                      _P(Checkpoint), c_vp]),
    "rsvd_step_spmm": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp]),
    "rsvd_residual": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "rsvd_plan_destroy": (None, [c_vp]),
    "rsvd_plan_set_streams": (c_i32, [c_vp, c_vp, c_vp]),
    "rsvd_status_str": (ctypes.c_char_p, [c_i32]),
    "rsvd_last_error": (ctypes.c_char_p, [c_vp]),
    "rsvd_version": (ctypes.c_char_p, []),
    "rsvd_tile_map": (c_i32, [c_vp, _P(c_i64), c_sz, _P(c_sz)]),
    "rsvd_visit_order": (c_i32, [c_vp, c_i64, _P(c_i64), c_sz, _P(c_sz)]),
    "rsvd_philox_raw": (c_i32, [c_u64, c_u32, c_i64, c_i64, c_i64, c_vp, c_vp]),
    "rsvd_omega": (c_i32, [c_u64, c_i64, c_i64, c_i64, c_i64, c_i32, c_vp, c_i64, c_vp]),
    "rsvd_step_product": (c_i32, [c_vp, c_i32, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp]),
    "rsvd_step_orth": (c_i32, [c_vp, c_i32, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp]),
    "rsvd_step_gram": (c_i32, [c_vp, c_i32, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "rsvd_step_small_svd": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp]),
}

_lock = threading.Lock()
_lib = None


class RsvdError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"rsvd status {status}: {message}")
        self.status = status


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                                   "(__graft_entry__.build())")
            h = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(h, name)
                fn.restype = res
                fn.argtypes = args
            _lib = h
        return _lib


def exported_symbols():
    return list(_SIGS)


def check(status, plan=None, allow_warnings=True):
    """Raise RsvdError for error statuses; return the status otherwise."""
    if status < 0 or (status > 0 and not allow_warnings):
        L = lib()
        msg = L.rsvd_last_error(plan).decode(errors="replace")
        text = L.rsvd_status_str(status).decode()
        raise RsvdError(status, f"{text}: {msg}")
    return status
