"""Helpers for the GPU parity tests (inputs come from workloads/, expected
values from oracle/)."""
import sys

import numpy as np
import pytest
import torch


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch.device("cuda:0")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def col_major_from_numpy(X, device, dtype=torch.float32):
    """Column-major device tensor (rows, cols) with stride (1, rows)."""
    t = torch.as_tensor(np.ascontiguousarray(np.asarray(X).T), dtype=dtype, device=device)
    return t.T


def rand_panel(rows, cols, seed, scale=None):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((rows, cols))
    if scale is not None:
        X = X * scale[None, :]
    return X.astype(np.float32)


def gamma_bound(K, absprod, u=2.0 ** -24):
    """Componentwise bound |fl(AX) - AX| <= gamma_K |A||X| (Higham, Thm 3.5)."""
    g = K * u / (1.0 - K * u)
    return g * absprod
