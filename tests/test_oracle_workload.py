"""The oracle on the 2000 x 1000 plain workload (sigma_i = exp(-i/50)):
runs in seconds and stays within rSVD accuracy of the known spectrum."""
import time

import numpy as np

import workloads
from oracle import metrics
from oracle.rsvd import rsvd


def test_plain_small_workload_recovers_known_spectrum():
    A, meta = workloads.make("plain_small")
    A = A.numpy()
    t0 = time.time()
    out = rsvd(A, meta["k"], meta["p"], meta["q"], seed=0)
    assert time.time() - t0 < 30.0
    s_true = np.linalg.svd(A, compute_uv=False)
    # interlacing; the spectrum decays slowly (sigma_31/sigma_20 = e^-0.22,
    # raised to 2q+1 = 5 only gives 0.33), so rSVD sits a few percent below
    # the exact values, more so towards k
    assert np.all(out["S"] <= s_true[:20] * (1 + 1e-13))
    assert metrics.sigma_err(out["S"], s_true[:20]) < 0.05
    assert metrics.sigma_err(out["S"][:5], s_true[:5]) < 0.005
    assert abs(s_true[0] - np.exp(-1 / 50)) < 1e-3
