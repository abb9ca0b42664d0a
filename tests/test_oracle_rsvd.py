"""Pins of the oracle randomized SVD (Sections 2.1-2.2) against mathematics:
exact recovery, full-sketch equality with the SVD, interlacing, the
U^T A = S V^T identity, Eckart-Young and the power-matrix identity."""
import numpy as np
import pytest

from oracle import metrics
from oracle.jacobi import jacobi_svd
from oracle.rsvd import rsvd, range_finder


def lowrank(m, n, sig, seed, noise=0.0):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, len(sig))))
    V, _ = np.linalg.qr(rng.standard_normal((n, len(sig))))
    A = (U * np.asarray(sig)) @ V.T
    if noise:
        A = A + noise * rng.standard_normal((m, n))
    return A, U, V


@pytest.mark.parametrize("q", [0, 1, 2])
def test_exact_recovery_rank_le_k(q):
    sig = np.array([5.0, 3.0, 2.0, 1.0, 0.5, 0.25])
    A, U0, V0 = lowrank(120, 80, sig, seed=10)
    out = rsvd(A, k=6, p=4, q=q, seed=3)
    assert np.allclose(out["S"], sig, rtol=1e-12)
    assert np.max(np.abs(A @ out["V"] - out["U"] * out["S"])) < 1e-12
    assert metrics.sin_theta(U0, out["U"]) < 1e-12
    assert metrics.sin_theta(V0, out["V"]) < 1e-12
    assert metrics.orth_err(out["U"]) < 1e-13 and metrics.orth_err(out["V"]) < 1e-13


def test_full_sketch_equals_lapack_svd():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((60, 25))
    out = rsvd(A, k=10, p=15, q=1, seed=9)         # l = n: the sketch spans everything
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    assert np.allclose(out["S"], s[:10], rtol=1e-12)
    assert metrics.sin_theta(U[:, :10], out["U"]) < 1e-10
    assert metrics.sin_theta(Vt[:10].T, out["V"]) < 1e-10


@pytest.mark.parametrize("shape", [(8, 6), (6, 8), (7, 7), (5, 3)])
def test_tiny_full_sketch_equals_bruteforce_jacobi(shape):
    rng = np.random.default_rng(sum(shape))
    A = rng.standard_normal(shape)
    mn = min(shape)
    out = rsvd(A, k=mn, p=0, q=2, seed=1)
    Uj, sj, Vj = jacobi_svd(A)
    assert np.allclose(out["S"], sj, rtol=1e-12)
    Ua, Va = metrics.align_signs(Uj, out["U"], out["V"])
    assert np.allclose(Ua, Uj, atol=1e-11) and np.allclose(Va, Vj, atol=1e-11)


def test_interlacing_identity_and_eckart_young():
    sig = 1.0 / np.arange(1, 41)
    A, _, _ = lowrank(300, 200, sig, seed=2, noise=1e-3)
    s_true = np.linalg.svd(A, compute_uv=False)
    for q in (0, 1, 3):
        out = rsvd(A, k=10, p=5, q=q, seed=5, full=True)
        # compressions of A cannot exceed its singular values
        assert np.all(out["Sl"] <= s_true[:15] + 1e-13 * s_true[0])
        # U_l^T A = S_l V_l^T exactly (B = Q^T A and U_l = Q U_B)
        lhs = out["Ul"].T @ A
        assert np.max(np.abs(lhs - out["Sl"][:, None] * out["Vl"].T)) < 1e-13
        r = metrics.residual_fro(A, out["U"], out["S"], out["V"])
        assert r >= np.sqrt(np.sum(s_true[10:] ** 2)) * (1 - 1e-12)


def test_power_iteration_improves_accuracy():
    sig = 1.0 / np.arange(1, 201) ** 0.5
    A, _, _ = lowrank(400, 300, sig, seed=8, noise=1e-4)
    s_true = np.linalg.svd(A, compute_uv=False)[:10]
    errs = [metrics.sigma_err(rsvd(A, 10, 5, q, seed=1)["S"], s_true) for q in (0, 1, 3)]
    assert errs[0] > errs[1] > errs[2]


@pytest.mark.parametrize("q", [1, 2])
def test_power_matrix_identity(q):
    # Section 2.2: A_q = (A A^T)^q A has the singular vectors of A and
    # singular values sigma^(2q+1)
    rng = np.random.default_rng(q)
    A = rng.standard_normal((9, 6)) / 3.0
    Aq = A.copy()
    for _ in range(q):
        Aq = A @ (A.T @ Aq)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    Uq, sq, Vqt = np.linalg.svd(Aq, full_matrices=False)
    assert np.allclose(sq, s ** (2 * q + 1), rtol=1e-10)
    assert np.allclose(np.abs(np.sum(U * Uq, axis=0)), 1.0, atol=1e-8)
    assert np.allclose(np.abs(np.sum(Vt * Vqt, axis=1)), 1.0, atol=1e-8)


def test_schedules_span_the_same_subspace():
    # Eq. (2) as printed (orthonormalise once at the end) and the
    # re-orthonormalised schedule span the same subspace in exact arithmetic
    sig = np.array([1.0, 0.9, 0.8, 0.7, 0.6, 0.5, 0.45, 0.4])
    A, _, _ = lowrank(50, 40, sig, seed=6, noise=1e-3)
    Qe = range_finder(A, 8, 1, seed=2, ortho="each")
    Qf = range_finder(A, 8, 1, seed=2, ortho="final_only")
    assert metrics.sin_theta(Qe, Qf) < 1e-9


def test_invalid_arguments():
    A = np.zeros((10, 5))
    for k, p, q in [(0, 1, 0), (3, 3, 0), (2, -1, 0), (2, 1, -1)]:
        with pytest.raises(ValueError):
            rsvd(A, k, p, q)


def test_sign_convention():
    sig = np.array([3.0, 2.0, 1.0])
    A, _, _ = lowrank(30, 20, sig, seed=12)
    out = rsvd(A, 3, 2, 1, seed=0)
    for i in range(3):
        j = np.argmax(np.abs(out["V"][:, i]))
        assert out["V"][j, i] > 0


# ---- automatic iteration parameter (Section 2.2) ------------------------------
from oracle.rsvd import rsvd_auto_q  # noqa: E402


def _graded(m, n, decay, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.arange(1, n + 1, dtype=np.float64) ** (-decay)
    return (U * s) @ V.T


def test_auto_q_equals_fixed_q_at_the_chosen_q():
    A = _graded(300, 120, 0.7, 1)
    auto = rsvd_auto_q(A, 10, 5, 6, tol=1e-6)
    fixed = rsvd(A, 10, 5, auto["q_used"])
    assert 1 <= auto["q_used"] <= 6
    for key in ("U", "S", "V"):
        assert np.array_equal(auto[key], fixed[key])


def test_auto_q_zero_tolerance_runs_to_the_maximum():
    A = _graded(200, 90, 0.5, 2)
    auto = rsvd_auto_q(A, 8, 4, 3, tol=0.0)
    assert auto["q_used"] == 3 and len(auto["deltas"]) == 3
    assert np.array_equal(auto["S"], rsvd(A, 8, 4, 3)["S"])


def test_auto_q_follows_the_decay_of_the_spectrum():
    # fast decay: the sketch already captures the top k, q stops at 1;
    # slow decay: more steps before the values settle
    fast = rsvd_auto_q(_graded(300, 150, 3.0, 3), 10, 10, 8, tol=1e-8)
    slow = rsvd_auto_q(_graded(300, 150, 0.3, 3), 10, 10, 8, tol=1e-8)
    assert fast["q_used"] < slow["q_used"]
    # the singular values grow toward the exact ones as q increases
    exact = np.linalg.svd(_graded(300, 150, 0.3, 3), compute_uv=False)[:10]
    assert np.all(slow["S"] <= exact * (1 + 1e-12))
    assert np.max(np.abs(slow["S"] - exact) / exact) < np.max(
        np.abs(rsvd(_graded(300, 150, 0.3, 3), 10, 10, 0)["S"] - exact) / exact)
