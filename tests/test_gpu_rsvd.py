"""End-to-end parity of rsvd_factor (through the C ABI) with the FP64 oracle
on the same input and the same Gaussian test matrix.  FP32 form: sigma
relative error <= 1e-5 (the stated target); subspace angles are reported and
only loosely bounded (they depend on the gaps of the spectrum)."""
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

SIGMA_TOL_FP32 = 1e-5


def run_and_compare(A_host, k, p, q, seed=0, tile=None, flags=0, dtype=torch.float32,
                    expect_status=None, angle_tol=1e-3):
    dev = need_gpu()
    m, n = A_host.shape
    A = torch.as_tensor(A_host, dtype=dtype).to(dev)
    plan = Plan(m, n, k, p, q, seed=seed, dtype=dtype, tile=tile, flags=flags)
    U, S, V, info = plan.factor(A)
    torch.cuda.synchronize()
    U, S, V = U.cpu().double().numpy(), S.cpu().numpy(), V.cpu().double().numpy()
    Aref = A.cpu().double().numpy()          # the exact bytes the GPU saw
    ref = oracle_rsvd(Aref, k, p, q, seed=seed)
    err = metrics.sigma_err(S, ref["S"])
    su, sv = metrics.sin_theta(ref["U"], U), metrics.sin_theta(ref["V"], V)
    say(f"m={m} n={n} k={k} p={p} q={q}: sigma err {err:.2e}, sin U {su:.1e}, sin V {sv:.1e}, "
        f"status {info['status']}, dropped {info['dropped']}, sweeps {info['jacobi_sweeps']}, "
        f"{info['total_ms']:.2f} ms")
    assert err <= SIGMA_TOL_FP32
    assert su <= angle_tol and sv <= angle_tol
    assert metrics.orth_err(U) < 1e-5 and metrics.orth_err(V) < 1e-4
    # U^T A = S V^T holds exactly for the randomized SVD (B = Q^T A, U = Q U_B)
    lhs = U.T @ Aref
    assert np.max(np.abs(lhs - S[:, None] * V.T)) <= 1e-5 * S[0] * max(1.0, np.sqrt(n) / 100)
    for i in range(k):                      # sign convention
        j = int(np.argmax(np.abs(V[:, i])))
        assert V[j, i] > 0 or np.isclose(np.abs(V[:, i]).max(), np.sort(np.abs(V[:, i]))[-2])
    if expect_status is not None:
        assert info["status"] == expect_status
    return S, ref, info


def test_plain_small_workload():
    A, meta = workloads.make("plain_small")
    run_and_compare(A.numpy(), meta["k"], meta["p"], meta["q"], seed=0, dtype=torch.float64)


def test_plain_small_workload_fp32_storage():
    A, meta = workloads.make("plain_small", out_dtype=torch.float32)
    run_and_compare(A.numpy(), meta["k"], meta["p"], meta["q"], seed=0, tile=(512, 256))


@pytest.mark.parametrize("m,n,k,p,q,tile", [
    (1500, 900, 15, 10, 1, (256, 160)),
    (900, 1500, 15, 10, 2, (192, 256)),
    (1000, 1000, 40, 24, 0, (0, 0)),
    (3000, 400, 100, 90, 1, (1024, 128)),
    (140000, 300, 40, 24, 1, (0, 0)),    # tall: the m-side panel products stage W in LDS
])
def test_ragged_tiles_and_shapes(m, n, k, p, q, tile):
    sigma = workloads.spectrum_pow(min(m, n), 1.0)
    A = workloads.dense_lowrank(m, n, sigma, 1e-4, seed=m + n, out_dtype=torch.float32)
    run_and_compare(A.numpy(), k, p, q, tile=tile)


def test_full_sketch_equals_exact_svd():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((200, 48)).astype(np.float32)
    S, ref, _ = run_and_compare(A, 16, 32, 1)
    s_true = np.linalg.svd(A.astype(np.float64), compute_uv=False)[:16]
    assert metrics.sigma_err(S, s_true) < 1e-5


def test_tiny_matrix():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((8, 6)).astype(np.float32)
    run_and_compare(A, 3, 3, 2)


@pytest.mark.parametrize("k,p", [(1, 0), (1, 1), (2, 0)])
def test_sketch_widths_one_and_two(k, p):
    """l = 1 and l = 2: the tridiagonal small SVD has no reduction step (its
    tail block is all of C)."""
    sig = np.array([5.0, 2.0, 1.0, 0.5, 0.25, 0.1])
    A = workloads.dense_lowrank(400, 300, sig, 1e-3, seed=13, out_dtype=torch.float32).numpy()
    _, _, info = run_and_compare(A, k, p, 2)
    assert info["jacobi_sweeps"] == 0


def test_exact_recovery_of_low_rank_input_drops_directions():
    sig = np.array([4.0, 3.0, 2.0, 1.5, 1.0, 0.7, 0.5, 0.3])
    A = workloads.dense_lowrank(1200, 700, sig, 0.0, seed=11, out_dtype=torch.float32).numpy()
    S, _, info = run_and_compare(A, 8, 8, 1, expect_status=L.W_RANK_DEFICIENT)
    assert np.all(np.abs(S - sig) <= 1e-5 * sig)
    assert info["dropped"] > 0


def test_scaled_plain_gpu_workload():
    A, meta = workloads.make("plain_gpu", scale=0.2)
    run_and_compare(A.numpy(), meta["k"], meta["p"], meta["q"], tile=(1024, 1024))


def test_cholqr1_flag_same_result():
    A, meta = workloads.make("plain_gpu", scale=0.1)
    run_and_compare(A.numpy(), 50, 10, 2, flags=L.FLAG_CHOLQR1)


def test_small_svd_tridiagonal_matches_jacobi():
    """Widths <= 128 solve the small eigenproblem of C = B B^T through its
    tridiagonal form (Householder, bisection, inverse iteration) and keep the
    result only when W^T W = I and C W = W diag(lambda) hold to 1e-12; the
    Cholesky + one-sided Jacobi path (forced here by RSVD_FLAG_JACOBI_ONLY)
    gives the same factors."""
    dev = need_gpu()
    A, _ = workloads.make("plain_gpu", scale=0.1)
    A = A.to(dev)
    m, n = A.shape
    outs = []
    for flags in (0, L.FLAG_JACOBI_ONLY):
        plan = Plan(m, n, 100, 20, 2, tile=(1024, 1024), flags=flags)
        outs.append(plan.factor(A))
        torch.cuda.synchronize()
    (U1, S1, V1, i1), (U2, S2, V2, i2) = outs
    S1, S2 = S1.cpu().double().numpy(), S2.cpu().double().numpy()
    su = metrics.sin_theta(U2.cpu().double().numpy(), U1.cpu().double().numpy())
    sv = metrics.sin_theta(V2.cpu().double().numpy(), V1.cpu().double().numpy())
    say(f"tridiagonal vs Jacobi: sigma diff {np.max(np.abs(S1 - S2)) / S2[0]:.2e}, sin U {su:.1e}, "
        f"sin V {sv:.1e}, sweeps {i1['jacobi_sweeps']} / {i2['jacobi_sweeps']}")
    assert i1["jacobi_sweeps"] == 0 and i2["jacobi_sweeps"] > 0
    assert np.max(np.abs(S1 - S2)) <= 1e-6 * S2[0]
    assert su <= 1e-4 and sv <= 1e-4


@pytest.mark.parametrize("l", [33, 80, 97, 128])
def test_small_svd_tridiagonal_widths(l):
    """The tridiagonal small SVD keeps its register blocks of 32 rows and 16
    columns only while they hold live entries: width 33 takes two row blocks,
    80 three, 97 and 128 (the largest) four.  sigma_i = i^-1/2 with little
    noise keeps the eigenvalues of C apart, so the result must pass the
    kernel's own checks (no Jacobi sweeps), match the oracle, and give the
    factors of the Cholesky + one-sided Jacobi path."""
    dev = need_gpu()
    m, n, k, p = 3000, 1200, l - 10, 10
    A = workloads.dense_lowrank(m, n, np.arange(1, n + 1) ** -0.5, 1e-8, seed=21,
                                out_dtype=torch.float32)
    S1, _, info = run_and_compare(A.numpy(), k, p, 2, tile=(1024, 1024))
    assert info["jacobi_sweeps"] == 0
    plan = Plan(m, n, k, p, 2, tile=(1024, 1024), flags=L.FLAG_JACOBI_ONLY)
    U2, S2, V2, info2 = plan.factor(A.to(dev))
    torch.cuda.synchronize()
    plan1 = Plan(m, n, k, p, 2, tile=(1024, 1024))
    U1, _, V1, _ = plan1.factor(A.to(dev))
    torch.cuda.synchronize()
    S2 = S2.cpu().double().numpy()
    su = metrics.sin_theta(U2.cpu().double().numpy(), U1.cpu().double().numpy())
    sv = metrics.sin_theta(V2.cpu().double().numpy(), V1.cpu().double().numpy())
    say(f"l={l}: tridiagonal vs Jacobi sigma diff {np.max(np.abs(S1 - S2)) / S2[0]:.2e}, "
        f"sin U {su:.1e}, sin V {sv:.1e}, sweeps {info2['jacobi_sweeps']}")
    assert info2["jacobi_sweeps"] > 0
    assert np.max(np.abs(S1 - S2)) <= 1e-6 * S2[0]
    assert su <= 1e-4 and sv <= 1e-4


def test_small_svd_falls_back_to_jacobi_on_repeated_eigenvalues():
    """Rank 8 with l = 16: the dropped directions give C a repeated zero
    eigenvalue, independent inverse iterations are not orthogonal there, and
    the Jacobi path runs instead (on the device, no host decision)."""
    sig = np.array([4.0, 3.0, 2.0, 1.5, 1.0, 0.7, 0.5, 0.3])
    A = workloads.dense_lowrank(1200, 700, sig, 0.0, seed=12, out_dtype=torch.float32).numpy()
    S, _, info = run_and_compare(A, 8, 8, 1, expect_status=L.W_RANK_DEFICIENT)
    assert np.all(np.abs(S - sig) <= 1e-5 * sig)
    assert info["jacobi_sweeps"] > 0


def test_zero_matrix_gives_zero_factorisation():
    """A = 0: every direction is dropped and C = 0, where the tridiagonal
    path's inverse iterations overflow and its checks hand the call to the
    Jacobi path; S = 0 and U, V stay finite."""
    dev = need_gpu()
    A = torch.zeros(300, 200, device=dev)
    U, S, V, info = Plan(300, 200, 5, 5, 1).factor(A)
    torch.cuda.synchronize()
    say(f"zero matrix: status {info['status']}, sweeps {info['jacobi_sweeps']}")
    assert torch.all(S == 0)
    assert bool(torch.isfinite(U).all()) and bool(torch.isfinite(V).all())
    assert info["status"] in (L.OK, L.W_RANK_DEFICIENT)


def test_bitwise_deterministic():
    dev = need_gpu()
    A, _ = workloads.make("plain_gpu", scale=0.1)
    A = A.to(dev)
    plan = Plan(A.shape[0], A.shape[1], 50, 10, 2, tile=(512, 512))
    outs = [plan.factor(A)[:3] for _ in range(3)]
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert torch.equal(a, b)


def test_nonfinite_input_is_reported():
    dev = need_gpu()
    A = torch.randn(300, 200, device=dev)
    A[17, 33] = float("nan")
    plan = Plan(300, 200, 5, 5, 1)
    with pytest.raises(L.RsvdError) as e:
        plan.factor(A)
    assert e.value.status == L.E_NUMERIC


def test_unaligned_leading_dimension_is_accepted():
    dev = need_gpu()
    base = torch.randn(300 * 203, device=dev)
    A = base.as_strided((300, 201), (203, 1))
    plan = Plan(300, 201, 5, 5, 1)
    U, S, V, info = plan.factor(A)
    ref = oracle_rsvd(A.cpu().double().numpy(), 5, 5, 1, seed=0)
    assert metrics.sigma_err(S.cpu().numpy(), ref["S"]) <= SIGMA_TOL_FP32


def test_misaligned_base_pointer_is_rejected():
    import ctypes
    dev = need_gpu()
    base = torch.randn(300 * 201 + 4, device=dev)
    plan = Plan(300, 201, 5, 5, 1)
    ws = plan.workspace(dev)
    U = torch.empty(5, 300, device=dev)
    S = torch.empty(5, dtype=torch.float64, device=dev)
    V = torch.empty(5, 201, device=dev)
    st = L.lib().rsvd_factor(plan.handle, ctypes.c_void_p(base.data_ptr() + 2), 201,
                             ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(U.data_ptr()), 300,
                             ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(V.data_ptr()), 201,
                             None, None)
    assert st == L.E_INVALID_ARG
