"""Pins of the oracle's accuracy measures and of its Box-Muller step with
hand-computed answers (every parity verdict goes through these functions).

* sigma_err: the relative error of the leading singular values, with the
  floor that keeps near-zero values from dividing by zero.
* sin_theta: the sine of the largest principal angle between two subspaces,
  checked on two planes in R^4 that meet at a known angle.
* residual_fro: ||A - U diag(S) V^T||_F of a matrix whose difference from
  the factors is a known rank-1 matrix.
* orth_err: max |U^T U - I| of column pairs with a known inner product.
* box_muller (Section 2.1, step 1: independent N(0, 1) entries): the uniform
  that feeds the logarithm and the cos / sin order are fixed by inputs whose
  outputs are exact in closed form.
"""

import math

import numpy as np
import pytest

from oracle import metrics, philox


def test_sigma_err_three_values():
    s_ref = np.array([4.0, 2.0, 1.0])
    s_hat = np.array([4.4, 1.9, 1.0])
    # |0.4| / 4 = 0.1, |0.1| / 2 = 0.05, 0
    assert metrics.sigma_err(s_hat, s_ref) == pytest.approx(0.1, rel=1e-15)
    assert metrics.sigma_err(s_hat, s_ref, k=1) == pytest.approx(0.1, rel=1e-15)
    assert metrics.sigma_err(s_hat[1:], s_ref[1:]) == pytest.approx(0.05, rel=1e-14)


def test_sigma_err_floor():
    # the second value is below floor * s_1 = 1e-6: the error is measured
    # against 1e-6, not against 1e-8
    s_ref = np.array([1.0, 1e-8, 0.5])
    s_hat = np.array([1.0, 2e-8, 0.5])
    assert metrics.sigma_err(s_hat, s_ref) == pytest.approx(1e-2, rel=1e-9)


@pytest.mark.parametrize("theta", [0.0, 1e-6, 0.3, math.pi / 4, 1.2, math.pi / 2])
def test_sin_theta_two_planes(theta):
    e = np.eye(4)
    U_ref = e[:, :2]
    # the plane spanned by e1 and cos(t) e2 + sin(t) e3 meets span(e1, e2) at angle t
    U_hat = np.stack([e[:, 0], math.cos(theta) * e[:, 1] + math.sin(theta) * e[:, 2]], axis=1)
    assert metrics.sin_theta(U_ref, U_hat) == pytest.approx(math.sin(theta), rel=1e-12, abs=1e-15)
    # basis invariance: mix the columns of U_hat by a rotation and scale them
    c, s = math.cos(0.7), math.sin(0.7)
    mixed = U_hat @ np.array([[c, -s], [s, c]]) @ np.diag([3.0, 0.5])
    assert metrics.sin_theta(U_ref, mixed) == pytest.approx(math.sin(theta), rel=1e-12, abs=1e-15)
    assert metrics.sin_theta(mixed, U_ref) == pytest.approx(math.sin(theta), rel=1e-12, abs=1e-15)


def test_residual_fro_rank_one_difference():
    rng = np.random.default_rng(3)
    U, _ = np.linalg.qr(rng.standard_normal((7, 3)))
    V, _ = np.linalg.qr(rng.standard_normal((5, 3)))
    S = np.array([3.0, 2.0, 0.5])
    x = np.array([1.0, 0.0, -2.0, 0.0, 0.0, 0.0, 2.0])    # ||x|| = 3
    y = np.array([0.0, 4.0, 0.0, 3.0, 0.0])               # ||y|| = 5
    A = (U * S) @ V.T + 0.1 * np.outer(x, y)
    # ||0.1 x y^T||_F = 0.1 * 3 * 5
    assert metrics.residual_fro(A, U, S, V, block=3) == pytest.approx(1.5, rel=1e-13)
    assert metrics.residual_fro((U * S) @ V.T, U, S, V) == pytest.approx(0.0, abs=1e-13)


def test_residual_fro_truncation():
    A = np.diag([3.0, 2.0, 1.0])
    e = np.eye(3)
    # keeping the first singular triplet leaves sqrt(2^2 + 1^2)
    assert metrics.residual_fro(A, e[:, :1], np.array([3.0]), e[:, :1]) == pytest.approx(math.sqrt(5.0))


def test_orth_err_known_pairs():
    a = 0.3
    U = np.array([[1.0, math.cos(a)], [0.0, math.sin(a)]])
    # U^T U - I has cos(a) off the diagonal and zero on it
    assert metrics.orth_err(U) == pytest.approx(math.cos(a), rel=1e-14)
    assert metrics.orth_err(np.diag([2.0, 1.0])) == pytest.approx(3.0)
    assert metrics.orth_err(np.eye(5)[:, :3]) == 0.0


def test_box_muller_known_answers():
    # u_a = e^-2 gives radius sqrt(-2 ln u_a) = 2; u_b = 1/4 gives angle pi / 2
    za, zb = philox.box_muller(np.array([math.exp(-2.0)]), np.array([0.25]))
    assert abs(za[0]) < 1e-15
    assert zb[0] == pytest.approx(2.0, rel=1e-15)
    # u_b = 1/8: angle pi / 4, both values sqrt(2)
    za, zb = philox.box_muller(np.array([math.exp(-2.0)]), np.array([0.125]))
    assert za[0] == pytest.approx(math.sqrt(2.0), rel=1e-15)
    assert zb[0] == pytest.approx(math.sqrt(2.0), rel=1e-15)
    # u_b = 1/2: angle pi, (-radius, 0); the radius uses u_a only
    za, zb = philox.box_muller(np.array([math.exp(-4.5)]), np.array([0.5]))
    assert za[0] == pytest.approx(-3.0, rel=1e-15)
    assert abs(zb[0]) < 1e-15
