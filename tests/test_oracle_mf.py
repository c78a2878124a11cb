"""Pins for the FP64 CSR matrix factorisation (Eq. 1-5, Alg. 1, Alg. 2)."""
import numpy as np
import pytest

from oracle import mf
import workloads


def _small():
    # 2 users x 3 items: user 0 rated items 0 and 2, user 1 rated item 1
    row_ptr = np.array([0, 2, 3])
    col_idx = np.array([0, 2, 1])
    vals = np.array([4.0, 2.0, 5.0])
    U = np.array([[0.1, 0.2], [0.3, -0.1]])
    V = np.array([[0.5, 0.0], [0.2, 0.4], [-0.3, 0.1]])
    return row_ptr, col_idx, vals, U, V


def test_r1_single_step_by_hand():
    row_ptr, col_idx, vals, U, V = _small()
    a, lam = 0.1, 0.5
    U2, V2, rhat = mf.epoch(U, V, row_ptr, col_idx, vals, a, lam, rule="R1")
    # by hand: predictions <u0,v0> = 0.05, <u0,v2> = -0.01, <u1,v1> = 0.02
    assert np.allclose(rhat, [0.05, -0.01, 0.02])
    e00, e02, e11 = 4 - 0.05, 2 + 0.01, 5 - 0.02
    u0 = (1 - a * lam * 2) * np.array([0.1, 0.2]) + a * (e00 * np.array([0.5, 0.0]) + e02 * np.array([-0.3, 0.1]))
    u1 = (1 - a * lam * 1) * np.array([0.3, -0.1]) + a * (e11 * np.array([0.2, 0.4]))
    v0 = (1 - a * lam * 1) * np.array([0.5, 0.0]) + a * e00 * np.array([0.1, 0.2])
    v1 = (1 - a * lam * 1) * np.array([0.2, 0.4]) + a * e11 * np.array([0.3, -0.1])
    v2 = (1 - a * lam * 1) * np.array([-0.3, 0.1]) + a * e02 * np.array([0.1, 0.2])
    assert np.allclose(U2, [u0, u1], atol=1e-15)
    assert np.allclose(V2, [v0, v1, v2], atol=1e-15)


def test_r1_is_gradient_step_of_per_rating_loss():
    """R1 = U - a * dL/dU for L = 1/2 sum_NZR [(r - <u,v>)^2 + lam (|u|^2 + |v|^2)]."""
    csr = workloads.tiny_ratings()
    U, V = workloads.init_factors(32, 64, 4)
    a, lam = 0.01, 0.02

    def L(U, V):
        e = csr.values - mf.predict(U, V, csr.row_ptr, csr.col_idx)
        rows = mf.csr_rows(csr.row_ptr)
        return 0.5 * np.sum(e ** 2) + 0.5 * lam * (np.sum(U[rows] ** 2) + np.sum(V[csr.col_idx] ** 2))

    U2, V2, _ = mf.epoch(U, V, csr.row_ptr, csr.col_idx, csr.values, a, lam, rule="R1")
    h = 1e-6
    for (i, f) in [(0, 0), (5, 3), (17, 1)]:
        Up, Um = U.copy(), U.copy()
        Up[i, f] += h
        Um[i, f] -= h
        g = (L(Up, V) - L(Um, V)) / (2 * h)
        assert abs(U2[i, f] - (U[i, f] - a * g)) < 1e-8
    for (j, f) in [(0, 0), (40, 2)]:
        Vp, Vm = V.copy(), V.copy()
        Vp[j, f] += h
        Vm[j, f] -= h
        g = (L(U, Vp) - L(U, Vm)) / (2 * h)
        assert abs(V2[j, f] - (V[j, f] - a * g)) < 1e-8


def test_eq4_eq5_are_half_the_gradient_of_eq1():
    csr = workloads.tiny_ratings()
    U, V = workloads.init_factors(32, 64, 4)
    lam, mu = 0.02, 0.03
    gU, gV = mf.grad_eq4_eq5(U, V, csr.row_ptr, csr.col_idx, csr.values, lam, mu)
    h = 1e-6
    for (i, f) in [(0, 0), (9, 2)]:
        Up, Um = U.copy(), U.copy()
        Up[i, f] += h
        Um[i, f] -= h
        fd = (mf.loss_eq1(Up, V, csr.row_ptr, csr.col_idx, csr.values, lam, mu)
              - mf.loss_eq1(Um, V, csr.row_ptr, csr.col_idx, csr.values, lam, mu)) / (2 * h)
        assert abs(fd - 2 * gU[i, f]) < 1e-7
    for (j, f) in [(3, 1)]:
        Vp, Vm = V.copy(), V.copy()
        Vp[j, f] += h
        Vm[j, f] -= h
        fd = (mf.loss_eq1(U, Vp, csr.row_ptr, csr.col_idx, csr.values, lam, mu)
              - mf.loss_eq1(U, Vm, csr.row_ptr, csr.col_idx, csr.values, lam, mu)) / (2 * h)
        assert abs(fd - 2 * gV[j, f]) < 1e-7


def test_r2_equals_r1_when_all_degrees_equal():
    # every user rates exactly 2 items and every item is rated by exactly 2 users
    row_ptr = np.array([0, 2, 4, 6])
    col_idx = np.array([0, 1, 1, 2, 0, 2])
    vals = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 1.0])
    U, V = workloads.init_factors(3, 3, 2, seed=3)
    a, lam = 0.05, 0.1
    U1, V1, _ = mf.epoch(U, V, row_ptr, col_idx, vals, a, lam, rule="R1")
    U2, V2, _ = mf.epoch(U, V, row_ptr, col_idx, vals, 2 * a, lam, rule="R2")
    assert np.allclose(U1, U2, atol=1e-15) and np.allclose(V1, V2, atol=1e-15)


def test_synchronous_epoch_equals_accumulated_sequential_sum():
    """Alg. 2 accumulator: summing the per-rating gradient terms (all evaluated at
    the epoch-start factors) and applying once equals the synchronous epoch."""
    csr = workloads.tiny_ratings()
    U, V = workloads.init_factors(32, 64, 4)
    a, lam = 0.01, 0.02
    U2, V2, _ = mf.epoch(U, V, csr.row_ptr, csr.col_idx, csr.values, a, lam, rule="R1")
    accU = np.zeros_like(U)
    accV = np.zeros_like(V)
    rows = mf.csr_rows(csr.row_ptr)
    for idx, (i, j) in enumerate(zip(rows, csr.col_idx)):
        err = csr.values[idx] - U[i] @ V[j]
        accU[i] += a * (err * V[j] - lam * U[i])
        accV[j] += a * (err * U[i] - lam * V[j])
    assert np.allclose(U + accU, U2, atol=1e-15) and np.allclose(V + accV, V2, atol=1e-15)


def test_dampened_rate_and_empty_rows_r2():
    csr = workloads.tiny_ratings()
    U, V = workloads.init_factors(32, 64, 4)
    d = np.diff(csr.row_ptr)
    c = np.bincount(csr.col_idx, minlength=64)
    U2, V2, _ = mf.epoch(U, V, csr.row_ptr, csr.col_idx, csr.values, 0.01, 0.02, t=3, damp=0.1, rule="R2")
    assert np.array_equal(U2[d == 0], U[d == 0]) and np.array_equal(V2[c == 0], V[c == 0])
    Ua, _, _ = mf.epoch(U, V, csr.row_ptr, csr.col_idx, csr.values, 0.01 / 1.3, 0.02, rule="R2")
    assert np.allclose(Ua, U2, atol=1e-15)


def test_training_reduces_rmse():
    csr = workloads.tiny_ratings()
    U, V = workloads.init_factors(32, 64, 4, sigma=0.5)
    r0 = mf.rmse(mf.predict(U, V, csr.row_ptr, csr.col_idx), csr.values)
    U2, V2, _ = mf.train(U, V, csr.row_ptr, csr.col_idx, csr.values, 0.02, 0.02, 200)
    r1 = mf.rmse(mf.predict(U2, V2, csr.row_ptr, csr.col_idx), csr.values)
    assert r1 < 0.5 * r0


def test_rmse_eq10():
    assert mf.rmse([1.0, 2.0, 4.0], [1.0, 3.0, 2.0]) == pytest.approx(np.sqrt(5 / 3))
