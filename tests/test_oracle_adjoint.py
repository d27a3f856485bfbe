"""Pins of the adjoint oracle (gradient of a loss on the eigenpairs in an interval).

Independent references: central finite differences of the loss evaluated with
scipy's tridiagonal eigensolver (a different library routine from the oracle's
dense eigh), the Hellmann-Feynman closed form for the eigenvalue part, and the
agreement of the two formulations (explicit eigen-sum and deflated solves).
"""

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import adjoint as adj
from workloads import generators as gen


def _loss_tridiagonal(v, c, emin, emax):
    lam, X = sla.eigh_tridiagonal(2.0 + v, -np.ones(v.size - 1), select="v", select_range=(emin, emax))
    return lam.sum() + float(np.sum(c[:, None] * X ** 2))


def _small_problem(n=300, seed=7):
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.0, 1.0, n)
    c = rng.standard_normal(n)
    lam = np.linalg.eigvalsh(adj.tridiag_dense(v))
    # an interval holding the 3rd..8th eigenvalues with clear gaps at both ends
    emin, emax = 0.5 * (lam[1] + lam[2]), 0.5 * (lam[7] + lam[8])
    return v, c, emin, emax


def test_gradient_matches_central_differences():
    v, c, emin, emax = _small_problem()
    L, gv, lamS, XS = adj.loss_and_grad_v(v, c, emin, emax)
    assert lamS.size == 6
    assert abs(L - _loss_tridiagonal(v, c, emin, emax)) < 1e-10 * abs(L)
    h = 1e-6
    fd = np.empty(v.size)
    for k in range(v.size):
        e = np.zeros(v.size)
        e[k] = h
        fd[k] = (_loss_tridiagonal(v + e, c, emin, emax) - _loss_tridiagonal(v - e, c, emin, emax)) / (2 * h)
    # central differences: O(h^2) truncation plus roundoff ~ eps |L| / h
    assert np.max(np.abs(fd - gv)) < 2e-7 * max(1.0, np.max(np.abs(gv))), np.max(np.abs(fd - gv))


def test_eigenvalue_part_is_hellmann_feynman():
    """With c = 0 the loss is sum of lambda_i and dL/dv_k = sum_i x_ik^2 exactly."""
    v, c, emin, emax = _small_problem(seed=9)
    L, gv, lamS, XS = adj.loss_and_grad_v(v, np.zeros_like(c), emin, emax)
    np.testing.assert_allclose(gv, np.sum(XS ** 2, axis=1), atol=1e-14)


def test_deflated_solves_equal_eigen_sum():
    v, c, emin, emax = _small_problem(n=240, seed=11)
    A = adj.tridiag_dense(v)
    lam, V, inside = adj.interval_pairs(A, emin, emax)
    XS = V[:, inside]
    g = np.ones(XS.shape[1])
    G = 2.0 * c[:, None] * XS
    gA1, Y1 = adj.grad_by_eigensum(lam, V, inside, g, G)
    gA2, Y2 = adj.grad_by_solves(A, lam[inside], XS, g, G)
    np.testing.assert_allclose(Y2, Y1, atol=1e-10 * np.max(np.abs(Y1)))
    np.testing.assert_allclose(gA2, gA1, atol=1e-10 * np.max(np.abs(gA1)))
    # y_i is orthogonal to span(X_S)
    assert np.max(np.abs(XS.T @ Y2)) < 1e-10 * np.max(np.abs(Y2))


def test_gradient_is_sign_invariant_and_symmetric():
    v, c, emin, emax = _small_problem(n=200, seed=13)
    A = adj.tridiag_dense(v)
    lam, V, inside = adj.interval_pairs(A, emin, emax)
    XS = V[:, inside].copy()
    g = np.ones(XS.shape[1])
    gA1, _ = adj.grad_by_solves(A, lam[inside], XS, g, 2.0 * c[:, None] * XS)
    XS[:, ::2] *= -1.0
    gA2, _ = adj.grad_by_solves(A, lam[inside], XS, g, 2.0 * c[:, None] * XS)
    np.testing.assert_allclose(gA1, gA2, atol=1e-12)
    np.testing.assert_allclose(gA1, gA1.T, atol=1e-14)


def test_workload_generator_and_interval_count():
    v, c, A = gen.differentiation_problem(512, seed=3)
    np.testing.assert_array_equal(A, adj.tridiag_dense(v))
    assert np.all((v >= 0) & (v < 1))
