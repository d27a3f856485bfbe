"""Pins of the stochastic eigenvalue-count oracle (fpm(14)=2) against facts that do
not come from the oracle itself: the published SplitMix64 test vector (probe signs),
the zero-variance case of Rademacher probes on a diagonal matrix (exact sum of the
filter, and with 32 nodes the exact integer count), identity probes (the filter
trace from a library eigendecomposition, real and complex Hermitian, which also
catches a dropped conjugate-node term) and Hutchinson's variance bound.
"""

import json
import os

import numpy as np

from oracle.contour import half_contour, rational_filter
from oracle.splitmix import rademacher_block
from oracle.stochastic import filtered_trace, stochastic_count
from workloads import generators as gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_probe_signs_follow_published_splitmix_outputs():
    with open(os.path.join(GOLDEN, "splitmix64.json")) as fh:
        gold = json.load(fh)
    want = np.array([-1.0 if int(v) >> 63 else 1.0 for v in gold["seed_1234567"]])
    got = rademacher_block(5, 1, 1234567)[:, 0]
    np.testing.assert_array_equal(got, want)
    # column-major counter: entry (i, j) uses output i + j n
    Y = rademacher_block(2, 2, 1234567)
    np.testing.assert_array_equal(Y[:, 0], want[:2])
    np.testing.assert_array_equal(Y[:, 1], want[2:4])


def test_diagonal_matrix_gives_the_filter_sum_exactly():
    # with y_r^2 = 1 every probe sees sum_r rho(a_r): no variance at all
    rng = np.random.default_rng(11)
    a = np.sort(rng.uniform(-2.0, 2.0, 60))
    A = np.diag(a)
    for seed in (0, 5, 123):
        est, M = stochastic_count(A, None, -0.6, 0.9, 7, ne=3, seed=seed)
        z, w = half_contour(-0.6, 0.9, 3)
        assert abs(est - rational_filter(a, z, w).sum()) < 1e-12
        assert M == int(np.floor(est + 0.5))


def test_diagonal_matrix_with_many_nodes_counts_exactly():
    # entries kept 0.1 away from the interval ends: a 32-node filter is 1 inside and 0
    # outside to within 1e-4, so the estimate is the integer count
    a = np.concatenate([np.linspace(-3.0, -0.7, 9), np.linspace(-0.5, 0.5, 13), np.linspace(0.7, 3.0, 8)])
    est, M = stochastic_count(np.diag(a), None, -0.6, 0.6, 5, ne=32, seed=2)
    assert abs(est - 13.0) < 1e-3
    assert M == 13


def _filter_trace_by_eigs(A, B, z, w):
    lam = np.linalg.eigvalsh(A) if B is None else np.linalg.eigvals(np.linalg.solve(B, A)).real
    return rational_filter(lam, z, w).sum()


def test_identity_probes_give_the_filter_trace_real_pencil():
    rng = np.random.default_rng(3)
    n = 40
    A, _, _ = gen.prescribed_real_problem(n, rng, -2.0, 2.0)
    C = rng.standard_normal((n, n))
    B = np.eye(n) + 0.1 * C @ C.T / n
    z, w = half_contour(-0.8, 0.5, 4)
    got = filtered_trace(A, B, np.eye(n), z, w)
    assert abs(got - _filter_trace_by_eigs(A, B, z, w)) < 1e-10 * n


def test_identity_probes_give_the_filter_trace_complex_pencil():
    n = 30
    A, B, lam, _ = gen.prescribed_complex_pencil(n, seed=4, lam_lo=-2.0, lam_hi=2.0)
    z, w = half_contour(-0.8, 0.5, 3)
    got = filtered_trace(A, B, np.eye(n), z, w)
    assert abs(got - rational_filter(lam, z, w).sum()) < 1e-10 * n


def test_random_probes_within_hutchinson_bound():
    # Var(y^T F y) = 2 (||F||_F^2 - sum_i F_ii^2) for Rademacher y and symmetric F
    rng = np.random.default_rng(8)
    n, m0 = 80, 400
    A, _, _ = gen.prescribed_real_problem(n, rng, -1.0, 1.0)
    z, w = half_contour(-0.4, 0.3, 3)
    lam, V = np.linalg.eigh(A)
    F = (V * rational_filter(lam, z, w)[None, :]) @ V.T
    sigma = np.sqrt(2.0 * (np.sum(F * F) - np.sum(np.diag(F) ** 2)) / m0)
    est, _ = stochastic_count(A, None, -0.4, 0.3, m0, ne=3, seed=9)
    assert abs(est - np.trace(F)) < 5.0 * sigma, (est, np.trace(F), sigma)
