"""Pins of the oracle's polynomial FEAST (Section 3.4): matrix polynomials built with known
eigenpairs, the reduction to the linear non-Hermitian oracle for degree 1, and the
algebraic identity behind the residual form."""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import nonhermitian as nh
from oracle import polynomial as po
from workloads import generators as gen


def _sin(X, Y):
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    return float(np.linalg.norm(qx - qy @ (qy.conj().T @ qx), 2))


def test_generator_eigenpairs():
    """The construction's eigenpairs satisfy P(lambda) x = 0 (checks the generator)."""
    As, lam, X = gen.prescribed_polynomial(40, 3, 1, leading=True)
    for i in range(0, lam.size, 7):
        assert np.linalg.norm(po.poly_eval(As, lam[i]) @ X[:, i]) < 1e-11


@pytest.mark.parametrize("p,leading,extra", [(2, False, 10), (2, True, 20), (3, False, 20)])
def test_prescribed_polynomial_eigenpairs(p, leading, extra):
    As, lam, Xe = gen.prescribed_polynomial(100, p, 3, leading=leading)
    emid, r = 0.2 - 0.1j, 0.8
    inside = nh.inside_ellipse(lam, emid, r)
    cnt = int(inside.sum())
    out = po.feast_polynomial(As, emid, r, cnt + extra)
    assert out["info"] == 0 and out["M"] == cnt
    E = out["E"][:cnt]
    li = lam[inside]
    Xi = Xe[:, inside]
    for q, e in enumerate(E):
        i = int(np.argmin(np.abs(li - e)))
        assert abs(li[i] - e) <= 1e-10 * (abs(emid) + r)
        assert _sin(out["X"][:, [q]], Xi[:, [i]]) <= 1e-8
    assert np.max(out["res"][:cnt]) < 1e-12


def test_degree_one_is_the_linear_problem():
    """P(lambda) = -A + lambda B: the eigenvalues of the non-Hermitian oracle (one-sided)."""
    A, B, lam, V, Y = gen.prescribed_nonnormal(120, 8, generalized=True)
    emid, r = 0.1 + 0.2j, 1.0
    cnt = int(nh.inside_ellipse(lam, emid, r).sum())
    out = po.feast_polynomial([-A, B], emid, r, cnt + 10)
    fpm = nh.nfeastinit()
    fpm[14] = 1
    ref = nh.feast_general(A, B, emid, r, cnt + 10, fpm)
    assert out["info"] == ref["info"] == 0 and out["M"] == ref["M"] == cnt
    np.testing.assert_allclose(np.sort_complex(out["E"][:cnt]), np.sort_complex(ref["E"][:cnt]), atol=1e-11)


def test_residual_form_is_the_divided_difference_contour():
    """For any X and values lambda: rho(l) x - sum_j w_j/(z_j - l) P(z_j)^-1 P(l) x equals
    sum_j w_j P(z_j)^-1 [(P(z_j) - P(l)) / (z_j - l)] x (the divided difference), exactly."""
    rng = np.random.default_rng(2)
    n, m = 30, 5
    As = [(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n) for _ in range(3)]
    z, w = nh.full_contour(0.3 + 0.1j, 1.2, 10)
    facts = [sla.lu_factor(po.poly_eval(As, zj)) for zj in z]
    X = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    lam = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    Q = po.contour_residual(facts, z, w, As, X, lam)
    ref = np.zeros_like(X)
    for i in range(m):
        for j in range(len(z)):
            Dd = (po.poly_eval(As, z[j]) - po.poly_eval(As, lam[i])) / (z[j] - lam[i])
            ref[:, i] += w[j] * np.linalg.solve(po.poly_eval(As, z[j]), Dd @ X[:, i])
    np.testing.assert_allclose(Q, ref, rtol=1e-10, atol=1e-12)


def test_argument_checks():
    A = np.eye(8, dtype=complex)
    assert po.feast_polynomial([A], 0.0, 1.0, 4)["info"] == -102
    f = po.pfeastinit()
    f[14] = 0
    assert po.feast_polynomial([A, A], 0.0, 1.0, 4, f)["info"] == 115
    assert po.feast_polynomial([A, A], 0.0, 0.0, 4)["info"] == 200


@pytest.mark.parametrize("n,p,seed,leading,emid,r,extra", [
    (333, 2, 5, True, -0.3 + 0.4j, 0.9, {}),
    (120, 3, 7, False, 0.1 + 0.1j, 1.0, {17: 70, 18: 20}),
])
def test_found_pairs_are_eigenpairs_at_every_iteration(n, p, seed, leading, emid, r, extra):
    """R-pfound: over the whole history, every pair counted in M is within 1e-5 alpha of a
    constructed eigenvalue inside the contour (no spurious value of the linearization is
    counted), and the run ends with all of them (M0 = 1.5 times the count)."""
    As, lam, Xe = gen.prescribed_polynomial(n, p, seed, leading=leading)
    fpm = po.pfeastinit()
    for k, v in extra.items():
        fpm[k] = v
    inside = nh.inside_ellipse(lam, emid, r, int(fpm[17]), int(fpm[18]))
    cnt = int(inside.sum())
    out = po.feast_polynomial(As, emid, r, int(np.ceil(1.5 * cnt)), fpm)
    assert out["info"] == 0 and out["M"] == cnt
    alpha = abs(emid) + r
    li = lam[inside]
    for h in out["history"]:
        assert h["M"] <= cnt
        for e in h["E"]:
            assert np.min(np.abs(li - e)) <= 1e-5 * alpha


def test_subspace_crowded_by_the_linearization_gives_info_3():
    """M0 a little above the count: the 2 M0 values of the quadratic's linearization put
    at least M0 inside the contour at the first iteration, which reports info 3; M0 below
    the count does too."""
    As, lam, Xe = gen.prescribed_polynomial(333, 2, 5, leading=True)
    emid, r = -0.3 + 0.4j, 0.9
    cnt = int(nh.inside_ellipse(lam, emid, r).sum())
    assert po.feast_polynomial(As, emid, r, cnt + 20)["info"] == 3
    assert po.feast_polynomial(As, emid, r, cnt // 3)["info"] == 3
