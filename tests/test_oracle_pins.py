"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a closed form, a value printed in
the FEAST v4.0 User Guide (fixtures under tests/golden/), a published generator
test vector, an independent textbook method (Sylvester inertia, brute-force
Jacobi), or an exact algebraic identity.  Chosen so that a dropped term, a
wrong sign, a wrong conjugation or a transposed operand in the oracle fails at
least one of them.
"""

import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle.feast import _Factored, _contour_classic, _contour_residual
from workloads import generators as gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


# ----------------------------------------------------------------------------
# independent helpers (textbook methods, not the oracle's code path)
# ----------------------------------------------------------------------------

def jacobi_eigh_bruteforce(H, sweeps=60):
    """Cyclic two-sided Jacobi for a small Hermitian matrix, written out in Python loops."""
    H = np.array(H, dtype=np.complex128)
    n = H.shape[0]
    V = np.eye(n, dtype=np.complex128)
    for _ in range(sweeps):
        off = np.sqrt(max(0.0, np.sum(np.abs(H) ** 2) - np.sum(np.abs(np.diag(H)) ** 2)))
        if off < 1e-15 * np.linalg.norm(H):
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                b = H[p, q]
                if abs(b) == 0.0:
                    continue
                a = H[p, p].real
                d = H[q, q].real
                ph = b / abs(b)
                tau = (d - a) / (2.0 * abs(b))
                if abs(tau) > 1e150:
                    t = 0.5 / tau
                else:
                    t = (1.0 if tau >= 0 else -1.0) / (abs(tau) + np.sqrt(1.0 + tau * tau))
                c = 1.0 / np.sqrt(1.0 + t * t)
                s = t * c
                # J acts on columns p, q: [c, s*ph; -s*conj(ph), c]
                J = np.array([[c, s * ph], [-s * np.conj(ph), c]])
                cols = H[:, [p, q]] @ J
                H[:, p], H[:, q] = cols[:, 0], cols[:, 1]
                rows = J.conj().T @ H[[p, q], :]
                H[p, :], H[q, :] = rows[0, :], rows[1, :]
                vc = V[:, [p, q]] @ J
                V[:, p], V[:, q] = vc[:, 0], vc[:, 1]
    return np.real(np.diag(H)), V


def cholesky_bruteforce(B):
    n = B.shape[0]
    L = np.zeros_like(B, dtype=np.complex128)
    for j in range(n):
        s = B[j, j] - np.sum(np.abs(L[j, :j]) ** 2)
        L[j, j] = np.sqrt(s.real)
        for i in range(j + 1, n):
            L[i, j] = (B[i, j] - np.sum(L[i, :j] * np.conj(L[j, :j]))) / L[j, j]
    return L


def inertia_count(A, B, a, b):
    """#eigenvalues of (A, B) in [a, b] by Sylvester's law: nu(A - bB) - nu(A - aB)."""
    def neg(M):
        _, D, _ = sla.ldl(M)
        return int(np.sum(np.linalg.eigvalsh(D) < 0))
    return neg(A - b * B) - neg(A - a * B)


def subspace_angle(X, Y, B=None):
    """Largest principal angle between span(X) and span(Y) in the B-inner product."""
    if B is not None:
        L = np.linalg.cholesky(B)
        X = L.conj().T @ X
        Y = L.conj().T @ Y
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    # sine form: accurate for small angles (arccos of a cosine is not)
    s = np.linalg.norm(qx - qy @ (qy.conj().T @ qx), 2)
    return float(np.arcsin(min(1.0, s)))


def clusters(lam, tol):
    groups, cur = [], [0]
    for i in range(1, len(lam)):
        if lam[i] - lam[i - 1] < tol:
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    groups.append(cur)
    return groups


# ----------------------------------------------------------------------------
# contour (quadrature) pins
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("ne", [4, 8, 16])
def test_trapezoid_circle_matches_closed_form_filter(ne):
    """Trapezoidal rule on a circle gives rho(lambda) = 1 / (1 + t^(2 ne)), t = (lambda-c)/r."""
    emin, emax = -0.3, 1.7
    z, w = oracle.half_contour(emin, emax, ne, rule=1, ratio_pct=100)
    c, r = 0.5 * (emin + emax), 0.5 * (emax - emin)
    lam = np.linspace(-2.0, 3.5, 57)
    lam = lam[np.abs(np.abs((lam - c) / r) - 1.0) > 1e-3]
    t = (lam - c) / r
    np.testing.assert_allclose(oracle.rational_filter(lam, z, w), 1.0 / (1.0 + t ** (2 * ne)),
                               rtol=1e-12, atol=1e-14)
    # exactly one half at both ends of the interval
    np.testing.assert_allclose(oracle.rational_filter([emin, emax], z, w), [0.5, 0.5], atol=1e-14)


def test_gauss_circle_centre_is_one_and_filter_symmetric():
    """Circle + Gauss: rho(c) = sum(om)/2 = 1 exactly; rho(c+t) = rho(c-t)."""
    z, w = oracle.half_contour(2.0, 6.0, 8, rule=0, ratio_pct=100)
    assert abs(oracle.rational_filter([4.0], z, w)[0] - 1.0) < 1e-14
    t = np.linspace(0.05, 5.0, 40)
    np.testing.assert_allclose(oracle.rational_filter(4.0 + t, z, w),
                               oracle.rational_filter(4.0 - t, z, w), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("ratio", [30, 100])
def test_gauss_quadrature_cauchy_integrals(ratio):
    """sum_j w_j g(z_j) + conj(w_j) g(conj z_j) -> (1/2 pi i) contour integral of g.

    g = 1/(z - a): 1 for a inside, 0 outside; g = polynomial: 0 (Cauchy's theorem).
    """
    z, w = oracle.half_contour(-1.0, 3.0, 56, rule=0, ratio_pct=ratio)

    def integ(g):
        return np.sum(w * g(z) + np.conj(w) * g(np.conj(z)))

    for a, expect in [(1.0, 1.0), (0.2, 1.0), (2.4, 1.0), (4.5, 0.0), (-3.0, 0.0)]:
        val = integ(lambda zz: 1.0 / (zz - a))
        assert abs(val - expect) < 1e-9, (a, val)
    for k in range(0, 5):
        assert abs(integ(lambda zz: zz ** k)) < 1e-10


def test_contour_node_order_and_count():
    z, w = oracle.half_contour(0.0, 0.5, 8)
    assert len(z) == 8 and np.all(np.diff(z.real) > 0) and np.all(z.imag > 0)
    x, om = oracle.gauss_legendre_rule(8)
    assert abs(np.sum(om) - 2.0) < 1e-14 and np.all(np.diff(x) > 0)


# ----------------------------------------------------------------------------
# generator pins
# ----------------------------------------------------------------------------

def test_splitmix64_published_vectors():
    gold = _load("splitmix64.json")
    got = oracle.splitmix.splitmix64_raw(1234567, 5)
    assert [int(v) for v in got] == [int(s) for s in gold["seed_1234567"]]
    got0 = oracle.splitmix.splitmix64_raw(0, 2)
    assert [int(v) for v in got0] == [int(s) for s in gold["seed_0"]]


def test_initial_subspace_layout():
    Y = oracle.initial_subspace(5, 3, 7, False)
    flat = oracle.splitmix64_uniform(7, 15)
    assert Y[2, 1] == flat[2 + 1 * 5]
    Yc = oracle.initial_subspace(5, 3, 7, True)
    flatc = oracle.splitmix64_uniform(7, 30)
    assert Yc[4, 2] == flatc[2 * (4 + 2 * 5)] + 1j * flatc[2 * (4 + 2 * 5) + 1]
    assert np.all(np.abs(Y) <= 1.0)


# ----------------------------------------------------------------------------
# whole-method pins
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("form", ["residual", "classic"])
def test_helloworld_matches_guide_output(form):
    g = _load("helloworld.json")
    A = np.array(g["A"], dtype=np.float64)
    assert np.allclose(np.linalg.eigvalsh(A), g["all_eigenvalues"], atol=1e-12)
    r = oracle.feast_dense(A, None, g["emin"], g["emax"], g["m0"], form=form)
    p = g["printed"]
    assert r["info"] == 0
    assert r["M"] == p["M"]
    np.testing.assert_allclose(r["E"][:r["M"]], p["E"], atol=1e-13)
    assert abs(np.sum(r["E"][:r["M"]]) - p["trace_final"]) < 1e-13
    assert r["loop"] == p["loop"]
    assert np.max(r["res"][:r["M"]]) < 1e-12
    X = r["X"][:, :r["M"]]
    np.testing.assert_allclose(A @ X, 4.0 * X, atol=1e-12)
    np.testing.assert_allclose(X.T @ X, np.eye(2), atol=1e-12)
    assert r["history"][0]["epsout"] == 1.0


@pytest.mark.parametrize("form", ["residual", "classic"])
def test_laplacian_1d_closed_form(form):
    """tridiag(-1,2,-1), n=200, [0, 0.5]: 46 eigenvalues 2-2cos(k pi/201), sine eigenvectors."""
    n = 200
    A = gen.laplacian_1d_dense(n)
    r = oracle.feast_dense(A, None, 0.0, 0.5, 70, form=form)
    assert r["info"] == 0
    k = np.arange(1, n + 1)
    lam = 2.0 - 2.0 * np.cos(k * np.pi / (n + 1))
    inside = np.sort(lam[(lam >= 0) & (lam <= 0.5)])
    assert r["M"] == 46 == inside.size
    np.testing.assert_allclose(r["E"][:46], inside, rtol=0, atol=1e-13)
    assert abs(np.sum(r["E"][:46]) - 7.972983218787455) < 1e-12
    i = np.arange(1, n + 1)[:, None]
    Xex = np.sqrt(2.0 / (n + 1)) * np.sin(i * k[None, :46] * np.pi / (n + 1))
    X = r["X"][:, :46]
    for col in range(46):
        assert abs(abs(X[:, col] @ Xex[:, col]) - 1.0) < 1e-12
    assert np.max(r["res"][:46]) < 1e-12


def test_classic_and_residual_forms_agree_per_iteration():
    A, B, lam, X = gen.prescribed_complex_pencil(160, seed=5, lam_lo=-4, lam_hi=4)
    fpm = oracle.feastinit()
    fpm[2] = 14
    a = oracle.feast_dense(A, B, -0.5, 0.5, 30, fpm, form="classic")
    b = oracle.feast_dense(A, B, -0.5, 0.5, 30, fpm, form="residual")
    assert a["M"] == b["M"] and a["info"] == b["info"] == 0
    for ha, hb in zip(a["history"], b["history"]):
        assert ha["M"] == hb["M"]
        assert abs(ha["trace"] - hb["trace"]) < 1e-12 * max(1.0, abs(ha["trace"]))
    np.testing.assert_allclose(a["E"][:a["M"]], b["E"][:b["M"]], rtol=0, atol=1e-12)


def test_residual_contour_identity_exact():
    """For ANY X and diagonal Lambda the residual-form sum equals the classic sum on B X."""
    rng = np.random.default_rng(3)
    n, m = 40, 6
    A, B, _, _ = gen.prescribed_complex_pencil(n, seed=9, lam_lo=-2, lam_hi=2)
    z, w = oracle.half_contour(-0.7, 0.9, 8)
    facts = [_Factored(zj, A, B) for zj in z]
    X = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    lam = rng.uniform(-3, 3, m)
    R = A @ X - (B @ X) * lam[None, :]
    q_res = _contour_residual(facts, z, w, X, lam, R, False)
    q_cls = _contour_classic(facts, z, w, B @ X, False)
    np.testing.assert_allclose(q_res, q_cls, rtol=0, atol=1e-11 * np.abs(q_cls).max())
    # real symmetric version
    Ar = gen.laplacian_1d_dense(n)
    facts_r = [_Factored(zj, Ar, None) for zj in z]
    Xr = rng.standard_normal((n, m))
    Rr = Ar @ Xr - Xr * lam[None, :]
    np.testing.assert_allclose(_contour_residual(facts_r, z, w, Xr, lam, Rr, True),
                               _contour_classic(facts_r, z, w, Xr, True), atol=1e-11)


def test_diagonal_matrix_gives_filter_times_block():
    """A = diag(a), B = I: the subspace after one contour is diag(rho(a_ii)) Y exactly."""
    rng = np.random.default_rng(11)
    a = rng.uniform(-2.0, 3.0, 30)
    Y = rng.standard_normal((30, 5))
    fpm = oracle.feastinit()
    fpm[4] = 1    # fpm(5): use X0
    fpm[13] = 1   # fpm(14): return Q after one contour
    r = oracle.feast_dense(np.diag(a), None, -0.5, 1.0, 5, fpm, X0=Y)
    assert r["info"] == 4
    z, w = oracle.half_contour(-0.5, 1.0, 8)
    np.testing.assert_allclose(r["X"], oracle.rational_filter(a, z, w)[:, None] * Y,
                               rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("is_complex", [False, True])
def test_tiny_pencils_against_bruteforce_jacobi(is_complex):
    """n = 12 random generalized pencils: eigenvalues in the interval equal those of a
    hand-written Cholesky + cyclic Jacobi reduction; count equals Sylvester inertia."""
    rng = np.random.default_rng(21 + int(is_complex))
    n = 12
    G = rng.standard_normal((n, n)) + (1j * rng.standard_normal((n, n)) if is_complex else 0)
    A = 0.5 * (G + G.conj().T)
    H = rng.standard_normal((n, n)) + (1j * rng.standard_normal((n, n)) if is_complex else 0)
    B = np.eye(n) + 0.05 * (H @ H.conj().T)
    L = cholesky_bruteforce(B)
    Li = np.linalg.inv(L)
    lam_all, _ = jacobi_eigh_bruteforce(Li @ A @ Li.conj().T)
    lam_all = np.sort(lam_all)
    emin = 0.5 * (lam_all[3] + lam_all[4])
    emax = 0.5 * (lam_all[7] + lam_all[8])
    expect = lam_all[4:8]
    fpm = oracle.feastinit()
    r = oracle.feast_dense(A, B, emin, emax, 8, fpm)
    assert r["info"] == 0
    assert r["M"] == 4 == inertia_count(A, B, emin, emax)
    np.testing.assert_allclose(r["E"][:4], expect, atol=1e-12)
    X = r["X"][:, :4]
    np.testing.assert_allclose(X.conj().T @ B @ X, np.eye(4), atol=1e-12)


def test_prescribed_complex_pencil_exact_spectrum_and_vectors():
    n = 192
    A, B, lam, Xex = gen.prescribed_complex_pencil(n, seed=2, lam_lo=-5, lam_hi=5)
    emin, emax = -1.0, 1.0
    cnt = int(np.sum((lam >= emin) & (lam <= emax)))
    assert cnt == inertia_count(A, B, emin, emax)
    r = oracle.feast_dense(A, B, emin, emax, int(np.ceil(1.6 * cnt)) + 4)
    assert r["info"] == 0 and r["M"] == cnt
    inside = lam[(lam >= emin) & (lam <= emax)]
    np.testing.assert_allclose(r["E"][:cnt], inside, atol=1e-11)
    X = r["X"][:, :cnt]
    np.testing.assert_allclose(X.conj().T @ B @ X, np.eye(cnt), atol=1e-11)
    sel = Xex[:, (lam >= emin) & (lam <= emax)]
    for grp in clusters(inside, 1e-4):
        assert subspace_angle(X[:, grp], sel[:, grp], B) < 1e-8


def test_uplo_triangles_expand_to_full():
    A, B, _, _ = gen.prescribed_complex_pencil(24, seed=1)
    for uplo, T in (("L", np.tril(A)), ("U", np.triu(A))):
        np.testing.assert_allclose(oracle.expand_uplo(T, uplo), A, atol=1e-14)


# ----------------------------------------------------------------------------
# info codes (Table tab_info)
# ----------------------------------------------------------------------------

def test_argument_errors():
    A = gen.laplacian_1d_dense(10)
    fpm = oracle.feastinit()
    assert oracle.feast_dense(np.zeros((0, 0)), None, 0, 1, 1, fpm)["info"] == 202
    assert oracle.feast_dense(A, None, 0, 1, 11, fpm)["info"] == 201
    assert oracle.feast_dense(A, None, 0, 1, 0, fpm)["info"] == 201
    assert oracle.feast_dense(A, None, 1, 1, 4, fpm)["info"] == 200
    for idx, val, code in [(1, 21, 102), (2, 17, 103), (3, -1, 104), (4, 2, 105),
                           (5, 2, 106), (13, 3, 114), (15, 3, 116), (17, 0, 118), (41, 2, 142)]:
        f = fpm.copy()
        f[idx] = val
        assert oracle.feast_dense(A, None, 0, 1, 4, f)["info"] == code, (idx, val)
    f = fpm.copy()
    f[15] = 1
    f[1] = 21   # trapezoidal accepts any positive count
    assert oracle.feast_dense(A, None, 0, 1, 6, f)["info"] in (0, 2, 3)


def test_warnings_and_reduced_errors():
    A = gen.laplacian_1d_dense(40)
    # empty interval -> 1
    assert oracle.feast_dense(A, None, 5.0, 6.0, 4)["info"] == 1
    # M0 too small for the 10 eigenvalues in [0, 0.5] -> 3
    lam = gen.laplacian_1d_eigs(40)
    assert int(np.sum(lam <= 0.5)) > 3
    assert oracle.feast_dense(A, None, 0.0, 0.5, 3)["info"] == 3
    # no convergence within fpm(4)=0 loops at eps=1e-16 -> 2
    f = oracle.feastinit()
    f[2] = 16
    f[3] = 0
    assert oracle.feast_dense(A, None, 0.0, 0.5, 20, f)["info"] == 2
    # B not positive definite -> -3
    assert oracle.feast_dense(A, -np.eye(40), 0.0, 0.5, 20)["info"] == -3


def test_spurious_ritz_values_are_not_counted():
    """Uniform spectrum on [-10, 10], generalized complex pencil, M0 = 1.6 * count:
    the weakly filtered outer subspace yields Ritz values inside the interval with
    O(1) residuals; the count must still equal the prescribed one (R-spur reading)."""
    A, B, lam, X = gen.prescribed_complex_pencil(512, seed=0)
    cnt = int(np.sum((lam >= -1) & (lam <= 1)))
    r = oracle.feast_dense(A, B, -1.0, 1.0, 75, oracle.feastinit())
    assert r["info"] == 0 and r["M"] == cnt == inertia_count(A, B, -1.0, 1.0)
    np.testing.assert_allclose(r["E"][:cnt], lam[(lam >= -1) & (lam <= 1)], atol=1e-12)
    # iteration 0 did see more Ritz values in the interval than eigenvalues
    assert max(h["M"] for h in r["history"]) == cnt
    assert np.all(r["res"][:cnt] < 1e-12)
