"""Pins of the IFEAST oracle (sparse CSR, BiCGSTAB solves) against outside facts.

Closed forms (the scalar operator, finite termination of BiCG-type methods on an
operator with few distinct eigenvalues, the 3-D Laplacian spectrum and its
tensor-product sine eigenvectors), the guide's printed IFEAST HelloWorld run
(tests/golden/helloworld.json) and a library direct solve / dense eigensolver.
"""

import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from workloads import generators as gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _csr(nx, ny=None, nz=None):
    v, c, p = gen.laplacian_3d_csr(nx, ny, nz)
    n = len(p) - 1
    return sp.csr_matrix((v, c, p), shape=(n, n))


def _subspace_sin(X, Y):
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    return float(np.linalg.norm(qx - qy @ (qy.conj().T @ qx), 2))


def _laplacian_modes(nx, ny, nz):
    """All (eigenvalue, k1, k2, k3) of the Dirichlet 7-point Laplacian, ascending."""
    out = []
    for k1 in range(1, nx + 1):
        for k2 in range(1, ny + 1):
            for k3 in range(1, nz + 1):
                lam = sum(2.0 - 2.0 * np.cos(k * np.pi / (m + 1)) for k, m in ((k1, nx), (k2, ny), (k3, nz)))
                out.append((lam, k1, k2, k3))
    out.sort()
    return out


def _mode_vector(nx, ny, nz, k1, k2, k3):
    i = np.arange(1, nx + 1)
    j = np.arange(1, ny + 1)
    l = np.arange(1, nz + 1)
    sx = np.sin(i * k1 * np.pi / (nx + 1))
    sy = np.sin(j * k2 * np.pi / (ny + 1))
    sz = np.sin(l * k3 * np.pi / (nz + 1))
    v = (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).ravel()  # index i + nx (j + ny l)
    return v / np.linalg.norm(v)


# ----------------------------------------------------------------------------
# the generator (input, not oracle): CSR equals the Kronecker-sum construction
# ----------------------------------------------------------------------------

def test_laplacian_3d_csr_is_kronecker_sum():
    nx, ny, nz = 4, 3, 5
    T = lambda m: sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])  # noqa: E731
    I = lambda m: sp.identity(m)  # noqa: E731
    K = sp.kron(I(nz), sp.kron(I(ny), T(nx))) + sp.kron(I(nz), sp.kron(T(ny), I(nx))) + sp.kron(T(nz), sp.kron(I(ny), I(nx)))
    A = _csr(nx, ny, nz)
    assert abs(A - K).max() == 0.0
    assert np.all(np.diff(A.indptr) <= 7)
    lam = np.linalg.eigvalsh(K.toarray())
    assert np.max(np.abs(lam - gen.laplacian_3d_eigs(nx, ny, nz))) < 1e-13


# ----------------------------------------------------------------------------
# BiCGSTAB
# ----------------------------------------------------------------------------

def test_bicgstab_scalar_operator_one_step():
    """op = c I: one iteration gives x = b / c exactly (alpha = 1/c, s = 0)."""
    rng = np.random.default_rng(1)
    b = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    c = 0.3 - 1.7j
    x, it = oracle.ifeast.bicgstab(lambda v: c * v, b, 1e-14, 10)
    assert it == 1
    assert np.max(np.abs(x - b / c)) <= 1e-15 * np.max(np.abs(b / c)) * 10


@pytest.mark.parametrize("k", [2, 3])
def test_bicgstab_terminates_within_distinct_eigenvalue_count(k):
    """A diagonalizable operator with k distinct eigenvalues: the BiCG polynomial of
    degree k annihilates r0, so BiCGSTAB stops by iteration k (up to rounding)."""
    rng = np.random.default_rng(k)
    d = np.repeat(rng.uniform(1, 3, k) + 1j * rng.uniform(0.1, 1, k), 40)
    b = rng.standard_normal(d.size) + 1j * rng.standard_normal(d.size)
    x, it = oracle.ifeast.bicgstab(lambda v: d * v, b, 1e-12, 50)
    assert it <= k
    assert np.max(np.abs(x - b / d)) < 1e-10


def test_bicgstab_matches_direct_solve_and_meets_tolerance():
    A = _csr(7, 6, 5)
    n = A.shape[0]
    z = 0.6 + 0.05j
    K = (z * sp.identity(n) - A).tocsc()
    rng = np.random.default_rng(7)
    b = rng.standard_normal((n, 3)) + 0j
    xd = spla.spsolve(K, b)
    x, its = oracle.bicgstab_block(lambda v: K @ v, b, 1e-13, 2000)
    assert np.all(its < 2000)
    assert np.max(np.abs(x - xd)) / np.max(np.abs(xd)) < 1e-9
    for tol in (1e-1, 1e-4):
        x, its = oracle.bicgstab_block(lambda v: K @ v, b, tol, 2000)
        rel = np.linalg.norm(b - K @ x, axis=0) / np.linalg.norm(b, axis=0)
        assert np.all(rel <= tol * (1 + 1e-8)), rel
    # a looser tolerance never needs more iterations
    _, i1 = oracle.bicgstab_block(lambda v: K @ v, b, 1e-1, 2000)
    _, i4 = oracle.bicgstab_block(lambda v: K @ v, b, 1e-4, 2000)
    assert np.all(i1 <= i4)


def test_bicgstab_first_step_galerkin_and_minimal_residual():
    """One iteration from x0 = 0 (p = b): the BiCG half step makes s orthogonal to the
    shadow residual b, and omega minimizes ||s - omega t|| so r1 is orthogonal to t = K s."""
    A = _csr(4, 5, 3)
    n = A.shape[0]
    K = (0.4 - 0.3j) * sp.identity(n) - A
    rng = np.random.default_rng(5)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x1, it = oracle.ifeast.bicgstab(lambda v: K @ v, b, 1e-14, 1)
    assert it == 1
    r1 = b - K @ x1
    # x1 = alpha b + omega s with s = b - alpha K b: recover alpha from s being orthogonal to b
    Kb = K @ b
    alpha = np.vdot(b, b) / np.vdot(b, Kb)
    s = b - alpha * Kb
    assert abs(np.vdot(b, s)) < 1e-12 * np.linalg.norm(b) * np.linalg.norm(s)
    t = K @ s
    assert abs(np.vdot(t, r1)) < 1e-12 * np.linalg.norm(t) * np.linalg.norm(r1)
    assert np.linalg.norm(r1) < np.linalg.norm(s)


def test_bicgstab_zero_rhs_and_iteration_cap():
    K = _csr(5) * (-1.0) + 0.1j * sp.identity(125)
    x, it = oracle.ifeast.bicgstab(lambda v: K @ v, np.zeros(125, complex), 1e-4, 10)
    assert it == 0 and not np.any(x)
    b = np.ones(125, complex)
    _, it = oracle.ifeast.bicgstab(lambda v: K @ v, b, 1e-14, 3)
    assert it == 3


# ----------------------------------------------------------------------------
# IFEAST driver
# ----------------------------------------------------------------------------

def test_ifeast_defaults_follow_table():
    f = oracle.ifeastinit()
    # 4 nodes, 50 loops, trapezoidal, circle, BiCGStab 1e-1 / 40 iterations
    assert (f[1], f[3], f[15], f[17], f[44], f[45]) == (4, 50, 1, 100, 1, 40)


def test_ifeast_helloworld_matches_guide_output():
    g = json.load(open(os.path.join(GOLDEN, "helloworld.json")))
    p = g["ifeast_printed"]
    ia = np.array(p["csr_ia_1based"]) - 1
    ja = np.array(p["csr_ja_1based"]) - 1
    A = sp.csr_matrix((np.array(p["csr_values"], float), ja, ia), shape=(4, 4))
    assert np.array_equal(A.toarray(), np.array(g["A"], float))
    r = oracle.feast_csr(A, None, g["emin"], g["emax"], g["m0"])
    assert r["info"] == 0
    assert r["M"] == p["M"]
    assert np.max(np.abs(r["E"][:2] - 4.0)) < 1e-13
    # the guide's run (random start) took 4 loops and 31 inner iterations; every
    # node solve takes between 1 and fpm(46) = 40 iterations
    assert 2 <= r["loop"] <= 8
    nsolve = 4 * (r["loop"] + 1)
    assert nsolve <= r["fpm60"] <= 40 * nsolve
    X = r["X"][:, :2]
    assert np.max(np.abs(A @ X - X * 4.0)) < 1e-12
    assert np.max(np.abs(X.T @ X - np.eye(2))) < 1e-12


def test_ifeast_diagonal_pencil_gives_filter_times_block():
    """A = diag(a), B = diag(d): after one contour the subspace is diag(rho(a_i / d_i)) Y,
    since (z B - A)^-1 B = diag(1 / (z - a_i / d_i)); the solves are run to 1e-14."""
    rng = np.random.default_rng(3)
    a = rng.uniform(-2.0, 3.0, 40)
    d = rng.uniform(0.5, 2.0, 40)
    Y = rng.standard_normal((40, 6))
    fpm = oracle.ifeastinit()
    fpm[4] = 1    # fpm(5): use X0
    fpm[13] = 1   # fpm(14): return Q after one contour
    fpm[44] = 14
    fpm[45] = 400
    r = oracle.feast_csr(sp.diags(a), sp.diags(d), -0.5, 1.0, 6, fpm, X0=Y)
    assert r["info"] == 4
    z, w = oracle.half_contour(-0.5, 1.0, 4, rule=1, ratio_pct=100)
    np.testing.assert_allclose(r["X"], oracle.rational_filter(a / d, z, w)[:, None] * Y,
                               rtol=1e-10, atol=1e-12)


def test_ifeast_3d_laplacian_closed_form():
    nx, ny, nz = 9, 10, 11
    A = _csr(nx, ny, nz)
    modes = _laplacian_modes(nx, ny, nz)
    lam = np.array([m[0] for m in modes])
    cnt = 12
    assert lam[cnt] - lam[cnt - 1] > 1e-2
    emax = 0.5 * (lam[cnt - 1] + lam[cnt])
    f = oracle.ifeastinit()
    f[1] = 16       # 16 nodes
    f[44] = 4       # BiCGSTAB to 1e-4
    f[45] = 1000
    r = oracle.feast_csr(A, None, 0.0, emax, 20, f)
    assert r["info"] == 0 and r["M"] == cnt
    E = r["E"][:cnt]
    assert np.max(np.abs(E - lam[:cnt])) < 1e-12 * emax
    X = r["X"][:, :cnt]
    for g in _clusters(lam[:cnt], 1e-6):
        Xref = np.stack([_mode_vector(nx, ny, nz, *modes[i][1:]) for i in g], axis=1)
        assert _subspace_sin(X[:, g], Xref) < 1e-8
    assert r["fpm60"] > 0


def test_ifeast_generalized_against_dense_eigh():
    """B = diag(d) sparse SPD; the interval count and values from scipy's dense eigh."""
    A = _csr(6, 7, 8)
    n = A.shape[0]
    rng = np.random.default_rng(11)
    d = rng.uniform(0.8, 1.25, n)
    B = sp.diags(d).tocsr()
    lam = sla.eigh(A.toarray(), np.diag(d), eigvals_only=True)
    gaps = np.diff(lam[:30])
    cnt = 5 + int(np.argmax(gaps[4:])) + 1     # widest gap after the fifth eigenvalue
    emin, emax = lam[0] - 0.1, 0.5 * (lam[cnt - 1] + lam[cnt])
    f = oracle.ifeastinit()
    f[1] = 12
    f[44] = 6
    f[45] = 1000
    r = oracle.feast_csr(A, B, emin, emax, cnt + 8, f)
    assert r["info"] == 0 and r["M"] == cnt
    assert np.max(np.abs(r["E"][:cnt] - lam[:cnt])) < 1e-11 * max(abs(emin), abs(emax))
    X = r["X"][:, :cnt]
    assert np.max(np.abs(X.T @ (B @ X) - np.eye(cnt))) < 1e-11


def _clusters(lam, tol):
    groups, cur = [], [0]
    for i in range(1, len(lam)):
        if lam[i] - lam[i - 1] < tol:
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    groups.append(cur)
    return groups
