"""GPU parity of the adjoint (dL/dA of a loss on the eigenpairs in an interval).

The forward pass is mfeast_dsygv, the backward pass mfeast_dsy_adjoint, joined in
torch.autograd through paper_2002_04807_amd.feast_eigh.  The reference is the FP64
oracle (explicit eigen-sum over numpy's dense eigh), itself pinned by finite
differences; at full size a sample of coordinates is also checked against central
differences of the loss through scipy's tridiagonal eigensolver.
"""

import sys

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import adjoint as adj
from workloads import generators as gen

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2002_04807_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _gpu_grad(v, c, emin, emax, m0, precision):
    n = v.size
    vt = torch.tensor(v, dtype=torch.float64, device=DEV, requires_grad=True)
    A0 = (2.0 * torch.eye(n, dtype=torch.float64, device=DEV)
          - torch.diag(torch.ones(n - 1, dtype=torch.float64, device=DEV), 1)
          - torch.diag(torch.ones(n - 1, dtype=torch.float64, device=DEV), -1))
    A = A0 + torch.diag(vt)
    fpm = mf.mfeast_init()
    fpm[41] = 1
    E, X = mf.feast_eigh(A, emin, emax, m0, fpm=fpm, precision=precision)
    ct = torch.tensor(c, dtype=torch.float64, device=DEV)
    L = E.sum() + (ct[:, None] * X * X).sum()
    L.backward()
    torch.cuda.synchronize()
    return float(L.item()), vt.grad.cpu().numpy(), E.detach().cpu().numpy()


def _loss_tridiagonal(v, c, emin, emax):
    lam, X = sla.eigh_tridiagonal(2.0 + v, -np.ones(v.size - 1), select="v", select_range=(emin, emax))
    return lam.sum() + float(np.sum(c[:, None] * X ** 2))


@pytest.mark.parametrize("precision", [0, 1])
def test_small_problem_against_oracle(precision):
    rng = np.random.default_rng(7)
    n = 300
    v = rng.uniform(0.0, 1.0, n)
    c = rng.standard_normal(n)
    lam = np.linalg.eigvalsh(adj.tridiag_dense(v))
    emin, emax = 0.5 * (lam[1] + lam[2]), 0.5 * (lam[7] + lam[8])
    _say("adjoint n=300 precision=%d" % precision)
    L, g, E = _gpu_grad(v, c, emin, emax, 12, precision)
    Lr, gr, lamS, _ = adj.loss_and_grad_v(v, c, emin, emax)
    assert E.size == lamS.size == 6
    assert abs(L - Lr) < 1e-10 * abs(Lr)
    err = np.max(np.abs(g - gr)) / np.max(np.abs(gr))
    assert err < 1e-8, err


def test_full_dL_dA_against_oracle():
    """dL/dA (all n^2 entries) from the C interface, eigenvalue and eigenvector parts."""
    rng = np.random.default_rng(21)
    n = 257
    v = rng.uniform(0.0, 1.0, n)
    c = rng.standard_normal(n)
    A = adj.tridiag_dense(v)
    lam, V, inside = adj.interval_pairs(A, 0.0, 0.35)
    M = int(inside.sum())
    assert 3 <= M <= 12
    XS = V[:, inside]
    gE = rng.standard_normal(M)
    G = 2.0 * c[:, None] * XS
    want, _ = adj.grad_by_eigensum(lam, V, inside, gE, G)
    _say("adjoint full gA n=%d M=%d" % (n, M))
    h = mf.Handle(0)
    At = torch.tensor(np.asfortranarray(A), device=DEV)
    Et = torch.tensor(lam[inside], device=DEV)
    Xt = torch.tensor(XS.T.copy(), device=DEV).mT
    gEt = torch.tensor(gE, device=DEV)
    Gt = torch.tensor(G.T.copy(), device=DEV).mT
    gA = torch.zeros((n, n), dtype=torch.float64, device=DEV)
    gd = torch.zeros(n, dtype=torch.float64, device=DEV)
    for prec in (0, 1):
        info = mf.mfeast_dsy_adjoint(h, n, At, n, M, Et, Xt, n, gEt, Gt, n, prec, gA, n, gd)
        torch.cuda.synchronize()
        assert info == 0
        got = gA.cpu().numpy()
        assert np.max(np.abs(got - want)) < 1e-9 * np.max(np.abs(want))
        np.testing.assert_allclose(gd.cpu().numpy(), np.diag(want), atol=1e-9 * np.max(np.abs(want)))
    # eigenvalue part alone (gX = NULL): X diag(gE) X^T
    info = mf.mfeast_dsy_adjoint(h, n, At, n, M, Et, Xt, n, gEt, None, n, 0, gA, n, None)
    torch.cuda.synchronize()
    assert info == 0
    np.testing.assert_allclose(gA.cpu().numpy(), (XS * gE) @ XS.T, atol=1e-13)
    h.close()


@pytest.fixture(scope="module")
def workload():
    v, c, A = gen.differentiation_problem(4096, seed=3)
    out = {}
    for emin, emax in ((0.0, 0.2), (0.0, 0.3)):
        out[(emin, emax)] = adj.loss_and_grad_v(v, c, emin, emax)
    return v, c, out


@pytest.mark.parametrize("interval", [(0.0, 0.2), (0.0, 0.3)])
@pytest.mark.parametrize("precision", [0, 1])
def test_differentiation_workload(workload, interval, precision):
    """n = 4096, A = tridiag(-1, 2 + v, -1), v ~ U[0, 1] (seed 3): [0, 0.2] holds 2 eigenvalues;
    [0, 0.3] is a supplementary interval with more pairs.  M0 = 16 and 48."""
    v, c, ref = workload
    emin, emax = interval
    Lr, gr, lamS, _ = ref[interval]
    m0 = 16 if emax < 0.25 else 48
    _say("adjoint workload interval=%s precision=%d M=%d" % (interval, precision, lamS.size))
    L, g, E = _gpu_grad(v, c, emin, emax, m0, precision)
    assert E.size == lamS.size
    np.testing.assert_allclose(E, lamS, rtol=0, atol=1e-12)
    err = np.max(np.abs(g - gr)) / np.max(np.abs(gr))
    assert err < 1e-8, err
    if interval == (0.0, 0.2) and precision == 1:
        # central differences on a sample of coordinates, independent eigensolver
        ks = np.random.default_rng(0).choice(v.size, 6, replace=False)
        ks = np.concatenate([ks, [int(np.argmax(np.abs(gr)))]])
        h = 1e-6
        for k in ks:
            e = np.zeros(v.size)
            e[k] = h
            fd = (_loss_tridiagonal(v + e, c, emin, emax) - _loss_tridiagonal(v - e, c, emin, emax)) / (2 * h)
            assert abs(fd - g[k]) < 2e-7 * max(1.0, np.max(np.abs(gr))), (k, fd, g[k])
