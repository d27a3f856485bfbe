"""GPU parity of the Zolotarev rule (fpm(16) = 2) against the oracle.

The nodes, weights and constant term come from the library's own generator (checked
against the oracle's on the CPU in test_abi_cpu.py); here the whole iteration runs
with them: dense real and complex Hermitian problems in FP64 and FP32+IR, the sparse
driver's BiCGSTAB, and the stochastic count.  Same parity bar as the other tests.
"""

import sys

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle.stochastic import stochastic_count
from workloads import generators as gen

from parity import compare_eigenpairs

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2002_04807_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dense(A, B, emin, emax, m0, Y, fp32, ne=8, band=90):
    fpm = mf.mfeast_init()
    fpm[41] = 1 if fp32 else 0
    fpm[15], fpm[1], fpm[53] = 2, ne, band
    At = torch.from_numpy(np.asfortranarray(A)).to(DEV)
    Bt = None if B is None else torch.from_numpy(np.asfortranarray(B)).to(DEV)
    out = mf.feast(At, Bt, emin, emax, m0, fpm=fpm, X0=torch.from_numpy(np.ascontiguousarray(Y)).to(DEV))
    torch.cuda.synchronize()
    f = oracle.feastinit()
    f[4] = 1
    f[15], f[1], f[53] = 2, ne, band
    ref = oracle.feast_dense(A, B, emin, emax, m0, f, X0=Y)
    return out, ref


@pytest.mark.parametrize("fp32", [False, True])
def test_laplacian_1d(fp32):
    _say("zolotarev laplacian 1-D fp32=%s" % fp32)
    n, emin, emax, m0 = 200, 0.0, 0.5, 60
    A = gen.laplacian_1d_dense(n)
    Y = oracle.initial_subspace(n, m0, 0, False)
    out, ref = _dense(A, None, emin, emax, m0, Y, fp32)
    assert out["info"] == ref["info"] == 0 and out["M"] == ref["M"] == 46
    compare_eigenpairs(out["E"].cpu().numpy(), out["X"].cpu().numpy(), ref["E"], ref["X"], 46, emin, emax)
    np.testing.assert_allclose(out["E"].cpu().numpy()[:46], gen.laplacian_1d_eigs(n)[:46], rtol=0, atol=1e-12)
    assert float(out["res"][:46].max()) <= 1e-10


@pytest.mark.parametrize("fp32,ne,band", [(False, 8, 90), (True, 8, 90), (True, 12, 80)])
def test_complex_generalized(fp32, ne, band):
    _say("zolotarev complex pencil fp32=%s ne=%d band=%d" % (fp32, ne, band))
    n = 333
    A, B, lam, X = gen.prescribed_complex_pencil(n, 2)
    emin, emax = -1.0, 1.0
    cnt = int(np.sum((lam >= emin) & (lam <= emax)))
    m0 = int(1.3 * cnt) + 2
    Y = oracle.initial_subspace(n, m0, 2, True)
    out, ref = _dense(A, B, emin, emax, m0, Y, fp32, ne, band)
    assert out["info"] == ref["info"] == 0 and out["M"] == ref["M"] == cnt
    compare_eigenpairs(out["E"].cpu().numpy(), out["X"].cpu().numpy(), ref["E"], ref["X"], cnt, emin, emax, B=B)
    if not fp32:
        assert out["loop"] == ref["loop"]  # FP32 solves may need more iterations


def test_sparse_laplacian_3d():
    """9 x 10 x 11 grid, 12 eigenvalues, 8 Zolotarev nodes, BiCGSTAB to 1e-6 in FP32."""
    _say("zolotarev ifeast laplacian 9x10x11")
    nx, ny, nz = 9, 10, 11
    v, c, p = gen.laplacian_3d_csr(nx, ny, nz)
    lam = gen.laplacian_3d_eigs(nx, ny, nz)
    cnt = 12
    emax = 0.5 * (lam[cnt - 1] + lam[cnt])
    fpm = mf.mfeast_init_ifeast()
    fpm[15], fpm[1], fpm[44], fpm[45] = 2, 8, 6, 2000
    out = mf.feast_csr((v, p, c), 0.0, emax, 20, fpm=fpm)
    torch.cuda.synchronize()
    f = oracle.ifeastinit()
    f[15], f[1], f[44], f[45] = 2, 8, 6, 2000
    ref = oracle.feast_csr(sp.csr_matrix((v, c, p)), None, 0.0, emax, 20, f)
    assert out["info"] == ref["info"] == 0 and out["M"] == ref["M"] == cnt
    compare_eigenpairs(out["E"].cpu().numpy(), out["X"].cpu().numpy(), ref["E"], ref["X"], cnt, 0.0, emax)
    np.testing.assert_allclose(out["E"].cpu().numpy()[:cnt], lam[:cnt], rtol=0, atol=1e-12)


@pytest.mark.parametrize("fp32", [False, True])
def test_stochastic_count(fp32):
    """fpm(14) = 2 with 8 Zolotarev nodes on the 1-D Laplacian n = 200 (46 inside): the
    same 70 probes on both sides; the estimate includes the rule's constant term."""
    _say("zolotarev stochastic count fp32=%s" % fp32)
    n, m0 = 200, 70
    A = gen.laplacian_1d_dense(n)
    est_ref, M_ref = stochastic_count(A, None, 0.0, 0.5, m0, ne=8, rule=2, seed=0, band_pct=90)
    fpm = mf.mfeast_init_stochastic()
    fpm[41] = 1 if fp32 else 0
    fpm[15], fpm[1] = 2, 8
    out = mf.feast(torch.from_numpy(np.asfortranarray(A)).to(DEV), None, 0.0, 0.5, m0, fpm=fpm)
    torch.cuda.synchronize()
    assert out["info"] == 5
    est = float(out["E"][0].item())
    tol = 1e-3 if fp32 else 1e-10 * max(1.0, abs(est_ref))
    assert abs(est - est_ref) <= tol, (est, est_ref)
    assert out["M"] == M_ref
