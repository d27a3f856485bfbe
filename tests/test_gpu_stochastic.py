"""Stochastic eigenvalue count (fpm(14)=2) through the C-ABI against the oracle.

The library and the oracle draw the same +-1 probe block (SplitMix64 sign bits), so
the estimates compare value for value: to 1e-10 relative with FP64 solves, and with
FP32 solves (or the sparse path's complex-FP32 BiCGSTAB) to 1e-3 absolute, far below
the 0.5 that decides the rounded count (the FP32 solve error is about
kappa(z B - A) * 6e-8 relative per node, kappa of order 1e2 to 1e3 here).
"""

import sys

import numpy as np
import pytest

from oracle.stochastic import stochastic_count
from workloads import generators as gen

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2002_04807_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _count_gpu(A, B, emin, emax, m0, fp32, seed=0):
    fpm = mf.mfeast_init_stochastic()
    fpm[41] = 1 if fp32 else 0
    fpm[50] = seed
    At = torch.from_numpy(np.asfortranarray(A)).to(DEV)
    Bt = None if B is None else torch.from_numpy(np.asfortranarray(B)).to(DEV)
    out = mf.feast(At, Bt, emin, emax, m0, fpm=fpm)
    torch.cuda.synchronize()
    return out


def _check(out, est_ref, M_ref, fp32):
    assert out["info"] == 5, out["info"]
    assert out["loop"] == 0
    est = float(out["E"][0].item())
    if fp32:
        assert abs(est - est_ref) < 1e-3, (est, est_ref)
    else:
        assert abs(est - est_ref) <= 1e-10 * max(1.0, abs(est_ref)), (est, est_ref)
    if abs(est_ref - np.floor(est_ref) - 0.5) > 1e-2:
        assert out["M"] == M_ref, (out["M"], M_ref)
    # nothing but E[0] and M is written in this mode
    assert torch.count_nonzero(out["E"][1:]).item() == 0
    assert torch.count_nonzero(out["X"]).item() == 0
    assert torch.count_nonzero(out["res"]).item() == 0
    return est


@pytest.mark.parametrize("fp32", [False, True])
def test_count_laplacian_1d_n200(fp32):
    _say("stochastic count: 1-D Laplacian n=200 fp32=%s" % fp32)
    n, m0 = 200, 70
    A = gen.laplacian_1d_dense(n)
    est_ref, M_ref = stochastic_count(A, None, 0.0, 0.5, m0, ne=3, seed=0)
    est = _check(_count_gpu(A, None, 0.0, 0.5, m0, fp32), est_ref, M_ref, fp32)
    _say("  estimate %.6f (oracle %.6f, exact count 46)" % (est, est_ref))


@pytest.mark.parametrize("fp32", [False, True])
def test_count_complex_pencil_n512(fp32):
    _say("stochastic count: complex pencil n=512 fp32=%s" % fp32)
    n, m0 = 512, 64
    A, B, lam, _ = gen.prescribed_complex_pencil(n, seed=1)
    est_ref, M_ref = stochastic_count(A, B, -1.0, 1.0, m0, ne=3, seed=5)
    est = _check(_count_gpu(A, B, -1.0, 1.0, m0, fp32, seed=5), est_ref, M_ref, fp32)
    _say("  estimate %.6f (oracle %.6f, exact count %d)" % (est, est_ref, int(((lam >= -1) & (lam <= 1)).sum())))


def test_count_sparse_laplacian_8cube():
    _say("stochastic count: sparse 3-D Laplacian 8^3")
    v, c, p = gen.laplacian_3d_csr(8)
    n = len(p) - 1
    A = np.zeros((n, n))
    for r in range(n):
        A[r, c[p[r]:p[r + 1]]] = v[p[r]:p[r + 1]]
    m0 = 32
    est_ref, M_ref = stochastic_count(A, None, 0.0, 1.0, m0, ne=3, seed=0)
    fpm = mf.mfeast_init_stochastic()
    fpm[44] = 10   # BiCGSTAB to 1e-10
    fpm[45] = 400
    out = mf.feast_csr((v, p, c), 0.0, 1.0, m0, fpm=fpm)
    torch.cuda.synchronize()
    est = _check(out, est_ref, M_ref, True)
    _say("  estimate %.6f (oracle %.6f)" % (est, est_ref))


def test_count_batched_problems():
    _say("stochastic count: three batched real problems")
    rng = np.random.default_rng(21)
    probs = []
    for n in (96, 160, 257):
        A, lam, _ = gen.prescribed_real_problem(n, rng, -2.0, 2.0)
        probs.append((A, -0.7, 0.4, 24))
    fpm = mf.mfeast_init_stochastic()
    fpm[41] = 0
    As = [torch.from_numpy(np.ascontiguousarray(A)).to(DEV) for A, _, _, _ in probs]
    ret, outs, _ = mf.feast_batched(As, [p[1] for p in probs], [p[2] for p in probs], [p[3] for p in probs],
                                    fpm=fpm)
    torch.cuda.synchronize()
    assert ret == 5, ret
    for (A, emin, emax, m0), out in zip(probs, outs):
        est_ref, M_ref = stochastic_count(A, None, emin, emax, m0, ne=3, seed=0)
        _check(out, est_ref, M_ref, False)
