"""GPU parity of the stopping criteria and of the found-pair test against the oracle.

  * fpm(6) = 0 (trace criterion, Table tab_fpm): loop and epsout (Table tab-common1,
    |trace_k - trace_{k-1}| / max(|Emin|, |Emax|)) equal the oracle's on the same
    starting block, also when the run is cut off by fpm(4);
  * the found-pair test (r^H B^-1 r below the Kato-Temple bound of the interval) gives
    the same count and eigenvalues for (A, B) and (0.01 A, 0.01 B);
  * a complex generalized pencil against the oracle's classic form of the iteration
    (every contour solved with B X, Section 1.1), not only its residual form.
"""

import sys

import numpy as np
import pytest

import oracle
from workloads import generators as gen

from parity import compare_eigenpairs

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2002_04807_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _gpu(A, B, emin, emax, m0, Y, fp32, extra=None):
    fpm = mf.mfeast_init()
    fpm[41] = 1 if fp32 else 0
    for k, v in (extra or {}).items():
        fpm[k] = v
    At = torch.from_numpy(np.asfortranarray(A)).to(DEV)
    Bt = None if B is None else torch.from_numpy(np.asfortranarray(B)).to(DEV)
    out = mf.feast(At, Bt, emin, emax, m0, fpm=fpm, X0=torch.from_numpy(np.ascontiguousarray(Y)).to(DEV))
    torch.cuda.synchronize()
    return out


def _oracle(A, B, emin, emax, m0, Y, extra=None, form="residual"):
    f = oracle.feastinit()
    f[4] = 1
    for k, v in (extra or {}).items():
        f[k] = v
    return oracle.feast_dense(A, B, emin, emax, m0, f, X0=Y, form=form)


@pytest.mark.parametrize("p, maxloops", [(12, 20), (6, 20), (12, 1), (12, 2)])
def test_trace_criterion_loop_and_epsout(p, maxloops):
    """1-D Laplacian n = 200, [0, 0.5], M0 = 70, FP64 solves, fpm(6) = 0."""
    _say("trace criterion fpm(3)=%d fpm(4)=%d" % (p, maxloops))
    n, emin, emax, m0 = 200, 0.0, 0.5, 70
    A = gen.laplacian_1d_dense(n)
    Y = oracle.initial_subspace(n, m0, 0, False)
    extra = {2: p, 3: maxloops, 5: 0}
    out = _gpu(A, None, emin, emax, m0, Y, False, extra)
    ref = _oracle(A, None, emin, emax, m0, Y, extra)
    assert out["info"] == ref["info"], (out["info"], ref["info"])
    assert out["loop"] == ref["loop"], (out["loop"], ref["loop"])
    assert out["M"] == ref["M"] == 46
    e_gpu, e_ref = out["epsout"], ref["epsout"]
    # each trace is a sum of 46 eigenvalues, each within the parity bar 1e-10 max(|l|, alpha)
    # (alpha = 0.5 >= every |l| here), so two traces over alpha differ by at most 2 * 46e-10
    bar = 2.0 * 46 * 1e-10
    assert abs(e_gpu - e_ref) <= max(1e-9 * e_ref, bar), (e_gpu, e_ref)
    if ref["info"] == 0:
        assert e_gpu < 10.0 ** -p
    if ref["info"] == 0:
        compare_eigenpairs(out["E"].cpu().numpy(), out["X"].cpu().numpy(), ref["E"], ref["X"], 46, emin, emax)


@pytest.mark.parametrize("fp32", [False, True])
def test_found_pairs_unchanged_by_pencil_scaling(fp32):
    """Complex Hermitian pencil n = 200 (seed 5), [-1, 1], M0 = 28: (A, B) and
    (0.01 A, 0.01 B) give the same count and eigenvalues, and both match the oracle."""
    _say("pencil scaling fp32=%s" % fp32)
    A, B, lam, X = gen.prescribed_complex_pencil(200, 5)
    emin, emax, m0 = -1.0, 1.0, 28
    Y = oracle.initial_subspace(200, m0, 5, True)
    ref = _oracle(A, B, emin, emax, m0, Y)
    outs = [_gpu(beta * A, beta * B, emin, emax, m0, Y, fp32) for beta in (1.0, 0.01)]
    for out in outs:
        assert out["info"] == ref["info"] == 0, (out["info"], ref["info"])
        assert out["M"] == ref["M"] == 24
        compare_eigenpairs(out["E"].cpu().numpy(), out["X"].cpu().numpy(), ref["E"], ref["X"], 24, emin, emax, B=B)
    np.testing.assert_allclose(outs[0]["E"].cpu().numpy()[:24], outs[1]["E"].cpu().numpy()[:24], rtol=0, atol=1e-12)


@pytest.mark.parametrize("fp32", [False, True])
def test_complex_generalized_against_classic_form(fp32):
    """Complex Hermitian pencil n = 333 (seed 2; ragged tail of the 64-wide tiles), [-1, 1],
    M0 = 1.3 x count: the GPU's residual-form iteration against the oracle's classic one."""
    _say("complex generalized vs classic oracle fp32=%s" % fp32)
    n = 333
    A, B, lam, X = gen.prescribed_complex_pencil(n, 2)
    emin, emax = -1.0, 1.0
    cnt = int(np.sum((lam >= emin) & (lam <= emax)))
    m0 = int(1.3 * cnt) + 2
    Y = oracle.initial_subspace(n, m0, 2, True)
    ref = _oracle(A, B, emin, emax, m0, Y, form="classic")
    out = _gpu(A, B, emin, emax, m0, Y, fp32)
    assert out["info"] == ref["info"] == 0, (out["info"], ref["info"])
    assert out["M"] == ref["M"] == cnt
    compare_eigenpairs(out["E"].cpu().numpy(), out["X"].cpu().numpy(), ref["E"], ref["X"], cnt, emin, emax, B=B)
    assert float(out["res"][:cnt].max()) <= 1e-10
