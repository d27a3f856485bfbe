"""The allocation-free entry point mfeast_dsygv_noalloc against mfeast_dsygv.

Both are called through the C interface on the same seeded inputs and starting block:
two calls in a row on the no-allocation entry point (the second with a smaller
problem, so the static array holds the first call's data when the second starts),
each compared with the allocating entry point to the parity bar (exact count,
eigenvalues within 1e-10 max(|lambda|, alpha), cluster angles within 1e-8, residuals
below 1e-10), in FP32+IR and FP64; then a problem too large for the array is rejected
with -901 and leaves the outputs untouched.
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


def _call(fn, h, A, emin, emax, m0, Y, fp32):
    n = A.shape[0]
    fpm = mf.mfeast_init()
    fpm[41] = 1 if fp32 else 0
    fpm[4] = 1
    At = torch.from_numpy(np.asfortranarray(A)).to(DEV)
    X = torch.zeros((m0, n), dtype=torch.float64, device=DEV).mT
    X.copy_(torch.from_numpy(Y).to(DEV))
    E = torch.zeros(m0, dtype=torch.float64, device=DEV)
    res = torch.zeros(m0, dtype=torch.float64, device=DEV)
    out = fn(h, "F", n, At, n, None, n, fpm, emin, emax, m0, E, X, n, res)
    torch.cuda.synchronize()
    m = out["m0"]
    out.update(E=E[:m].cpu().numpy(), X=X[:, :m].cpu().numpy(), res=res[:m].cpu().numpy())
    return out


def _problem(n, seed):
    """Real symmetric A = U diag(lambda) U^T (lambda ~ U[-2, 2]); interval around the
    lower middle of the spectrum holding about a quarter of it."""
    rng = np.random.default_rng(seed)
    A, lam, _ = gen.prescribed_real_problem(n, rng, -2.0, 2.0)
    k0, k1 = n // 4, n // 2
    emin = 0.5 * (lam[k0 - 1] + lam[k0])
    emax = 0.5 * (lam[k1 - 1] + lam[k1])
    return A, emin, emax, k1 - k0


@pytest.mark.parametrize("fp32", [True, False])
def test_noalloc_matches_allocating_entry_point(fp32):
    h = mf.Handle(0)
    try:
        for n, seed in ((200, 11), (120, 12)):
            A, emin, emax, cnt = _problem(n, seed)
            m0 = int(1.5 * cnt) + 4
            Y = oracle.initial_subspace(n, m0, seed, False)
            _say("noalloc n=%d m0=%d fp32=%s" % (n, m0, fp32))
            ref = _call(mf.mfeast_dsygv, h, A, emin, emax, m0, Y, fp32)
            out = _call(mf.mfeast_dsygv_noalloc, h, A, emin, emax, m0, Y, fp32)
            assert ref["info"] == 0 and out["info"] == 0, (ref["info"], out["info"])
            assert out["M"] == ref["M"] == cnt
            compare_eigenpairs(out["E"], out["X"], ref["E"], ref["X"], cnt, emin, emax)
            assert np.all(out["res"][:cnt] <= 1e-10)
    finally:
        h.close()


def test_noalloc_rejects_a_problem_beyond_its_array():
    _say("noalloc too large")
    h = mf.Handle(0)
    try:
        n, m0 = 700, 300
        A, emin, emax, _ = _problem(n, 13)
        Y = oracle.initial_subspace(n, m0, 13, False)
        out = _call(mf.mfeast_dsygv_noalloc, h, A, emin, emax, m0, Y, False)
        assert out["info"] == -901, out["info"]
        assert np.all(out["E"] == 0.0)
    finally:
        h.close()
