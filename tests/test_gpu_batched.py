"""GPU parity of the batched entry point (many independent dense problems, B = I).

Inputs: the seeded prescribed-spectrum problems of workloads (known eigenvalues and
eigenvectors: A = U diag(lambda) U^T with Haar U), each with an interval holding an
exact number of eigenvalues.  Every problem is held to the parity bar against its
closed form (count, eigenvalues within 1e-10 * max(|lambda|, alpha), cluster subspace
angles within 1e-8, residuals <= 1e-10); a sample is also compared with the oracle,
and with single-problem calls of mfeast_dsygv.
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


def _check(o, p, res_tol):
    c = p["count"]
    assert o["info"] == 0, o["info"]
    assert o["M"] == c
    lam = p["lam"][p["start"]:p["start"] + c]
    U = p["U"][:, p["start"]:p["start"] + c]
    E = o["E"].cpu().numpy()
    X = o["X"].cpu().numpy()
    err = compare_eigenpairs(E, X, lam, U, c, p["emin"], p["emax"])
    assert np.all(o["res"].cpu().numpy()[:c] <= res_tol)
    return err


def test_small_batch_against_closed_form_oracle_and_single_calls():
    probs = gen.batched_real_problems(12, seed=5, n_lo=180, n_hi=520, c_lo=8, c_hi=20)
    _say("batched small: n = %s" % [p["A"].shape[0] for p in probs])
    fpm = mf.mfeast_init()
    fpm[2] = 10
    As = [torch.from_numpy(p["A"]).to(DEV) for p in probs]
    ret, outs, secs = mf.feast_batched(As, [p["emin"] for p in probs], [p["emax"] for p in probs],
                                       [p["m0"] for p in probs], fpm=fpm)
    torch.cuda.synchronize()
    assert ret == 0
    for o, p in zip(outs, probs):
        _check(o, p, 1e-10)
    # two problems against the oracle and against single-problem calls
    for k in (0, 7):
        p = probs[k]
        f = oracle.feastinit()
        f[2] = 10
        ref = oracle.feast_dense(p["A"], None, p["emin"], p["emax"], p["m0"], f)
        assert ref["M"] == outs[k]["M"]
        compare_eigenpairs(outs[k]["E"].cpu().numpy(), outs[k]["X"].cpu().numpy(), ref["E"], ref["X"], ref["M"],
                           p["emin"], p["emax"])
        single = mf.feast(As[k], None, p["emin"], p["emax"], p["m0"], fpm=fpm)
        compare_eigenpairs(outs[k]["E"].cpu().numpy(), outs[k]["X"].cpu().numpy(), single["E"].cpu().numpy(),
                           single["X"].cpu().numpy(), single["M"], p["emin"], p["emax"])


def test_bad_problem_reports_its_own_info():
    probs = gen.batched_real_problems(3, seed=2, n_lo=100, n_hi=150, c_lo=5, c_hi=8)
    As = [torch.from_numpy(p["A"]).to(DEV) for p in probs]
    emins = [p["emin"] for p in probs]
    emaxs = [p["emax"] for p in probs]
    m0s = [p["m0"] for p in probs]
    emaxs[1] = emins[1] - 1.0   # empty interval: 200 for problem 1 only
    ret, outs, _ = mf.feast_batched(As, emins, emaxs, m0s)
    torch.cuda.synchronize()
    assert outs[1]["info"] == 200
    assert outs[0]["info"] == 0 and outs[2]["info"] == 0
    assert ret == 200


def test_full_batched_workload():
    """128 problems, n ~ U{256..2048}, 24-48 eigenvalues each, M0 = ceil(1.5 count), 8 Gauss
    nodes, FP32 solves with the FP64 residual form, res <= 1e-10."""
    probs = gen.batched_real_problems(128, seed=0)
    _say("batched full: sum n^3 = %.3e" % sum(float(p["A"].shape[0]) ** 3 for p in probs))
    fpm = mf.mfeast_init()
    fpm[2] = 10
    As = [torch.from_numpy(p["A"]).to(DEV) for p in probs]
    ret, outs, secs = mf.feast_batched(As, [p["emin"] for p in probs], [p["emax"] for p in probs],
                                       [p["m0"] for p in probs], fpm=fpm)
    torch.cuda.synchronize()
    _say("batched full: %.3f s, loops %s" % (secs, np.bincount([o["loop"] for o in outs])))
    assert ret == 0
    for o, p in zip(outs, probs):
        _check(o, p, 1e-10)
