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
import scipy.linalg as sla

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


def test_graph_replay_repeats_the_first_call_and_follows_new_intervals():
    """The first call factors every (problem, node) item in padded size classes with the
    tile autotuner on and captures the launches in a graph; the second call replays it and
    must return the same results bit for bit (the problems run concurrently on several
    worker streams, so this also checks that no kernel's result depends on what runs beside
    it); a third call with other intervals (same sizes, so the same graph, new nodes
    uploaded) must match the single-problem driver."""
    probs = gen.batched_real_problems(10, seed=11, n_lo=200, n_hi=700, c_lo=6, c_hi=14)
    _say("batched graph replay: n = %s" % [p["A"].shape[0] for p in probs])
    fpm = mf.mfeast_init()
    fpm[2] = 10
    As = [torch.from_numpy(p["A"]).to(DEV) for p in probs]
    h = mf.Handle(0)
    args = ([p["emin"] for p in probs], [p["emax"] for p in probs], [p["m0"] for p in probs])
    r1, o1, _ = mf.feast_batched(As, *args, fpm=fpm, handle=h)
    torch.cuda.synchronize()
    r2, o2, _ = mf.feast_batched(As, *args, fpm=fpm, handle=h)
    torch.cuda.synchronize()
    assert r1 == r2 == 0
    for a, b, p in zip(o1, o2, probs):
        _check(b, p, 1e-10)
        assert a["loop"] == b["loop"] and a["M"] == b["M"] and a["info"] == b["info"]
        assert torch.equal(a["E"], b["E"]) and torch.equal(a["X"], b["X"]) and torch.equal(a["res"], b["res"])
    # new intervals: the lower half of each problem's eigenvalues (edges mid-gap)
    emins, emaxs, m0s, counts = [], [], [], []
    for p in probs:
        lam = np.sort(p["lam"])
        lo = p["start"]
        c = max(2, p["count"] // 2)
        emins.append(0.5 * (lam[lo - 1] + lam[lo]) if lo > 0 else lam[0] - 1.0)
        emaxs.append(0.5 * (lam[lo + c - 1] + lam[lo + c]))
        m0s.append(int(np.ceil(1.5 * c)) + 2)
        counts.append(c)
    r3, o3, _ = mf.feast_batched(As, emins, emaxs, m0s, fpm=fpm, handle=h)
    torch.cuda.synchronize()
    assert r3 == 0
    for k in range(len(probs)):
        assert o3[k]["M"] == counts[k]
        single = mf.feast(As[k], None, emins[k], emaxs[k], m0s[k], fpm=fpm)
        compare_eigenpairs(o3[k]["E"].cpu().numpy(), o3[k]["X"].cpu().numpy(), single["E"].cpu().numpy(),
                           single["X"].cpu().numpy(), single["M"], emins[k], emaxs[k])
    h.close()


@pytest.mark.parametrize("fp32", [True, False])
def test_generalized_batch_against_single_calls(fp32):
    """Problems with B = I + 0.1 C C^T / n (one more factored item per problem for the
    found-pair test): every problem against the single-problem driver, FP32 and FP64."""
    rng = np.random.default_rng(21)
    sizes = [150, 300, 301, 520, 257]
    As, Bs, ivs = [], [], []
    for n in sizes:
        G = rng.standard_normal((n, n))
        A = 0.5 * (G + G.T) / np.sqrt(n)
        C = rng.standard_normal((n, n))
        B = np.eye(n) + 0.1 * (C @ C.T) / n
        lam = np.sort(sla.eigh(A, B, eigvals_only=True))
        i0 = n // 2 - 5
        ivs.append((0.5 * (lam[i0 - 1] + lam[i0]), 0.5 * (lam[i0 + 9] + lam[i0 + 10]), 10))
        As.append(torch.from_numpy(A).to(DEV))
        Bs.append(torch.from_numpy(B).to(DEV))
    _say("batched generalized fp32=%s: n = %s" % (fp32, sizes))
    fpm = mf.mfeast_init()
    fpm[2] = 10
    fpm[41] = 1 if fp32 else 0
    ret, outs, _ = mf.feast_batched(As, [v[0] for v in ivs], [v[1] for v in ivs], [20] * len(sizes), fpm=fpm,
                                    Bs=Bs)
    torch.cuda.synchronize()
    assert ret == 0
    for k in range(len(sizes)):
        o = outs[k]
        assert o["info"] == 0 and o["M"] == 10
        single = mf.feast(As[k], Bs[k], ivs[k][0], ivs[k][1], 20, fpm=fpm)
        Bn = Bs[k].cpu().numpy()
        compare_eigenpairs(o["E"].cpu().numpy(), o["X"].cpu().numpy(), single["E"].cpu().numpy(),
                           single["X"].cpu().numpy(), single["M"], ivs[k][0], ivs[k][1], B=Bn)
        assert float(o["res"][:10].max()) <= 1e-10
