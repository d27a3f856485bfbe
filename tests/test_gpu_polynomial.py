"""GPU parity of the polynomial driver (mfeast_zgepev, Section 3.4) against the oracle.

Inputs are matrix polynomials built with known eigenpairs
(workloads.generators.prescribed_polynomial); the GPU and the oracle start from the same
block (fpm(5)=1).  Bar: equal info and count inside the contour, every eigenvalue within
1e-10 alpha of the oracle's and of the constructed one (alpha = |Emid| + r), eigenvectors
within sin 1e-8 of the constructed ones, residuals below 1e-10 (the oracle reaches about
1e-14; the bar leaves room for the FP32 solves, whose error the FP64 residual form removes
at the rate of the filter).
"""

import sys

import numpy as np
import pytest

from oracle import nonhermitian as nh
from oracle import polynomial as po
from oracle.splitmix import initial_subspace
from workloads import generators as gen

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2002_04807_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sin(X, Y):
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    return float(np.linalg.norm(qx - qy @ (qy.conj().T @ qx), 2))


def _run(n, p, seed, leading, emid, r, fp32, extra=None):
    As, lam, Xe = gen.prescribed_polynomial(n, p, seed, leading=leading)
    fpm_o = po.pfeastinit()
    fpm_g = mf.mfeast_init_polynomial()
    for f in (fpm_o, fpm_g):
        for k, v in (extra or {}).items():
            f[k] = v
    inside = nh.inside_ellipse(lam, emid, r, int(fpm_o[17]), int(fpm_o[18]))
    cnt = int(inside.sum())
    m0 = int(np.ceil(1.5 * cnt))
    X0 = initial_subspace(n, m0, seed, True)
    fpm_o[4] = 1
    ref = po.feast_polynomial(As, emid, r, m0, fpm_o, X0=X0)
    fpm_g[41] = 1 if fp32 else 0
    At = [torch.from_numpy(np.asfortranarray(a)).to(DEV) for a in As]
    out = mf.feast_polynomial(At, emid, r, m0, fpm=fpm_g, X0=torch.from_numpy(X0).to(DEV))
    torch.cuda.synchronize()
    assert ref["M"] == cnt
    return out, ref, lam[inside], Xe[:, inside]


def _compare(out, ref, lam_in, X_in, emid, r, same_loop=True):
    alpha = abs(emid) + r
    M = ref["M"]
    assert out["info"] == ref["info"] == 0, (out["info"], ref["info"])
    assert out["M"] == M
    if same_loop and out["loop"] != ref["loop"]:
        # the trace criterion at 1e-12 sits near the rounding of the trace: one iteration
        # apart is allowed when the oracle's change at the earlier stop was within 10x of it
        lo = min(out["loop"], ref["loop"])
        eps = 10.0 ** -int(out["fpm"][2])
        assert abs(out["loop"] - ref["loop"]) == 1, (out["loop"], ref["loop"])
        assert ref["history"][lo]["epsout"] < 10.0 * eps, (out["loop"], ref["loop"], ref["history"][lo]["epsout"])
    E = out["E"].cpu().numpy()[:M]
    Er = ref["E"][:M]
    match = [int(np.argmin(np.abs(Er - e))) for e in E]
    assert sorted(match) == list(range(M))
    err = max(abs(E[i] - Er[match[i]]) for i in range(M)) / alpha
    assert err <= 1e-10, err
    X = out["X"].cpu().numpy()[:, :M]
    worst = 0.0
    for q in range(M):
        i = int(np.argmin(np.abs(lam_in - E[q])))
        assert abs(lam_in[i] - E[q]) <= 1e-10 * alpha
        worst = max(worst, _sin(X[:, [q]], X_in[:, [i]]))
    assert worst <= 1e-8, worst
    res = out["res"].cpu().numpy()
    assert float(res[:M].max()) <= 1e-10
    np.testing.assert_allclose(np.linalg.norm(X, axis=0), 1.0, atol=1e-12)
    return err, worst


@pytest.mark.parametrize("fp32", [False, True])
def test_quadratic(fp32):
    _say("polynomial quadratic fp32=%s" % fp32)
    emid, r = 0.2 - 0.1j, 0.8
    out, ref, li, Xi = _run(100, 2, 3, False, emid, r, fp32)
    _compare(out, ref, li, Xi, emid, r, same_loop=not fp32)


def test_quadratic_leading_coefficient_ragged_n():
    """n = 333 (several 64-wide tiles and a ragged tail), A_2 != I, FP32 solves."""
    _say("polynomial quadratic leading n=333")
    emid, r = -0.3 + 0.4j, 0.9
    out, ref, li, Xi = _run(333, 2, 5, True, emid, r, True)
    _compare(out, ref, li, Xi, emid, r, same_loop=False)


def test_cubic_rotated_ellipse():
    _say("polynomial cubic rotated ellipse")
    emid, r = 0.1 + 0.1j, 1.0
    out, ref, li, Xi = _run(120, 3, 7, False, emid, r, False, extra={17: 70, 18: 20})
    _compare(out, ref, li, Xi, emid, r)


def test_gauss_full_contour_fpm6():
    """Gauss-Legendre full contour (fpm(16)=0, 24 nodes), residual criterion fpm(6)=1."""
    _say("polynomial gauss 24 nodes, residual criterion")
    emid, r = 0.0, 0.9
    out, ref, li, Xi = _run(100, 2, 9, True, emid, r, False, extra={15: 0, 7: 24, 5: 1, 2: 10})
    _compare(out, ref, li, Xi, emid, r)
    assert float(out["res"][:out["M"]].max()) < 1e-10


def test_degree_one_matches_linear_driver():
    """P(lambda) = -A + lambda B on the GPU: the eigenvalues of mfeast_zgegv (one-sided)
    from the same starting block."""
    _say("polynomial degree one vs zgegv")
    n, seed = 150, 8
    A, B, lam, V, Yv = gen.prescribed_nonnormal(n, seed, generalized=True)
    emid, r = 0.1 + 0.2j, 1.0
    cnt = int(nh.inside_ellipse(lam, emid, r).sum())
    m0 = int(np.ceil(1.5 * cnt))
    X0 = torch.from_numpy(initial_subspace(n, m0, seed, True)).to(DEV)
    At = torch.from_numpy(np.asfortranarray(A)).to(DEV)
    Bt = torch.from_numpy(np.asfortranarray(B)).to(DEV)
    fg = mf.mfeast_init_general()
    fg[14] = 1
    fg[41] = 0
    fp = mf.mfeast_init_polynomial()
    fp[41] = 0
    a = mf.feast_general(At, Bt, emid, r, m0, fpm=fg, X0=X0)
    b = mf.feast_polynomial([-At, Bt], emid, r, m0, fpm=fp, X0=X0)
    torch.cuda.synchronize()
    assert a["info"] == b["info"] == 0 and a["M"] == b["M"] == cnt
    Ea = np.sort_complex(a["E"].cpu().numpy()[:cnt])
    Eb = np.sort_complex(b["E"].cpu().numpy()[:cnt])
    np.testing.assert_allclose(Ea, Eb, rtol=0, atol=1e-10 * (abs(emid) + r))


def test_random_start_and_info_codes():
    """fpm(5)=0 (the driver's own start, SplitMix64 seed fpm(51)) converges to the same
    eigenvalues; an empty contour gives info 1 and M = 0; M0 below the count gives info 3,
    as in the oracle."""
    _say("polynomial random start, info 1 and 3")
    n, p, seed = 100, 2, 3
    As, lam, Xe = gen.prescribed_polynomial(n, p, seed)
    At = [torch.from_numpy(np.asfortranarray(a)).to(DEV) for a in As]
    emid, r = 0.2 - 0.1j, 0.8
    inside = nh.inside_ellipse(lam, emid, r)
    cnt = int(inside.sum())
    out = mf.feast_polynomial(At, emid, r, int(np.ceil(1.5 * cnt)))
    torch.cuda.synchronize()
    assert out["info"] == 0 and out["M"] == cnt
    E = out["E"].cpu().numpy()[:cnt]
    li = lam[inside]
    assert max(min(abs(li - e)) for e in E) <= 1e-10 * (abs(emid) + r)
    far = mf.feast_polynomial(At, 20.0 + 20.0j, 0.5, 8)
    torch.cuda.synchronize()
    assert far["info"] == 1 and far["M"] == 0
    few = mf.feast_polynomial(At, emid, r, max(cnt // 3, 1))
    torch.cuda.synchronize()
    ref = po.feast_polynomial(As, emid, r, max(cnt // 3, 1))
    assert few["info"] == ref["info"] == 3
