"""GPU parity of the non-Hermitian driver (mfeast_zgegv, Section 3.3) against the oracle.

Inputs are pencils built with a known spectrum and known right and left eigenvectors
(workloads.generators.prescribed_nonnormal); the GPU and the oracle start from the same
blocks (fpm(5)=1).  Bar: equal count inside the contour, every eigenvalue within
1e-10 alpha of the oracle's (alpha = |Emid| + r), right and left eigenvector subspaces of
clusters of close eigenvalues within sin 1e-8 of the oracle's, residuals below 1e-10.
"""

import sys

import numpy as np
import pytest

from oracle import nonhermitian as nh
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


def _groups(lam, tol):
    """Connected components of eigenvalues closer than tol (complex plane)."""
    n = len(lam)
    label = list(range(n))

    def find(i):
        while label[i] != i:
            label[i] = label[label[i]]
            i = label[i]
        return i
    for i in range(n):
        for j in range(i + 1, n):
            if abs(lam[i] - lam[j]) < tol:
                label[find(i)] = find(j)
    groups = {}
    for i in range(n):
        groups.setdefault(find(i), []).append(i)
    return list(groups.values())


def _compare(out, ref, emid, r, two):
    alpha = abs(emid) + r
    M = ref["M"]
    assert out["info"] == ref["info"] == 0, (out["info"], ref["info"])
    assert out["M"] == M
    E = out["E"].cpu().numpy()[:M]
    Er = ref["E"][:M]
    match = [int(np.argmin(np.abs(Er - e))) for e in E]
    assert sorted(match) == list(range(M))
    err = max(abs(E[i] - Er[match[i]]) for i in range(M)) / alpha
    assert err <= 1e-10, err
    X = out["X"].cpu().numpy()[:, :M]
    Y = out["Y"].cpu().numpy()[:, :M] if two else None
    worst = 0.0
    for g in _groups(Er, 1e-4 * alpha):
        gi = [i for i in range(M) if match[i] in g]
        worst = max(worst, _sin(X[:, gi], ref["X"][:, g]))
        if two:
            worst = max(worst, _sin(Y[:, gi], ref["Y"][:, g]))
    assert worst <= 1e-8, worst
    assert float(out["res"][:M].max()) <= 1e-10
    if two:
        assert float(out["res_left"][:M].max()) <= 1e-10
    return err, worst


def _run(n, seed, generalized, emid, r, two, fp32, extra=None, m0_extra=10):
    A, B, lam, V, Yv = gen.prescribed_nonnormal(n, seed, generalized=generalized)
    fpm_o = nh.nfeastinit()
    fpm_g = mf.mfeast_init_general()
    for f in (fpm_o, fpm_g):
        f[14] = 0 if two else 1
        for k, v in (extra or {}).items():
            f[k] = v
    cnt = int(nh.inside_ellipse(lam, emid, r, int(fpm_o[17]), int(fpm_o[18])).sum())
    m0 = cnt + m0_extra
    X0 = initial_subspace(n, m0, seed, True)
    if two:
        X0 = np.concatenate([X0, initial_subspace(n, m0, seed + 1, True)], axis=1)
    fpm_o[4] = 1
    ref = nh.feast_general(A, B, emid, r, m0, fpm_o, X0=X0)
    fpm_g[41] = 1 if fp32 else 0
    At = torch.from_numpy(np.asfortranarray(A)).to(DEV)
    Bt = None if B is None else torch.from_numpy(np.asfortranarray(B)).to(DEV)
    out = mf.feast_general(At, Bt, emid, r, m0, fpm=fpm_g, X0=torch.from_numpy(X0).to(DEV))
    torch.cuda.synchronize()
    assert ref["M"] == cnt
    return out, ref


@pytest.mark.parametrize("fp32", [False, True])
def test_standard_two_sided(fp32):
    _say("nonhermitian standard two-sided fp32=%s" % fp32)
    out, ref = _run(150, 3, False, 0.2 - 0.3j, 0.9, True, fp32)
    _compare(out, ref, 0.2 - 0.3j, 0.9, True)


@pytest.mark.parametrize("fp32", [False, True])
def test_generalized_rotated_ellipse_two_sided(fp32):
    """n = 200 (a ragged tail of the 64-wide tiles), ellipse ratio 0.6 rotated 30 degrees."""
    _say("nonhermitian generalized rotated ellipse fp32=%s" % fp32)
    emid, r = -0.4 + 0.2j, 1.1
    out, ref = _run(200, 4, True, emid, r, True, fp32, extra={17: 60, 18: 30})
    _compare(out, ref, emid, r, True)


def test_generalized_one_sided():
    _say("nonhermitian generalized one-sided")
    emid, r = 0.5 + 0.5j, 1.0
    out, ref = _run(180, 5, True, emid, r, False, False)
    _compare(out, ref, emid, r, False)
    assert out["Y"] is None


def test_gauss_full_contour():
    _say("nonhermitian gauss 24 nodes")
    emid, r = 0.0, 0.8
    out, ref = _run(160, 6, False, emid, r, True, True, extra={15: 0, 7: 24})
    _compare(out, ref, emid, r, True)


def test_contour_matches_oracle_on_device_call():
    """The nodes the driver uses are those of mfeast_gcontour (host logic checked on the
    CPU against the oracle); an expert call with them gives the same result."""
    _say("nonhermitian expert contour")
    n, seed = 150, 3
    A, B, lam, V, Yv = gen.prescribed_nonnormal(n, seed)
    emid, r = 0.2 - 0.3j, 0.9
    info, z, w = mf.mfeast_gcontour(emid, r, 16, 1, 100, 0)
    assert info == 0
    cnt = int(nh.inside_ellipse(lam, emid, r).sum())
    m0 = cnt + 10
    X0 = np.concatenate([initial_subspace(n, m0, seed, True), initial_subspace(n, m0, seed + 1, True)], axis=1)
    At = torch.from_numpy(np.asfortranarray(A)).to(DEV)
    f = mf.mfeast_init_general()
    f[41] = 0
    a = mf.feast_general(At, None, emid, r, m0, fpm=f, X0=torch.from_numpy(X0).to(DEV))
    b = mf.feast_general(At, None, emid, r, m0, fpm=f, X0=torch.from_numpy(X0).to(DEV), zne=z, wne=w)
    torch.cuda.synchronize()
    assert a["info"] == b["info"] == 0 and a["M"] == b["M"] == cnt
    assert torch.equal(a["E"], b["E"])
