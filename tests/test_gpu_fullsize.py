"""The benchmark configuration at full size: generalized complex Hermitian pencil n = 4096,
M0 = 600, 8-node Gauss-Legendre half contour, [-1, 1], default tolerance 1e-12, with FP32
solves (the default fpm(42) = 1) and in plain FP64, called as bench.py calls it (one
handle reused across calls).

The oracle cannot run at this size within a test, so the reference is the pencil's
construction: A = L U diag(lambda) U^H L^H with B = L L^H gives the exact eigenvalues
lambda and B-orthonormal eigenvectors X = L^-H U.  Checked properties:
  * the count equals the number of exact eigenvalues in the interval;
  * every eigenvalue within 1e-10 * max(|lambda|, alpha) of the exact one;
  * every reported residual below 1e-12, and the residuals recomputed here in FP64
    (torch on the device) agree with the reported ones;
  * every cluster subspace (clusters: runs of exact eigenvalues closer than 1e-4 alpha)
    within sin(angle) <= 1e-8 of the exact one in the B inner product, the parity bar
    for eigenvectors, at the default tolerance fpm(3) = 12; and within the Davis-Kahan
    bound sin(angle) <= ||A x - lambda B x|| / (|x|_B * gap), gap the distance to the
    nearest exact eigenvalue outside the cluster (times 2 for rounding headroom, plus
    1e-12).
"""

import sys

import numpy as np
import pytest

from workloads import generators as gen

from parity import clusters

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2002_04807_amd")

pytestmark = pytest.mark.gpu

N, M0, EMIN, EMAX, SEED = 4096, 600, -1.0, 1.0, 0


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pencil():
    _say("full size: building the n=4096 pencil (seed 0) on the host")
    A, B, lam, X = gen.prescribed_complex_pencil(N, seed=SEED)
    dev = torch.device("cuda:0")
    At = torch.from_numpy(np.asfortranarray(A)).to(dev)
    Bt = torch.from_numpy(np.asfortranarray(B)).to(dev)
    Lc = np.linalg.cholesky(B)
    h = mf.Handle(0)
    yield dict(A=A, B=B, lam=lam, X=X, At=At, Bt=Bt, Lc=Lc, h=h)
    h.close()


def _check(p, out):
    lam = p["lam"]
    inside = (lam >= EMIN) & (lam <= EMAX)
    cnt = int(inside.sum())
    assert out["info"] == 0, out["info"]
    assert out["M"] == cnt, (out["M"], cnt)
    lam_in = lam[inside]
    E = out["E"].cpu().numpy()[:cnt]
    alpha = max(abs(EMIN), abs(EMAX))
    eig_err = float(np.max(np.abs(E - lam_in) / np.maximum(np.abs(lam_in), alpha)))
    assert eig_err <= 1e-10, eig_err
    res = out["res"].cpu().numpy()[:cnt]
    assert float(res.max()) <= 1e-12, float(res.max())

    # residuals recomputed in FP64 on the device
    Xg = out["X"][:, :cnt].contiguous()
    Eg = out["E"][:cnt].to(Xg.dtype)
    BX = p["Bt"] @ Xg
    R = p["At"] @ Xg - BX * Eg[None, :]
    rnorm = torch.linalg.vector_norm(R, dim=0).cpu().numpy()
    bxn = torch.linalg.vector_norm(BX, dim=0).cpu().numpy()
    res_here = rnorm / (alpha * bxn)
    assert np.allclose(res_here, res, rtol=1e-2, atol=1e-14), float(np.max(np.abs(res_here - res)))

    # Davis-Kahan in the B inner product against the exact eigenvectors
    Xc = Xg.cpu().numpy()
    xb = np.sqrt(np.real(np.sum(np.conj(Xc) * (p["B"] @ Xc), axis=0)))
    Xt = p["Lc"].conj().T @ Xc
    Xr = p["Lc"].conj().T @ p["X"][:, inside]
    idx_in = np.flatnonzero(inside)
    worst_ratio = 0.0
    worst_sin = 0.0
    for g in clusters(lam_in, 1e-4 * alpha):
        gl = idx_in[g]
        others = np.delete(lam, gl)
        gap = float(np.min(np.abs(others[:, None] - lam[gl][None, :])))
        qx, _ = np.linalg.qr(Xt[:, g])
        qy, _ = np.linalg.qr(Xr[:, g])
        s = float(np.linalg.norm(qx - qy @ (qy.conj().T @ qx), 2))
        bound = 2.0 * float(np.max(rnorm[g] / xb[g])) / gap + 1e-12
        assert s <= bound, (g, s, bound)
        assert s <= 1e-8, (g, s, bound)
        worst_ratio = max(worst_ratio, s / bound)
        worst_sin = max(worst_sin, s)
    return eig_err, float(res.max()), worst_ratio, worst_sin


@pytest.mark.parametrize("fp32", [True, False])
def test_pencil_4096_m600_against_construction(pencil, fp32):
    _say("full size: mfeast_zhegv n=4096 M0=600 fp32=%s" % fp32)
    fpm = mf.mfeast_init()
    fpm[41] = 1 if fp32 else 0
    out = mf.feast(pencil["At"], pencil["Bt"], EMIN, EMAX, M0, fpm=fpm, handle=pencil["h"])
    torch.cuda.synchronize()
    _say("full size: loop %d, M %d; checking" % (out["loop"], out["M"]))
    eig_err, res_max, ratio, sin_max = _check(pencil, out)
    _say("full size: eig err %.1e, max res %.1e, worst cluster sin %.1e, worst angle / bound %.2f"
         % (eig_err, res_max, sin_max, ratio))
    # a second call on the same handle (reused workspace) gives the same answer
    out2 = mf.feast(pencil["At"], pencil["Bt"], EMIN, EMAX, M0, fpm=fpm, handle=pencil["h"])
    torch.cuda.synchronize()
    assert out2["M"] == out["M"] and out2["loop"] == out["loop"]
    assert torch.equal(out2["E"], out["E"])
