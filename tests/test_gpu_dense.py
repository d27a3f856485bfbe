"""GPU parity of the dense Hermitian FEAST path against the FP64 oracle.

Every case calls the C interface through the thin binding and compares with the
oracle on identical seeded inputs and an identical starting block (fpm(5)=1):
exact count, eigenvalues within 1e-10 * max(|lambda|, alpha), cluster subspace
angles within 1e-8, residuals below 1e-10 for every reported pair.  Sizes span
several 64-wide LU/GEMM tiles and a ragged tail.
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


def _run_gpu(A, B, emin, emax, m0, Y, fp32, extra=None, uplo="F", zne=None, wne=None):
    fpm = mf.mfeast_init()
    fpm[41] = 1 if fp32 else 0
    if extra:
        for k, v in extra.items():
            fpm[k] = v
    At = torch.from_numpy(np.asfortranarray(A)).to(DEV)
    Bt = None if B is None else torch.from_numpy(np.asfortranarray(B)).to(DEV)
    X0 = None if Y is None else torch.from_numpy(np.ascontiguousarray(Y)).to(DEV)
    out = mf.feast(At, Bt, emin, emax, m0, fpm=fpm, X0=X0, uplo=uplo, zne=zne, wne=wne)
    torch.cuda.synchronize()
    return out


def _run_oracle(A, B, emin, emax, m0, Y, extra=None, uplo="F", zne=None, wne=None):
    f = oracle.feastinit()
    if Y is not None:
        f[4] = 1
    if extra:
        for k, v in extra.items():
            f[k] = v
    return oracle.feast_dense(A, B, emin, emax, m0, f, X0=Y, uplo=uplo, zne=zne, wne=wne)


def _check(out, ref, emin, emax, B=None, res_tol=1e-10):
    assert out["info"] == ref["info"] == 0, (out["info"], ref["info"])
    M = ref["M"]
    assert out["M"] == M
    E = out["E"].cpu().numpy()
    X = out["X"].cpu().numpy()
    err = compare_eigenpairs(E, X, ref["E"], ref["X"], M, emin, emax, B=B)
    res = out["res"].cpu().numpy()[:M]
    assert np.all(res <= res_tol), res.max()
    return err


@pytest.mark.parametrize("fp32", [False, True])
def test_helloworld(fp32):
    _say("helloworld fp32=%s" % fp32)
    A = gen.helloworld()
    Y = oracle.initial_subspace(4, 3, 0, False)
    out = _run_gpu(A, None, 3.0, 5.0, 3, Y, fp32)
    ref = _run_oracle(A, None, 3.0, 5.0, 3, Y)
    _check(out, ref, 3.0, 5.0)
    np.testing.assert_allclose(out["E"].cpu().numpy()[:2], [4.0, 4.0], atol=1e-12)


@pytest.mark.parametrize("fp32", [False, True])
def test_first_contour_subspace_matches_oracle(fp32):
    """fpm(14)=1: Q after one contour equals the oracle's classic contour sum."""
    _say("first contour fp32=%s" % fp32)
    n, m0 = 200, 70
    A = gen.laplacian_1d_dense(n)
    Y = oracle.initial_subspace(n, m0, 3, False)
    out = _run_gpu(A, None, 0.0, 0.5, m0, Y, fp32, extra={13: 1})
    ref = _run_oracle(A, None, 0.0, 0.5, m0, Y, extra={13: 1})
    assert out["info"] == ref["info"] == 4
    Q = out["X"].cpu().numpy()
    rel = np.abs(Q - ref["X"]).max() / np.abs(ref["X"]).max()
    assert rel < (2e-5 if fp32 else 1e-12), rel


def test_random_start_block_matches_oracle_generator():
    """fpm(5)=0: the library draws the same SplitMix64 block as the oracle (seen through Q)."""
    _say("random start")
    n, m0 = 96, 12
    A = gen.laplacian_1d_dense(n)
    out = _run_gpu(A, None, 0.0, 0.3, m0, None, False, extra={13: 1, 50: 77})
    f = oracle.feastinit()
    f[13] = 1
    f[50] = 77
    ref = oracle.feast_dense(A, None, 0.0, 0.3, m0, f)
    Q = out["X"].cpu().numpy()
    assert np.abs(Q - ref["X"]).max() < 1e-12 * np.abs(ref["X"]).max()


@pytest.mark.parametrize("fp32", [False, True])
def test_laplacian_1d_n200(fp32):
    _say("laplacian n=200 fp32=%s" % fp32)
    n, m0 = 200, 70
    A = gen.laplacian_1d_dense(n)
    Y = oracle.initial_subspace(n, m0, 0, False)
    out = _run_gpu(A, None, 0.0, 0.5, m0, Y, fp32)
    ref = _run_oracle(A, None, 0.0, 0.5, m0, Y)
    _check(out, ref, 0.0, 0.5)
    k = np.arange(1, n + 1)
    exact = np.sort(2 - 2 * np.cos(k * np.pi / (n + 1)))[:46]
    assert out["M"] == 46
    assert np.max(np.abs(out["E"].cpu().numpy()[:46] - exact)) < 1e-12


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("n", [130, 333])
def test_complex_generalized(fp32, n):
    _say("complex generalized n=%d fp32=%s" % (n, fp32))
    A, B, lam, _ = gen.prescribed_complex_pencil(n, seed=n, lam_lo=-5, lam_hi=5)
    emin, emax = -1.0, 1.0
    cnt = int(np.sum((lam >= emin) & (lam <= emax)))
    m0 = int(np.ceil(1.5 * cnt)) + 3
    Y = oracle.initial_subspace(n, m0, 1, True)
    out = _run_gpu(A, B, emin, emax, m0, Y, fp32)
    ref = _run_oracle(A, B, emin, emax, m0, Y)
    assert ref["M"] == cnt
    _check(out, ref, emin, emax, B=B)
    np.testing.assert_allclose(out["E"].cpu().numpy()[:cnt], lam[(lam >= emin) & (lam <= emax)], atol=1e-10)


@pytest.mark.parametrize("uplo", ["L", "U"])
def test_triangle_storage(uplo):
    _say("uplo %s" % uplo)
    n = 150
    A, B, lam, _ = gen.prescribed_complex_pencil(n, seed=4, lam_lo=-4, lam_hi=4)
    T = np.tril if uplo == "L" else np.triu
    At, Bt = T(A), T(B)
    emin, emax = -0.8, 0.9
    cnt = int(np.sum((lam >= emin) & (lam <= emax)))
    m0 = cnt + 12
    Y = oracle.initial_subspace(n, m0, 2, True)
    out = _run_gpu(At, Bt, emin, emax, m0, Y, True, uplo=uplo)
    ref = _run_oracle(At, Bt, emin, emax, m0, Y, uplo=uplo)
    _check(out, ref, emin, emax, B=B)


def test_real_generalized_odd_m0_and_trapezoid():
    _say("real generalized odd m0 trapezoid")
    rng = np.random.default_rng(8)
    n = 97
    A, lam, U = gen.prescribed_real_problem(n, rng, -3, 3)
    H = rng.standard_normal((n, n))
    B = np.eye(n) + 0.3 * H @ H.T / n
    emin, emax = -0.5, 0.7
    lam_pencil = np.linalg.eigvalsh(np.linalg.solve(np.linalg.cholesky(B), np.linalg.solve(
        np.linalg.cholesky(B), A).T))
    cnt = int(np.sum((lam_pencil >= emin) & (lam_pencil <= emax)))
    m0 = int(np.ceil(1.6 * cnt)) + 5
    m0 += 1 - (m0 % 2)  # odd M0: the Jacobi ordering pads a phantom index
    Y = oracle.initial_subspace(n, m0, 5, False)
    extra = {15: 1, 17: 100, 1: 12}  # trapezoidal rule, circle, 12 nodes
    out = _run_gpu(A, B, emin, emax, m0, Y, True, extra=extra)
    ref = _run_oracle(A, B, emin, emax, m0, Y, extra=extra)
    _check(out, ref, emin, emax, B=B)


def test_expert_contour_and_warnings():
    _say("expert contour and warnings")
    n = 80
    A = gen.laplacian_1d_dense(n)
    z, w = oracle.half_contour(0.0, 0.4, 10, rule=0, ratio_pct=50)
    Y = oracle.initial_subspace(n, 20, 9, False)
    out = _run_gpu(A, None, 0.0, 0.4, 20, Y, True, zne=z, wne=w, extra={1: 10})
    ref = _run_oracle(A, None, 0.0, 0.4, 20, Y, zne=z, wne=w, extra={1: 10})
    _check(out, ref, 0.0, 0.4)
    # no eigenvalue in the interval -> 1; M0 too small -> 3; loop cap -> 2
    assert _run_gpu(A, None, 5.0, 6.0, 4, None, True)["info"] == 1
    assert _run_gpu(A, None, 0.0, 0.5, 3, None, True)["info"] == 3
    assert _run_gpu(A, None, 0.0, 0.5, 20, None, True, extra={2: 16, 3: 0})["info"] == 2
    assert _run_gpu(A, -np.eye(n), 0.0, 0.5, 20, None, False)["info"] == -3


@pytest.mark.parametrize("steps,bound", [(1, 1e-8), (2, 1e-11)])
def test_first_contour_with_refined_fp32_solves(steps, bound):
    """fpm(50) extra refinement steps: the FP32 solves of the first contour approach the
    oracle's FP64 contour sum (a single FP32 solve stays near 1e-5, see above)."""
    _say("first contour refined steps=%d" % steps)
    n, m0 = 200, 70
    A = gen.laplacian_1d_dense(n)
    Y = oracle.initial_subspace(n, m0, 3, False)
    out = _run_gpu(A, None, 0.0, 0.5, m0, Y, True, extra={13: 1, 49: steps})
    ref = _run_oracle(A, None, 0.0, 0.5, m0, Y, extra={13: 1})
    assert out["info"] == ref["info"] == 4
    Q = out["X"].cpu().numpy()
    rel = np.abs(Q - ref["X"]).max() / np.abs(ref["X"]).max()
    assert rel < bound, rel


def test_complex_generalized_with_refined_fp32_solves():
    """fpm(50)=1 on a complex generalized pencil (both solve directions refined): the
    result matches the oracle and converges no later than the plain FP64 form."""
    n = 333
    _say("complex generalized refined n=%d" % n)
    A, B, lam, _ = gen.prescribed_complex_pencil(n, seed=n, lam_lo=-5, lam_hi=5)
    emin, emax = -1.0, 1.0
    cnt = int(np.sum((lam >= emin) & (lam <= emax)))
    m0 = int(np.ceil(1.5 * cnt)) + 3
    Y = oracle.initial_subspace(n, m0, 1, True)
    out = _run_gpu(A, B, emin, emax, m0, Y, True, extra={49: 1})
    ref = _run_oracle(A, B, emin, emax, m0, Y)
    _check(out, ref, emin, emax, B=B)
    out64 = _run_gpu(A, B, emin, emax, m0, Y, False)
    assert out["loop"] <= out64["loop"], (out["loop"], out64["loop"])


def test_four_product_scheme_matches_oracle():
    """fpm(53)=1: the complex FP32 products use four real products instead of Gauss's
    three; same parity bar on a complex generalized pencil with a ragged tail."""
    n = 333
    _say("complex generalized four-product n=%d" % n)
    A, B, lam, _ = gen.prescribed_complex_pencil(n, seed=n + 1, lam_lo=-5, lam_hi=5)
    emin, emax = -1.0, 1.0
    cnt = int(np.sum((lam >= emin) & (lam <= emax)))
    m0 = int(np.ceil(1.5 * cnt)) + 3
    Y = oracle.initial_subspace(n, m0, 2, True)
    out = _run_gpu(A, B, emin, emax, m0, Y, True, extra={52: 1})
    ref = _run_oracle(A, B, emin, emax, m0, Y)
    _check(out, ref, emin, emax, B=B)


@pytest.mark.parametrize("fp32", [False, True])
def test_repeated_calls_are_bit_for_bit_equal(fp32):
    """A complex generalized pencil (its forward and conjugate-transpose solves run on two
    streams at once) solved three times on one handle: count, loop, eigenvalues, vectors and
    residuals equal bit for bit, so no kernel's result depends on scheduling."""
    _say("dense repeated calls fp32=%s" % fp32)
    A, B, lam, _ = gen.prescribed_complex_pencil(333, 2)
    cnt = int(np.sum((lam >= -1.0) & (lam <= 1.0)))
    At = torch.from_numpy(np.asfortranarray(A)).to(DEV)
    Bt = torch.from_numpy(np.asfortranarray(B)).to(DEV)
    h = mf.Handle(0)
    outs = []
    for _ in range(3):
        fpm = mf.mfeast_init()
        fpm[41] = 1 if fp32 else 0
        o = mf.feast(At, Bt, -1.0, 1.0, int(1.5 * cnt) + 8, fpm=fpm, handle=h)
        torch.cuda.synchronize()
        outs.append(o)
    h.close()
    a = outs[0]
    assert a["info"] == 0 and a["M"] == cnt
    for b in outs[1:]:
        assert (b["info"], b["M"], b["loop"]) == (a["info"], a["M"], a["loop"])
        assert torch.equal(a["E"], b["E"]) and torch.equal(a["X"], b["X"]) and torch.equal(a["res"], b["res"])


@pytest.mark.parametrize("fp32", [False, True])
def test_large_subspace_tridiagonal_eigensolver(fp32):
    """M0 = 260 with about 100 eigenvalues inside: the first iteration's reduced problem and
    the block of the pairs not yet found (about 160) are both solved through the real
    tridiagonal form (order >= 128); parity with the oracle as in every dense case."""
    _say("large subspace fp32=%s" % fp32)
    n = 520
    A, B, lam, _ = gen.prescribed_complex_pencil(n, seed=77, lam_lo=-5, lam_hi=5)
    emin, emax = -1.0, 1.0
    cnt = int(np.sum((lam >= emin) & (lam <= emax)))
    m0 = 260
    Y = oracle.initial_subspace(n, m0, 3, True)
    out = _run_gpu(A, B, emin, emax, m0, Y, fp32)
    ref = _run_oracle(A, B, emin, emax, m0, Y)
    assert ref["M"] == cnt
    _check(out, ref, emin, emax, B=B)
    np.testing.assert_allclose(out["E"].cpu().numpy()[:cnt], lam[(lam >= emin) & (lam <= emax)], atol=1e-10)


def test_multiple_eigenvalues_large_subspace():
    """Real symmetric A with eigenvalue 0.3 of multiplicity 80 and 0.6 of multiplicity 20
    (the rest spread over [-4, 4]), M0 >= 128: the reduced problems hold nearly repeated
    Ritz values, which the tridiagonal solver orthogonalizes together in groups (a group
    of more than 64 goes to the Jacobi solver).  Exact count, the repeated eigenvalues to
    1e-12, and oracle parity of every cluster subspace."""
    _say("multiple eigenvalues")
    rng = np.random.default_rng(21)
    n = 400
    lam = np.concatenate([np.full(80, 0.3), np.full(20, 0.6), rng.uniform(-4.0, 4.0, n - 100)])
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (U * lam[None, :]) @ U.T
    A = 0.5 * (A + A.T)
    emin, emax = -1.0, 1.0
    cnt = int(np.sum((lam >= emin) & (lam <= emax)))
    m0 = max(128, cnt + 40)
    Y = oracle.initial_subspace(n, m0, 4, False)
    out = _run_gpu(A, None, emin, emax, m0, Y, False)
    ref = _run_oracle(A, None, emin, emax, m0, Y)
    assert ref["M"] == cnt
    _check(out, ref, emin, emax)
    E = np.sort(out["E"].cpu().numpy()[:cnt])
    np.testing.assert_allclose(E, np.sort(lam[(lam >= emin) & (lam <= emax)]), atol=1e-12)


def test_fp32_solves_below_their_floor():
    """Tolerance 1e-13 with FP32 solves: below the residual floor that FP32 solves reach on
    their own, so the loop refines the solves once in FP64 when it gets there; it must
    converge (info 0) with every residual below 1e-13 and match the oracle."""
    _say("fp32 tolerance 1e-13")
    n = 333
    A, B, lam, _ = gen.prescribed_complex_pencil(n, seed=n, lam_lo=-5, lam_hi=5)
    emin, emax = -1.0, 1.0
    cnt = int(np.sum((lam >= emin) & (lam <= emax)))
    m0 = int(np.ceil(1.5 * cnt)) + 3
    Y = oracle.initial_subspace(n, m0, 1, True)
    out = _run_gpu(A, B, emin, emax, m0, Y, True, extra={2: 13})
    ref = _run_oracle(A, B, emin, emax, m0, Y, extra={2: 13})
    assert ref["M"] == cnt
    _check(out, ref, emin, emax, B=B, res_tol=1e-13)
