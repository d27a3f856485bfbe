"""CPU-side checks of the C interface: the library loads, exports every declared
symbol, and its host logic (defaults, contour, argument checks) agrees with the
guide's tables.  No call here touches a GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfeast.h")

mf = pytest.importorskip("paper_2002_04807_amd")


def _declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void)\s+(mfeast_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = mf.library()
    names = _declared_symbols()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(mf.EXPORTED)


def test_defaults_match_feastinit_table():
    got = mf.mfeast_init()
    want = oracle.feastinit()
    np.testing.assert_array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("rule,ratio,ne", [(0, 30, 8), (0, 100, 16), (0, 50, 5), (1, 100, 4), (1, 100, 16),
                                           (0, 30, 56), (0, 30, 1)])
def test_contour_matches_oracle(rule, ratio, ne):
    info, z, w = mf.mfeast_contour(-0.7, 2.2, ne, rule, ratio)
    assert info == 0
    zo, wo = oracle.half_contour(-0.7, 2.2, ne, rule=rule, ratio_pct=ratio)
    np.testing.assert_allclose(z, zo, rtol=0, atol=1e-14)
    np.testing.assert_allclose(w, wo, rtol=0, atol=1e-14)


def test_contour_errors():
    assert mf.mfeast_contour(1.0, 1.0, 8)[0] == 200
    assert mf.mfeast_contour(0.0, 1.0, 21, 0)[0] == 102
    assert mf.mfeast_contour(0.0, 1.0, 21, 1)[0] == 0
    assert mf.mfeast_contour(0.0, 1.0, 8, 3)[0] == 116
    assert mf.mfeast_contour(0.0, 1.0, 21, 2, 90)[0] == 102
    assert mf.mfeast_contour(0.0, 1.0, 8, 2, 100)[0] == 154
    assert mf.mfeast_contour(0.0, 1.0, 8, 0, 0)[0] == 118
    assert mf.mfeast_zolotarev(0.0, 1.0, 8, 0)[0] == 154
    assert mf.mfeast_zolotarev(0.0, 1.0, 9, 90)[0] == 0
    assert mf.mfeast_zolotarev(0.0, 1.0, 21, 90)[0] == 102


@pytest.mark.parametrize("ne,band", [(1, 90), (2, 50), (4, 90), (8, 90), (8, 75), (16, 95), (56, 90)])
def test_zolotarev_matches_oracle(ne, band):
    """The library's Zolotarev rule (its own elliptic functions by the arithmetic-geometric
    mean) against the oracle's (SciPy's elliptic functions): nodes, weights, constant."""
    info, z, w, ci = mf.mfeast_zolotarev(-0.7, 2.2, ne, band)
    assert info == 0
    zo, wo, co = oracle.zolotarev_contour(-0.7, 2.2, ne, band)
    # The oracle hands SciPy the parameter m = 1 - l^2 of the Jacobi functions, rounded
    # in FP64: a relative error of about 1e-16 / l^2 in the complementary parameter l^2
    # (l = 0.0028 for a 90% band, 1.7e-4 for 95%), which moves the coefficients by up to
    # about 1e-10; the library starts from the complementary modulus l itself.
    tol = 1e-10
    np.testing.assert_allclose(z, zo, rtol=0, atol=tol)
    np.testing.assert_allclose(w, wo, rtol=0, atol=tol)
    assert abs(ci - co) <= tol
    info, z2, w2 = mf.mfeast_contour(-0.7, 2.2, ne, 2, band)
    assert info == 0
    np.testing.assert_array_equal(z2, z)
    np.testing.assert_array_equal(w2, w)


def _call(name, n=10, m0=4, emin=0.0, emax=1.0, fpm=None, handle=None, **kw):
    """Invoke a dense entry point with host dummies and a NULL handle: only the
    host-side argument checks can run (no device pointer is ever dereferenced)."""
    fpm = oracle.feastinit().astype(np.int32) if fpm is None else fpm
    dummy = np.zeros(8)
    args = dict(uplo="F", A=dummy, lda=max(n, 1), B=None, ldb=max(n, 1), E=dummy, X=dummy, ldx=max(n, 1),
                res=dummy)
    args.update(kw)
    out = getattr(mf, name)(handle, args["uplo"], n, args["A"], args["lda"], args["B"], args["ldb"], fpm,
                            emin, emax, m0, args["E"], args["X"], args["ldx"], args["res"])
    return out["info"]


@pytest.mark.parametrize("name", ["mfeast_dsygv", "mfeast_zhegv"])
def test_argument_checks_in_table_order(name):
    assert _call(name, n=0) == 202
    assert _call(name, m0=0) == 201
    assert _call(name, m0=11) == 201
    # the kernels' limits: n <= 16384 (dense LU), M0 <= 1024 (reduced eigensolver)
    assert _call(name, n=16385, m0=4) == 202
    assert _call(name, n=2000, m0=1025) == 201
    assert _call(name, emin=1.0, emax=1.0) == 200
    for idx, val, code in [(1, 21, 102), (2, 17, 103), (3, -1, 104), (4, 2, 105), (5, 2, 106),
                           (13, 3, 114), (15, 3, 116), (17, 0, 118), (41, 2, 142), (49, 9, 150),
                           (49, -1, 150), (52, 2, 153)]:
        f = oracle.feastinit().astype(np.int32)
        f[idx] = val
        assert _call(name, fpm=f) == code, (idx, val)
    # a consistent call reaches the handle check
    assert _call(name) == -101
    assert _call(name, handle=ctypes.c_void_p(1), uplo="X") == -102
    assert _call(name, handle=ctypes.c_void_p(1), A=None) == -104
    assert _call(name, handle=ctypes.c_void_p(1), lda=5) == -105
    assert _call(name, handle=ctypes.c_void_p(1), B=np.zeros(4), ldb=3) == -107
    assert _call(name, handle=ctypes.c_void_p(1), E=None) == -112
    assert _call(name, handle=ctypes.c_void_p(1), X=None) == -113
    assert _call(name, handle=ctypes.c_void_p(1), ldx=2) == -114
    assert _call(name, handle=ctypes.c_void_p(1), res=None) == -116


def test_create_without_device_reports_minus_900():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert mf.library().mfeast_create(ctypes.byref(h), 0, None) == -900


def test_ifeast_defaults_match_oracle():
    got = mf.mfeast_init_ifeast()
    np.testing.assert_array_equal(got.astype(np.int64), oracle.ifeastinit())


def test_stochastic_defaults_match_oracle():
    from oracle.stochastic import stochasticinit
    got = mf.mfeast_init_stochastic()
    np.testing.assert_array_equal(got.astype(np.int64), stochasticinit())


def _csr_call(n=10, m0=4, emin=0.0, emax=1.0, fpm=None, handle=None, **kw):
    """mfeast_dcsrgv with host dummies: only the host-side argument checks run."""
    fpm = oracle.ifeastinit().astype(np.int32) if fpm is None else fpm
    dummy = np.zeros(8)
    idx = np.zeros(8, dtype=np.int32)
    args = dict(uplo="F", a=dummy, ia=idx, ja=idx, base=0, b=None, ib=None, jb=None, E=dummy, X=dummy,
                ldx=max(n, 1), res=dummy)
    args.update(kw)
    out = mf.mfeast_dcsrgv(handle, args["uplo"], n, args["a"], args["ia"], args["ja"], args["base"], args["b"],
                           args["ib"], args["jb"], fpm, emin, emax, m0, args["E"], args["X"], args["ldx"],
                           args["res"])
    return out["info"]


def test_csr_argument_checks_in_table_order():
    assert _csr_call(n=0) == 202
    assert _csr_call(m0=0) == 201
    assert _csr_call(emin=2.0, emax=1.0) == 200
    for idx, val, code in [(1, 0, 102), (2, 17, 103), (15, 3, 116), (44, -1, 145), (44, 17, 145), (45, 0, 146)]:
        f = oracle.ifeastinit().astype(np.int32)
        f[idx] = val
        assert _csr_call(fpm=f) == code, (idx, val)
    assert _csr_call() == -101
    h = ctypes.c_void_p(1)
    assert _csr_call(handle=h, uplo="Q") == -102
    assert _csr_call(handle=h, a=None) == -104
    assert _csr_call(handle=h, ia=None) == -105
    assert _csr_call(handle=h, ja=None) == -106
    assert _csr_call(handle=h, base=2) == -107
    assert _csr_call(handle=h, b=np.zeros(4)) == -109
    assert _csr_call(handle=h, b=np.zeros(4), ib=np.zeros(4, dtype=np.int32)) == -110
    assert _csr_call(handle=h, E=None) == -115
    assert _csr_call(handle=h, X=None) == -116
    assert _csr_call(handle=h, ldx=3) == -117
    assert _csr_call(handle=h, res=None) == -119


def test_adjoint_argument_checks():
    d = np.zeros(16)
    f = mf.mfeast_dsy_adjoint
    h = ctypes.c_void_p(1)
    # (h, n, A, lda, M, E, X, ldx, gE, gX, ldgx, precision, gA, ldga, gdiag)
    assert f(None, 0, d, 1, 1, d, d, 1, None, None, 1, 0, d, 1, None) == 202
    assert f(None, 4, d, 4, 0, d, d, 4, None, None, 4, 0, d, 4, None) == 201
    assert f(None, 4, d, 4, 5, d, d, 4, None, None, 4, 0, d, 4, None) == 201
    assert f(None, 4, d, 4, 2, d, d, 4, None, None, 4, 0, d, 4, None) == -101
    assert f(h, 4, None, 4, 2, d, d, 4, None, None, 4, 0, d, 4, None) == -103
    assert f(h, 4, d, 3, 2, d, d, 4, None, None, 4, 0, d, 4, None) == -104
    assert f(h, 4, d, 4, 2, None, d, 4, None, None, 4, 0, d, 4, None) == -106
    assert f(h, 4, d, 4, 2, d, None, 4, None, None, 4, 0, d, 4, None) == -107
    assert f(h, 4, d, 4, 2, d, d, 3, None, None, 4, 0, d, 4, None) == -108
    assert f(h, 4, d, 4, 2, d, d, 4, None, d, 3, 0, d, 4, None) == -111
    assert f(h, 4, d, 4, 2, d, d, 4, None, None, 4, 2, d, 4, None) == -112
    assert f(h, 4, d, 4, 2, d, d, 4, None, None, 4, 0, None, 4, None) == -113
    assert f(h, 4, d, 4, 2, d, d, 4, None, None, 4, 0, d, 3, None) == -114


@pytest.mark.parametrize("rule,ne,ratio,angle", [(1, 16, 100, 0), (1, 7, 60, -45), (0, 24, 100, 0), (0, 12, 40, 170)])
def test_full_contour_matches_oracle(rule, ne, ratio, angle):
    from oracle import nonhermitian as nh
    info, z, w = mf.mfeast_gcontour(0.3 - 1.2j, 0.7, ne, rule, ratio, angle)
    assert info == 0
    zo, wo = nh.full_contour(0.3 - 1.2j, 0.7, ne, rule=rule, ratio_pct=ratio, angle_deg=angle)
    np.testing.assert_allclose(z, zo, rtol=0, atol=1e-14)
    np.testing.assert_allclose(w, wo, rtol=0, atol=1e-14)


def test_general_driver_argument_checks():
    """mfeast_zgegv's host checks in Table tab_info order, with host dummies and a NULL
    handle (no device pointer is dereferenced)."""
    from oracle import nonhermitian as nh
    dummy = np.zeros(8)

    def call(n=10, m0=4, r=1.0, fpm=None, handle=None, lda=None, X=dummy, res=dummy, ldx=None):
        f = nh.nfeastinit().astype(np.int32) if fpm is None else fpm
        return mf.mfeast_zgegv(handle, n, dummy, lda or max(n, 1), None, max(n, 1), f, 0.0, r, m0, dummy, X,
                               ldx or max(n, 1), res)["info"]
    assert call(n=0) == 202
    assert call(m0=0) == 201
    assert call(m0=11) == 201
    assert call(n=1000, m0=513) == 201
    assert call(r=0.0) == 200
    for idx, val, code in [(7, 1, 108), (15, 2, 116), (17, 0, 118), (18, 181, 119), (14, 2, 115), (13, 1, 114),
                           (2, 17, 103), (3, -1, 104)]:
        f = nh.nfeastinit().astype(np.int32)
        f[idx] = val
        assert call(fpm=f) == code, (idx, val)
    assert call() == -101
    assert call(handle=ctypes.c_void_p(1), lda=5) == -104
    assert call(handle=ctypes.c_void_p(1), ldx=5) == -115
    assert call(handle=ctypes.c_void_p(1), res=None) == -117
    np.testing.assert_array_equal(mf.mfeast_init_general().astype(np.int64), nh.nfeastinit())


def test_polynomial_driver_argument_checks():
    """mfeast_zgepev's host checks with host dummies and a NULL or dummy handle (every call
    below stops at a check before any device access)."""
    from oracle import polynomial as pl
    dummy = np.zeros(8)

    def call(p=2, n=10, m0=4, r=1.0, fpm=None, handle=None, lda=None, X=dummy, res=dummy, ldx=None):
        f = pl.pfeastinit().astype(np.int32) if fpm is None else fpm
        return mf.mfeast_zgepev(handle, p, n, dummy, lda or max(n, 1), f, 0.0, r, m0, dummy, X, ldx or max(n, 1),
                                res)["info"]
    assert call(p=0) == -102
    assert call(p=9) == -102
    assert call(n=0) == 202
    assert call(m0=0) == 201
    assert call(m0=11) == 201
    assert call(p=3, n=1000, m0=171) == 201  # p M0 > 512
    assert call(p=3, n=1000, m0=170, handle=ctypes.c_void_p(1), lda=5) == -105
    assert call(r=-1.0) == 200
    f = pl.pfeastinit().astype(np.int32)
    f[14] = 0
    assert call(fpm=f) == 115
    for idx, val, code in [(7, 1, 108), (15, 2, 116), (17, 0, 118), (18, 181, 119), (2, 17, 103)]:
        f = pl.pfeastinit().astype(np.int32)
        f[idx] = val
        assert call(fpm=f) == code, (idx, val)
    assert call() == -101
    assert call(handle=ctypes.c_void_p(1), ldx=5) == -114
    assert call(handle=ctypes.c_void_p(1), res=None) == -116
    assert call(handle=ctypes.c_void_p(1), X=None) == -113
    np.testing.assert_array_equal(mf.mfeast_init_polynomial().astype(np.int64), pl.pfeastinit())
