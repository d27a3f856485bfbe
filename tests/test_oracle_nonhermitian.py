"""Pins of the oracle's non-Hermitian FEAST (Section 3.3) against what fixes the answer
independently: closed forms of the full-contour filter, exact quadrature cases, pencils
built with a known spectrum and known right and left eigenvectors, the Hermitian oracle
on a Hermitian matrix, and the algebraic identity behind the residual form."""

import numpy as np
import pytest

import oracle
from oracle import nonhermitian as nh
from workloads import generators as gen

from parity import clusters


def _sin(X, Y):
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    return float(np.linalg.norm(qx - qy @ (qy.conj().T @ qx), 2))


@pytest.mark.parametrize("ne,angle", [(8, 0), (16, 0), (12, 30), (7, -75)])
def test_trapezoidal_circle_filter_closed_form(ne, angle):
    """On a circle, the trapezoidal full contour gives rho = 1 / (1 + u^ne) with
    u = e^{-i phi} (lambda - Emid) / r, for every complex lambda off the nodes."""
    emid, r = 0.4 - 0.7j, 1.3
    z, w = nh.full_contour(emid, r, ne, rule=1, ratio_pct=100, angle_deg=angle)
    rng = np.random.default_rng(1)
    lam = emid + r * (rng.uniform(-2, 2, 200) + 1j * rng.uniform(-2, 2, 200))
    u = np.exp(-1j * np.deg2rad(angle)) * (lam - emid) / r
    np.testing.assert_allclose(nh.full_filter(lam, z, w), 1.0 / (1.0 + u ** ne), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(np.abs(z - emid), r, rtol=0, atol=1e-14)


@pytest.mark.parametrize("ne", [4, 10, 32])
def test_gauss_full_circle_centre_is_exact(ne):
    """At the centre of a circle the integrand (1/2pi) is constant in theta, so every
    Gauss rule integrates it exactly: rho(Emid) = 1."""
    emid, r = -1.0 + 2.0j, 0.5
    z, w = nh.full_contour(emid, r, ne, rule=0)
    assert abs(nh.full_filter(np.array([emid]), z, w)[0] - 1.0) < 1e-13


@pytest.mark.parametrize("rule", [0, 1])
def test_ellipse_filter_converges_to_indicator(rule):
    """Rotated ellipse (ratio 0.4, 35 degrees): with many nodes the filter is the
    indicator of the ellipse (Cauchy's formula) away from the boundary."""
    emid, r = 0.2 + 0.1j, 1.0
    z, w = nh.full_contour(emid, r, 112 if rule == 0 else 200, rule=rule, ratio_pct=40, angle_deg=35)
    rot = np.exp(1j * np.deg2rad(35))
    t = np.linspace(0, 2 * np.pi, 50, endpoint=False)
    inner = emid + rot * 0.6 * (np.cos(t) + 0.4j * np.sin(t))
    outer = emid + rot * 1.6 * (np.cos(t) + 0.4j * np.sin(t))
    # Gauss-Legendre in theta does not have the trapezoidal rule's geometric convergence
    # on periodic integrands
    tol = 1e-5 if rule == 0 else 1e-8
    np.testing.assert_allclose(nh.full_filter(inner, z, w), 1.0, atol=tol)
    np.testing.assert_allclose(nh.full_filter(outer, z, w), 0.0, atol=tol)
    assert np.all(nh.inside_ellipse(inner, emid, r, 40, 35))
    assert not np.any(nh.inside_ellipse(outer, emid, r, 40, 35))


@pytest.mark.parametrize("generalized", [False, True])
@pytest.mark.parametrize("two_sided", [True, False])
def test_prescribed_pencil_eigenpairs(generalized, two_sided):
    n = 150
    A, B, lam, V, Y = gen.prescribed_nonnormal(n, 3, generalized=generalized)
    emid, r = 0.2 - 0.3j, 0.9
    inside = nh.inside_ellipse(lam, emid, r)
    cnt = int(inside.sum())
    fpm = nh.nfeastinit()
    fpm[14] = 0 if two_sided else 1
    out = nh.feast_general(A, B, emid, r, cnt + 10, fpm)
    assert out["info"] == 0 and out["M"] == cnt
    E = out["E"][:cnt]
    li = lam[inside]
    # match each computed value to the exact one
    for e in E:
        assert np.min(np.abs(li - e)) <= 1e-10 * (abs(emid) + r)
    # right (and left) vectors against the construction, per cluster of close values
    order = np.argsort(E.real)
    alpha = abs(emid) + r
    for g in clusters(E.real[order], 1e-4 * alpha):
        idx = order[g]
        ex = [int(np.argmin(np.abs(lam - E[i]))) for i in idx]
        assert _sin(out["X"][:, idx], V[:, ex]) <= 1e-8
        if two_sided:
            assert _sin(out["Y"][:, idx], Y[:, ex]) <= 1e-8
    assert np.max(out["res"][:cnt]) < 1e-12
    if two_sided:
        assert np.max(out["res_left"][:cnt]) < 1e-12
        Bm = np.eye(n) if B is None else B
        G = out["Y"][:, :cnt].conj().T @ Bm @ out["X"][:, :cnt]
        np.testing.assert_allclose(G, np.eye(cnt), atol=1e-9)


def test_hermitian_matrix_matches_hermitian_oracle():
    """A Hermitian pencil searched with a circle around [Emin, Emax]: the non-Hermitian
    path finds the same (real) eigenvalues as the Hermitian oracle."""
    A, B, lam, X = gen.prescribed_complex_pencil(160, 7)
    # interval edges half-way between eigenvalues, about [-1, 1]
    i0 = int(np.searchsorted(lam, -1.0))
    i1 = int(np.searchsorted(lam, 1.0))
    emin, emax = 0.5 * (lam[i0 - 1] + lam[i0]), 0.5 * (lam[i1 - 1] + lam[i1])
    ref = oracle.feast_dense(A, B, emin, emax, 40)
    assert ref["info"] == 0
    fpm = nh.nfeastinit()
    out = nh.feast_general(A, B, 0.5 * (emin + emax), 0.5 * (emax - emin), 40, fpm)
    assert out["info"] == 0 and out["M"] == ref["M"]
    np.testing.assert_allclose(np.sort(out["E"][:out["M"]].real), ref["E"][:ref["M"]], atol=1e-11)
    assert np.max(np.abs(out["E"][:out["M"]].imag)) < 1e-11


def test_classic_and_residual_forms_agree_per_iteration():
    n = 120
    A, B, lam, V, Y = gen.prescribed_nonnormal(n, 5, generalized=True)
    emid, r = 0.0, 1.0
    cnt = int(nh.inside_ellipse(lam, emid, r).sum())
    fpm = nh.nfeastinit()
    fpm[2] = 14
    fpm[3] = 3
    a = nh.feast_general(A, B, emid, r, cnt + 8, fpm, form="residual")
    b = nh.feast_general(A, B, emid, r, cnt + 8, fpm, form="classic")
    for ha, hb in zip(a["history"], b["history"]):
        assert ha["M"] == hb["M"]
        np.testing.assert_allclose(np.sort_complex(ha["E"]), np.sort_complex(hb["E"]), atol=1e-11)


def test_epsout_divisor_and_trace_criterion():
    """epsout is |trace_k - trace_{k-1}| / (|Emid| + r) (Table tab-common2); with
    fpm(6) = 0 the run stops at the first iteration below 10^-fpm(3)."""
    A, B, lam, V, Y = gen.prescribed_nonnormal(100, 9)
    emid, r = 0.5 + 0.5j, 1.0
    cnt = int(nh.inside_ellipse(lam, emid, r).sum())
    fpm = nh.nfeastinit()
    fpm[5] = 0
    fpm[2] = 10
    out = nh.feast_general(A, B, emid, r, cnt + 8, fpm)
    h = out["history"]
    assert out["info"] == 0
    for k in range(1, len(h)):
        d = abs(np.sum(h[k]["E"]) - np.sum(h[k - 1]["E"])) / (abs(emid) + r)
        assert h[k]["epsout"] == pytest.approx(d, rel=1e-12, abs=1e-300)
    assert out["loop"] == next(k for k in range(1, len(h)) if h[k]["epsout"] < 1e-10)


def test_argument_checks():
    A = np.eye(10, dtype=complex)
    f = nh.nfeastinit()
    assert nh.feast_general(np.zeros((0, 0)), None, 0, 1, 1, f)["info"] == 202
    assert nh.feast_general(A, None, 0, 1, 11, f)["info"] == 201
    assert nh.feast_general(A, None, 0, 0.0, 4, f)["info"] == 200
    for idx, val, code in [(7, 1, 108), (15, 2, 116), (17, 0, 118), (18, 200, 119), (14, 2, 115), (13, 1, 114)]:
        g = f.copy()
        g[idx] = val
        assert nh.feast_general(A, None, 0, 1, 4, g)["info"] == code, (idx, val)
