"""Pins of the oracle's Zolotarev rule (fpm(16) = 2) against what the construction fixes.

  * Best approximation: the error 1 - Z of the sign approximation equioscillates on
    [l, 1] at 2m + 1 points (found here by dense sampling, not from the elliptic
    formulas), the characterization of the best odd type (2m-1, 2m) approximation.
  * The filter in partial fractions (nodes, weights, constant) equals (1 + Z)/2 of the
    product form, is exactly 1/2 at Emin and Emax, is symmetric about the centre, and
    stays within the measured error level of 1 inside the flat band and of 0 beyond it.
  * The nodes lie on the circle through Emin and Emax.
  * FEAST with the rule reaches the closed-form spectrum of the 1-D Laplacian.
"""

import numpy as np
import pytest

import oracle
from oracle.zolotarev import zolotarev_contour, zolotarev_filter, zolotarev_sign
from workloads import generators as gen


def _sign_approx(m, ell):
    c, C, _ = zolotarev_sign(m, ell)

    def Z(x):
        x = np.asarray(x, dtype=np.float64)
        out = C * x / (x * x + c[2 * m - 2])
        for q in range(1, m):
            out = out * (x * x + c[2 * q - 1]) / (x * x + c[2 * q - 2])
        return out
    return Z


def _local_extrema(x, e):
    """Values of e at its local extrema along x, endpoints included."""
    idx = [0]
    for i in range(1, len(e) - 1):
        if (e[i] - e[i - 1]) * (e[i + 1] - e[i]) <= 0:
            idx.append(i)
    idx.append(len(e) - 1)
    return np.array([e[i] for i in idx])


@pytest.mark.parametrize("m,a", [(2, 0.5), (4, 0.8), (6, 0.9), (8, 0.9)])
def test_sign_error_equioscillates_at_2m_plus_1_points(m, a):
    kappa = (1 - a) / (1 + a)
    ell = kappa * kappa
    Z = _sign_approx(m, ell)
    x = np.exp(np.linspace(np.log(ell), 0.0, 400001))
    e = 1.0 - Z(x)
    ext = _local_extrema(x, e)
    # merge runs of samples at one flat extremum: keep alternating signs only
    vals = [ext[0]]
    for v in ext[1:]:
        if np.sign(v) != np.sign(vals[-1]):
            vals.append(v)
        elif abs(v) > abs(vals[-1]):
            vals[-1] = v
    vals = np.array(vals)
    assert vals.size == 2 * m + 1, vals
    level = np.max(np.abs(vals))
    assert np.all(np.abs(np.abs(vals) - level) <= 1e-6 * level + 1e-15), vals
    assert np.all(vals[:-1] * vals[1:] < 0)
    # the odd extension: the same level on [-1, -l]
    assert np.max(np.abs(-1.0 - Z(-x))) == pytest.approx(level, rel=1e-9)


@pytest.mark.parametrize("ne,band", [(4, 90), (8, 90), (8, 70), (16, 95)])
def test_filter_from_nodes_and_weights(ne, band):
    emin, emax = -0.7, 2.2
    c, r = 0.5 * (emin + emax), 0.5 * (emax - emin)
    z, w, c_inf = zolotarev_contour(emin, emax, ne, band)
    assert np.allclose(np.abs(z - c), r, rtol=0, atol=1e-13)
    assert np.all(z.imag > 0)

    def f(lam):
        return oracle.rational_filter(lam, z, w) + c_inf

    # partial fractions = product form
    lam = np.linspace(emin - 3 * r, emax + 3 * r, 3001)
    lam = lam[np.abs(np.abs(lam - c) - r) > 1e-9 * r]   # the product form has x = inf at t = 1
    np.testing.assert_allclose(f(lam), zolotarev_filter((lam - c) / r, ne, band / 100.0).real, rtol=0, atol=1e-13)
    # exactly 1/2 at the ends, symmetric about the centre
    np.testing.assert_allclose(f(np.array([emin, emax])), 0.5, rtol=0, atol=1e-13)
    s = np.linspace(0.0, 3.0 * r, 1001)
    # symmetric nodes come from coefficients c_j and c_(2m-j) evaluated apart, each with the
    # rounding of the Jacobi functions' parameter 1 - l^2 (relative error ~ u / l^2)
    a = band / 100.0
    ell = ((1 - a) / (1 + a)) ** 2
    np.testing.assert_allclose(f(c + s), f(c - s), rtol=0, atol=1e-13 + 2.3e-16 / ell ** 2)
    # flat band: the measured equioscillation level delta of the sign approximation
    kappa = (1 - a) / (1 + a)
    x = np.exp(np.linspace(np.log(kappa * kappa), 0.0, 200001))
    delta = float(np.max(np.abs(1.0 - _sign_approx(ne, kappa * kappa)(x))))
    inside = np.linspace(c - a * r, c + a * r, 4001)
    assert np.max(np.abs(f(inside) - 1.0)) <= 0.5 * delta * (1 + 1e-9) + 1e-15
    outside = np.concatenate([c + r * np.geomspace(1 / a, 1e4, 4001), c - r * np.geomspace(1 / a, 1e4, 4001)])
    assert np.max(np.abs(f(outside))) <= 0.5 * delta * (1 + 1e-9) + 1e-15
    # the constant term is the filter at infinity (product form far away)
    far = zolotarev_filter(np.array([1e9]), ne, band / 100.0).real[0]
    assert c_inf == pytest.approx(far, abs=1e-8 * max(delta, 1e-12))
    assert abs(c_inf) <= 0.5 * delta * (1 + 1e-9)


@pytest.mark.parametrize("form", ["residual", "classic"])
def test_feast_with_zolotarev_reaches_laplacian_closed_form(form):
    n, emin, emax, m0 = 200, 0.0, 0.5, 60
    lam = gen.laplacian_1d_eigs(n)
    inside = lam[(lam >= emin) & (lam <= emax)]
    fpm = oracle.feastinit()
    fpm[15] = 2
    out = oracle.feast_dense(gen.laplacian_1d_dense(n), None, emin, emax, m0, fpm, form=form)
    assert out["info"] == 0 and out["M"] == inside.size == 46
    np.testing.assert_allclose(out["E"][:46], inside, rtol=0, atol=1e-12)
    assert np.max(out["res"][:46]) < 1e-12


def test_zolotarev_count_estimate_is_filter_trace():
    """Stochastic count with the Zolotarev rule on a diagonal matrix: Rademacher probes
    give exactly sum_i f(a_i) (no variance on a diagonal), with the constant term."""
    from oracle.stochastic import stochastic_count
    a = np.linspace(-2.0, 3.0, 40)
    A = np.diag(a)
    est, M = stochastic_count(A, None, 0.0, 1.0, 16, ne=8, rule=2, seed=3)
    z, w, c_inf = zolotarev_contour(0.0, 1.0, 8, 90)
    assert est == pytest.approx(float(np.sum(oracle.rational_filter(a, z, w) + c_inf)), rel=1e-12)
    assert M == int(np.sum((a >= 0) & (a <= 1)))
