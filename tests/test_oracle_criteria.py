"""Pins of the oracle's parameter defaults, trace criterion and found-pair test.

What fixes each expected value:
  * Table tab_fpm's default column (tests/golden/tab_fpm_defaults.json);
  * the HelloWorld run printed in Section 2.4 (its Trace and Error-Trace columns fix
    the divisor of epsout as max(|Emin|, |Emax|));
  * the closed-form spectrum of the 1-D Laplacian (the trace the fpm(6)=0 run must
    reach);
  * a closed form of the Kato-Temple residual for a mixture of two eigenvectors, and
    the invariance of the eigenproblem under (A, B) -> (beta A, beta B).
"""

import json
import os

import numpy as np
import pytest

import oracle
from oracle import feast as ofeast
from oracle.ifeast import ifeastinit
from oracle.stochastic import stochasticinit
from workloads import generators as gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    with open(os.path.join(GOLDEN, "tab_fpm_defaults.json")) as fh:
        return json.load(fh)


def _check_defaults(fpm, table):
    for key, val in table.items():
        i = int(key)
        assert int(fpm[i - 1]) == val, ("fpm(%d)" % i, int(fpm[i - 1]), val)


def test_feastinit_matches_table_tab_fpm():
    g = _golden()
    _check_defaults(oracle.feastinit(), g["hermitian"])


def test_ifeast_and_stochastic_defaults_match_table_tab_fpm():
    g = _golden()
    ifeast = dict(g["hermitian"], **g["ifeast_overrides"])
    _check_defaults(ifeastinit(), ifeast)
    stoch = dict(g["hermitian"], **g["stochastic_overrides"])
    _check_defaults(stochasticinit(), stoch)


def _trace_divisor():
    """max(|Emin|, |Emax|) as fixed by the printed HelloWorld run: Error-Trace of
    iteration 1 times the divisor is the printed change of the trace."""
    run = _golden()["helloworld_run"]
    d_trace = abs(run["trace"][1] - run["trace"][0])
    divisor = d_trace / run["error_trace"][1]
    assert divisor == pytest.approx(max(abs(run["emin"]), abs(run["emax"])), rel=1e-12)
    assert run["error_trace"][0] == 1.0  # iteration 0 prints epsout = 1
    return divisor


def test_helloworld_epsout_follows_printed_error_trace():
    """The oracle's epsout on HelloWorld is its own trace change divided by the divisor
    the guide's printed run fixes (5 for [3, 5]); iteration 0 reports 1."""
    divisor = _trace_divisor()
    A = gen.helloworld()
    fpm = oracle.feastinit()
    fpm[5] = 0  # fpm(6) = 0: trace criterion
    out = oracle.feast_dense(A, None, 3.0, 5.0, 3, fpm)
    h = out["history"]
    assert h[0]["epsout"] == 1.0
    for k in range(1, len(h)):
        d = abs(np.sum(h[k]["E"]) - np.sum(h[k - 1]["E"]))
        assert h[k]["epsout"] == pytest.approx(d / divisor, rel=1e-12, abs=1e-300)
    assert out["M"] == 2 and np.allclose(out["E"][:2], 4.0, atol=1e-12)


@pytest.mark.parametrize("form", ["residual", "classic"])
def test_trace_criterion_on_laplacian_closed_form(form):
    """fpm(6) = 0 on the 1-D Laplacian (n = 200, [0, 0.5], 46 eigenvalues): the run stops
    at the first iteration whose relative trace change, recomputed here from the
    eigenvalues of consecutive iterations with the printed divisor's rule, is below
    10^-fpm(3); the final trace is the closed form's."""
    n, emin, emax, m0 = 200, 0.0, 0.5, 70
    lam = gen.laplacian_1d_eigs(n)
    exact_trace = float(np.sum(lam[(lam >= emin) & (lam <= emax)]))
    assert exact_trace == pytest.approx(7.972983218787455, rel=1e-14)
    divisor = max(abs(emin), abs(emax))
    for p in (12, 6):
        fpm = oracle.feastinit()
        fpm[2] = p
        fpm[5] = 0
        out = oracle.feast_dense(gen.laplacian_1d_dense(n), None, emin, emax, m0, fpm, form=form)
        assert out["info"] == 0 and out["M"] == 46
        h = out["history"]
        eps = [1.0] + [abs(np.sum(h[k]["E"]) - np.sum(h[k - 1]["E"])) / divisor for k in range(1, len(h))]
        for k in range(len(h)):
            assert h[k]["epsout"] == pytest.approx(eps[k], rel=1e-12, abs=1e-300)
        stop = next(k for k in range(len(eps)) if eps[k] < 10.0 ** -p and h[k]["M"] > 0)
        assert out["loop"] == stop == len(h) - 1
        assert out["epsout"] == h[-1]["epsout"]
        assert np.sum(out["E"][:46]) == pytest.approx(exact_trace, rel=10.0 ** -min(p, 12) * 10)


def _two_vector_mixture(beta):
    """A B-unit mixture of two eigenvectors of a prescribed pencil (beta A, beta B), one
    below Emin and one above Emax, with its Rayleigh quotient inside [Emin, Emax]."""
    A, B, lam, X = gen.prescribed_complex_pencil(60, 4, b_scale=0.5)
    A, B = beta * A, beta * B
    X = X / np.sqrt(beta)  # B-orthonormal for the scaled pencil
    emin, emax = -1.0, 1.0
    ia = int(np.searchsorted(lam, emin)) - 1       # largest eigenvalue below Emin
    ib = int(np.searchsorted(lam, emax, side="right"))  # smallest above Emax
    la, lb = lam[ia], lam[ib]
    theta = 0.5 * (emin + emax) + 0.1
    # x = ca xa + cb xb, |ca|^2 + |cb|^2 = 1, Rayleigh quotient |ca|^2 la + |cb|^2 lb = theta
    pa = (lb - theta) / (lb - la)
    x = np.sqrt(pa) * X[:, ia] + np.sqrt(1.0 - pa) * 1j * X[:, ib]
    r = A @ x - theta * (B @ x)
    return A, B, emin, emax, la, lb, theta, x, r


@pytest.mark.parametrize("beta", [1.0, 0.01])
def test_kato_temple_term_of_two_vector_mixture_is_closed_form(beta):
    """For x = ca xa + cb xb (B-unit eigenvectors, |ca|^2 + |cb|^2 = 1) with Rayleigh
    quotient theta, B^-1 r = ca (la - theta) xa + cb (lb - theta) xb, so
    r^H B^-1 r = (lb - theta)(theta - la), at least (Emax - theta)(theta - Emin) when
    la < Emin and lb > Emax: such a pair must not count as found, at any scale of the
    pencil.  The Euclidean ||r||^2 does not have this property (it scales with beta)."""
    A, B, emin, emax, la, lb, theta, x, r = _two_vector_mixture(beta)
    assert abs(np.vdot(x, B @ x) - 1.0) < 1e-12
    assert np.vdot(x, A @ x).real == pytest.approx(theta, abs=1e-12)
    kt = ofeast.kato_temple_terms(r[:, None], ofeast._dense_b_solver(B))[0]
    assert kt == pytest.approx((lb - theta) * (theta - la), rel=1e-10)
    bound = (emax - theta) * (theta - emin)
    assert kt >= bound
    lam = np.array([theta])
    res = np.array([1e-3])  # below the relative-residual threshold: only R-spur decides
    _, M, n_inside = ofeast._ordered(lam, res, emin, emax, np.array([kt]))
    assert n_inside == 1 and M == 0
    if beta == 0.01:
        # the scaled pencil makes the Euclidean residual small enough to pass a 2-norm test
        assert np.linalg.norm(r) ** 2 < bound


def test_found_counts_do_not_depend_on_the_scale_of_the_pencil():
    """(beta A, beta B) has the eigenpairs of (A, B), and every FEAST iterate is the same
    up to rounding: the found count of every iteration must not change.  On this pencil
    (complex Hermitian, n = 200, seed 5, M0 = 28) a found test on the Euclidean residual
    drops a pair at iteration 0 for beta = 100."""
    A, B, lam, X = gen.prescribed_complex_pencil(200, 5)
    emin, emax, m0 = -1.0, 1.0, 28
    Y = oracle.initial_subspace(200, m0, 5, True)
    fpm = oracle.feastinit()
    fpm[4] = 1
    hist = {}
    for beta in (1.0, 0.01, 100.0):
        out = oracle.feast_dense(beta * A, beta * B, emin, emax, m0, fpm, X0=Y)
        assert out["info"] == 0 and out["M"] == 24
        hist[beta] = [h["M"] for h in out["history"]]
        assert np.allclose(out["E"][:24], lam[(lam >= emin) & (lam <= emax)], atol=1e-12)
    assert hist[0.01] == hist[1.0] == hist[100.0]
    assert hist[1.0][0] == 24
