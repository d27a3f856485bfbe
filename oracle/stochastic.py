"""Stochastic estimate of the number of eigenvalues inside the search contour (oracle).

Test infrastructure only (see the package docstring).

With fpm(14)=2 (Table tab_fpm) the solver returns in M an estimate of the number of
eigenvalues in [Emin, Emax] instead of the eigenpairs (info 5, Table tab_info), with
few contour nodes (fpm(2)=3 half-contour nodes by default in that mode).  The guide
names the method (Di Napoli, Polizzi, Saad, "Efficient estimation of eigenvalue
counts in an interval", NLAA 2016) but prints no formula.  Reading used here, the
rational-filter form of Hutchinson's trace estimator from that line of work:

  For B-orthonormal eigenvectors X of the pencil, the first contour of FEAST maps a
  block Y to Q = X diag(rho(lambda)) X^H B Y (rho the quadrature filter, see
  contour.py), and for a random vector y with E[y y^H] = I,
      E[y^H X rho X^H B y] = trace(rho X^H B X) = sum_i rho(lambda_i),
  which counts the eigenvalues inside up to the filter's smearing at the interval
  ends.  Over m0 probe vectors (the columns of Y, Rademacher entries, see
  splitmix.py) the estimate is
      est = Re(trace(Y^H Q)) / m0,
  and M is est rounded to the nearest integer (at least 0).
"""

import numpy as np

from .contour import half_contour
from .feast import _Factored, _contour_classic, feastinit
from .splitmix import rademacher_block
from .zolotarev import zolotarev_contour


def stochasticinit():
    """fpm[64] defaults of the stochastic count (Table tab_fpm, entries marked "using
    Stochastic fpm(14)=2"): feastinit, then fpm(2)=3 half-contour nodes, fpm(8)=6
    full-contour nodes, fpm(14)=2 and fpm(15)=1 (one-sided contour).  0-based array."""
    fpm = feastinit()
    fpm[1] = 3
    fpm[7] = 6
    fpm[13] = 2
    fpm[14] = 1
    return fpm


def filtered_trace(A, B, Y, z, w, c_inf=0.0):
    """Re(trace(Y^H Q)) with Q the first contour of FEAST applied to the block Y
    (nodes z, half-contour weights w, constant term c_inf; B None for B = I)."""
    real_problem = np.isrealobj(A) and (B is None or np.isrealobj(B))
    facts = [_Factored(zj, A, B) for zj in z]
    BY = Y if B is None else B @ Y
    Q = _contour_classic(facts, z, w, BY, real_problem, Y=Y, c_inf=c_inf)
    return float(np.real(np.sum(np.conj(Y) * Q)))


def stochastic_count(A, B, emin, emax, m0, ne=3, rule=0, ratio_pct=30, seed=0, band_pct=90):
    """(estimate, M) for the pencil (A, B) on [emin, emax] with m0 Rademacher probes
    drawn with the given seed (fpm(51)) and ne half-contour nodes (rule 2: Zolotarev
    with flat band band_pct, fpm(54))."""
    n = A.shape[0]
    if rule == 2:
        z, w, c_inf = zolotarev_contour(emin, emax, ne, band_pct)
    else:
        z, w = half_contour(emin, emax, ne, rule, ratio_pct)
        c_inf = 0.0
    Y = rademacher_block(n, m0, seed)
    est = filtered_trace(A, B, Y, z, w, c_inf) / m0
    return est, max(0, int(np.floor(est + 0.5)))
