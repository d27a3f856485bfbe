"""Zolotarev half-contour rule for Hermitian FEAST (oracle).

Test infrastructure only (see the package docstring).

The guide lists Zolotarev quadrature as integration type fpm(16) = 2, for Hermitian
problems only, with the same permitted node counts as the Gauss rule (Table tab_fpm),
and cites Guettel, Polizzi, Tang and Viaud (SIAM J. Sci. Comput. 2015) for it; it prints
no construction.  The construction used here (written from that method and from
Zolotarev's best approximation of the sign function, in the form of Akhiezer's
"Elements of the theory of elliptic functions"):

1. Best uniform approximation of sign(x) on [-1, -l] u [l, 1] among odd rational
   functions of type (2m-1, 2m), 0 < l < 1:
       Z(x) = C x prod_{q=1}^{m-1} (x^2 + c_{2q}) / prod_{q=1}^{m} (x^2 + c_{2q-1}),
       c_i = l^2 sn^2(i K'/(2m); l') / cn^2(i K'/(2m); l'),  i = 1..2m-1,
   with l' = sqrt(1 - l^2) the modulus of the Jacobi functions sn, cn, dn and
   K' = K(l') the complete elliptic integral.  Its error 1 - Z equioscillates on [l, 1]
   at x_k = l / dn(k K'/(2m); l'), k = 0..2m (x_0 = l, x_2m = 1), so C follows from
   Z(x_0) - 1 = -(Z(x_1) - 1): C = 2 / (Zt(x_0) + Zt(x_1)) with Zt the product for C = 1,
   and the error level is delta = (Zt(x_1) - Zt(x_0)) / (Zt(x_1) + Zt(x_0)).

2. Indicator of the interval.  With t = (lambda - c)/r (c, r the centre and half-width
   of [Emin, Emax]) and the Moebius map x(t) = (1 + t)/(1 - t), which sends (-1, 1) to
   (0, inf) and the outside of [-1, 1] to (-inf, 0), the filter is
       f(t) = (1 + Z(kappa x(t))) / 2,   kappa = (1 - a)/(1 + a),  l = kappa^2,
   so that |t| <= a maps to kappa x in [l, 1] (f within delta/2 of 1) and |t| >= 1/a to
   kappa x in [-1, -l] (f within delta/2 of 0).  Reading R-zolo-band: a = fpm(54)/100
   (a project slot; default 90, i.e. the filter is flat to delta/2 inside 90% of the
   half-width and beyond 1/0.9 of it).  f(+-1) = 1/2 exactly (Z(0) = Z(inf) = 0), and
   f(-t) = f(t): t -> -t is x -> 1/x, i.e. kappa x -> l/(kappa x), which maps the
   approximation set onto itself and keeps the rational type (2m-1, 2m), so by the
   uniqueness of the best approximation Z(l/y) = Z(y).

3. Nodes and weights.  The poles of Z are x_q = +-i sqrt(c_{2q-1})/kappa, mapped by
   t = (x - 1)/(x + 1) onto the unit circle: t_q = (y_q^2 - 1 + 2 i y_q)/(y_q^2 + 1) with
   y_q = sqrt(c_{2q-1})/kappa (upper half for y_q > 0).  Partial fractions give
       f(t) = c_inf + sum_q [ -w_q/r / (t - t_q) + conj(...) ],  i.e. in lambda
       f(lambda) = c_inf + sum_q 2 Re( w_q / (z_q - lambda) ),  z_q = c + r t_q,
   with w_q = -r * Res_{t_q} f and c_inf = f(infinity) = (1 + Z(-kappa))/2.  Reading
   R-zolo-const: the constant c_inf (of size delta/2) is part of the filter; the contour
   sum applies it as c_inf * Y (classic form) and inside rho(lambda) (residual form).
   Nodes are listed with t_q's real part ascending (the node nearest Emin first).
"""

import numpy as np
from scipy.special import ellipj, ellipk


def zolotarev_sign(m, ell):
    """Coefficients c_1..c_{2m-1}, normalization C and error level delta of the best
    type (2m-1, 2m) approximation of sign on [-1, -ell] u [ell, 1] (step 1 above)."""
    m = int(m)
    lp2 = 1.0 - ell * ell                     # (l')^2, the parameter of scipy's functions
    Kp = ellipk(lp2)
    i = np.arange(1, 2 * m, dtype=np.float64)
    sn, cn, _, _ = ellipj(i * Kp / (2 * m), lp2)
    c = ell * ell * sn ** 2 / cn ** 2
    _, _, dn01, _ = ellipj(np.array([0.0, Kp / (2 * m)]), lp2)
    x01 = ell / dn01
    zt = np.array([_product(x, c, m) for x in x01]).real
    C = 2.0 / (zt[0] + zt[1])
    delta = (zt[1] - zt[0]) / (zt[1] + zt[0])
    return c, C, delta


def _product(x, c, m):
    """x prod_{q<m} (x^2 + c_{2q}) / prod_{q<=m} (x^2 + c_{2q-1}) (c 0-based: c[i-1] = c_i),
    formed as a product of ratios so that no partial product under- or overflows."""
    x = complex(x)
    out = x / (x * x + c[2 * m - 2])
    for q in range(1, m):
        out *= (x * x + c[2 * q - 1]) / (x * x + c[2 * q - 2])
    return out


def zolotarev_filter(t, m, a):
    """f(t) = (1 + Z(kappa x(t)))/2 from the product form (step 2); t real or complex array."""
    kappa = (1.0 - a) / (1.0 + a)
    c, C, _ = zolotarev_sign(m, kappa * kappa)
    t = np.atleast_1d(np.asarray(t, dtype=np.complex128))
    out = np.empty(t.shape, dtype=np.complex128)
    for k, tk in enumerate(t):
        out[k] = 0.5 * (1.0 + C * _product(kappa * (1.0 + tk) / (1.0 - tk), c, m))
    return out


def zolotarev_contour(emin, emax, ne, a_pct=90):
    """Nodes z_q, half-contour weights w_q (q = 1..ne) and the constant c_inf (step 3)."""
    m = int(ne)
    a = a_pct / 100.0
    kappa = (1.0 - a) / (1.0 + a)
    ell = kappa * kappa
    c, C, _ = zolotarev_sign(m, ell)
    cen = 0.5 * (emin + emax)
    r = 0.5 * (emax - emin)
    podd = c[0::2]                            # c_1, c_3, ..., c_{2m-1}: the poles' squares
    peven = c[1::2]                           # c_2, ..., c_{2m-2}: the zeros' squares
    z = np.empty(m, dtype=np.complex128)
    w = np.empty(m, dtype=np.complex128)
    for q in range(m):
        xt = 1j * np.sqrt(podd[q])            # pole of Z in the scaled variable kappa x
        # residue of Z at xt: C xt N(xt^2) / (2 xt D'(xt^2)) with N, D the products over
        # the zeros' and poles' squares, D' the derivative in u = x^2
        others = np.delete(podd, q)
        res_x = C * np.prod((peven - podd[q]) / (others - podd[q])) / 2.0
        y = np.sqrt(podd[q]) / kappa
        tq = (y * y - 1.0 + 2j * y) / (y * y + 1.0)
        # kappa x(t) = kappa (1 + t)/(1 - t): d/dt = 2 kappa / (1 - t)^2
        res_t = 0.5 * res_x * (1.0 - tq) ** 2 / (2.0 * kappa)
        z[q] = cen + r * tq
        w[q] = -r * res_t
    order = np.argsort(z.real, kind="stable")
    c_inf = 0.5 * (1.0 + C * _product(-kappa, c, m).real)
    return z[order], w[order], float(c_inf)
