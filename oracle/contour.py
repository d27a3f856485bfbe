"""Half-contour quadrature nodes and weights for Hermitian FEAST (oracle).

Test infrastructure only (see the package docstring).

The guide (Section "Search contour", Table tab_contour, Table tab_fpm entries
fpm(2), fpm(16), fpm(18)) fixes the *shape*: an ellipse centred on the real
axis through Emin and Emax, symmetric about the real axis, with only the upper
half sampled; fpm(2) nodes; Gauss-Legendre (fpm(16)=0) or trapezoidal
(fpm(16)=1); vertical/horizontal axis ratio fpm(18)/100.  It prints no node or
weight formula.  Reading used here (derived from the Cauchy integral of the
resolvent, not printed in the guide):

  centre c = (Emin+Emax)/2, half-axis r = (Emax-Emin)/2, ratio e = fpm(18)/100
  z(theta) = c + r cos(theta) + i e r sin(theta),   theta in [0, pi]
  (1/2 pi i) z'(theta) dtheta = (1/2 pi) (e r cos(theta) + i r sin(theta)) dtheta

  Gauss-Legendre, nodes x_j / weights om_j on [-1, 1] (ascending x):
      theta_j = (pi/2)(1 - x_j),   w_j = (om_j / 4)(e r cos theta_j + i r sin theta_j)
  Trapezoidal on the full ellipse with 2*ne points theta = pi (j - 1/2)/ne,
  upper half listed from Emin towards Emax:
      theta_j = pi (ne - j + 1/2)/ne, w_j = (1/(2 ne))(e r cos theta_j + i r sin theta_j)

  w_j is the weight of node z_j on the upper half; the lower half node conj(z_j)
  carries conj(w_j).  The spectral projector applied to a block V is therefore
      P V  ~  sum_j [ w_j f(z_j) + conj(w_j) f(conj z_j) ],  f(z) = (zB - A)^-1 B V,
  and the scalar filter seen by an eigenpair (lambda, x) is
      rho(lambda) = sum_j 2 Re( w_j / (z_j - lambda) ).

Nodes are listed with j = 1 nearest Emin; every accumulation runs in node order.
"""

import numpy as np

# Permitted Gauss-Legendre node counts (Table tab_fpm, fpm(2)).
GAUSS_ALLOWED = tuple(range(1, 21)) + (24, 32, 40, 48, 56)


def gauss_legendre_rule(ne):
    """Gauss-Legendre nodes (ascending) and weights on [-1, 1] (library primitive)."""
    x, om = np.polynomial.legendre.leggauss(int(ne))
    return np.asarray(x, dtype=np.float64), np.asarray(om, dtype=np.float64)


def half_contour(emin, emax, ne, rule=0, ratio_pct=30):
    """Nodes z_j and half-contour weights w_j, j = 1..ne (see module docstring).

    rule: 0 = Gauss-Legendre, 1 = trapezoidal (Table tab_fpm, fpm(16)).
    ratio_pct: fpm(18), the ellipse ratio in percent.
    Returns two complex128 arrays of length ne.
    """
    emin = float(emin)
    emax = float(emax)
    ne = int(ne)
    c = 0.5 * (emin + emax)
    r = 0.5 * (emax - emin)
    e = ratio_pct / 100.0
    if rule == 0:
        x, om = gauss_legendre_rule(ne)
        theta = 0.5 * np.pi * (1.0 - x)
        scale = om / 4.0
    elif rule == 1:
        j = np.arange(1, ne + 1, dtype=np.float64)
        theta = np.pi * (ne - j + 0.5) / ne
        scale = np.full(ne, 1.0 / (2.0 * ne))
    else:
        raise ValueError("rule must be 0 (Gauss) or 1 (trapezoidal)")
    z = (c + r * np.cos(theta)) + 1j * (e * r * np.sin(theta))
    w = scale * ((e * r * np.cos(theta)) + 1j * (r * np.sin(theta)))
    return z.astype(np.complex128), w.astype(np.complex128)


def rational_filter(lam, z, w):
    """rho(lambda) = sum_j 2 Re(w_j / (z_j - lambda)) for real lambda (array-valued)."""
    lam = np.asarray(lam, dtype=np.float64)
    out = np.zeros(lam.shape, dtype=np.float64)
    for zj, wj in zip(z, w):
        out += 2.0 * np.real(wj / (zj - lam))
    return out
