"""Plain FP64 non-Hermitian FEAST for dense matrices (oracle).

Test infrastructure only (see the package docstring).

What is computed follows the guide's Section 3.3 "FEAST Non-Hermitian" and its tables:
  * the problem A x = lambda B x with A, B complex general, eigenvalues searched inside
    a full contour (an ellipse centred at Emid with horizontal radius r, axis ratio
    fpm(18)/100, rotation fpm(19) degrees) with fpm(8) nodes, trapezoidal (fpm(16)=1,
    the non-Hermitian default) or Gauss (fpm(16)=0) (Table tab_fpm, zfeast_gcontour);
  * the non-Hermitian RCI template: per node, factor Az = Ze B - A (case 10), solve
    with the right block (case 11) and, for left eigenvectors, with Az^H reusing the
    factorization (cases 20/21); products A X, A^H X, B X, B^H X (cases 30/31/40/41);
  * Table tab-common2: outputs E (complex), X (right vectors, then left vectors when
    fpm(15)=0), M, res (right, then left), epsout = |trace_k - trace_{k-1}| / alpha,
    alpha = |Emid| + r; res_i = ||A x_i - lambda_i B x_i|| / ||alpha B x_i|| (right) and
    ||A^H y_i - conj(lambda_i) B^H y_i|| / ||alpha B^H y_i|| (left).

Readings where the guide is silent (listed with their reasons in the design notes):
  R-ncontour  z(theta) = Emid + e^{i phi} (r cos theta + i e r sin theta), theta in
              [0, 2 pi), e = fpm(18)/100, phi = fpm(19) degrees (counter-clockwise);
              (1/2 pi i) z'(theta) dtheta = (1/2 pi) e^{i phi} (e r cos theta + i r sin theta)
              dtheta.  Trapezoidal: theta_j = 2 pi (j - 1/2)/ne, w_j = (1/ne) e^{i phi}(...);
              Gauss: theta_j = pi (1 + x_j) with Legendre nodes x_j, weights omega_j on
              [-1, 1], w_j = (omega_j / 2) e^{i phi}(...).  Filter rho(lambda) =
              sum_j w_j / (z_j - lambda).
  R-left      left subspace: Q~ = sum_j conj(w_j) (z_j B - A)^-H B^H Y~ (the projector of
              the pencil (A^H, B^H) on the conjugate contour; scalar filter conj(rho)).
  R-equil     the columns of Q and Q~ are scaled to unit 2-norm before the reduced
              matrices are formed (a change of basis inside the same subspaces, so the Ritz
              pairs are unchanged in exact arithmetic; it evens out the columns' scales,
              which the filter spreads over many orders of magnitude).
  R-nrank     the equilibrated Q and Q~ are replaced by orthonormal bases of their numerical
              ranges (singular values above 1e-13 times the largest); for two-sided runs
              both keep the smaller of the two ranks, and M0 shrinks to it ("new suitable
              M0", Table tab-common2).  info = -3 if nothing is kept or the reduced pencil
              has non-finite eigenvalues.
  R-rr        two-sided (fpm(15)=0): Aq = Q~^H A Q, Bq = Q~^H B Q, right and left
              eigenvectors W, W~ of (Aq, Bq); one-sided (fpm(15)=1): Q~ = Q and only right
              vectors.  X = Q W with unit 2-norm columns; Y = Q~ W~ scaled so that
              y_i^H B x_i = 1.
  R-inside    M = number of found pairs: Ritz values inside the (closed) ellipse whose
              relative residual (right, and left when two-sided) is below SPURIOUS_RES = 0.1;
              spurious Ritz values of a projected non-normal problem can fall inside the
              contour with residuals of order one (the Hermitian reading's first test).
              info = 1 when no Ritz value lies inside, 3 when all do (whatever their
              residuals); convergence needs at least one found pair.
  R-order     inside values first, then the others, each ascending by real part, then by
              imaginary part; X (and Y, res) follow E.
  R-conv      fpm(6)=1: max residual (right, and left when two-sided) over the inside
              pairs below 10^-fpm(3); fpm(6)=0: epsout below it.  epsout = 1 at iteration 0.
  R-start     Y (and Y~) from fpm(5)=1, else the complex SplitMix64 block of seed fpm(51)
              (right) and of seed fpm(51) + 1 (left).
  R-resid     iteration k > 0 runs the residual form: with R = A X - B X Lambda and
              R~ = A^H Y - B^H Y conj(Lambda), Q = X rho(Lambda) + sum_j w_j (z_j B - A)^-1 R
              (z_j - Lambda)^-1 and Q~ = Y conj(rho(Lambda)) + sum_j conj(w_j) (z_j B - A)^-H R~
              (conj(z_j) - conj(Lambda))^-1, the same subspaces as the classic form in exact
              arithmetic (the identity of the Hermitian oracle holds for any diagonal Lambda).
"""

import numpy as np
import scipy.linalg as sla

from .contour import gauss_legendre_rule
from .splitmix import initial_subspace

GAUSS_FULL_ALLOWED = tuple(range(2, 41)) + (48, 64, 80, 96, 112)
SPURIOUS_RES = 1.0e-1


def full_contour(emid, r, ne, rule=1, ratio_pct=100, angle_deg=0):
    """Nodes z_j and weights w_j of the full contour (R-ncontour); complex128 arrays."""
    emid = complex(emid)
    e = ratio_pct / 100.0
    rot = np.exp(1j * np.deg2rad(angle_deg))
    if rule == 1:
        j = np.arange(1, ne + 1, dtype=np.float64)
        theta = 2.0 * np.pi * (j - 0.5) / ne
        scale = np.full(ne, 1.0 / ne)
    elif rule == 0:
        x, om = gauss_legendre_rule(ne)
        theta = np.pi * (1.0 + x)
        scale = om / 2.0
    else:
        raise ValueError("rule must be 0 (Gauss) or 1 (trapezoidal)")
    z = emid + rot * (r * np.cos(theta) + 1j * e * r * np.sin(theta))
    w = scale * rot * (e * r * np.cos(theta) + 1j * r * np.sin(theta))
    return z.astype(np.complex128), w.astype(np.complex128)


def full_filter(lam, z, w):
    """rho(lambda) = sum_j w_j / (z_j - lambda) for complex lambda (array)."""
    lam = np.asarray(lam, dtype=np.complex128)
    out = np.zeros(lam.shape, dtype=np.complex128)
    for zj, wj in zip(z, w):
        out += wj / (zj - lam)
    return out


def inside_ellipse(lam, emid, r, ratio_pct=100, angle_deg=0):
    """True where lambda lies in the closed (rotated) ellipse."""
    u = np.exp(-1j * np.deg2rad(angle_deg)) * (np.asarray(lam, dtype=np.complex128) - emid)
    e = ratio_pct / 100.0
    return (u.real / r) ** 2 + (u.imag / (e * r)) ** 2 <= 1.0


def nfeastinit():
    """fpm defaults for the non-Hermitian drivers (Table tab_fpm): feastinit, then
    fpm(15)=0 (two-sided), fpm(16)=1 (trapezoidal), fpm(18)=100 (circle)."""
    from .feast import feastinit
    fpm = feastinit()
    fpm[14] = 0
    fpm[15] = 1
    fpm[17] = 100
    return fpm


def validate_general(n, m0, r, fpm, have_expert_contour=False):
    """Argument checks in the order of Table tab_info; returns info or 0."""
    f = lambda i: int(fpm[i - 1])  # noqa: E731
    if n < 1:
        return 202
    if m0 < 1 or m0 > n:
        return 201
    if not (r > 0):
        return 200
    if not have_expert_contour:
        if f(16) not in (0, 1):
            return 116
        if f(16) == 0 and f(8) not in GAUSS_FULL_ALLOWED:
            return 108
        if f(16) == 1 and f(8) < 2:
            return 108
        if f(18) <= 0:
            return 118
        if not (-180 <= f(19) <= 180):
            return 119
    elif f(8) < 1:
        return 108
    if not (0 <= f(3) <= 16):
        return 103
    if f(4) < 0:
        return 104
    if f(5) not in (0, 1):
        return 105
    if f(6) not in (0, 1):
        return 106
    if f(15) not in (0, 1):
        return 115
    if f(14) != 0:
        return 114
    return 0


def _order(lam, inside):
    idx_in = np.where(inside)[0]
    idx_out = np.where(~inside)[0]
    key = lambda idx: idx[np.lexsort((lam[idx].imag, lam[idx].real))]  # noqa: E731
    return np.concatenate([key(idx_in), key(idx_out)])


RANK_TOL = 1.0e-13


def _range_basis(Q):
    """Orthonormal basis of the numerical range of Q: left singular vectors with singular
    value above RANK_TOL times the largest, in decreasing order (R-nrank)."""
    U, sv, _ = np.linalg.svd(Q, full_matrices=False)
    keep = sv > RANK_TOL * sv[0] if sv.size else sv > 0
    return U[:, keep]


def feast_general(A, B, emid, r, m0, fpm=None, X0=None, zne=None, wne=None, form="residual"):
    """Non-Hermitian FEAST on dense complex A (and B; None means identity).

    X0: n x m0 (one-sided) or n x 2 m0 (right block, then left block) starting vectors,
    used when fpm(5) = 1.  Returns a dict with E, X (right), Y (left or None), M, res
    (right), res_left, epsout, loop, info, history.
    """
    fpm = nfeastinit() if fpm is None else np.asarray(fpm, dtype=np.int64)
    f = lambda i: int(fpm[i - 1])  # noqa: E731
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    info = validate_general(n, m0, r, fpm, have_expert_contour=zne is not None)
    out = {"info": info, "E": None, "X": None, "Y": None, "M": 0, "res": None, "res_left": None,
           "epsout": 1.0, "loop": 0, "history": []}
    if info:
        return out
    Bm = np.eye(n, dtype=np.complex128) if B is None else np.asarray(B, dtype=np.complex128)
    two = f(15) == 0
    if zne is None:
        z, w = full_contour(emid, r, f(8), rule=f(16), ratio_pct=f(18), angle_deg=f(19))
    else:
        z, w = np.asarray(zne, np.complex128), np.asarray(wne, np.complex128)
    alpha = abs(emid) + r
    eps = 10.0 ** (-f(3))
    if f(5) == 1:
        X = np.asarray(X0, dtype=np.complex128)[:, :m0].copy()
        Yl = np.asarray(X0, dtype=np.complex128)[:, m0:2 * m0].copy() if two else X.copy()
    else:
        X = initial_subspace(n, m0, f(51), True)
        Yl = initial_subspace(n, m0, f(51) + 1, True) if two else X.copy()
    facts = [sla.lu_factor(zj * Bm - A) for zj in z]
    lam = None
    trace_prev = None
    k = 0
    while True:
        if k == 0 or form == "classic":
            BX = Bm @ X
            BYl = Bm.conj().T @ Yl
            Q = np.zeros_like(X)
            Ql = np.zeros_like(Yl)
            for j in range(len(z)):
                Q += w[j] * sla.lu_solve(facts[j], BX)
                if two:
                    Ql += np.conj(w[j]) * sla.lu_solve(facts[j], BYl, trans=2)
        else:
            R = A @ X - (Bm @ X) * lam[None, :]
            rho = full_filter(lam, z, w)
            Q = X * rho[None, :]
            if two:
                Rl = A.conj().T @ Yl - (Bm.conj().T @ Yl) * np.conj(lam)[None, :]
                Ql = Yl * np.conj(rho)[None, :]
            for j in range(len(z)):
                Q += w[j] * sla.lu_solve(facts[j], R) / (z[j] - lam)[None, :]
                if two:
                    Ql += np.conj(w[j]) * sla.lu_solve(facts[j], Rl, trans=2) / np.conj(z[j] - lam)[None, :]
        if not two:
            Ql = Q
        # R-equil / R-nrank: unit columns, then orthonormal bases of the numerical ranges
        Q = _range_basis(Q / np.linalg.norm(Q, axis=0)[None, :])
        if two:
            Ql = _range_basis(Ql / np.linalg.norm(Ql, axis=0)[None, :])
            kept = min(Q.shape[1], Ql.shape[1])
            Q, Ql = Q[:, :kept], Ql[:, :kept]
        else:
            Ql = Q
        if Q.shape[1] == 0:
            out.update(info=-3, loop=k)
            return out
        m0 = Q.shape[1]
        Aq = Ql.conj().T @ (A @ Q)
        Bq = Ql.conj().T @ (Bm @ Q)
        if two:
            lam, Wl, Wr = sla.eig(Aq, Bq, left=True, right=True)
        else:
            lam, Wr = sla.eig(Aq, Bq, right=True)
            Wl = None
        if not np.all(np.isfinite(lam)):
            out.update(info=-3, loop=k)
            return out
        X = Q @ Wr
        X = X / np.linalg.norm(X, axis=0)[None, :]
        BX = Bm @ X
        R = A @ X - BX * lam[None, :]
        res = np.linalg.norm(R, axis=0) / (alpha * np.linalg.norm(BX, axis=0))
        res_l = None
        if two:
            Yl = Ql @ Wl
            d = np.sum(np.conj(Yl) * BX, axis=0)
            Yl = Yl / np.conj(d)[None, :]
            BhY = Bm.conj().T @ Yl
            Rl = A.conj().T @ Yl - BhY * np.conj(lam)[None, :]
            res_l = np.linalg.norm(Rl, axis=0) / (alpha * np.linalg.norm(BhY, axis=0))
        ok = res < SPURIOUS_RES
        if two:
            ok = ok & (res_l < SPURIOUS_RES)
        geo = inside_ellipse(lam, emid, r, f(18), f(19))
        n_inside = int(np.sum(geo))
        inside = geo & ok
        perm = _order(lam, inside)
        lam, X, res = lam[perm], X[:, perm], res[perm]
        if two:
            Yl, res_l = Yl[:, perm], res_l[perm]
        else:
            Yl = X.copy()
        M = int(np.sum(inside))
        trace = complex(np.sum(lam[:M]))
        epsout = 1.0 if trace_prev is None else abs(trace - trace_prev) / alpha
        trace_prev = trace
        maxres = float(np.max(res[:M])) if M else 0.0
        if two and M:
            maxres = max(maxres, float(np.max(res_l[:M])))
        out["history"].append({"it": k, "M": M, "trace": trace, "epsout": epsout, "maxres": maxres,
                               "E": lam[:M].copy()})
        out.update(E=lam, X=X, Y=Yl if two else None, M=M, res=res, res_left=res_l, epsout=epsout, loop=k,
                   m0=X.shape[1])
        if n_inside == 0:
            out["info"] = 1
            return out
        if n_inside >= X.shape[1]:
            out["info"] = 3
            return out
        if M > 0 and ((maxres < eps) if f(6) == 1 else (epsout < eps)):
            out["info"] = 0
            return out
        if k >= f(4):
            out["info"] = 2
            return out
        k += 1
