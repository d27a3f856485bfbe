"""Plain FP64 polynomial FEAST for dense matrices (oracle).

Test infrastructure only (see the package docstring).

The guide's Section 3.4 "FEAST Polynomial" solves sum_{k=0}^{p} lambda^k A_k x = 0 with the
eigenvalues inside a full contour (Emid, r, fpm(18), fpm(19), fpm(8) nodes; the common
arguments of Table tab-common2 and the matrix layout of Table tab-spec3: A(LDA, N, p+1),
A_k = A(:, :, k+1)).  Its RCI template needs only two operations: form and factor
P(Ze) = sum_k Ze^k A_k at every node (case 10), solve with it (case 11), and products
A_k X (case 30).  Readings (listed with their reasons in the design notes):

  R-pcontour  the full contour of the non-Hermitian oracle (nonhermitian.full_contour).
  R-pfirst    iteration 0: Q = sum_j w_j P(z_j)^-1 Y (the contour integral of the resolvent
              P(z)^-1 applied to the starting block; for P(z) = z I - A it is the filter of
              the linear problem).
  R-presid    iteration k > 0, from the Ritz pairs (lambda_i, x_i) with residuals
              r_i = P(lambda_i) x_i:  Q_i = rho(lambda_i) x_i - sum_j w_j / (z_j - lambda_i)
              P(z_j)^-1 r_i, rho the full-contour filter.  This is sum_j w_j P(z_j)^-1 (z_j -
              lambda_i)^-1 [P(z_j) - P(lambda_i)] x_i, the residual inverse iteration of the
              nonlinear problem; for P(z) = z B - A it is exactly the linear contour sum
              sum_j w_j (z_j B - A)^-1 B x_i.
  R-prr       Rayleigh-Ritz on an orthonormal basis Qo of the numerical range of Q (unit
              columns first; singular values above 1e-13 times the largest): the reduced
              polynomial sum_k lambda^k (Qo^H A_k Qo) w = 0, linearized in companion form
              L0 z = lambda L1 z of size p m (m = kept columns) with z = [w; lambda w; ...;
              lambda^(p-1) w], L0 = [[0, I, ...], ..., [-Aq_0, ..., -Aq_(p-1)]], L1 =
              diag(I, ..., I, Aq_p).  Of its p m eigenvalues the m with the smallest ellipse
              metric ((Re u / r)^2 + (Im u / (e r))^2, u = e^{-i phi}(lambda - Emid)) are kept;
              x = Qo w / ||Qo w|| with w the first block of z.
  R-pres      res_i = ||P(lambda_i) x_i|| / sum_k |lambda_i|^k ||A_k x_i|| (a backward-error
              style relative residual; the linear case's ||alpha B x|| has no polynomial
              analogue).  Convergence: max res over the inside pairs below 10^-fpm(3)
              (fpm(6) = 1) or epsout = |trace_k - trace_{k-1}| / (|Emid| + r) below it.
  R-pone      right eigenvectors only (fpm(15) = 1); ordering and info codes as in the
              non-Hermitian oracle (info 3 when every kept Ritz value lies inside the
              contour: the p m values of the linearization then crowd the subspace, and M0
              must grow; about 1.5 times the count inside suffices in practice).
  R-pfound    a Ritz pair counts as found (in M, the trace and the residual criterion) when
              its value lies inside the contour and its residual is below min(0.1,
              10^(-fpm(3)/2)).  The linearization of the projected polynomial has p m
              eigenvalues, and those inside the contour that belong to no eigenpair of the
              full problem keep relative residuals of 1e-2 to 1e-1 (this relative residual
              is small for any vector when the coefficients differ in scale); the square
              root of the target tolerance separates them from converging pairs, which
              pass it on their way to 10^-fpm(3).
"""

import numpy as np
import scipy.linalg as sla

from .nonhermitian import full_contour, full_filter, inside_ellipse, nfeastinit, validate_general
from .splitmix import initial_subspace

RANK_TOL = 1.0e-13
SPURIOUS_RES = 1.0e-1


def found_tol(fpm):
    """R-pfound: a Ritz pair inside the contour counts as found below this residual,
    min(0.1, 10^(-fpm(3)/2))."""
    return min(SPURIOUS_RES, 10.0 ** (-0.5 * int(fpm[2])))


def pfeastinit():
    """Defaults of the polynomial drivers: the non-Hermitian ones with fpm(15) = 1."""
    fpm = nfeastinit()
    fpm[14] = 1
    return fpm


def poly_eval(As, z):
    """P(z) = sum_k z^k A_k."""
    P = np.zeros_like(As[0], dtype=np.complex128)
    for k, Ak in enumerate(As):
        P = P + (z ** k) * Ak
    return P


def ellipse_metric(lam, emid, r, ratio_pct, angle_deg):
    u = np.exp(-1j * np.deg2rad(angle_deg)) * (np.asarray(lam, dtype=np.complex128) - emid)
    e = ratio_pct / 100.0
    return (u.real / r) ** 2 + (u.imag / (e * r)) ** 2


def contour_first(facts, z, w, Y):
    """R-pfirst: Q = sum_j w_j P(z_j)^-1 Y (facts[j]: LU of P(z_j))."""
    Q = np.zeros_like(Y, dtype=np.complex128)
    for j in range(len(z)):
        Q += w[j] * sla.lu_solve(facts[j], Y)
    return Q


def contour_residual(facts, z, w, As, X, lam):
    """R-presid: Q_i = rho(lambda_i) x_i - sum_j w_j / (z_j - lambda_i) P(z_j)^-1 P(lambda_i) x_i."""
    R = np.zeros_like(X, dtype=np.complex128)
    for k, Ak in enumerate(As):
        R += (Ak @ X) * (lam ** k)[None, :]
    Q = X * full_filter(lam, z, w)[None, :]
    for j in range(len(z)):
        Q -= w[j] * sla.lu_solve(facts[j], R) / (z[j] - lam)[None, :]
    return Q


def feast_polynomial(As, emid, r, m0, fpm=None, X0=None, zne=None, wne=None):
    """Polynomial FEAST on dense complex A_0..A_p (list).  Returns a dict with E, X, M, res,
    epsout, loop, info, m0, history."""
    fpm = pfeastinit() if fpm is None else np.asarray(fpm, dtype=np.int64)
    f = lambda i: int(fpm[i - 1])  # noqa: E731
    As = [np.asarray(a, dtype=np.complex128) for a in As]
    p = len(As) - 1
    n = As[0].shape[0]
    out = {"info": 0, "E": None, "X": None, "M": 0, "res": None, "epsout": 1.0, "loop": 0, "history": []}
    if p < 1:
        out["info"] = -102
        return out
    info = validate_general(n, m0, r, fpm, have_expert_contour=zne is not None)
    if info == 0 and f(15) != 1:
        info = 115
    if info:
        out["info"] = info
        return out
    if zne is None:
        z, w = full_contour(emid, r, f(8), rule=f(16), ratio_pct=f(18), angle_deg=f(19))
    else:
        z, w = np.asarray(zne, np.complex128), np.asarray(wne, np.complex128)
    alpha = abs(emid) + r
    eps = 10.0 ** (-f(3))
    ftol = found_tol(fpm)
    X = np.asarray(X0, dtype=np.complex128)[:, :m0].copy() if f(5) == 1 else initial_subspace(n, m0, f(51), True)
    facts = [sla.lu_factor(poly_eval(As, zj)) for zj in z]
    lam = None
    trace_prev = None
    k = 0
    while True:
        Q = contour_first(facts, z, w, X) if k == 0 else contour_residual(facts, z, w, As, X, lam)
        Qn = Q / np.linalg.norm(Q, axis=0)[None, :]
        U, sv, _ = np.linalg.svd(Qn, full_matrices=False)
        Qo = U[:, sv > RANK_TOL * sv[0]]
        m = Qo.shape[1]
        if m == 0:
            out.update(info=-3, loop=k)
            return out
        Aq = [Qo.conj().T @ (Ak @ Qo) for Ak in As]
        pm = p * m
        L0 = np.zeros((pm, pm), dtype=np.complex128)
        L1 = np.zeros((pm, pm), dtype=np.complex128)
        for b in range(p - 1):
            L0[b * m:(b + 1) * m, (b + 1) * m:(b + 2) * m] = np.eye(m)
            L1[b * m:(b + 1) * m, b * m:(b + 1) * m] = np.eye(m)
        for b in range(p):
            L0[(p - 1) * m:, b * m:(b + 1) * m] = -Aq[b]
        L1[(p - 1) * m:, (p - 1) * m:] = Aq[p]
        mu, Z = sla.eig(L0, L1)
        metric = ellipse_metric(mu, emid, r, f(18), f(19))
        metric = np.where(np.isfinite(metric), metric, np.inf)
        sel = np.argsort(metric, kind="stable")[:m]
        lam = mu[sel]
        if not np.all(np.isfinite(lam)):
            out.update(info=-3, loop=k)
            return out
        X = Qo @ Z[:m, sel]
        X = X / np.linalg.norm(X, axis=0)[None, :]
        R = np.zeros_like(X)
        den = np.zeros(m)
        for kk, Ak in enumerate(As):
            AkX = Ak @ X
            R += AkX * (lam ** kk)[None, :]
            den += np.abs(lam) ** kk * np.linalg.norm(AkX, axis=0)
        res = np.linalg.norm(R, axis=0) / den
        geo = inside_ellipse(lam, emid, r, f(18), f(19))
        n_inside = int(np.sum(geo))
        inside = geo & (res < ftol)
        idx_in = np.where(inside)[0]
        idx_out = np.where(~inside)[0]
        key = lambda idx: idx[np.lexsort((lam[idx].imag, lam[idx].real))]  # noqa: E731
        perm = np.concatenate([key(idx_in), key(idx_out)])
        lam, X, res = lam[perm], X[:, perm], res[perm]
        M = int(idx_in.size)
        trace = complex(np.sum(lam[:M]))
        epsout = 1.0 if trace_prev is None else abs(trace - trace_prev) / alpha
        trace_prev = trace
        maxres = float(np.max(res[:M])) if M else 0.0
        out["history"].append({"it": k, "M": M, "n_inside": n_inside, "epsout": epsout, "maxres": maxres,
                               "E": lam[:M].copy()})
        out.update(E=lam, X=X, M=M, res=res, epsout=epsout, loop=k, m0=m)
        if n_inside == 0:
            out["info"] = 1
            return out
        if n_inside >= m:
            out["info"] = 3
            return out
        if M > 0 and ((maxres < eps) if f(6) == 1 else (epsout < eps)):
            out["info"] = 0
            return out
        if k >= f(4):
            out["info"] = 2
            return out
        k += 1
