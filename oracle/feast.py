"""Plain FP64 Hermitian FEAST for dense matrices (oracle).

Test infrastructure only (see the package docstring).

What is computed follows the guide:
  * Section 1.1 "The FEAST Algorithm": a quadrature of the resolvent along a
    contour around [Emin, Emax] applied to an M0-column block, followed by a
    Rayleigh-Ritz step on the reduced M0 x M0 problem, iterated.
  * Hermitian RCI templates (Section 3.2): per node, factor Az = Ze*B - A
    (case 10), solve with the block (case 11); for complex Hermitian problems the
    conjugate node is handled by a solve with Az^H that reuses the same
    factorization (cases 20/21); A*X and B*X products (cases 30/40).
  * Table tab-common1: outputs E, X, M, res, epsout, loop; res_i =
    ||A x_i - lambda_i B x_i|| / ||alpha B x_i||, alpha = max(|Emin|, |Emax|);
    epsout = |trace_k - trace_{k-1}| / alpha; M0 in/out.
  * Table tab_fpm defaults (feastinit) and Table tab_info return codes.
  * Section 1.2 / 3.1 "Tips": v4.0 runs residual inverse iterations.  The
    residual form implemented in ``form="residual"`` rests on the identity, for
    any X and diagonal Lambda with R = A X - B X Lambda:
        (zB - A)^-1 B X = X (z - Lambda)^-1 + (zB - A)^-1 R (z - Lambda)^-1,
    so the contour sum of the classic iteration started from Y = X equals
        X diag(rho(lambda)) + sum_j [w_j d_j diag(1/(z_j - lambda))
                                     + conj(w_j) e_j diag(1/(conj z_j - lambda))]
    with d_j = (z_j B - A)^-1 R and e_j = (z_j B - A)^-H R.  Both forms give the
    same subspace in exact arithmetic; iteration 0 always uses the classic form
    on the starting block.

Readings where the guide is silent (each is listed with its reason in the
design notes of the repository):
  R-spur    a Ritz pair (theta, x), x B-normalized, counts as found (one of the M)
            when theta lies in [Emin, Emax], its relative residual is below
            SPURIOUS_RES = 0.1, and its residual r = A x - theta B x satisfies
            r^H B^-1 r < (Emax - theta)(theta - Emin).  Ritz values inside the
            interval that fail either test are spurious: their Ritz vectors mix
            eigenvectors from both sides of the interval whose filter weights are
            small and nearly equal, so they carry no eigenvalue; they are listed with
            the outside values.  The second test is the Kato-Temple bound for the
            operator B^-1 A, self-adjoint in the B inner product, whose residual norm
            for x is ||B^-1 r||_B = (r^H B^-1 r)^(1/2): a B-unit vector B-orthogonal
            to every eigenvector in the interval (the pencil restricted to their
            complement has no eigenvalue there) has r^H B^-1 r >= (Emax - theta)
            (theta - Emin), so a pair below it is not such a mixture.  The test is
            unchanged under (A, B) -> (beta A, beta B), as the eigenpairs are.
            M, the trace and the convergence test use the found pairs only.
  R-order   E(1:M) are the found Ritz values ascending, followed by all others
            ascending; X columns follow E.
  R-closed  the interval is closed.
  R-rank    the reduced overlap S = Q^H B Q is equilibrated (unit diagonal), then
            eigen-decomposed; directions with eigenvalue <= RANK_TOL * max are
            dropped and M0 shrinks to the kept count ("new suitable M0",
            Table tab-common1).  info = -3 if S has a non-positive diagonal or
            nothing is kept.
  R-loop    loop is the index of the last iteration; iteration 0 is the first
            contour (HelloWorld output prints rows 0 and 1, then loop = 1).
  R-info1   info = 1 when no Ritz value at all lies in the interval (after any
            iteration); found pairs are required before convergence is declared.
  R-info3   info = 3 when every Ritz value lies in the interval (no outside
            value shows that the subspace holds all of them; M0 too small).
  R-conv    convergence is tested on the M pairs inside the interval only; at
            iteration 0 epsout = 1.
"""

import numpy as np
import scipy.linalg as sla

from .contour import GAUSS_ALLOWED, half_contour, rational_filter
from .splitmix import initial_subspace
from .zolotarev import zolotarev_contour

RANK_TOL = 1.0e-13
SPURIOUS_RES = 1.0e-1


def feastinit():
    """fpm[64] defaults of the Hermitian FEAST drivers (Table tab_fpm), 1-based view.

    Returned as a 0-based int array: fpm[i-1] holds fpm(i).
    Project slot fpm(51) (reserved in the guide) holds the seed of the random
    starting block; default 0.
    """
    fpm = np.zeros(64, dtype=np.int64)
    fpm[0] = 0     # fpm(1)  runtime comments off
    fpm[1] = 8     # fpm(2)  half-contour nodes
    fpm[2] = 12    # fpm(3)  eps = 1e-12
    fpm[3] = 20    # fpm(4)  max refinement loops
    fpm[4] = 0     # fpm(5)  no initial guess
    fpm[5] = 1     # fpm(6)  residual criterion
    fpm[7] = 16    # fpm(8)  full-contour nodes (non-Hermitian; unused)
    fpm[9] = 1     # fpm(10) factorizations stored
    fpm[13] = 0    # fpm(14) normal execution
    fpm[14] = 2    # fpm(15) one-sided contour, left = right* (Hermitian drivers)
    fpm[15] = 0    # fpm(16) Gauss-Legendre
    fpm[17] = 30   # fpm(18) ellipse ratio 0.30
    fpm[18] = 0    # fpm(19) rotation (non-Hermitian only)
    fpm[39] = 0    # fpm(40) user interval
    fpm[40] = 1    # fpm(41) matrix scaling (sparse drivers)
    fpm[41] = 1    # fpm(42) single-precision solves
    fpm[42] = 0    # fpm(43) no automatic IFEAST switch
    fpm[44] = 1    # fpm(45) BiCGStab accuracy 1e-1
    fpm[45] = 40   # fpm(46) BiCGStab max iterations
    fpm[50] = 0    # fpm(51) seed of the random starting block (project slot)
    fpm[53] = 90   # fpm(54) Zolotarev flat band, percent of the half-width (project slot)
    return fpm


def validate(n, m0, emin, emax, fpm, have_expert_contour=False):
    """Host-side argument checks in the order of Table tab_info; returns info or 0."""
    if n < 1:
        return 202
    if m0 < 1 or m0 > n:
        return 201
    if not (emin < emax):
        return 200
    f = lambda i: int(fpm[i - 1])  # noqa: E731  (1-based access as in the guide)
    if not have_expert_contour:
        if f(16) not in (0, 1, 2):
            return 116
        if f(16) in (0, 2) and f(2) not in GAUSS_ALLOWED:
            return 102
        if f(16) == 1 and f(2) < 1:
            return 102
        if f(18) <= 0:
            return 118
        if f(16) == 2 and not (1 <= f(54) <= 99):
            return 154
    elif f(2) < 1:
        return 102
    if not (0 <= f(3) <= 16):
        return 103
    if f(4) < 0:
        return 104
    if f(5) not in (0, 1):
        return 105
    if f(6) not in (0, 1):
        return 106
    if f(14) not in (0, 1):
        return 114
    if f(42) not in (0, 1):
        return 142
    return 0


def expand_uplo(A, uplo):
    """Full Hermitian matrix from the triangle named by UPLO (Table tab-spec1)."""
    A = np.asarray(A)
    if uplo in ("F", "f"):
        return A.copy()
    if uplo in ("L", "l"):
        T = np.tril(A, -1)
    elif uplo in ("U", "u"):
        T = np.triu(A, 1)
    else:
        raise ValueError("uplo must be F, L or U")
    D = np.diag(np.real(np.diag(A))).astype(A.dtype)
    return T + T.conj().T + D


def _ordered(lam, res, emin, emax, rbinv2):
    """Permutation: found pairs (R-spur) ascending, then all others ascending.

    rbinv2: r^H B^-1 r per column, r = A x - lambda B x of the B-normalized Ritz
    vectors (||r||^2 for B = I).
    Returns (perm, M, n_inside) with n_inside the count of Ritz values in the
    interval regardless of their residual."""
    inside = (lam >= emin) & (lam <= emax)
    certified = rbinv2 < (emax - lam) * (lam - emin)
    found = inside & (res < SPURIOUS_RES) & certified
    idx_in = np.where(found)[0]
    idx_out = np.where(~found)[0]
    idx_in = idx_in[np.argsort(lam[idx_in], kind="stable")]
    idx_out = idx_out[np.argsort(lam[idx_out], kind="stable")]
    return np.concatenate([idx_in, idx_out]), int(idx_in.size), int(np.sum(inside))


def rayleigh_ritz(Q, A, B):
    """Reduced problem on span(Q) (Section 1.1; Table tab-rci1 Aq, Bq).

    Aq = Q^H A Q, Bq = Q^H B Q; solve Aq W = Bq W Lambda with the R-rank reading.
    Returns (lam, W, info) with lam unsorted as produced by the dense solver.
    """
    BQ = Q if B is None else B @ Q
    AQ = A @ Q
    S = Q.conj().T @ BQ
    T = Q.conj().T @ AQ
    S = 0.5 * (S + S.conj().T)
    T = 0.5 * (T + T.conj().T)
    sd = np.real(np.diag(S))
    if np.any(~(sd > 0)):
        return None, None, -3
    d = 1.0 / np.sqrt(sd)
    Sp = (d[:, None] * S) * d[None, :]
    Tp = (d[:, None] * T) * d[None, :]
    s, V = np.linalg.eigh(Sp)
    keep = s > RANK_TOL * s.max()
    if s.max() <= 0 or not np.any(keep):
        return None, None, -3
    G = V[:, keep] / np.sqrt(s[keep])[None, :]
    C = G.conj().T @ Tp @ G
    C = 0.5 * (C + C.conj().T)
    lam, Z = np.linalg.eigh(C)
    W = d[:, None] * (G @ Z)
    return lam, W, 0


def kato_temple_terms(R, b_solve=None):
    """r^H B^-1 r for every column r of R (R-spur); b_solve(R) = B^-1 R, None for B = I."""
    if b_solve is None:
        return np.sum(np.abs(R) ** 2, axis=0)
    return np.real(np.sum(np.conj(R) * b_solve(R), axis=0))


def _dense_b_solver(B):
    """B^-1 rhs by a Cholesky factorization of the positive definite B (library routine)."""
    if B is None:
        return None
    cf = sla.cho_factor(B, lower=True)
    return lambda rhs: sla.cho_solve(cf, rhs)


class _Factored:
    """LU factorization of Az = z B - A kept for reuse (fpm(10)=1)."""

    def __init__(self, z, A, B):
        n = A.shape[0]
        Bm = np.eye(n) if B is None else B
        self.lu = sla.lu_factor(z * Bm - A)

    def solve(self, rhs):
        return sla.lu_solve(self.lu, rhs, trans=0)

    def solve_h(self, rhs):
        # (z B - A)^H y = rhs with the same LU (case 21 of the Hermitian RCI)
        return sla.lu_solve(self.lu, rhs, trans=2)


def _contour_classic(facts, z, w, BY, real_problem, Y=None, c_inf=0.0):
    """Q = c_inf Y + sum_j [w_j (z_j B - A)^-1 BY + conj(w_j) (z_j B - A)^-H BY] in node
    order (c_inf: the constant term of the Zolotarev filter, else 0)."""
    n, m = BY.shape
    Q = np.zeros((n, m), dtype=np.float64 if real_problem else np.complex128)
    if c_inf != 0.0:
        Q += c_inf * Y
    for j in range(len(z)):
        Qj = facts[j].solve(BY.astype(np.complex128))
        if real_problem:
            # lower-half node is the complex conjugate for real A, B, Y
            Q += 2.0 * np.real(w[j] * Qj)
        else:
            Qt = facts[j].solve_h(BY.astype(np.complex128))
            Q += w[j] * Qj + np.conj(w[j]) * Qt
    return Q


def _contour_residual(facts, z, w, X, lam, R, real_problem, c_inf=0.0):
    """Residual form of the same contour sum (identity in the module docstring); the
    constant term c_inf acts on X exactly, so it only enters rho."""
    rho = rational_filter(lam, z, w) + c_inf
    Q = X * rho[None, :]
    Q = Q.astype(np.float64 if real_problem else np.complex128)
    for j in range(len(z)):
        dj = facts[j].solve(R.astype(np.complex128))
        cj = 1.0 / (z[j] - lam)
        if real_problem:
            Q += 2.0 * np.real(w[j] * dj * cj[None, :])
        else:
            ej = facts[j].solve_h(R.astype(np.complex128))
            ct = 1.0 / (np.conj(z[j]) - lam)
            Q += w[j] * dj * cj[None, :] + np.conj(w[j]) * ej * ct[None, :]
    return Q


def feast_dense(A, B, emin, emax, m0, fpm=None, X0=None, zne=None, wne=None,
                form="residual", uplo="F"):
    """Hermitian FEAST on dense A (and B; None means B = I).

    A, B: real symmetric or complex Hermitian (n x n), storage per ``uplo``.
    X0: n x m0 initial block, used when fpm(5) = 1.
    zne, wne: expert contour (nodes, half-contour weights); else built from fpm.
    form: "residual" (v4.0 residual inverse iteration) or "classic".
    Returns a dict with E, X, M, res, epsout, loop, info, m0, history; with
    fpm(14) = 1 it returns Q after one contour in X and info = 4.
    """
    fpm = feastinit() if fpm is None else np.asarray(fpm, dtype=np.int64)
    A = np.asarray(A)
    n = A.shape[0]
    info = validate(n, m0, emin, emax, fpm, have_expert_contour=zne is not None)
    if info:
        return _empty(info, m0)
    real_problem = not (np.iscomplexobj(A) or (B is not None and np.iscomplexobj(B)))
    dt = np.float64 if real_problem else np.complex128
    A = expand_uplo(A, uplo).astype(dt)
    if B is not None:
        B = expand_uplo(np.asarray(B), uplo).astype(dt)
    z, w, c_inf = _nodes(emin, emax, fpm, zne, wne)
    try:
        b_solve = _dense_b_solver(B)
    except np.linalg.LinAlgError:
        return _empty(-3, m0)  # Table tab_info -3: B may not be positive definite
    facts = [_Factored(zj, A, B) for zj in z]
    return iterate(A, B, n, real_problem, emin, emax, m0, fpm, X0, z, w, facts, form,
                   b_solve=b_solve, c_inf=c_inf)


def _empty(info, m0):
    return {"info": info, "E": None, "X": None, "M": 0, "res": None, "epsout": 1.0,
            "loop": 0, "m0": m0, "history": []}


def _nodes(emin, emax, fpm, zne, wne):
    """(z, w, c_inf): the rule of fpm(16) (Zolotarev with its constant term), or the
    caller's expert nodes and weights (no constant term)."""
    f = lambda i: int(fpm[i - 1])  # noqa: E731
    if zne is None:
        if f(16) == 2:
            return zolotarev_contour(emin, emax, f(2), f(54))
        z, w = half_contour(emin, emax, f(2), rule=f(16), ratio_pct=f(18))
        return z, w, 0.0
    return np.asarray(zne, np.complex128), np.asarray(wne, np.complex128), 0.0


def iterate(A, B, n, real_problem, emin, emax, m0, fpm, X0, z, w, solvers, form="residual",
            b_solve=None, c_inf=0.0):
    """The subspace iteration shared by the dense and the sparse drivers.

    A, B: objects supporting ``@`` with an n x m block (B None means identity).
    solvers[j]: object with solve(rhs) for (z_j B - A)^-1 rhs and, for complex
    Hermitian problems, solve_h(rhs) for (z_j B - A)^-H rhs.
    b_solve: B^-1 applied to a block (needed when B is given; R-spur).
    c_inf: constant term of the filter (Zolotarev rule), applied to the block itself.
    """
    if B is not None and b_solve is None:
        raise ValueError("a B^-1 solver is needed for the found-pair test when B is given")
    f = lambda i: int(fpm[i - 1])  # noqa: E731
    dt = np.float64 if real_problem else np.complex128
    out = _empty(0, m0)
    alpha = max(abs(emin), abs(emax))
    eps = 10.0 ** (-f(3))
    if f(5) == 1:
        Y = np.asarray(X0, dtype=dt)[:, :m0].copy()
    else:
        Y = initial_subspace(n, m0, f(51), not real_problem).astype(dt)
    facts = solvers

    trace_prev = None
    X = Y
    lam_sorted = None
    k = 0
    while True:
        if k == 0 or form == "classic":
            BY = X if B is None else B @ X
            Q = _contour_classic(facts, z, w, BY, real_problem, Y=X, c_inf=c_inf)
        else:
            BX = X if B is None else B @ X
            R = A @ X - BX * lam_sorted[None, :]
            Q = _contour_residual(facts, z, w, X, lam_sorted, R, real_problem, c_inf=c_inf)
        if f(14) == 1:
            out.update(info=4, X=Q, loop=0, m0=Q.shape[1])
            return out
        lam, W, rinfo = rayleigh_ritz(Q, A, B)
        if rinfo:
            out.update(info=rinfo, loop=k)
            return out
        X = Q @ W
        BX = X if B is None else B @ X
        R = A @ X - BX * lam[None, :]
        res = np.linalg.norm(R, axis=0) / (alpha * np.linalg.norm(BX, axis=0))
        perm, M, n_inside = _ordered(lam, res, emin, emax, kato_temple_terms(R, b_solve))
        lam_sorted, X, res = lam[perm], X[:, perm], res[perm]
        trace = float(np.sum(lam_sorted[:M]))
        epsout = 1.0 if trace_prev is None else abs(trace - trace_prev) / alpha
        trace_prev = trace
        maxres = float(np.max(res[:M])) if M > 0 else 0.0
        out["history"].append({"it": k, "M": M, "trace": trace, "epsout": epsout,
                               "maxres": maxres, "m0": X.shape[1], "E": lam_sorted[:M].copy()})
        out.update(E=lam_sorted, X=X, M=M, res=res, epsout=epsout, loop=k, m0=X.shape[1])
        if n_inside == 0:
            out["info"] = 1
            return out
        if n_inside >= X.shape[1]:
            out["info"] = 3
            return out
        converged = M > 0 and ((maxres < eps) if f(6) == 1 else (epsout < eps))
        if converged:
            out["info"] = 0
            return out
        if k >= f(4):
            out["info"] = 2
            return out
        k += 1
