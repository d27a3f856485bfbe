"""IFEAST (FEAST without factorization) for sparse CSR matrices (oracle).

Test infrastructure only (see the package docstring).

The guide's Section 3.5 (IFEAST) replaces the sparse direct solver of the FEAST
sparse drivers by a built-in BiCGStab that solves every shifted system only to the
accuracy 10^-fpm(45) within fpm(46) iterations, reports the total number of
BiCGStab iterations in fpm(60), and uses its own defaults: 4 half-contour nodes,
trapezoidal rule, circle (Table tab_fpm).  The subspace iteration itself is the
one of the dense drivers (oracle.feast.iterate); only the solver changes.

BiCGSTAB follows van der Vorst (SIAM J. Sci. Stat. Comput. 13, 1992) for each
column independently, in complex128, with x0 = 0 and shadow residual r_hat = r0 = b,
inner product <a, b> = a^H b.
Readings where the guide is silent:
  R-bicg-stop   a column stops when ||r|| <= 10^-fpm(45) ||b|| (also checked on the
                half step s) or after fpm(46) iterations.
  R-bicg-break  a column whose rho, omega or r_hat^H v vanishes exactly stops where
                it is (no restart); the subspace iteration tolerates inexact solves.
  R-fpm60       fpm(60) is the sum over loops and nodes of the iterations one node's
                block needed (the largest count among its columns), as in the
                guide's IFEAST example output (4+3+2+2+...+1 = 31).
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .feast import _empty, _nodes, feastinit, iterate, validate


def ifeastinit():
    """IFEAST defaults of Table tab_fpm: 4 nodes, trapezoidal, circle, 50 loops."""
    fpm = feastinit()
    fpm[1] = 4      # fpm(2)
    fpm[3] = 50     # fpm(4)
    fpm[15] = 1     # fpm(16)
    fpm[17] = 100   # fpm(18)
    return fpm


def bicgstab(op, b, tol, maxit):
    """One column of op(x) = b by BiCGSTAB.  Returns (x, iterations used)."""
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0
    r = b.copy()
    r_hat = b.copy()
    rho = alpha = omega = 1.0 + 0.0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    for it in range(1, maxit + 1):
        rho_new = np.vdot(r_hat, r)
        if rho_new == 0 or omega == 0:
            return x, it - 1                    # R-bicg-break
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = op(p)
        den = np.vdot(r_hat, v)
        if den == 0:
            return x, it
        alpha = rho_new / den
        s = r - alpha * v
        if np.linalg.norm(s) <= tol * bnorm:
            return x + alpha * p, it
        t = op(s)
        tt = np.vdot(t, t)
        omega = np.vdot(t, s) / tt if tt != 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        if np.linalg.norm(r) <= tol * bnorm:
            return x, it
    return x, maxit


def bicgstab_block(op, b, tol, maxit):
    """Every column of b (n x m) solved on its own; returns x and the per-column counts."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    its = np.zeros(b.shape[1], dtype=np.int64)
    for c in range(b.shape[1]):
        x[:, c], its[c] = bicgstab(op, b[:, c], tol, maxit)
    return x, its


class _ShiftedBiCG:
    """(z B - A)^-1 rhs by BiCGSTAB; real symmetric A, B: the conjugate node is the
    complex conjugate, so no solve with the conjugate transpose is needed."""

    def __init__(self, z, A, B, tol, maxit, counter):
        self.z, self.A, self.B, self.tol, self.maxit = z, A, B, tol, maxit
        self.counter = counter

    def op(self, v):
        Bv = v if self.B is None else self.B @ v
        return self.z * Bv - self.A @ v

    def solve(self, rhs):
        x, its = bicgstab_block(self.op, rhs.astype(np.complex128), self.tol, self.maxit)
        self.counter[0] += int(its.max()) if its.size else 0
        return x


def feast_csr(A, B, emin, emax, m0, fpm=None, X0=None, zne=None, wne=None, form="residual"):
    """IFEAST on a real symmetric sparse A (scipy.sparse; full storage) and B (or None).

    Returns the dict of oracle.feast.iterate plus "fpm60", the total BiCGSTAB count.
    """
    fpm = ifeastinit() if fpm is None else np.asarray(fpm, dtype=np.int64)
    f = lambda i: int(fpm[i - 1])  # noqa: E731
    A = sp.csr_matrix(A, dtype=np.float64)
    n = A.shape[0]
    info = validate(n, m0, emin, emax, fpm, have_expert_contour=zne is not None)
    if info:
        return _empty(info, m0)
    Bm = None if B is None else sp.csr_matrix(B, dtype=np.float64)
    z, w, c_inf = _nodes(emin, emax, fpm, zne, wne)
    counter = [0]
    tol = 10.0 ** (-f(45))
    solvers = [_ShiftedBiCG(zj, A, Bm, tol, f(46), counter) for zj in z]
    b_solve = None
    if Bm is not None:
        try:
            lu = spla.splu(Bm.tocsc())
        except RuntimeError:
            return _empty(-3, m0)  # B singular (Table tab_info -3)
        b_solve = lambda rhs: lu.solve(np.asarray(rhs, dtype=np.float64))  # noqa: E731
    out = iterate(A, Bm, n, True, emin, emax, m0, fpm, X0, z, w, solvers, form, b_solve=b_solve, c_inf=c_inf)
    out["fpm60"] = counter[0]
    return out
