"""Comparison helpers for GPU-versus-oracle parity (test code only)."""

import numpy as np


def clusters(lam, tol):
    """Maximal runs of sorted values whose neighbour gaps are below tol."""
    if len(lam) == 0:
        return []
    groups, cur = [], [0]
    for i in range(1, len(lam)):
        if lam[i] - lam[i - 1] < tol:
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    groups.append(cur)
    return groups


def subspace_sin(X, Y, B=None):
    """sin of the largest principal angle between span(X) and span(Y) (B-inner product)."""
    if B is not None:
        L = np.linalg.cholesky(B)
        X = L.conj().T @ X
        Y = L.conj().T @ Y
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    return float(np.linalg.norm(qx - qy @ (qy.conj().T @ qx), 2))


def compare_eigenpairs(E, X, Eref, Xref, M, emin, emax, B=None, eig_tol=1e-10, angle_tol=1e-8):
    """Parity bar: equal count, |dE| <= eig_tol * max(|E|, alpha), cluster angles <= angle_tol."""
    alpha = max(abs(emin), abs(emax))
    E = np.asarray(E)[:M]
    Eref = np.asarray(Eref)[:M]
    scale = np.maximum(np.abs(Eref), alpha)
    eig_err = float(np.max(np.abs(E - Eref) / scale)) if M else 0.0
    assert eig_err <= eig_tol, ("eigenvalue error", eig_err)
    worst = 0.0
    for g in clusters(Eref, 1e-4 * alpha):
        worst = max(worst, subspace_sin(np.asarray(X)[:, g], np.asarray(Xref)[:, g], B))
    assert worst <= angle_tol, ("subspace angle", worst)
    return eig_err, worst
