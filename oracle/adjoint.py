"""Gradient of a loss on the eigenpairs inside [Emin, Emax] with respect to A (oracle).

Test infrastructure only (see the package docstring).

Real symmetric A, B = I.  S is the set of eigenpairs (lambda_i, x_i) with lambda_i in
the interval, x_i of unit norm.  For a loss L(lambda_S, X_S) with gradients
g_i = dL/dlambda_i and G_i = dL/dx_i, first-order perturbation of a symmetric
eigenproblem (A -> A + E) gives
    d lambda_i = x_i^T E x_i,
    d x_i      = sum_{j != i} x_j (x_j^T E x_i) / (lambda_i - lambda_j).
When the loss is invariant under rotations inside span(X_S) (for instance
sum_i lambda_i + sum_i x_i^T C x_i with C symmetric), the terms with j in S cancel
pairwise and
    dL/dA = sum_{i in S} [ g_i x_i x_i^T + (x_i y_i^T + y_i x_i^T) / 2 ],
    y_i   = sum_{j not in S} x_j (x_j^T G_i) / (lambda_i - lambda_j).
y_i is also the unique solution orthogonal to span(X_S) of
    (lambda_i I - A + sigma X_S X_S^T) y_i = (I - X_S X_S^T) G_i,
for any sigma with sigma != lambda_j - lambda_i (j in S): the deflated shifted solve
that the HIP path performs.  Two functions below compute dL/dA both ways:
``grad_by_eigensum`` (the explicit sum over a dense eigendecomposition, the
definition) and ``grad_by_solves`` (the deflated solves with a library LU).
"""

import numpy as np
import scipy.linalg as sla


def interval_pairs(A, emin, emax):
    """All eigenpairs of symmetric A (numpy eigh) and the boolean mask of S."""
    lam, V = np.linalg.eigh(A)
    inside = (lam >= emin) & (lam <= emax)
    return lam, V, inside


def grad_by_eigensum(lam, V, inside, g, G):
    """dL/dA from the full eigendecomposition (lam, V); g: (M,), G: (n, M) for the
    pairs of S in ascending order."""
    XS = V[:, inside]
    lS = lam[inside]
    Xo = V[:, ~inside]
    lo = lam[~inside]
    Y = np.zeros_like(XS)
    for i in range(XS.shape[1]):
        coef = (Xo.T @ G[:, i]) / (lS[i] - lo)
        Y[:, i] = Xo @ coef
    gA = (XS * g[None, :]) @ XS.T + 0.5 * (XS @ Y.T + Y @ XS.T)
    return gA, Y


def grad_by_solves(A, lamS, XS, g, G, sigma=None):
    """dL/dA from the deflated shifted solves, one scipy LU per eigenvalue of S."""
    n, M = XS.shape
    if sigma is None:
        sigma = np.abs(A).sum(axis=0).max()  # ||A||_1 exceeds every |lambda_j - lambda_i|
    P = XS @ XS.T
    Y = np.zeros_like(XS)
    for i in range(M):
        K = lamS[i] * np.eye(n) - A + sigma * P
        rhs = G[:, i] - XS @ (XS.T @ G[:, i])
        Y[:, i] = sla.lu_solve(sla.lu_factor(K), rhs)
    gA = (XS * g[None, :]) @ XS.T + 0.5 * (XS @ Y.T + Y @ XS.T)
    return gA, Y


# ----------------------------------------------------------------------------
# the differentiation workload: A = tridiag(-1, 2 + v, -1), L = sum lambda_i + sum_i sum_k c_k x_ik^2
# ----------------------------------------------------------------------------

def tridiag_dense(v):
    n = v.size
    return np.diag(2.0 + v) - np.eye(n, k=1) - np.eye(n, k=-1)


def loss_and_grad_v(v, c, emin, emax):
    """Loss and dL/dv for the workload (dense eigendecomposition, explicit sum).
    dL/dv = diag(dL/dA) since dA/dv_k = e_k e_k^T."""
    A = tridiag_dense(v)
    lam, V, inside = interval_pairs(A, emin, emax)
    XS = V[:, inside]
    L = lam[inside].sum() + float(np.sum(c[:, None] * XS ** 2))
    g = np.ones(XS.shape[1])
    G = 2.0 * c[:, None] * XS
    gA, _ = grad_by_eigensum(lam, V, inside, g, G)
    return L, np.diag(gA).copy(), lam[inside], XS
