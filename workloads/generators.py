"""Seeded synthetic matrices for the FEAST workloads (no FEAST arithmetic here).

All generation runs in FP64 on the host with ``numpy.random.default_rng``.
Draw order per workload is fixed so that a seed names one input exactly.
"""

import numpy as np


def column_major(M):
    """Fortran-ordered copy: element (i, j) at i + j * n, as the C interface expects."""
    return np.asfortranarray(M)


def helloworld():
    """4 x 4 real symmetric matrix of the guide's HelloWorld example (Section 2.4)."""
    return np.array([[2.0, -1.0, -1.0, 0.0],
                     [-1.0, 3.0, -1.0, -1.0],
                     [-1.0, -1.0, 3.0, -1.0],
                     [0.0, -1.0, -1.0, 2.0]])


def laplacian_1d_dense(n, diag_shift=None):
    """Dense tridiag(-1, 2, -1) of order n; optional diagonal added (vector of length n)."""
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    if diag_shift is not None:
        A = A + np.diag(np.asarray(diag_shift, dtype=np.float64))
    return A


def laplacian_1d_eigs(n):
    """Eigenvalues 2 - 2 cos(k pi / (n + 1)), k = 1..n, ascending (closed form)."""
    k = np.arange(1, n + 1, dtype=np.float64)
    return np.sort(2.0 - 2.0 * np.cos(k * np.pi / (n + 1)))


def _haar_unitary(rng, n, complex_):
    """Haar-distributed orthogonal/unitary matrix: QR of a Gaussian with R-diagonal phase fix."""
    if complex_:
        Z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    else:
        Z = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    ph = d / np.abs(d)
    return Q * ph[None, :]


def prescribed_complex_pencil(n, seed, lam_lo=-10.0, lam_hi=10.0, b_scale=0.1):
    """Generalized complex Hermitian pencil with a known spectrum.

    Draw order from default_rng(seed): lambda ~ U[lam_lo, lam_hi]^n, then C (complex
    Gaussian n x n), then the Haar unitary U.  B = I + b_scale * C C^H / n,
    L = chol(B), A = L U diag(lambda) U^H L^H symmetrised.  Exact eigenvectors are
    X = L^-H U (B-orthonormal).  Returns (A, B, lam_sorted, X_sorted).
    """
    rng = np.random.default_rng(seed)
    lam = rng.uniform(lam_lo, lam_hi, n)
    C = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    U = _haar_unitary(rng, n, True)
    B = np.eye(n, dtype=np.complex128) + b_scale * (C @ C.conj().T) / n
    B = 0.5 * (B + B.conj().T)
    L = np.linalg.cholesky(B)
    LU = L @ U
    A = (LU * lam[None, :]) @ LU.conj().T
    A = 0.5 * (A + A.conj().T)
    order = np.argsort(lam)
    X = np.linalg.solve(L.conj().T, U)
    return A, B, lam[order], X[:, order]


def prescribed_real_problem(n, rng, lam_lo=-10.0, lam_hi=10.0):
    """Real symmetric A = U diag(lambda) U^T with Haar-orthogonal U (draws: lambda, U)."""
    lam = rng.uniform(lam_lo, lam_hi, n)
    U = _haar_unitary(rng, n, False)
    A = (U * lam[None, :]) @ U.T
    A = 0.5 * (A + A.T)
    order = np.argsort(lam)
    return A, lam[order], U[:, order]


def batched_real_problems(nprob, seed, n_lo=256, n_hi=2048, c_lo=24, c_hi=48):
    """Independent real symmetric problems of uneven size, each with a known interval.

    Draw order from default_rng(seed): all sizes n_p ~ U{n_lo..n_hi} first; then per
    problem lambda, U (see prescribed_real_problem), the count c_p ~ U{c_lo..c_hi}
    and the start index s_p ~ U{1..n_p - c_p - 1} in the sorted spectrum.  The interval
    edges are midpoints between sorted neighbours, so it holds exactly c_p
    eigenvalues; M0_p = ceil(1.5 c_p).
    Returns a list of dicts with A, lam (sorted), emin, emax, count, m0.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=nprob)
    probs = []
    for p in range(nprob):
        n = int(ns[p])
        A, lam, U = prescribed_real_problem(n, rng)
        c = int(rng.integers(c_lo, c_hi + 1))
        s = int(rng.integers(1, n - c))
        emin = 0.5 * (lam[s - 1] + lam[s])
        emax = 0.5 * (lam[s + c - 1] + lam[s + c])
        probs.append({"A": A, "lam": lam, "U": U, "emin": emin, "emax": emax,
                      "count": c, "m0": int(np.ceil(1.5 * c)), "start": s})
    return probs


def laplacian_3d_csr(nx, ny=None, nz=None):
    """7-point Laplacian (6 on the diagonal, -1 to each grid neighbour, Dirichlet) on an
    nx x ny x nz grid, natural ordering i + nx (j + ny k); CSR arrays (0-based):
    (values float64, column indices int32, row pointers int32), full storage."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    idx = np.arange(n)
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    rows, cols, vals = [idx], [idx], [np.full(n, 6.0)]
    for di, dj, dk, stride in ((1, 0, 0, 1), (0, 1, 0, nx), (0, 0, 1, nx * ny)):
        ok_p = (i + di < nx) & (j + dj < ny) & (k + dk < nz)
        rows += [idx[ok_p], idx[ok_p] + stride]
        cols += [idx[ok_p] + stride, idx[ok_p]]
        vals += [np.full(int(ok_p.sum()), -1.0)] * 2
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, r + 1, 1)
    indptr = np.cumsum(indptr)
    return v.astype(np.float64), c.astype(np.int32), indptr.astype(np.int32)


def laplacian_3d_eigs(nx, ny=None, nz=None):
    """All eigenvalues sum_d 2 - 2 cos(k_d pi / (n_d + 1)), ascending (closed form)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    ex = 2.0 - 2.0 * np.cos(np.arange(1, nx + 1) * np.pi / (nx + 1))
    ey = 2.0 - 2.0 * np.cos(np.arange(1, ny + 1) * np.pi / (ny + 1))
    ez = 2.0 - 2.0 * np.cos(np.arange(1, nz + 1) * np.pi / (nz + 1))
    return np.sort((ex[:, None, None] + ey[None, :, None] + ez[None, None, :]).ravel())


def differentiation_problem(n=4096, seed=3):
    """Tridiagonal A = tridiag(-1, 2 + v, -1) and loss weights for the differentiation
    workload.  Draw order from default_rng(seed): v ~ U[0, 1]^n, then c ~ N(0, 1)^n.
    Returns (v, c, A dense float64)."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.0, 1.0, n)
    c = rng.standard_normal(n)
    A = 2.0 * np.eye(n) + np.diag(v) - np.eye(n, k=1) - np.eye(n, k=-1)
    return v, c, A


def prescribed_nonnormal(n, seed, generalized=False, spread=2.0, coupling=0.3):
    """Complex general matrix (pencil) with a known spectrum and known eigenvectors.

    Draw order from default_rng(seed): lambda (real parts, then imaginary parts, each
    U[-spread, spread]), then G (complex Gaussian n x n) for V = I + coupling G / sqrt(n),
    then, for a pencil, C (complex Gaussian n x n) for B = I + 0.1 C C^H / n.
    A = B V diag(lambda) V^-1 (B = I for the standard problem), so the right
    eigenvectors are the columns of V and the left ones, y_i^H A = lambda_i y_i^H B, the
    columns of Y = (V^-1 B^-1)^H.  Returns (A, B or None, lambda, V, Y)."""
    rng = np.random.default_rng(seed)
    lam = rng.uniform(-spread, spread, n) + 1j * rng.uniform(-spread, spread, n)
    G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    V = np.eye(n) + coupling * G / np.sqrt(n)
    Vinv = np.linalg.inv(V)
    if generalized:
        C = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
        B = np.eye(n) + 0.1 * (C @ C.conj().T) / n
        B = 0.5 * (B + B.conj().T)
    else:
        B = None
    K = (V * lam[None, :]) @ Vinv
    A = K if B is None else B @ K
    Binv = np.eye(n) if B is None else np.linalg.inv(B)
    Y = (Vinv @ Binv).conj().T
    return A, B, lam, V, Y


def prescribed_polynomial(n, p, seed, leading=False, spread=2.0, coupling=0.3, vectors=True):
    """Matrix polynomial sum_k lambda^k A_k (k = 0..p) with known eigenpairs.

    Draw order from default_rng(seed): for t = 1..p the spectrum D_t (real parts, then
    imaginary parts, each U[-spread, spread]) and G_t for V_t = I + coupling G_t / sqrt(n);
    then, with leading=True, C for L = I + 0.1 C C^H / n.  With S_t = V_t diag(D_t) V_t^-1,
    P(lambda) = L (lambda I - S_p) ... (lambda I - S_1), expanded into the coefficients A_k
    of lambda^k (L = I without leading).  Its eigenvalues are those of every S_t; for
    lambda in eig(S_t) with eigenvector v of S_t, the right eigenvector is
    x = (lambda I - S_1)^-1 ... (lambda I - S_(t-1))^-1 v.
    Returns (As, lam (p n values, S_1's first), X (n x p n, unit columns; None with
    vectors=False, which skips the n (p - 1) solves of large problems))."""
    rng = np.random.default_rng(seed)
    S, D, Vs = [], [], []
    for t in range(p):
        d = rng.uniform(-spread, spread, n) + 1j * rng.uniform(-spread, spread, n)
        G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
        V = np.eye(n) + coupling * G / np.sqrt(n)
        S.append((V * d[None, :]) @ np.linalg.inv(V))
        D.append(d)
        Vs.append(V)
    L = np.eye(n, dtype=np.complex128)
    if leading:
        C = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
        L = np.eye(n) + 0.1 * (C @ C.conj().T) / n
    # coefficients of (lambda - S_p) ... (lambda - S_1), lowest degree first
    coef = [np.eye(n, dtype=np.complex128)]
    for t in range(p):
        new = [np.zeros((n, n), dtype=np.complex128) for _ in range(len(coef) + 1)]
        for k, Ck in enumerate(coef):
            new[k + 1] += Ck
            new[k] -= S[t] @ Ck
        coef = new
    As = [L @ Ck for Ck in coef]
    if not vectors:
        return As, np.concatenate(D), None
    lam, X = [], []
    for t in range(p):
        for i in range(n):
            x = Vs[t][:, i].astype(np.complex128)
            for u in range(t - 1, -1, -1):
                x = np.linalg.solve(D[t][i] * np.eye(n) - S[u], x)
            lam.append(D[t][i])
            X.append(x / np.linalg.norm(x))
    return As, np.array(lam), np.stack(X, axis=1)
