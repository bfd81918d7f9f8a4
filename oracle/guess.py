"""Start-vector estimators of Sec. IV, FP64 reference (test infrastructure only).

* ``mgs`` - eq. (4): modified Gram-Schmidt turns the last n (possibly linearly
  dependent) solutions into m <= n orthonormal columns V.
* ``galerkin_start`` - eq. (5): x0 = V (V^T M V)^{-1} V^T b, the small m x m
  system solved directly on the host.
* ``pod_basis`` - the POD variant: the snapshot matrix is decomposed by an SVD
  and the m left singular vectors with the largest singular values are kept.
* ``pod_from_gram`` - the same basis from the eigen-decomposition of the Gram
  matrix S^T S (the route a GPU takes with one pass over the snapshots):
  S^T S = U diag(sigma^2) U^T  =>  V = S U diag(1/sigma).
"""

from __future__ import annotations

import numpy as np


def mgs(X, drop_tol: float = 1e-10):
    """Eq. (4): orthonormalise the columns of X by modified Gram-Schmidt.

    A column whose remaining norm falls below drop_tol times its original norm
    is treated as linearly dependent and dropped."""
    X = np.asarray(X, dtype=np.float64)
    cols = []
    for j in range(X.shape[1]):
        v = X[:, j].copy()
        n0 = np.linalg.norm(v)
        if n0 == 0.0:
            continue
        for q in cols:
            v -= (q @ v) * q
        nv = np.linalg.norm(v)
        if nv <= drop_tol * n0:
            continue
        cols.append(v / nv)
    return np.stack(cols, axis=1) if cols else np.zeros((X.shape[0], 0))


def galerkin_start(V, M, b):
    """Eq. (5): x0 = V (V^T M V)^{-1} V^T b."""
    MV = M @ V
    G = V.T @ MV
    c = np.linalg.solve(G, V.T @ b)
    return V @ c


def pod_basis(S, m: int, rel_tol: float = 1e-12):
    """POD: the m dominant left singular vectors of the snapshot matrix S
    (columns with sigma_k <= rel_tol * sigma_1 are dropped)."""
    U, sig, _ = np.linalg.svd(np.asarray(S, dtype=np.float64), full_matrices=False)
    keep = min(m, int((sig > rel_tol * sig[0]).sum())) if sig.size and sig[0] > 0 else 0
    return U[:, :keep], sig[:keep]


def pod_from_gram(S, m: int, rel_tol: float = 1e-7):
    """The POD basis from the Gram matrix: G = S^T S = W diag(lam) W^T,
    V = S W diag(lam^{-1/2}) for the m largest eigenvalues lam = sigma^2.
    Eigenvalues of G are resolved to ~1e-16 of the largest, so singular values
    below ~1e-7 of the largest are dropped. Returns (V, sigma, W_kept)."""
    S = np.asarray(S, dtype=np.float64)
    G = S.T @ S
    lam, W = np.linalg.eigh(G)
    order = np.argsort(lam)[::-1]
    lam, W = lam[order], W[:, order]
    sig = np.sqrt(np.clip(lam, 0.0, None))
    keep = min(m, int((sig > rel_tol * sig[0]).sum())) if sig.size and sig[0] > 0 else 0
    W = W[:, :keep]
    sig = sig[:keep]
    return S @ (W / sig), sig, W
