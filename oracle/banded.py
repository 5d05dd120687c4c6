"""Textbook banded Cholesky and band solves (oracle).

The paper factors each local matrix once and reuses the factor for all
2|I^l|+1 right-hand sides (Sec. 2.2.3, "LocalSolver"; it uses a sparse LDL^T).
For an SPD matrix with lower bandwidth b the Cholesky factor L has the same
bandwidth, and is unique, so a band factor computed anywhere can be compared
entry by entry with this one (in the same row ordering).

Band storage here is "by column": ``Lb[j, t] = L[j + t, j]`` for
``t = 0..b`` (zero beyond the matrix).
"""
from __future__ import annotations

import numpy as np


def to_band(M, b):
    """Lower band of a dense or sparse symmetric matrix, by column."""
    M = M.toarray() if hasattr(M, "toarray") else np.asarray(M)
    n = M.shape[0]
    Lb = np.zeros((n, b + 1))
    for t in range(b + 1):
        Lb[: n - t, t] = np.diagonal(M, -t)
    return Lb


def band_cholesky(Ab):
    """Right-looking Cholesky on band storage: for each column j, take the
    square root of the pivot, scale the column, and subtract the outer product
    from the (b x b) trailing triangle.  Raises on a non-positive pivot."""
    A = np.array(Ab, dtype=np.float64, copy=True)
    n, bp1 = A.shape
    b = bp1 - 1
    for j in range(n):
        piv = A[j, 0]
        if not piv > 0.0:
            raise np.linalg.LinAlgError(f"non-positive pivot {piv} at column {j}")
        d = np.sqrt(piv)
        A[j, 0] = d
        w = min(b, n - 1 - j)
        A[j, 1:w + 1] /= d
        col = A[j, 1:w + 1]  # L[j+1 .. j+w, j]
        for t in range(1, w + 1):
            # column j+t, rows j+t .. j+w: subtract L[i,j] L[j+t,j]
            A[j + t, 0:w + 1 - t] -= col[t - 1:w] * col[t - 1]
    return A


def band_solve(Lb, B):
    """Solve L L^T X = B with the band factor (forward then backward)."""
    n, bp1 = Lb.shape
    b = bp1 - 1
    X = np.array(B, dtype=np.float64, copy=True)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    for j in range(n):
        X[j] /= Lb[j, 0]
        w = min(b, n - 1 - j)
        X[j + 1:j + 1 + w] -= np.outer(Lb[j, 1:w + 1], X[j])
    for j in range(n - 1, -1, -1):
        w = min(b, n - 1 - j)
        X[j] -= Lb[j, 1:w + 1] @ X[j + 1:j + 1 + w]
        X[j] /= Lb[j, 0]
    return X[:, 0] if squeeze else X


def bandwidth(M):
    """Largest |i - j| over the nonzeros of M."""
    C = M.tocoo()
    return int(np.max(np.abs(C.row - C.col))) if C.nnz else 0
