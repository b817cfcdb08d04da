"""All eigenpairs of a tiny pencil (A, B).  Test infrastructure.

The plain definition of what the method computes (Section 1): every eigenpair
of A x = lambda B x with lambda in (0, gamma], eigenvectors B-normalised.
Cholesky reduction: B = G G^T, C = G^{-1} A G^{-T}, C = Y diag(lambda) Y^T,
X = G^{-T} Y (then X^T B X = I).  The dense symmetric eigensolver is the library
primitive used for the middle step.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def all_eigenpairs(A, B):
    """Ascending eigenvalues and B-orthonormal eigenvectors of a small pencil."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A, dtype=np.float64)
    Bd = B.toarray() if hasattr(B, "toarray") else np.asarray(B, dtype=np.float64)
    G = np.linalg.cholesky(Bd)
    Ginv = sla.solve_triangular(G, np.eye(G.shape[0]), lower=True)
    C = Ginv @ Ad @ Ginv.T
    C = 0.5 * (C + C.T)
    lam, Y = np.linalg.eigh(C)
    X = Ginv.T @ Y
    return lam, X


def interval_eigenpairs(A, B, gamma: float):
    """Eigenpairs with lambda in (0, gamma]."""
    lam, X = all_eigenpairs(A, B)
    sel = (lam > 0) & (lam <= gamma)
    return lam[sel], X[:, sel]
