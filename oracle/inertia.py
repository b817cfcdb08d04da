"""Number of eigenvalues of the pencil (A, B) below gamma.  Test infrastructure.

Sylvester's law of inertia: with B symmetric positive definite, A - gamma B is
congruent to B^{-1/2} A B^{-1/2} - gamma I, so the number of negative pivots of
any symmetric LDL^T factorisation of A - gamma B equals #{lambda_i < gamma}.
The paper's problem (Section 1) asks for every eigenvalue in (0, gamma]; with A
positive definite that is this count whenever gamma is not an eigenvalue.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as sla


def sturm_count_tridiagonal(A, B, gamma: float) -> int:
    """LDL^T of the tridiagonal A - gamma B (Sturm sequence): d_1 = m_11,
    d_i = m_ii - m_{i,i-1}^2 / d_{i-1}; returns the number of d_i < 0."""
    M = (A - gamma * B).tocsr()
    diag = M.diagonal()
    sub = M.diagonal(-1)
    count = 0
    d = diag[0]
    count += d < 0
    for i in range(1, len(diag)):
        d = diag[i] - sub[i - 1] * sub[i - 1] / d
        count += d < 0
    return int(count)


def dense_ldl_count(A, B, gamma: float) -> int:
    """Unpivoted dense LDL^T of A - gamma B, counting negative pivots (small n)."""
    M = (A - gamma * B).toarray() if hasattr(A, "toarray") else np.array(A - gamma * B)
    n = M.shape[0]
    count = 0
    for k in range(n):
        d = M[k, k]
        count += d < 0
        l = M[k + 1:, k] / d
        M[k + 1:, k + 1:] -= np.outer(l, M[k, k + 1:])
    return int(count)


def sparse_ldl_count(A, B, gamma: float) -> int:
    """Negative pivots of a symmetric sparse factorisation of A - gamma B.

    SuperLU with diagonal pivoting only (diag_pivot_thresh = 0, SymmetricMode)
    and a symmetric fill-reducing ordering computes P M P^T = L U with
    U = D L^T, so sign(diag U) gives the inertia.  The symmetric permutation is
    verified (perm_r == perm_c).
    """
    M = (A - gamma * B).tocsc()
    lu = sla.splu(M, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                  options=dict(SymmetricMode=True))
    if not np.array_equal(lu.perm_r, lu.perm_c):
        raise RuntimeError("SuperLU used a non-symmetric pivot order")
    d = lu.U.diagonal()
    if not np.all(np.isfinite(d)) or np.any(d == 0):
        raise RuntimeError("zero or non-finite pivot: gamma too close to an eigenvalue")
    return int((d < 0).sum())
