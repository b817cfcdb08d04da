"""Rational filter application with exact solves.  Test infrastructure.

Paper Section 3: applying Phi(A, B) = sum_j w_j (A - sigma_j B)^{-1} B to a
vector multiplies its component along eigenvector x_i by Phi(lambda_i).  With
conjugate pairs (sigma_{N+j} = conj(sigma_j), w_{N+j} = conj(w_j)) only the N
upper-half-plane systems are solved and the filtered block is
U = sum_j 2 Re(w_j Y_j), Y_j = (A - sigma_j B)^{-1} B V   (Algorithm 1).

The shifted systems are solved exactly by a sparse LU factorisation (the setting
of the paper's Figure 3 experiment, "complete LU factorization"); SuperLU is the
library primitive used for that step.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla


def shifted_solve(A, B, sigma: complex, F: np.ndarray) -> np.ndarray:
    """Y = (A - sigma B)^{-1} F, complex128, exact (sparse LU)."""
    S = (A.astype(np.complex128) - sigma * B.astype(np.complex128)).tocsc()
    lu = sla.splu(S)
    F = np.asarray(F, dtype=np.complex128)
    return lu.solve(F)


def filter_apply(A, B, X: np.ndarray, sigma, w):
    """U = sum_j 2 Re(w_j (A - sigma_j B)^{-1} B X)  (Algorithm 1).

    Returns (U, [Y_j]).  X is (n, L) float64.
    """
    F = B @ X
    U = np.zeros(X.shape, dtype=np.float64)
    Ys = []
    for sj, wj in zip(sigma, w):
        Y = shifted_solve(A, B, complex(sj), F)
        Ys.append(Y)
        U += 2.0 * np.real(wj * Y)
    return U, Ys
