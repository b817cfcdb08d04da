"""Algorithm 1 of the paper (rational filter subspace iteration), FP64, exact
shifted solves.  Test infrastructure.

Per outer iteration k:
  1. Y_j = (A - sigma_j B)^{-1} B V_k for j = 1..N        (sparse LU, cached)
  2. U = sum_j 2 Re(w_j Y_j)
  3. Rayleigh-Ritz on span(U): the paper forms U^T A U and U^T B U and solves the
     projected pencil.  Reading: U is first B-orthonormalised (modified
     Gram-Schmidt in the B inner product, two passes), so the projected pencil
     is (Q^T A Q, I) -- the same subspace, hence the same Ritz pairs in exact
     arithmetic, without forming an ill-conditioned U^T B U.
  4. theta ascending, x_i = Q s_i
  5. rho_i = ||A x_i - theta_i B x_i||_2 / (|theta_i| ||B x_i||_2)
  6. V_{k+1} = [x_1 .. x_L]
Stopping (reading of the paper's test, restricted to the wanted interval): every
Ritz value in (0, gamma] has rho_i <= tol, and the number of Ritz values in
(0, gamma] is the same as in the previous iteration and smaller than L.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as sla


def relative_residuals(A, B, X, theta):
    """rho_i = ||A x_i - theta_i B x_i|| / (|theta_i| ||B x_i||)  (Algorithm 1)."""
    AX = A @ X
    BX = B @ X
    R = AX - BX * theta[None, :]
    return np.linalg.norm(R, axis=0) / (np.abs(theta) * np.linalg.norm(BX, axis=0))


def mgs_b(U, B, drop: float = 1e-13):
    """Modified Gram-Schmidt in the B inner product, applied twice.

    Raises if a column's B-norm after projection falls below ``drop`` times its
    norm before (numerically dependent filtered block)."""
    Q = np.array(U, dtype=np.float64, copy=True)
    n, L = Q.shape
    for _ in range(2):
        for i in range(L):
            q = Q[:, i]
            before = np.sqrt(q @ (B @ q))
            for j in range(i):
                q = q - (Q[:, j] @ (B @ q)) * Q[:, j]
            nrm = np.sqrt(q @ (B @ q))
            if not (nrm > drop * before):
                raise RuntimeError(f"filtered block numerically rank deficient at column {i}")
            Q[:, i] = q / nrm
    return Q


@dataclass
class SolveResult:
    theta: np.ndarray        # Ritz values in (0, gamma], ascending
    X: np.ndarray            # their Ritz vectors, B-orthonormal
    rho: np.ndarray          # their relative residuals
    iterations: int
    converged: bool
    theta_all: np.ndarray    # all L Ritz values of the last iteration
    history: list            # max rho over the wanted Ritz values, per iteration


class ShiftedSolvers:
    """Cached sparse LU factors of A - sigma_j B for a fixed pole set."""

    def __init__(self, A, B, sigma):
        self.A, self.B = A, B
        self.lus = []
        for s in sigma:
            S = (A.astype(np.complex128) - complex(s) * B.astype(np.complex128)).tocsc()
            self.lus.append(sla.splu(S))

    def filter(self, V, w):
        F = (self.B @ V).astype(np.complex128)
        U = np.zeros(V.shape)
        for lu, wj in zip(self.lus, w):
            U += 2.0 * np.real(wj * lu.solve(F))
        return U


def solve_interval(A, B, gamma: float, sigma, w, V0, tol: float = 1e-8,
                   maxit: int = 50, solvers: ShiftedSolvers | None = None) -> SolveResult:
    """Rational filter subspace iteration (Algorithm 1) on (0, gamma]."""
    L = V0.shape[1]
    solvers = solvers or ShiftedSolvers(A, B, sigma)
    V = np.array(V0, dtype=np.float64)
    prev_count = -1
    history = []
    for k in range(1, maxit + 1):
        U = solvers.filter(V, w)
        Q = mgs_b(U, B)
        H = Q.T @ (A @ Q)
        H = 0.5 * (H + H.T)
        theta, S = np.linalg.eigh(H)
        X = Q @ S
        rho = relative_residuals(A, B, X, theta)
        inside = (theta > 0) & (theta <= gamma)
        count = int(inside.sum())
        history.append(float(rho[inside].max()) if count else 0.0)
        if count == L:
            raise RuntimeError("subspace too small: every Ritz value lies in (0, gamma]")
        if count == prev_count and np.all(rho[inside] <= tol):
            return SolveResult(theta[inside], X[:, inside], rho[inside], k, True, theta,
                               history)
        prev_count = count
        V = X
    return SolveResult(theta[inside], X[:, inside], rho[inside], maxit, False, theta, history)
