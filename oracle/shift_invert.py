"""Eigenpairs in (0, gamma] of a large banded pencil by shift-invert subspace
iteration with shift 0.  Test infrastructure.

The paper's Algorithm 1 with the filter Phi(lambda) = 1/lambda: one real pole at
the origin.  This is the shift-and-invert subspace iteration the paper's
introduction cites (Ericsson and Ruhe), and it needs only one factorisation, of
A itself (SPD), where the rational filter would need one complex factorisation
per pole.  It converges to the same set {(lambda_i, x_i): lambda_i in (0, gamma]}
(the plain definition of the paper's problem, Section 1) once the subspace is
larger than the number of wanted eigenvalues, at the rate lambda_i/lambda_{p+1}
per iteration.

Each iteration (the subspace iteration method of Bathe and Wilson):
  1. Z = A^{-1} B X                         (banded Cholesky solves)
  2. A_hat = Z^T A Z = Z^T (B X),  B_hat = Z^T B Z
  3. all eigenpairs of the small pencil (A_hat, B_hat)  (oracle.dense)
  4. X = Z S (B-orthonormal since S^T B_hat S = I); A X = (B X_old) S,
     B X = (B Z) S
  5. rho_i = ||A x_i - theta_i B x_i|| / (|theta_i| ||B x_i||) (Algorithm 1)
Stop when every Ritz value in (0, gamma] has rho_i <= tol and their count is the
same as in the previous iteration and below the subspace size.  The returned
residuals are recomputed from explicit products A X and B X.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import banded, dense


@dataclass
class LargeResult:
    theta: np.ndarray       # eigenvalues in (0, gamma], ascending
    X: np.ndarray           # their eigenvectors, B-orthonormal
    rho: np.ndarray         # their relative residuals (explicit products)
    theta_all: np.ndarray   # all p Ritz values of the last iteration
    rho_all: np.ndarray     # their residuals (from the iteration's products)
    iterations: int
    converged: bool
    history: list


def _residuals(AX, BX, theta):
    R = AX - BX * theta[None, :]
    return np.linalg.norm(R, axis=0) / (np.abs(theta) * np.linalg.norm(BX, axis=0))


def subspace_iteration(A, B, gamma: float, V0, tol: float = 1e-10, maxit: int = 300,
                       factor: banded.BandCholesky | None = None, log=None) -> LargeResult:
    """Shift-invert (shift 0) subspace iteration on (A, B) from the block V0."""
    F = factor if factor is not None else banded.band_cholesky(A)
    X = np.array(V0, dtype=np.float64)
    p = X.shape[1]
    BX = B @ X
    prev = -1
    history = []
    for k in range(1, maxit + 1):
        t0 = time.time()
        Z = banded.band_solve(F, BX)
        Ahat = Z.T @ BX
        BZ = B @ Z
        Bhat = Z.T @ BZ
        theta, S = dense.all_eigenpairs(0.5 * (Ahat + Ahat.T), 0.5 * (Bhat + Bhat.T))
        AX = BX @ S
        X = Z @ S
        BX = BZ @ S
        rho = _residuals(AX, BX, theta)
        inside = (theta > 0) & (theta <= gamma)
        count = int(inside.sum())
        worst = float(rho[inside].max()) if count else 0.0
        history.append(worst)
        if log:
            log(f"iteration {k}: {count} in (0, gamma], max rho {worst:.3e}, "
                f"theta_p {theta[-1]:.6g}, {time.time() - t0:.1f} s")
        if count >= p:
            raise RuntimeError("subspace too small: every Ritz value lies in (0, gamma]")
        if count == prev and worst <= tol:
            break
        prev = count
    conv = count == prev and worst <= tol
    Xi = X[:, inside]
    rho_in = _residuals(A @ Xi, B @ Xi, theta[inside])
    return LargeResult(theta[inside], Xi, rho_in, theta, rho, k, conv, history)
