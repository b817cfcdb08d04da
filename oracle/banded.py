"""Band-limited block elimination for the large-pencil oracle.  Test infrastructure.

The structured-grid pencils number their unknowns lexicographically, so every
nonzero a_ij has |i - j| <= kd with kd about m^(d-1) (the bandwidth).  Gaussian
elimination then creates no fill outside the band.  Two plain uses of that fact:

* ``band_cholesky`` / ``band_solve``: the Cholesky factor of an SPD matrix (a
  library Cholesky on each diagonal block, the textbook block-column update for
  the rest) and forward/backward substitution with it.  This is the direct solve
  with A that the shift-invert subspace iteration needs (paper Section 1, the
  Ericsson-Ruhe shift-and-invert approach, with shift 0).
* ``band_inertia``: the number of negative eigenvalues of a symmetric matrix by
  block elimination and Haynsworth's inertia additivity,
  In(M) = In(M_11) + In(M / M_11), where M / M_11 is the Schur complement.
  Applied to A - gamma B it gives #{lambda < gamma} by Sylvester's law (B SPD),
  the count that checks the paper's interval (0, gamma] (Section 1).

Both keep one dense window of kd + nb rows and columns: the columns being
eliminated plus every row and column they can still touch.  Rows that enter
the window later hold untouched entries of the input matrix, because an
elimination step only updates entries within kd of the eliminated columns.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def bandwidth(M) -> int:
    """max |i - j| over the stored entries of a sparse matrix."""
    C = sp.coo_matrix(M)
    return int(np.abs(C.row.astype(np.int64) - C.col).max()) if C.nnz else 0


def _windows(M, kd: int, nb: int):
    """Yield (j0, b, W) for the block columns [j0, j0 + b): W is the current dense
    window on rows/cols [j0, hi) of the partially eliminated matrix.  The caller
    overwrites W[b:, b:] with the Schur complement before the next step."""
    M = sp.csr_matrix(M)
    n = M.shape[0]
    w = min(n, kd + nb)
    W = M[0:w, 0:w].toarray()
    j0 = 0
    while j0 < n:
        b = min(nb, n - j0)
        hi = j0 + W.shape[0]
        yield j0, b, W
        lo, new_hi = j0 + b, min(n, j0 + b + w)
        if lo >= n:
            break
        k = hi - lo
        Wn = np.empty((new_hi - lo, new_hi - lo))
        Wn[:k, :k] = W[b:, b:]
        if new_hi > hi:
            Wn[k:, :] = M[hi:new_hi, lo:new_hi].toarray()
            Wn[:k, k:] = Wn[k:, :k].T
        W = Wn
        j0 = lo


@dataclass
class BandCholesky:
    """Block columns of the lower Cholesky factor L (A = L L^T): for block
    [j0, j0 + b) the b x b diagonal block and the rows below it (at most kd)."""
    n: int
    kd: int
    panels: list   # (j0, b, L_jj (b x b lower), L_below (r x b))


def band_cholesky(A, kd: int | None = None, nb: int = 1024) -> BandCholesky:
    """Cholesky factor of an SPD band matrix by block columns:
    L_jj = chol(W_jj), L_below = W_below L_jj^{-T}, W_rest -= L_below L_below^T."""
    kd = bandwidth(A) if kd is None else kd
    panels = []
    for j0, b, W in _windows(A, kd, nb):
        Ljj = np.linalg.cholesky(W[:b, :b])
        if W.shape[0] > b:
            Lb = sla.solve_triangular(Ljj, W[b:, :b].T, lower=True).T
            W[b:, b:] -= Lb @ Lb.T
        else:
            Lb = np.zeros((0, b))
        panels.append((j0, b, Ljj, np.ascontiguousarray(Lb)))
    return BandCholesky(A.shape[0], kd, panels)


def band_solve(F: BandCholesky, R) -> np.ndarray:
    """Z with A Z = R: forward substitution L Y = R, then backward L^T Z = Y,
    one block of rows at a time."""
    Z = np.array(R, dtype=np.float64, copy=True)
    for j0, b, Ljj, Lb in F.panels:
        Z[j0:j0 + b] = sla.solve_triangular(Ljj, Z[j0:j0 + b], lower=True)
        r = Lb.shape[0]
        if r:
            Z[j0 + b:j0 + b + r] -= Lb @ Z[j0:j0 + b]
    for j0, b, Ljj, Lb in reversed(F.panels):
        r = Lb.shape[0]
        if r:
            Z[j0:j0 + b] -= Lb.T @ Z[j0 + b:j0 + b + r]
        Z[j0:j0 + b] = sla.solve_triangular(Ljj, Z[j0:j0 + b], lower=True, trans="T")
    return Z


def band_inertia(M, kd: int | None = None, nb: int = 1024, min_rel_pivot: float = 1e-12):
    """Number of negative eigenvalues of a symmetric band matrix.

    Block elimination without pivoting across blocks: the inertia of each
    diagonal block (symmetric eigenvalues, a library routine) is added, and the
    block is eliminated into the Schur complement (Haynsworth).  Raises if a
    diagonal block is numerically singular (then the count could be wrong);
    a different nb places the block boundaries elsewhere."""
    kd = bandwidth(M) if kd is None else kd
    neg = 0
    for j0, b, W in _windows(M, kd, nb):
        D = W[:b, :b]
        ev = np.linalg.eigvalsh(D)
        if np.abs(ev).min() <= min_rel_pivot * np.abs(ev).max():
            raise RuntimeError(f"near-singular diagonal block at row {j0}: try another nb")
        neg += int((ev < 0).sum())
        if W.shape[0] > b:
            C = W[b:, :b]
            W[b:, b:] -= C @ np.linalg.solve(D, C.T)
    return neg


def inertia_count(A, B, gamma: float, nb: int = 1024) -> int:
    """#{lambda < gamma} for the pencil (A, B), B SPD (Sylvester's law)."""
    M = (sp.csr_matrix(A) - gamma * sp.csr_matrix(B)).tocsr()
    return band_inertia(M, max(bandwidth(A), bandwidth(B)), nb)
