"""Right-preconditioned BiCGStab for the complex-shifted systems.  Test infrastructure.

The paper solves each shifted system (A - sigma_j B) y = f with BiCGStab
(van der Vorst, SIAM J. Sci. Stat. Comput. 13 (1992)), Sections 2 and 4.2, with an
ILU preconditioner of the shifted operator.  Three preconditioners M_j of
S_j = A - sigma_j B are used here, all applied on the right:
  * point Jacobi, M_j = diag(A) - sigma_j diag(B);
  * ILU(0), M_j = L_j U_j with the sparsity pattern of S_j (no fill), which is
    the exact LU factorisation when S_j is tridiagonal;
  * node block Jacobi for vector problems with 3 unknowns per node
    (unknowns 3k, 3k+1, 3k+2 belong to node k): M_j = blockdiag of the 3x3
    diagonal blocks of S_j, exact when A and B are block diagonal.

Readings: the initial guess is x_0 = 0, so r_0 = f, and the shadow residual is
r_hat = f (real when f = B X is real, shared by all poles).  Inner products are
Hermitian, (u, v) = u^H v.  Convergence is tested on the recursively updated
residual after the half step (s) and the full step (r), relative to ||f||.

Steps per iteration (all columns in parallel, each column its own scalars):
    rho   = (r_hat, r)
    beta  = (rho / rho_prev) (alpha / omega)
    p     = r + beta (p - omega v)
    p_hat = M^{-1} p ;  v = S p_hat ;  alpha = rho / (r_hat, v)
    s     = r - alpha v                  -> stop if ||s|| <= tol ||f||, x += alpha p_hat
    s_hat = M^{-1} s ;  t = S s_hat ;  omega = (t, s) / (t, t)
    x     = x + alpha p_hat + omega s_hat
    r     = s - omega t                  -> stop if ||r|| <= tol ||f||
"""
from __future__ import annotations

import numpy as np

ACTIVE, CONVERGED, HALF_CONVERGED, BREAKDOWN, MAXIT = 0, 1, 2, 3, 4


def jacobi_diagonal(A, B, sigma: complex) -> np.ndarray:
    """Diagonal of the shifted operator, diag(A) - sigma diag(B)."""
    return A.diagonal().astype(np.complex128) - sigma * B.diagonal()


def union_pattern(A, B):
    """CSR pattern of A + B (union), sorted, as (indptr, indices)."""
    P = (abs(A) + abs(B)).tocsr()
    P.sort_indices()
    return P.indptr, P.indices


def ilu0(A, B, sigma: complex):
    """ILU(0) of S = A - sigma B on the union pattern (IKJ variant):
    for each row i and each k < i in the pattern, l_ik = s_ik / u_kk and
    s_ij -= l_ik u_kj for every j > k with (i, j) and (k, j) in the pattern.
    Returns (indptr, indices, values) with L (unit, strictly lower) and U
    (upper with diagonal) stored together."""
    indptr, indices = union_pattern(A, B)
    n = A.shape[0]
    Ad, Bd = A.tolil(), B.tolil()
    rows = []
    for i in range(n):
        cols = indices[indptr[i]:indptr[i + 1]]
        rows.append({int(j): complex(Ad[i, j]) - sigma * complex(Bd[i, j]) for j in cols})
    for i in range(n):
        ri = rows[i]
        for k in sorted(c for c in ri if c < i):
            ri[k] /= rows[k][k]
            lik = ri[k]
            for j, ukj in rows[k].items():
                if j > k and j in ri:
                    ri[j] -= lik * ukj
    vals = np.array([rows[i][int(j)] for i in range(n) for j in indices[indptr[i]:indptr[i + 1]]])
    return indptr, indices, vals


def block_jacobi3(A, B, sigma: complex) -> np.ndarray:
    """The (n/3, 3, 3) diagonal node blocks of S = A - sigma B."""
    n = A.shape[0]
    if n % 3:
        raise ValueError("block Jacobi needs 3 unknowns per node")
    S = (A.astype(np.complex128) - sigma * B).tocsr()
    blocks = np.zeros((n // 3, 3, 3), np.complex128)
    for r in range(3):
        for c in range(3):
            rows = np.arange(r, n, 3)
            blocks[:, r, c] = np.asarray(S[rows, rows - r + c]).ravel()
    return blocks


def block_jacobi3_solve(blocks, Y):
    """M^{-1} Y for M = blockdiag(blocks): one 3x3 solve per node and column."""
    n, m = Y.shape
    Z = np.asarray(Y, dtype=np.complex128).reshape(n // 3, 3, m)
    return np.linalg.solve(blocks, Z).reshape(n, m)


def ilu0_solve(fac, Y):
    """(L U)^{-1} Y by forward and backward substitution (Y is (n, m))."""
    indptr, indices, vals = fac
    n = len(indptr) - 1
    Z = np.array(Y, dtype=np.complex128, copy=True)
    for i in range(n):
        for k in range(indptr[i], indptr[i + 1]):
            j = indices[k]
            if j < i:
                Z[i] -= vals[k] * Z[j]
    for i in range(n - 1, -1, -1):
        d = None
        for k in range(indptr[i], indptr[i + 1]):
            j = indices[k]
            if j > i:
                Z[i] -= vals[k] * Z[j]
            elif j == i:
                d = vals[k]
        Z[i] /= d
    return Z


def node_graph(A, B, block: int):
    """Adjacency of the nodes (block = 1: every unknown is a node; block = 3:
    unknowns 3k, 3k+1, 3k+2 form node k) in the union pattern of A and B, as a
    list of neighbour sets (without the node itself)."""
    indptr, indices = union_pattern(A, B)
    n = A.shape[0]
    nodes = n // block
    nb = [set() for _ in range(nodes)]
    for i in range(n):
        k = i // block
        for j in indices[indptr[i]:indptr[i + 1]]:
            m = int(j) // block
            if m != k:
                nb[k].add(m)
    return nb


def greedy_colouring(A, B, block: int = 1) -> np.ndarray:
    """Colour of every node such that coupled nodes differ: nodes are taken in
    increasing index and each gets the smallest colour none of its already
    coloured neighbours has (greedy colouring)."""
    nb = node_graph(A, B, block)
    col = -np.ones(len(nb), np.int64)
    for k in range(len(nb)):
        used = {int(col[m]) for m in nb[k] if col[m] >= 0}
        c = 0
        while c in used:
            c += 1
        col[k] = c
    return col


class MulticolourSGS:
    """Symmetric Gauss-Seidel preconditioner of S = A - sigma B in a multicolour
    order (the shifted-operator preconditioner of Section 4.2 is an ILU; this is a
    symmetric one with parallel colour sweeps, usable inside COCG):

        M = (D + L) D^{-1} (D + U),

    D the block diagonal of S (1x1 or 3x3 node blocks), L (U) the couplings of a
    node to nodes of lower (higher) colour.  Nodes of one colour are not coupled,
    so M^{-1} r is a forward sweep over the colours, (D + L) y = r, i.e.
    y_k = D_k^{-1} (r_k - sum_{colour(m) < colour(k)} S_km y_m), then a backward
    sweep, (D + U) z = D y, i.e. z_k = y_k - D_k^{-1} sum_{colour(m) > colour(k)} S_km z_m.
    With S complex symmetric, U = L^T and M is complex symmetric too.

    omega != 1 gives symmetric SOR: D is replaced by D / omega in all three
    factors, M = (D/omega + L) (D/omega)^{-1} (D/omega + U) (the constant
    factor of the textbook form, which no CG iterate depends on, is left out);
    0 < omega < 2."""

    def __init__(self, A, B, sigma: complex, block: int = 1, colour=None, omega: float = 1.0):
        n = A.shape[0]
        if block not in (1, 3) or n % block:
            raise ValueError("block must be 1, or 3 with n divisible by 3")
        if not 0.0 < omega < 2.0:
            raise ValueError("omega must lie in (0, 2)")
        self.n, self.block = n, block
        self.colour = greedy_colouring(A, B, block) if colour is None else np.asarray(colour)
        S = (A.astype(np.complex128) - sigma * B).tocoo()
        cr = self.colour[S.row // block]
        cc = self.colour[S.col // block]
        import scipy.sparse as sp
        low, up, dia = cr > cc, cr < cc, cr == cc
        mk = lambda m: sp.csr_matrix((S.data[m], (S.row[m], S.col[m])), shape=(n, n))
        self.L, self.U, self.D = mk(low), mk(up), mk(dia)
        # same-colour entries can only be the node's own block
        if np.any((S.row[dia] // block) != (S.col[dia] // block)):
            raise ValueError("colouring couples two nodes of one colour")
        nodes = n // block
        blocks = np.zeros((nodes, block, block), np.complex128)
        Dc = self.D.tocoo()
        blocks[Dc.row // block, Dc.row % block, Dc.col % block] = Dc.data
        self.blocks = blocks / omega
        self.order = [np.flatnonzero(self.colour == c) for c in range(int(self.colour.max()) + 1)]

    def _rows(self, nodes):
        return (nodes[:, None] * self.block + np.arange(self.block)[None, :]).ravel()

    def _dsolve(self, nodes, Y):
        m = Y.shape[1]
        Z = np.linalg.solve(self.blocks[nodes], Y.reshape(len(nodes), self.block, m))
        return Z.reshape(len(nodes) * self.block, m)

    def apply(self, R):
        """M^{-1} R for an (n, m) block."""
        R = np.asarray(R, dtype=np.complex128)
        Y = np.zeros_like(R)
        for nodes in self.order:
            rows = self._rows(nodes)
            Y[rows] = self._dsolve(nodes, R[rows] - self.L[rows] @ Y)
        Z = np.zeros_like(R)
        for nodes in reversed(self.order):
            rows = self._rows(nodes)
            Z[rows] = Y[rows] - self._dsolve(nodes, self.U[rows] @ Z)
        return Z

    def matrix(self):
        """M itself, formed from its factors (for checks on small pencils)."""
        import scipy.sparse as sp
        n = self.n
        Db = sp.block_diag(list(self.blocks), format="csr")
        Dinv = sp.block_diag([np.linalg.inv(b) for b in self.blocks], format="csr")
        return ((Db + self.L) @ Dinv @ (Db + self.U)).toarray() if n <= 4000 else None


def bicgstab(A, B, sigmas, F, tol: float, maxit: int, fixed_iters: int | None = None,
             precond: str = "jacobi"):
    """Solve (A - sigma_c B) x_c = F[:, l(c)] for every pole and column.

    sigmas: N poles; F: (n, L) real.  Columns are ordered pole-major,
    c = j*L + l.  Returns (X (n, N*L) complex, iters[K], flags[K], relres[K]).
    If ``fixed_iters`` is given, runs exactly that many full iterations with no
    convergence test (for comparing intermediate iterates).
    """
    n, L = F.shape
    N = len(sigmas)
    K = N * L
    sig = np.repeat(np.asarray(sigmas, dtype=np.complex128), L)          # (K,)
    if precond == "jacobi":
        D = np.stack([jacobi_diagonal(A, B, s) for s in sigmas], axis=1)  # (n, N)
        Dc = np.repeat(D, L, axis=1)                                      # (n, K)

        def Minv(Y):
            return Y / Dc
    elif precond == "ilu0":
        facs = [ilu0(A, B, s) for s in sigmas]

        def Minv(Y):
            return np.concatenate([ilu0_solve(facs[j], Y[:, j * L:(j + 1) * L])
                                   for j in range(N)], axis=1)
    elif precond == "bjac3":
        blks = [block_jacobi3(A, B, s) for s in sigmas]

        def Minv(Y):
            return np.concatenate([block_jacobi3_solve(blks[j], Y[:, j * L:(j + 1) * L])
                                   for j in range(N)], axis=1)
    else:
        raise ValueError(precond)
    f = np.tile(F, (1, N)).astype(np.complex128)                          # (n, K)
    rhat = np.tile(F, (1, N)).astype(np.float64)

    def S(Y):
        return (A @ Y) - sig[None, :] * (B @ Y)

    fn = np.sqrt((np.abs(f) ** 2).sum(0))
    x = np.zeros((n, K), np.complex128)
    r = f.copy()
    p = np.zeros_like(x)
    v = np.zeros_like(x)
    rho_prev = np.ones(K, np.complex128)
    alpha = np.ones(K, np.complex128)
    omega = np.ones(K, np.complex128)
    flags = np.where(fn == 0.0, CONVERGED, ACTIVE)
    iters = np.zeros(K, np.int64)
    nsteps = fixed_iters if fixed_iters is not None else maxit
    for it in range(nsteps):
        act = flags == ACTIVE
        if not act.any():
            break
        rho = (rhat * r).sum(0)
        beta = (rho / rho_prev) * (alpha / omega)
        p = np.where(act, r + beta * (p - omega * v), p)
        ph = Minv(p)
        v = np.where(act, S(ph), v)
        rv = (rhat * v).sum(0)
        bad = act & ((rho == 0) | (rv == 0))
        alpha = np.where(act & ~bad, rho / np.where(rv == 0, 1, rv), alpha)
        s = r - alpha * v
        sn = np.sqrt((np.abs(s) ** 2).sum(0))
        half = act & ~bad & (sn <= tol * fn) & (fixed_iters is None)
        x = np.where(half, x + alpha * ph, x)
        iters = np.where(act & ~bad, iters + 1, iters)
        flags = np.where(half, HALF_CONVERGED, np.where(bad, BREAKDOWN, flags))
        act = flags == ACTIVE
        sh = Minv(s)
        t = S(sh)
        tt = (np.abs(t) ** 2).sum(0)
        ts = (np.conj(t) * s).sum(0)
        bad = act & (tt == 0)
        omega = np.where(act & ~bad, ts / np.where(tt == 0, 1, tt), omega)
        x = np.where(act & ~bad, x + alpha * ph + omega * sh, x)
        r = np.where(act & ~bad, s - omega * t, r)
        rn = np.sqrt((np.abs(r) ** 2).sum(0))
        conv = act & ~bad & (rn <= tol * fn) & (fixed_iters is None)
        flags = np.where(conv, CONVERGED, np.where(bad, BREAKDOWN, flags))
        rho_prev = np.where(act, rho, rho_prev)
    if fixed_iters is None:
        flags = np.where(flags == ACTIVE, MAXIT, flags)
    relres = np.sqrt((np.abs(f - S(x)) ** 2).sum(0)) / np.where(fn == 0, 1, fn)
    return x, iters, flags, relres


def cocg(A, B, sigmas, F, tol: float, maxit: int, fixed_iters: int | None = None,
         precond: str = "jacobi", omega: float = 1.0):
    """Conjugate orthogonal conjugate gradients (COCG; van der Vorst and Melissen,
    IEEE Trans. Magn. 26 (1990)) for every pole and column, an alternative to
    BiCGStab for the shifted systems of Section 3.

    With A and B real symmetric, S_j = A - sigma_j B is complex symmetric
    (S_j^T = S_j), and CG with the bilinear form [u, v] = u^T v (no conjugation)
    in place of the inner product applies; it needs one product with S_j per
    iteration.  The preconditioner must be complex symmetric as well: point
    Jacobi, node block Jacobi, or multicolour symmetric Gauss-Seidel with point
    ("mcsgs") or node ("mcsgs3") blocks, relaxed by omega (symmetric SOR; 1:
    plain SGS) (ILU(0) is not symmetric and is not offered).
    Same interface and conventions as ``bicgstab``: x_0 = 0, columns pole-major,
    convergence on the recursively updated residual ||r||_2 <= tol ||f||_2.

    Steps per iteration, each column with its own scalars:
        q = S p ;  alpha = rho / [p, q]
        x = x + alpha p ;  r = r - alpha q        -> stop if ||r|| <= tol ||f||
        z = M^{-1} r ;  rho' = [r, z] ;  beta = rho' / rho ;  p = z + beta p
    starting from r = f, z = M^{-1} f, p = z, rho = [r, z].
    """
    n, L = F.shape
    N = len(sigmas)
    K = N * L
    sig = np.repeat(np.asarray(sigmas, dtype=np.complex128), L)
    if precond == "jacobi":
        D = np.stack([jacobi_diagonal(A, B, s) for s in sigmas], axis=1)
        Dc = np.repeat(D, L, axis=1)

        def Minv(Y):
            return Y / Dc
    elif precond == "bjac3":
        blks = [block_jacobi3(A, B, s) for s in sigmas]

        def Minv(Y):
            return np.concatenate([block_jacobi3_solve(blks[j], Y[:, j * L:(j + 1) * L])
                                   for j in range(N)], axis=1)
    elif precond in ("mcsgs", "mcsgs3"):
        block = 3 if precond == "mcsgs3" else 1
        colour = greedy_colouring(A, B, block)      # depends on the pattern only
        sgs = [MulticolourSGS(A, B, s, block, colour=colour, omega=omega) for s in sigmas]

        def Minv(Y):
            return np.concatenate([sgs[j].apply(Y[:, j * L:(j + 1) * L]) for j in range(N)], axis=1)
    else:
        raise ValueError(f"COCG needs a symmetric preconditioner, not {precond}")
    f = np.tile(F, (1, N)).astype(np.complex128)

    def S(Y):
        return (A @ Y) - sig[None, :] * (B @ Y)

    fn = np.sqrt((np.abs(f) ** 2).sum(0))
    x = np.zeros((n, K), np.complex128)
    r = f.copy()
    p = Minv(r)
    rho = (r * p).sum(0)
    flags = np.where(fn == 0.0, CONVERGED, ACTIVE)
    iters = np.zeros(K, np.int64)
    nsteps = fixed_iters if fixed_iters is not None else maxit
    for it in range(nsteps):
        act = flags == ACTIVE
        if not act.any():
            break
        q = S(p)
        pq = (p * q).sum(0)
        bad = act & ((pq == 0) | (rho == 0))
        ok = act & ~bad
        alpha = np.where(ok, rho / np.where(pq == 0, 1, pq), 0)
        x = np.where(ok, x + alpha * p, x)
        r = np.where(ok, r - alpha * q, r)
        iters = np.where(ok, iters + 1, iters)
        rn = np.sqrt((np.abs(r) ** 2).sum(0))
        conv = ok & (rn <= tol * fn) & (fixed_iters is None)
        flags = np.where(conv, CONVERGED, np.where(bad, BREAKDOWN, flags))
        act = flags == ACTIVE
        z = Minv(r)
        rho_new = (r * z).sum(0)
        beta = np.where(act, rho_new / np.where(rho == 0, 1, rho), 0)
        p = np.where(act, z + beta * p, p)
        rho = np.where(act, rho_new, rho)
    if fixed_iters is None:
        flags = np.where(flags == ACTIVE, MAXIT, flags)
    relres = np.sqrt((np.abs(f - S(x)) ** 2).sum(0)) / np.where(fn == 0, 1, fn)
    return x, iters, flags, relres
