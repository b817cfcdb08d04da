"""Seeded synthetic inputs for the symmetric-definite eigenproblem A x = lambda B x.

This package is the only code shared between the FP64 CPU oracle (``oracle/``)
and the GPU library (``paper_2503_21618_amd``).  It holds no eigensolver
arithmetic: only finite-element assembly of stiffness/mass pencils (the kind of
vibration pencils the paper's experiments use, Section 4.1) and counter-based
random numbers (start blocks, coefficient fields).

Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), a counter-based mixer: the i-th output for a
seed s is mix64(s + (i+1)*0x9E3779B97F4A7C15).  Normal deviates by the
Box-Muller transform on pairs of uniforms in (0, 1].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs offset .. offset+count-1 of the SplitMix64 stream for ``seed``."""
    with np.errstate(over="ignore"):
        idx = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, count: int) -> np.ndarray:
    """Uniform deviates in (0, 1]: ((x >> 11) + 1) * 2^-53."""
    x = splitmix64(seed, count)
    return ((x >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)


def gaussian(seed: int, count: int) -> np.ndarray:
    """Standard normal deviates: Box-Muller on consecutive uniform pairs.

    Output 2k is sqrt(-2 ln u_{2k}) cos(2 pi u_{2k+1}); output 2k+1 uses sin.
    """
    npairs = (count + 1) // 2
    u = uniform(seed, 2 * npairs)
    r = np.sqrt(-2.0 * np.log(u[0::2]))
    t = 2.0 * math.pi * u[1::2]
    out = np.empty(2 * npairs)
    out[0::2] = r * np.cos(t)
    out[1::2] = r * np.sin(t)
    return out[:count]


def start_block(n: int, L: int, seed: int) -> np.ndarray:
    """Random start block V_1 (n, L), row-major, i.i.d. N(0, 1) entries."""
    return gaussian(seed, n * L).reshape(n, L)


@dataclass
class Pencil:
    """A sparse symmetric-definite pencil (A, B) in CSR form (float64)."""
    A: sp.csr_matrix
    B: sp.csr_matrix
    name: str
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]

    def csr_arrays(self, which: str):
        """(indptr int32, indices int32, data float64) of A or B, sorted columns."""
        M = self.A if which == "A" else self.B
        M.sort_indices()
        return (M.indptr.astype(np.int32), M.indices.astype(np.int32),
                np.ascontiguousarray(M.data, dtype=np.float64))


def _elem_1d(h: float):
    k1 = (1.0 / h) * np.array([[1.0, -1.0], [-1.0, 1.0]])
    m1 = (h / 6.0) * np.array([[2.0, 1.0], [1.0, 2.0]])
    return k1, m1


def _scalar_element(dim: int, h: float):
    """Q1 element stiffness and mass on a cube of side h (exact tensor products)."""
    k1, m1 = _elem_1d(h)
    if dim == 1:
        return k1, m1
    if dim == 2:
        K = np.kron(m1, k1) + np.kron(k1, m1)
        return K, np.kron(m1, m1)
    K = (np.kron(m1, np.kron(m1, k1)) + np.kron(m1, np.kron(k1, m1))
         + np.kron(k1, np.kron(m1, m1)))
    return K, np.kron(m1, np.kron(m1, m1))


def _assemble(dofs: np.ndarray, coef: np.ndarray, Ke: np.ndarray, n: int):
    """Sum coef[e] * Ke over elements, keeping only free (>= 0) dofs."""
    nl = Ke.shape[0]
    rows = np.repeat(dofs, nl, axis=1).reshape(-1, nl, nl)
    cols = np.tile(dofs, (1, nl)).reshape(-1, nl, nl)
    vals = coef[:, None, None] * Ke[None, :, :]
    keep = (rows >= 0) & (cols >= 0)
    M = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n)).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    # duplicate sums run in a different order for (i, j) and (j, i): symmetrise
    # exactly, keeping the structural pattern (explicit zeros included)
    Mt = M.T.tocsr()
    Mt.sort_indices()
    assert np.array_equal(M.indptr, Mt.indptr) and np.array_equal(M.indices, Mt.indices)
    M.data = 0.5 * (M.data + Mt.data)
    return M


def string_1d(n: int) -> Pencil:
    """1D linear FE string: n interior nodes on [0, 1], h = 1/(n+1).

    A = (1/h) tridiag(-1, 2, -1), B = (h/6) tridiag(1, 4, 1).
    """
    h = 1.0 / (n + 1)
    d = np.full(n, 2.0 / h)
    o = np.full(n - 1, -1.0 / h)
    A = sp.diags([o, d, o], [-1, 0, 1], format="csr")
    db = np.full(n, 4.0 * (h / 6.0))
    ob = np.full(n - 1, h / 6.0)
    B = sp.diags([ob, db, ob], [-1, 0, 1], format="csr")
    A.sort_indices()
    B.sort_indices()
    return Pencil(A, B, f"string1d_n{n}", {"h": h, "dim": 1, "m": n + 1})


def scalar_q1(m: int, dim: int, sigma_ln: float = 0.0, seed: int = 0) -> Pencil:
    """Scalar vibration pencil on the unit cube [0,1]^dim with m Q1 elements per side.

    Dirichlet boundary on every face, so n = (m-1)^dim interior nodes in
    lexicographic order (x fastest).  Element coefficient c_e = exp(sigma_ln g_e)
    with g_e i.i.d. N(0, 1) from ``gaussian(seed, m^dim)``; density 1.
    A_e = c_e * int grad(phi_a).grad(phi_b), B_e = int phi_a phi_b (2x2x2 Gauss
    is exact here, so the element matrices are tensor products of the 1D ones).
    """
    h = 1.0 / m
    Ke, Me = _scalar_element(dim, h)
    mi = m - 1
    # node (i0, i1, i2) -> interior dof or -1
    grids = np.meshgrid(*[np.arange(m) for _ in range(dim)], indexing="ij")
    # element (e0, e1, ...) with e0 fastest: flatten with x fastest
    ecoords = [g.transpose(*reversed(range(dim))).reshape(-1) for g in grids]
    nel = m ** dim
    dofs = np.empty((nel, 2 ** dim), dtype=np.int64)
    for l in range(2 ** dim):
        off = [(l >> a) & 1 for a in range(dim)]
        node = [ecoords[a] + off[a] for a in range(dim)]
        inside = np.ones(nel, dtype=bool)
        dof = np.zeros(nel, dtype=np.int64)
        stride = 1
        for a in range(dim):
            inside &= (node[a] >= 1) & (node[a] <= mi)
            dof += (node[a] - 1) * stride
            stride *= mi
        dofs[:, l] = np.where(inside, dof, -1)
    if sigma_ln != 0.0:
        coef = np.exp(sigma_ln * gaussian(seed, nel))
    else:
        coef = np.ones(nel)
    n = mi ** dim
    A = _assemble(dofs, coef, Ke, n)
    B = _assemble(dofs, np.ones(nel), Me, n)
    name = f"scalar{dim}d_m{m}" + (f"_ln{sigma_ln}_s{seed}" if sigma_ln else "_cc")
    return Pencil(A, B, name, {"h": h, "dim": dim, "m": m, "sigma_ln": sigma_ln,
                               "seed": seed})


def _elasticity_element(nu: float):
    """Trilinear hex element stiffness (E = 1, unit cube) by 2x2x2 Gauss, 24x24.

    Local dof 3*l + c, l = a + 2b + 4c' for corner (a, b, c') in {0,1}^3.
    """
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    g = 0.5 / math.sqrt(3.0)
    pts = [0.5 - g, 0.5 + g]
    K = np.zeros((24, 24))
    for x in pts:
        for y in pts:
            for z in pts:
                grad = np.zeros((8, 3))
                for l in range(8):
                    a, b, c = l & 1, (l >> 1) & 1, (l >> 2) & 1
                    fx = x if a else 1 - x
                    fy = y if b else 1 - y
                    fz = z if c else 1 - z
                    sx = 1.0 if a else -1.0
                    sy = 1.0 if b else -1.0
                    sz = 1.0 if c else -1.0
                    grad[l] = [sx * fy * fz, fx * sy * fz, fx * fy * sz]
                Bm = np.zeros((6, 24))
                for l in range(8):
                    gx, gy, gz = grad[l]
                    Bm[0, 3 * l + 0] = gx
                    Bm[1, 3 * l + 1] = gy
                    Bm[2, 3 * l + 2] = gz
                    Bm[3, 3 * l + 1] = gz
                    Bm[3, 3 * l + 2] = gy
                    Bm[4, 3 * l + 0] = gz
                    Bm[4, 3 * l + 2] = gx
                    Bm[5, 3 * l + 0] = gy
                    Bm[5, 3 * l + 1] = gx
                K += 0.125 * Bm.T @ D @ Bm
    return 0.5 * (K + K.T)


def elasticity_q1(nx: int, ny: int, nz: int, h: float, E_sigma_ln: float = 0.0,
                  nu: float = 0.3, rho_range=(1.0, 1.0), seed: int = 0) -> Pencil:
    """3D linear elasticity, trilinear hexes of side h, nx*ny*nz elements.

    Nodes (i, j, k), i in 0..nx, j in 0..ny, k in 0..nz; the x = 0 face is
    clamped, every other face is free.  Free nodes are numbered (i-1) + nx*(j +
    (ny+1)*k), three dofs per node interleaved (dof = 3*node + component).
    Young's modulus E_e = exp(E_sigma_ln g_e), g_e ~ N(0,1) from
    ``gaussian(seed, nel)``; density rho_e ~ U[rho_range] from
    ``uniform(seed + 1, nel)``; consistent mass.
    """
    Kref = _elasticity_element(nu) * h  # stiffness of a cube of side h, E = 1
    _, m1 = _elem_1d(1.0)
    Mref = np.kron(np.kron(m1, np.kron(m1, m1)), np.eye(3)) * h ** 3
    nel = nx * ny * nz
    ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ex = ex.transpose(2, 1, 0).reshape(-1)
    ey = ey.transpose(2, 1, 0).reshape(-1)
    ez = ez.transpose(2, 1, 0).reshape(-1)
    dofs = np.empty((nel, 24), dtype=np.int64)
    for l in range(8):
        i = ex + (l & 1)
        j = ey + ((l >> 1) & 1)
        k = ez + ((l >> 2) & 1)
        node = (i - 1) + nx * (j + (ny + 1) * k)
        free = i >= 1
        for c in range(3):
            dofs[:, 3 * l + c] = np.where(free, 3 * node + c, -1)
    E = np.exp(E_sigma_ln * gaussian(seed, nel)) if E_sigma_ln else np.ones(nel)
    lo, hi = rho_range
    rho = lo + (hi - lo) * uniform(seed + 1, nel) if hi > lo else np.full(nel, lo)
    n = 3 * nx * (ny + 1) * (nz + 1)
    A = _assemble(dofs, E, Kref, n)
    B = _assemble(dofs, rho, Mref, n)
    return Pencil(A, B, f"elast3d_{nx}x{ny}x{nz}_s{seed}",
                  {"h": h, "nx": nx, "ny": ny, "nz": nz, "nu": nu, "seed": seed})


# Named workloads -----------------------------------------------------------

def c1_string() -> Pencil:
    """1D string, n = 2000 interior nodes."""
    return string_1d(2000)


def c2_scalar3d(m: int = 64, sigma_ln: float = 0.5, seed: int = 2) -> Pencil:
    """3D scalar vibration, 64^3 Q1 elements, log-normal coefficient (sigma 0.5)."""
    return scalar_q1(m, 3, sigma_ln, seed)


def c3_elasticity(nodes: int = 48, seed: int = 3) -> Pencil:
    """3D elasticity, 48 x 47 x 47 hexes of side 1/48, 48^3 free nodes x 3 dofs."""
    return elasticity_q1(nodes, nodes - 1, nodes - 1, 1.0 / nodes, 0.7, 0.3,
                         (0.8, 1.2), seed)


# Batched workload ----------------------------------------------------------

def cc_spectrum(m: int, dim: int, count: int) -> np.ndarray:
    """The `count` smallest eigenvalues of the constant-coefficient Q1 pencil with m
    elements per side (Dirichlet): sums of the 1D linear-FE eigenvalues
    mu_k = (6/h^2)(1 - cos k pi h)/(2 + cos k pi h), k = 1..m-1, one per axis
    (stiffness and mass are Kronecker sums/products of the 1D matrices)."""
    h = 1.0 / m
    k = np.arange(1, m)
    mu = (6.0 / h ** 2) * 2.0 * np.sin(0.5 * k * np.pi * h) ** 2 / (2.0 + np.cos(k * np.pi * h))
    mu = mu[: min(len(mu), count)]
    s = mu
    for _ in range(dim - 1):
        s = (s[:, None] + mu[None, :]).ravel()
        s = np.sort(s)[:count]
    return np.sort(s)[:count]


def batch_instance(i: int, seed0: int = 1000, n_range=(5e3, 2e5), nev_range=(10, 80),
                   sigma_ln: float = 0.5):
    """Instance i of the batched workload: a 2D or 3D scalar vibration pencil.

    Seed s = seed0 + i.  Uniforms u = uniform(s, 3): dimension 2 if u0 < 1/2 else 3;
    target size n = exp(U[ln n_lo, ln n_hi]) rounded to the nearest grid (m-1)^dim;
    NEV uniform on {nev_lo..nev_hi}; log-normal element coefficient (sigma_ln, seed s).
    gamma lies halfway between the NEV-th eigenvalue of the constant-coefficient
    pencil of the same grid and the next larger distinct one, so the log-normal
    pencil has about NEV eigenvalues in (0, gamma].  L = ceil(1.2 NEV) rounded up
    to a multiple of 8.  Returns (pencil, gamma, L, NEV)."""
    s = seed0 + i
    u = uniform(s, 3)
    dim = 2 if u[0] < 0.5 else 3
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    n_t = math.exp(lo + (hi - lo) * u[1])
    m = int(round(n_t ** (1.0 / dim))) + 1
    nev = nev_range[0] + min(int(u[2] * (nev_range[1] - nev_range[0] + 1)), nev_range[1] - nev_range[0])
    lam = cc_spectrum(m, dim, nev + 64)
    above = lam[lam > lam[nev - 1] * (1 + 1e-12)]
    gamma = 0.5 * (lam[nev - 1] + above[0])
    L = int(math.ceil(math.ceil(1.2 * nev) / 8.0) * 8)
    return scalar_q1(m, dim, sigma_ln, s), float(gamma), L, nev


def serve_request(r: int, seed0: int = 5000, n_range=(1e4, 1e5), nev_range=(20, 100),
                  sigma_ln: float = 0.5):
    """Request r of the serving workload: a 3D scalar vibration pencil.

    Seed s = seed0 + r; uniforms u = uniform(s, 2): size log-uniform on n_range
    (rounded to the nearest grid (m-1)^3), NEV log-uniform on nev_range; gamma
    from the constant-coefficient spectrum as in batch_instance; L = ceil(1.2 NEV)
    rounded up to a multiple of 8.  Returns (pencil, gamma, L, NEV)."""
    s = seed0 + r
    u = uniform(s, 2)
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    m = int(round(math.exp(lo + (hi - lo) * u[0]) ** (1.0 / 3.0))) + 1
    a, b = math.log(nev_range[0]), math.log(nev_range[1])
    nev = int(round(math.exp(a + (b - a) * u[1])))
    lam = cc_spectrum(m, 3, nev + 64)
    above = lam[lam > lam[nev - 1] * (1 + 1e-12)]
    gamma = 0.5 * (lam[nev - 1] + above[0])
    L = int(math.ceil(math.ceil(1.2 * nev) / 8.0) * 8)
    return scalar_q1(m, 3, sigma_ln, s), float(gamma), L, nev


# Fitted power law of the elasticity family's low eigenvalues on the unit cube
# (lambda_k ~ a k^p, fitted to the 48^3-node pencil's eigenvalues k = 20..199):
# the serving mix uses it to pick gamma for about NEV eigenvalues.
ELASTICITY_SPECTRUM = (1.216, 0.839)


def serve_structure(sid: int, seed0: int = 7000, n_range=(1e4, 5e5), sigma_ln: float = 0.5):
    """Structure sid of the mixed serving workload: even sid a 3D scalar
    vibration pencil, odd sid a 3D elasticity pencil (log-normal Young's modulus
    sigma 0.7, nu 0.3, density U[0.8, 1.2], clamped x = 0 face), size log-uniform
    on n_range from uniform(seed0 + sid, 1), coefficient fields seeded seed0 + sid.
    Returns (pencil, kind, grid size m)."""
    s = seed0 + sid
    u = uniform(s, 1)[0]
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    n_t = math.exp(lo + (hi - lo) * u)
    if sid % 2 == 0:
        m = int(round(n_t ** (1.0 / 3.0))) + 1
        return scalar_q1(m, 3, sigma_ln, s), "scalar", m
    nodes = max(4, int(round((n_t / 3.0) ** (1.0 / 3.0))))
    return (elasticity_q1(nodes, nodes - 1, nodes - 1, 1.0 / nodes, 0.7, 0.3, (0.8, 1.2), s),
            "elasticity", nodes)


def serve_request_mix(r: int, structures: dict, seed0: int = 6000, nev_range=(20, 300)):
    """Request r of the mixed serving workload over a pool of structures
    (sid -> serve_structure(sid)): the structure is uniform over the pool, NEV
    log-uniform on nev_range (seed seed0 + r).  gamma: for a scalar pencil
    halfway between the NEV-th constant-coefficient eigenvalue of its grid and
    the next distinct one (as serve_request); for an elasticity pencil the
    fitted power law at NEV + 1/2, so that about NEV eigenvalues lie below it.
    L = ceil(1.2 NEV) rounded up to a multiple of 8.  Returns (sid, gamma, L, NEV)."""
    u = uniform(seed0 + r, 2)
    ids = sorted(structures)
    sid = ids[min(int(u[0] * len(ids)), len(ids) - 1)]
    a, b = math.log(nev_range[0]), math.log(nev_range[1])
    nev = int(round(math.exp(a + (b - a) * u[1])))
    _, kind, m = structures[sid]
    if kind == "scalar":
        lam = cc_spectrum(m, 3, nev + 64)
        above = lam[lam > lam[nev - 1] * (1 + 1e-12)]
        gamma = 0.5 * (lam[nev - 1] + above[0])
    else:
        ca, cp = ELASTICITY_SPECTRUM
        gamma = ca * (nev + 0.5) ** cp
    L = int(math.ceil(math.ceil(1.2 * nev) / 8.0) * 8)
    return sid, float(gamma), L, nev


def arrival_times(count: int, rate: float, seed: int = 4999) -> np.ndarray:
    """Poisson arrivals: cumulative sums of exponential gaps -ln(u)/rate."""
    return np.cumsum(-np.log(uniform(seed, count)) / rate)
