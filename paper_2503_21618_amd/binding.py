"""Python binding of libslrf (the gfx950 SLRF eigensolver): argument marshalling only.

Every step of the computation runs in the HIP library; torch provides device
memory (the workspace and the dense blocks) and the stream.  If the compiled
library is missing this module raises on import: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libslrf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2503_21618_amd.build`")
_lib = C.CDLL(LIB_PATH)

FP64, MIXED = 0, 1
PRECOND_AUTO, PRECOND_JACOBI, PRECOND_ILU0, PRECOND_BLOCK3 = 0, 1, 2, 3
PRECOND_SGS, PRECOND_SGS3 = 4, 5   # multicolour symmetric Gauss-Seidel, point / node blocks (COCG)
SOLVER_BICGSTAB, SOLVER_COCG = 0, 1
STATUS = {0: "OK", 1: "E_INVALID_ARG", 2: "E_NOT_SPD", 3: "E_WORKSPACE", 4: "E_DEVICE",
          5: "E_NOT_CONVERGED", 6: "E_SUBSPACE_TOO_SMALL", 7: "E_BREAKDOWN"}


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("inner_tol", C.c_double), ("inner_maxit", C.c_int32),
                ("outer_tol", C.c_double), ("outer_maxit", C.c_int32), ("check_every", C.c_int32),
                ("seed", C.c_uint64), ("precond", C.c_int32), ("profile", C.c_int32),
                ("graph", C.c_int32), ("tile_rows", C.c_int32), ("tile_wgs", C.c_int32),
                ("band_rows", C.c_int32), ("tune", C.c_int32), ("solver", C.c_int32), ("recycle", C.c_int32),
                ("sgs_omega", C.c_double)]


class Poles(C.Structure):
    _fields_ = [("n_poles", C.c_int32), ("sigma", C.POINTER(C.c_double)),
                ("weight", C.POINTER(C.c_double))]


class FilterStats(C.Structure):
    _fields_ = [("max_iterations", C.c_int32), ("mean_iterations", C.c_double), ("spmv", C.c_int64),
                ("n_breakdown", C.c_int32), ("n_maxit", C.c_int32), ("refinements", C.c_int32),
                ("max_relres", C.c_double), ("seconds", C.c_double),
                ("spmm_seconds", C.c_double), ("spmm_launches", C.c_int64), ("spmm_bytes", C.c_double),
                ("spmm_columns", C.c_double),
                ("update_seconds", C.c_double), ("update_launches", C.c_int64),
                ("update_bytes", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SolveStats(C.Structure):
    _fields_ = [("outer_iterations", C.c_int32), ("spmv_total", C.c_int64), ("n_found", C.c_int32),
                ("max_resid", C.c_double), ("seconds", C.c_double), ("filter_seconds", C.c_double),
                ("inner_iterations", C.c_double), ("kernels", FilterStats)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["kernels"] = self.kernels.as_dict()
        return d


_P = C.c_void_p
_lib.slrf_default_options.argtypes = [C.POINTER(Options)]
_lib.slrf_design_poles.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, _P, _P, _P]
_lib.slrf_quadrature_poles.argtypes = [C.c_int32, C.c_int32, C.c_double, _P, _P]
_lib.slrf_workspace_bytes.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_size_t)]
_lib.slrf_workspace_bytes_for.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.POINTER(Options),
                                          C.POINTER(C.c_size_t)]
_lib.slrf_create.argtypes = [C.POINTER(_P), C.c_int64, _P, _P, _P, _P, _P, _P, _P, C.c_size_t,
                             C.c_int64, C.c_int32, C.POINTER(Options), _P]
_lib.slrf_create_static.argtypes = [C.POINTER(_P), C.c_int64, _P, _P, _P, _P, _P, _P,
                                    C.c_int64, C.c_int32, C.POINTER(Options), _P]
_lib.slrf_filter_apply.argtypes = [_P, C.POINTER(Poles), C.c_int64, _P, _P, C.POINTER(FilterStats)]
_lib.slrf_solve_interval.argtypes = [_P, C.c_double, C.c_int64, C.POINTER(Poles), _P,
                                     C.POINTER(C.c_int64), _P, _P, _P, C.POINTER(SolveStats)]
_lib.slrf_destroy.argtypes = [_P]
_lib.slrf_status_string.argtypes = [C.c_int]
_lib.slrf_status_string.restype = C.c_char_p
_lib.slrf_last_error.argtypes = [_P]
_lib.slrf_last_error.restype = C.c_char_p
_lib.slrf_batch_footprint.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
_lib.slrf_batch_footprint_for.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.POINTER(Options),
                                          C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
_lib.slrf_batch_create.argtypes = [C.POINTER(_P), _P, C.c_size_t, C.c_size_t, C.c_int32,
                                   C.POINTER(Options), _P]
_lib.slrf_batch_add.argtypes = [_P, C.c_int64, _P, _P, _P, _P, _P, _P, C.c_double, C.c_int64,
                                C.POINTER(Poles), _P, C.POINTER(C.c_int32)]
_lib.slrf_batch_step.argtypes = [_P, C.POINTER(C.c_int32)]
_lib.slrf_batch_query.argtypes = [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
_lib.slrf_batch_result.argtypes = [_P, C.c_int32, C.POINTER(C.c_int64), _P, _P, _P,
                                   C.POINTER(SolveStats)]
_lib.slrf_batch_remove.argtypes = [_P, C.c_int32]
_lib.slrf_batch_restart.argtypes = [_P, C.c_int32, _P]
_lib.slrf_batch_destroy.argtypes = [_P]
_lib.slrf_batch_last_error.argtypes = [_P]
_lib.slrf_batch_last_error.restype = C.c_char_p
for _f in ("slrf_design_poles", "slrf_workspace_bytes", "slrf_workspace_bytes_for", "slrf_create",
           "slrf_create_static",
           "slrf_filter_apply",
           "slrf_solve_interval", "slrf_batch_footprint", "slrf_batch_footprint_for", "slrf_batch_create",
           "slrf_batch_add",
           "slrf_batch_step", "slrf_batch_query", "slrf_batch_result", "slrf_batch_remove",
           "slrf_batch_restart"):
    getattr(_lib, _f).restype = C.c_int

_lib.slrf_test_gram.argtypes = [C.c_int64, C.c_int64, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]
_lib.slrf_test_gram.restype = C.c_int
_lib.slrf_test_gemm.argtypes = [C.c_int64, C.c_int64, C.c_int64, _P, _P, _P, _P]
_lib.slrf_test_gemm.restype = C.c_int
_lib.slrf_test_gram_prec.argtypes = [C.c_int64, C.c_int64, _P, _P, _P, _P, _P, _P, C.c_size_t, C.c_int, _P]
_lib.slrf_test_gram_prec.restype = C.c_int
_lib.slrf_test_gram_scratch.argtypes = [C.c_int64, C.c_int64]
_lib.slrf_test_gram_scratch.restype = C.c_size_t

EXPORTED = ["slrf_default_options", "slrf_design_poles", "slrf_quadrature_poles", "slrf_workspace_bytes",
            "slrf_workspace_bytes_for",
            "slrf_create", "slrf_create_static",
            "slrf_filter_apply", "slrf_solve_interval", "slrf_destroy", "slrf_status_string",
            "slrf_last_error", "slrf_batch_footprint", "slrf_batch_footprint_for", "slrf_batch_create",
            "slrf_batch_add",
            "slrf_batch_step", "slrf_batch_query", "slrf_batch_result", "slrf_batch_remove",
            "slrf_batch_restart", "slrf_batch_destroy", "slrf_batch_last_error"]
TESTING_EXPORTED = ["slrf_test_gram", "slrf_test_gemm", "slrf_test_gram_prec", "slrf_test_gram_scratch"]


def test_gram(U, WA, WB, f32: bool = False):
    """Kernel-level hook: (U^T WA, U^T WB) by the library's MFMA Gram kernel
    (f32: the FP32 MFMA variant)."""
    import torch
    n, L = U.shape
    GA = torch.empty((L, L), dtype=torch.float64, device=U.device)
    GB = torch.empty_like(GA)
    nb = _lib.slrf_test_gram_scratch(n, L)
    scratch = torch.empty(max(nb, 8), dtype=torch.uint8, device=U.device)
    st = _lib.slrf_test_gram_prec(n, L, *[C.c_void_p(t.data_ptr()) for t in (U, WA, WB, GA, GB, scratch)],
                                  nb, 1 if f32 else 0, C.c_void_p(torch.cuda.current_stream(U.device).cuda_stream))
    if st:
        raise SlrfError(st, "test_gram")
    return GA, GB


def test_gemm(X, Z):
    """Kernel-level hook: X Z by the library's MFMA Ritz-update kernel."""
    import torch
    n, L = X.shape
    r = Z.shape[1]
    Y = torch.empty((n, r), dtype=torch.float64, device=X.device)
    st = _lib.slrf_test_gemm(n, L, r, *[C.c_void_p(t.data_ptr()) for t in (X, Z, Y)],
                             C.c_void_p(torch.cuda.current_stream(X.device).cuda_stream))
    if st:
        raise SlrfError(st, "test_gemm")
    return Y


class SlrfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def default_options(**kw) -> Options:
    o = Options()
    _lib.slrf_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def design_poles(N: int, alpha: float = 1.0, beta: float = 0.01, gamma: float = 1.0):
    """SLRF poles/weights (upper half plane) and separation factor."""
    s = np.zeros(2 * N)
    w = np.zeros(2 * N)
    sep = np.zeros(1)
    st = _lib.slrf_design_poles(N, alpha, beta, gamma, _ptr(s), _ptr(w), _ptr(sep))
    if st:
        raise SlrfError(st, "pole design")
    return s[0::2] + 1j * s[1::2], w[0::2] + 1j * w[1::2], float(sep[0])


QUAD_MIDPOINT, QUAD_GAUSS_LEGENDRE, QUAD_GAUSS_CHEBYSHEV = 0, 1, 2


def quadrature_poles(rule: int, N: int, gamma: float = 1.0):
    """Section 3.2 quadrature-rule filter on the circle over [0, gamma]: upper
    half-plane poles and weights (complex arrays, sorted by real part)."""
    s = np.zeros(2 * N)
    w = np.zeros(2 * N)
    st = _lib.slrf_quadrature_poles(rule, N, gamma, _ptr(s), _ptr(w))
    if st:
        raise SlrfError(st, "quadrature poles")
    return s[0::2] + 1j * s[1::2], w[0::2] + 1j * w[1::2]


def workspace_bytes(n: int, nnz: int, L: int, N: int, precision: int = FP64, options: Options | None = None) -> int:
    """Workspace bytes of a Solver; with options, for their precision and preconditioner."""
    b = C.c_size_t()
    if options is None:
        st = _lib.slrf_workspace_bytes(n, nnz, L, N, precision, C.byref(b))
    else:
        st = _lib.slrf_workspace_bytes_for(n, nnz, L, N, C.byref(options), C.byref(b))
    if st:
        raise SlrfError(st, "workspace size")
    return b.value


def _poles_struct(sigma, w):
    sigma = np.asarray(sigma, dtype=np.complex128)
    w = np.asarray(w, dtype=np.complex128)
    s = np.empty(2 * len(sigma))
    s[0::2], s[1::2] = sigma.real, sigma.imag
    ww = np.empty(2 * len(w))
    ww[0::2], ww[1::2] = w.real, w.imag
    p = Poles(len(sigma), s.ctypes.data_as(C.POINTER(C.c_double)),
              ww.ctypes.data_as(C.POINTER(C.c_double)))
    return p, (s, ww)


def _union_nnz(A, B) -> int:
    return int((abs(A) + abs(B)).nnz) if (A.nnz != B.nnz or (A.indices != B.indices).any()) else int(A.nnz)


def _csr_arrays(A, B):
    """Sorted CSR of A and B as the six host arrays the C ABI takes, plus n and the union nnz."""
    A = A.tocsr()
    B = B.tocsr()
    A.sort_indices()
    B.sort_indices()
    arrs = [np.ascontiguousarray(x) for x in (
        A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64),
        B.indptr.astype(np.int32), B.indices.astype(np.int32), B.data.astype(np.float64))]
    return A.shape[0], _union_nnz(A, B), arrs


@dataclass
class SolveResult:
    status: int
    evals: np.ndarray      # all L Ritz values, ascending
    evecs: object          # torch (n, L) float64 on the device
    resid: np.ndarray      # rho_i of all L Ritz pairs
    n_found: int
    stats: dict
    message: str


class Solver:
    """A context over one pencil (A, B) with a workspace sized for (max_L, max_poles)."""

    def __init__(self, A, B, max_L: int, max_poles: int, options: Options | None = None,
                 device: str = "cuda:0", stream=None, static_scratch: bool = False, workspace=None):
        """static_scratch: build the context with slrf_create_static (no workspace
        tensor; the library's per-device static array instead).  workspace: a
        caller-owned uint8 tensor on the device of at least workspace_bytes(...)
        bytes (default: one is allocated); the context uses it until close()."""
        import torch
        self.torch = torch
        self.n, nnz, arrs = _csr_arrays(A, B)
        self.device = torch.device(device)
        self.options = options or default_options()
        self.stream = stream or torch.cuda.current_stream(self.device)
        self._h = C.c_void_p()
        if static_scratch:
            self.ws_bytes, self.workspace = 0, None
            with torch.cuda.device(self.device):
                st = _lib.slrf_create_static(C.byref(self._h), self.n, *[_ptr(a) for a in arrs], max_L,
                                             max_poles, C.byref(self.options),
                                             C.c_void_p(self.stream.cuda_stream))
        else:
            self.ws_bytes = workspace_bytes(self.n, nnz, max_L, max_poles, options=self.options)
            if workspace is None:
                workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            elif (workspace.dtype != torch.uint8 or workspace.device != self.device
                  or not workspace.is_contiguous() or workspace.numel() < self.ws_bytes):
                raise ValueError(f"workspace must be a contiguous uint8 tensor on {self.device} "
                                 f"of at least {self.ws_bytes} bytes")
            self.workspace = workspace
            st = _lib.slrf_create(C.byref(self._h), self.n, *[_ptr(a) for a in arrs],
                                  C.c_void_p(self.workspace.data_ptr()), self.ws_bytes, max_L, max_poles,
                                  C.byref(self.options), C.c_void_p(self.stream.cuda_stream))
        if st:
            msg = self.last_error()
            self.close()
            raise SlrfError(st, msg)

    def last_error(self) -> str:
        if not self._h:
            return ""
        return _lib.slrf_last_error(self._h).decode()

    def close(self):
        if self._h:
            _lib.slrf_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, X):
        t = self.torch
        if not isinstance(X, t.Tensor):
            X = t.as_tensor(np.ascontiguousarray(X, dtype=np.float64))
        return X.to(device=self.device, dtype=t.float64).contiguous()

    def filter_apply(self, X, sigma, w):  # noqa: D401
        """U = sum_j 2 Re(w_j (A - sigma_j B)^{-1} B X); returns (U, stats dict)."""
        X = self._dev(X)
        n, L = X.shape
        U = self.torch.empty_like(X)
        p, keep = _poles_struct(sigma, w)
        stats = FilterStats()
        st = _lib.slrf_filter_apply(self._h, C.byref(p), L, C.c_void_p(X.data_ptr()),
                                    C.c_void_p(U.data_ptr()), C.byref(stats))
        if st:
            raise SlrfError(st, self.last_error())
        return U, stats.as_dict()

    def solve_interval(self, gamma: float, L: int, sigma=None, w=None, V0=None,
                       raise_on_error: bool = True) -> SolveResult:
        t = self.torch
        evecs = t.empty((self.n, L), dtype=t.float64, device=self.device)
        evals = np.zeros(L)
        resid = np.zeros(L)
        nf = C.c_int64()
        stats = SolveStats()
        pp = None
        keep = None
        if sigma is not None:
            p, keep = _poles_struct(sigma, w)
            pp = C.byref(p)
        v0 = None
        if V0 is not None:
            v0 = self._dev(V0)
        st = _lib.slrf_solve_interval(self._h, gamma, L, pp,
                                      C.c_void_p(v0.data_ptr()) if v0 is not None else None,
                                      C.byref(nf), _ptr(evals), C.c_void_p(evecs.data_ptr()),
                                      _ptr(resid), C.byref(stats))
        msg = self.last_error() if st else ""
        if st and raise_on_error and st not in (5,):
            raise SlrfError(st, msg)
        return SolveResult(st, evals, evecs, resid, nf.value, stats.as_dict(), msg)


def batch_footprint(n: int, nnz: int, L: int, N: int, precision: int = FP64, options: Options | None = None):
    """(persistent, transient) device bytes of one pencil in a Batch (with options:
    for their precision and preconditioner; precision is then ignored)."""
    p, t = C.c_size_t(), C.c_size_t()
    if options is None:
        st = _lib.slrf_batch_footprint(n, nnz, L, N, precision, C.byref(p), C.byref(t))
    else:
        st = _lib.slrf_batch_footprint_for(n, nnz, L, N, C.byref(options), C.byref(p), C.byref(t))
    if st:
        raise SlrfError(st, "batch footprint")
    return p.value, t.value


class Batch:
    """Many pencils solved together: one batched Krylov launch per step for all
    unfinished pencils; pencils may join between steps and leave when done."""

    def __init__(self, ws_bytes: int, arena_bytes: int, max_poles: int = 4,
                 options: Options | None = None, device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.options = options or default_options()
        self.ws_bytes = int(ws_bytes)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self._h = C.c_void_p()
        self.n_of = {}
        self.L_of = {}
        st = _lib.slrf_batch_create(C.byref(self._h), C.c_void_p(self.workspace.data_ptr()),
                                    self.ws_bytes, int(arena_bytes), max_poles,
                                    C.byref(self.options), C.c_void_p(self.stream.cuda_stream))
        if st:
            msg = self.last_error()
            self.close()
            raise SlrfError(st, msg)

    def last_error(self) -> str:
        if not self._h:
            return ""
        return _lib.slrf_batch_last_error(self._h).decode()

    def close(self):
        if self._h:
            _lib.slrf_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, A, B, gamma: float, L: int, sigma=None, w=None, V0=None, must_fit: bool = True):
        """Adds a pencil; returns its id, or None when it does not fit and must_fit is False."""
        t = self.torch
        n, _, arrs = _csr_arrays(A, B)
        pp = None
        keep = None
        if sigma is not None:
            p, keep = _poles_struct(sigma, w)
            pp = C.byref(p)
        v0 = None
        if V0 is not None:
            if not isinstance(V0, t.Tensor):
                V0 = t.as_tensor(np.ascontiguousarray(V0, dtype=np.float64))
            v0 = V0.to(device=self.device, dtype=t.float64).contiguous()
        pid = C.c_int32()
        st = _lib.slrf_batch_add(self._h, n, *[_ptr(a) for a in arrs], gamma, L, pp,
                                 C.c_void_p(v0.data_ptr()) if v0 is not None else None, C.byref(pid))
        del keep
        if st == 3 and not must_fit:
            return None
        if st:
            raise SlrfError(st, self.last_error())
        self.n_of[pid.value] = n
        self.L_of[pid.value] = L
        return pid.value

    def step(self) -> int:
        act = C.c_int32()
        st = _lib.slrf_batch_step(self._h, C.byref(act))
        if st:
            raise SlrfError(st, self.last_error())
        return act.value

    def query(self, pid: int):
        """(done, outer iterations so far)."""
        d, k = C.c_int32(), C.c_int32()
        st = _lib.slrf_batch_query(self._h, pid, C.byref(d), C.byref(k))
        if st:
            raise SlrfError(st, self.last_error())
        return bool(d.value), k.value

    def result(self, pid: int) -> SolveResult:
        t = self.torch
        n, L = self.n_of[pid], self.L_of[pid]
        evecs = t.empty((n, L), dtype=t.float64, device=self.device)
        evals = np.zeros(L)
        resid = np.zeros(L)
        nf = C.c_int64()
        stats = SolveStats()
        st = _lib.slrf_batch_result(self._h, pid, C.byref(nf), _ptr(evals), C.c_void_p(evecs.data_ptr()),
                                    _ptr(resid), C.byref(stats))
        msg = self.last_error() if st else ""
        return SolveResult(st, evals, evecs, resid, nf.value, stats.as_dict(), msg)

    def restart(self, pid: int, V0=None):
        """Solve the pencil again from V0 (device (n, L) or host array; None: the
        seeded Gaussian block), keeping its device data."""
        v0 = None
        if V0 is not None:
            t = self.torch
            v0 = V0 if isinstance(V0, t.Tensor) else t.as_tensor(np.ascontiguousarray(V0, dtype=np.float64))
            v0 = v0.to(device=self.device, dtype=t.float64).contiguous()
        st = _lib.slrf_batch_restart(self._h, pid, C.c_void_p(v0.data_ptr()) if v0 is not None else None)
        if st:
            raise SlrfError(st, self.last_error())

    def remove(self, pid: int):
        st = _lib.slrf_batch_remove(self._h, pid)
        if st:
            raise SlrfError(st, self.last_error())
        self.n_of.pop(pid, None)
        self.L_of.pop(pid, None)
