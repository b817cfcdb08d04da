"""CPU checks of the compiled C-ABI library: exports, host-only entry points,
argument validation.  No GPU compute is called here."""
import ctypes as C
import json
import os
import re

import numpy as np
import scipy.sparse as sp
import pytest

import pencils

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


@pytest.fixture(scope="module")
def lib():
    import paper_2503_21618_amd as m
    return m


def header_symbols(name="slrf.h"):
    txt = open(os.path.join(ROOT, "include", name)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(slrf_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(lib):
    syms = header_symbols()
    assert len(syms) >= 9
    for s in syms:
        assert hasattr(lib._lib, s), s
    assert set(syms) == set(lib.EXPORTED)
    tsyms = header_symbols("slrf_testing.h")
    assert set(tsyms) == set(lib.TESTING_EXPORTED)
    for s in tsyms:
        assert hasattr(lib._lib, s), s


def test_default_options(lib):
    o = lib.default_options()
    assert o.precision == lib.FP64 and o.inner_maxit == 1000 and o.outer_tol == 1e-8
    assert o.solver == lib.SOLVER_BICGSTAB and o.recycle == 0


@pytest.mark.parametrize("rule", [0, 1, 2])
def test_quadrature_poles_match_oracle(lib, rule):
    """Section 3.2 quadrature filters: the library's host rule (Newton iteration
    for the Gauss-Legendre nodes) against the oracle's (numpy's leggauss)."""
    from oracle import poles
    name = {0: "midpoint", 1: "gauss-legendre", 2: "gauss-chebyshev"}[rule]
    for N in (1, 3, 4, 8, 16):
        s, w = lib.quadrature_poles(rule, N, 2.5)
        so, wo = poles.circle_quadrature(N, name, 2.5)
        assert np.abs(s - so).max() < 1e-14 * 2.5
        assert np.abs(w - wo).max() < 1e-14 * 2.5
    with pytest.raises(lib.SlrfError):
        lib.quadrature_poles(3, 4, 1.0)
    with pytest.raises(lib.SlrfError):
        lib.quadrature_poles(rule, 0, 1.0)


@pytest.mark.parametrize("N", [4, 6, 8])
def test_design_matches_oracle_tables(lib, N):
    """Product pole design (host C++) vs the oracle's design (stored tables).

    Section 3.1 admits abscissae x_j in (0, gamma], closed at gamma.  The N = 4
    optimum is interior and both designers reach it: tight tolerances.  For
    N = 6 and 8 the fit is flat along the largest abscissa near x = gamma: the
    product's Levenberg-Marquardt reaches x = gamma to rounding while SciPy's
    stops just inside; there the product's objective must be no worse than the
    oracle's and close to it, with the same arrangement of poles and the same
    separation factor."""
    with open(os.path.join(GOLDEN, f"poles_N{N}_a1_b0.01.json")) as f:
        d = json.load(f)
    s_or = np.array(d["sigma_re"]) + 1j * np.array(d["sigma_im"])
    w_or = np.array(d["w_re"]) + 1j * np.array(d["w_im"])
    s, w, sep = lib.design_poles(N, 1.0, 0.01, 1.0)
    from oracle import poles
    rows = poles.trapezoid_rows(0.01)
    J_prod = poles.objective(s.real, 1.0, rows)
    J_or = poles.objective(s_or.real, 1.0, rows)
    assert J_prod <= J_or * (1 + 1e-9)
    assert abs(sep - d["separation_factor"]) < 1e-3 * d["separation_factor"]
    if N == 4:
        assert np.abs(s - s_or).max() < 2e-5
        assert np.abs(w - w_or).max() < 1e-4 * np.abs(w_or).max()
    else:
        assert J_prod >= J_or * (1 - 1e-4)
        assert s.real.max() > 0.995 and s_or.real.max() > 0.995   # the end of the admissible range
        assert np.abs(s - s_or).max() < 5e-3
        assert np.abs(w - w_or).max() < 0.1 * np.abs(w_or).max()


def test_design_gamma_scaling(lib):
    s1, w1, _ = lib.design_poles(2, 1.0, 0.01, 1.0)
    s2, w2, _ = lib.design_poles(2, 1.0, 0.01, 421.0)
    assert np.abs(s2 / 421.0 - s1).max() < 1e-14
    assert np.abs(w2 / 421.0 - w1).max() < 1e-14
    assert np.all(s1.imag == s1.real)  # alpha = 1 line


def test_design_rejects_bad_args(lib):
    for args in [(0, 1.0, 0.01, 1.0), (2, -1.0, 0.01, 1.0), (2, 1.0, 0.0, 1.0), (2, 1.0, 0.01, 0.0)]:
        with pytest.raises(lib.SlrfError):
            lib.design_poles(*args)


def test_workspace_bytes_monotone(lib):
    a = lib.workspace_bytes(1000, 3000, 16, 2)
    b = lib.workspace_bytes(1000, 3000, 32, 2)
    c = lib.workspace_bytes(1000, 3000, 32, 4)
    assert 0 < a < b < c
    with pytest.raises(lib.SlrfError):
        lib.workspace_bytes(0, 3000, 16, 2)


def test_warm_start_blocks_in_the_sizes(lib):
    """Warm starts keep each pencil's previous Y (n x N L complex FP64, the mixed
    form's columns padded to whole tiles of 128) and B X (n x L real FP64): the
    workspace with recycle = 1 and the mixed batch footprint hold at least that
    much more than without."""
    n, nnz, L, N = 5000, 5000 * 27, 40, 6
    kp = -(-N * L // 128) * 128
    need = n * kp * 16 + n * L * 8
    cold = lib.workspace_bytes(n, nnz, L, N, options=lib.default_options(precision=lib.MIXED, recycle=0))
    warm = lib.workspace_bytes(n, nnz, L, N, options=lib.default_options(precision=lib.MIXED, recycle=1))
    assert need <= warm - cold <= need + 4096
    f64, _ = lib.batch_footprint(n, nnz, L, N, lib.FP64)
    mixed, _ = lib.batch_footprint(n, nnz, L, N, lib.MIXED)
    assert need <= mixed - f64 <= need + 4096


def _create(lib, A, B, ws_ptr=0x100000, ws_bytes=1 << 40):
    """slrf_create with a fake device pointer: validation runs before any device use."""
    arrs = [np.ascontiguousarray(x) for x in (
        A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64),
        B.indptr.astype(np.int32), B.indices.astype(np.int32), B.data.astype(np.float64))]
    h = C.c_void_p()
    opt = lib.default_options()
    st = lib._lib.slrf_create(C.byref(h), A.shape[0], *[a.ctypes.data_as(C.c_void_p) for a in arrs],
                              C.c_void_p(ws_ptr), ws_bytes, 8, 2, C.byref(opt), None)
    msg = lib._lib.slrf_last_error(h).decode() if h else ""
    if h:
        lib._lib.slrf_destroy(h)
    return st, msg


def test_create_rejects_bad_matrices(lib):
    p = pencils.string_1d(20)
    B0 = p.B.copy()
    B0.data[B0.indptr[3]:B0.indptr[4]] *= 0.0          # zero row => zero diagonal
    st, msg = _create(lib, p.A, B0)
    assert st == 2 and "diagonal" in msg
    An = p.A.copy()
    An.data[5] = np.nan
    st, msg = _create(lib, An, p.B)
    assert st == 1 and "non-finite" in msg
    Au = p.A.copy()
    Au.indices[Au.indptr[5]], Au.indices[Au.indptr[5] + 1] = Au.indices[Au.indptr[5] + 1], Au.indices[Au.indptr[5]]
    st, msg = _create(lib, Au, p.B)
    assert st == 1 and "increasing" in msg
    st, msg = _create(lib, p.A, p.B, ws_ptr=0x100001)
    assert st == 3
    st, msg = _create(lib, p.A, p.B, ws_bytes=1024)
    assert st == 3 and "needs" in msg


def test_create_rejects_non_symmetric_pencils(lib):
    """A and B must be symmetric (the pencil of Section 1): entry (i, j) against
    (j, i) to 1e-10 of sqrt(m_ii m_jj), an entry stored on one side only
    counting as zero.  Accepted pencils pass on to the workspace-size check."""
    p = pencils.string_1d(20)
    Aa = p.A.tolil()
    Aa[0, 1] = Aa[0, 1] * (1 + 1e-6)                  # relative 1e-6: rejected
    st, msg = _create(lib, Aa.tocsr(), p.B, ws_bytes=1024)
    assert st == 1 and "A is not symmetric" in msg and "(0, 1)" in msg
    Bb = p.B.tolil()
    Bb[0, 5] = 1e-3 * Bb[0, 0]                        # stored on one side only
    st, msg = _create(lib, p.A, Bb.tocsr(), ws_bytes=1024)
    assert st == 1 and "B is not symmetric" in msg
    Az = p.A.tocoo()
    Az = sp.csr_matrix((np.append(Az.data, 0.0), (np.append(Az.row, 0), np.append(Az.col, 7))), shape=Az.shape)
    assert Az.nnz == p.A.nnz + 1                      # an explicit zero at (0, 7) only: accepted
    st, msg = _create(lib, Az, p.B, ws_bytes=1024)
    assert st == 3 and "needs" in msg
    Ar = p.A.tolil()
    Ar[0, 1] = Ar[0, 1] * (1 + 1e-14)                 # rounding-level asymmetry: accepted
    st, msg = _create(lib, Ar.tocsr(), p.B, ws_bytes=1024)
    assert st == 3 and "needs" in msg


def test_batch_footprint_monotone(lib):
    p0, t0 = lib.batch_footprint(10000, 70000, 16, 4, lib.FP64)
    p1, t1 = lib.batch_footprint(10000, 70000, 32, 4, lib.FP64)
    p2, t2 = lib.batch_footprint(10000, 70000, 32, 6, lib.FP64)
    assert 0 < p0 < p1 and p1 == p2 and 0 < t0 < t1 < t2
    pm, tm = lib.batch_footprint(10000, 70000, 32, 6, lib.MIXED)
    assert tm != t2
    # a one-pencil context needs no more than persistent + transient (+ timer
    # counters); for an ILU(0)-sized pattern the two agree
    ws = lib.workspace_bytes(10000, 70000, 32, 6, lib.FP64)
    assert ws <= p2 + t2 + 8192
    pi, ti = lib.batch_footprint(10000, 30000, 32, 6, lib.FP64)
    wi = lib.workspace_bytes(10000, 30000, 32, 6, lib.FP64)
    assert pi + ti <= wi <= pi + ti + 8192
    with pytest.raises(lib.SlrfError):
        lib.batch_footprint(0, 1, 1, 1)


def test_batch_create_and_add_validate_before_device_use(lib):
    opt = lib.default_options()
    h = C.c_void_p()
    # misaligned and too-small workspaces are refused
    st = lib._lib.slrf_batch_create(C.byref(h), C.c_void_p(0x100001), 1 << 30, 1 << 20, 4, C.byref(opt), None)
    assert st == 3 and "aligned" in lib._lib.slrf_batch_last_error(h).decode()
    lib._lib.slrf_batch_destroy(h)
    st = lib._lib.slrf_batch_create(C.byref(h), C.c_void_p(0x100000), 1 << 20, 1 << 24, 4, C.byref(opt), None)
    assert st == 3
    lib._lib.slrf_batch_destroy(h)
    st = lib._lib.slrf_batch_create(C.byref(h), C.c_void_p(0x100000), 1 << 30, 1 << 20, 0, C.byref(opt), None)
    assert st == 1
    lib._lib.slrf_batch_destroy(h)
    # a valid batch over a fake pointer: add rejects bad matrices before touching memory
    st = lib._lib.slrf_batch_create(C.byref(h), C.c_void_p(0x100000), 1 << 30, 1 << 20, 4, C.byref(opt), None)
    assert st == 0
    p = pencils.string_1d(50)
    B0 = p.B.tolil()
    B0[3, 3] = 0.0
    B0 = B0.tocsr()
    n, _, arrs = lib.binding._csr_arrays(p.A, B0)
    pid = C.c_int32(-1)
    st = lib._lib.slrf_batch_add(h, n, *[a.ctypes.data_as(C.c_void_p) for a in arrs], 1.0, 8, None, None,
                                 C.byref(pid))
    assert st == 2 and "diagonal" in lib._lib.slrf_batch_last_error(h).decode()
    n, _, arrs = lib.binding._csr_arrays(p.A, p.B)
    st = lib._lib.slrf_batch_add(h, n, *[a.ctypes.data_as(C.c_void_p) for a in arrs], -1.0, 8, None, None,
                                 C.byref(pid))
    assert st == 1
    # a pencil whose filter arena exceeds the batch's arena is refused before upload
    q = pencils.scalar_q1(40, 3)
    n, _, arrs = lib.binding._csr_arrays(q.A, q.B)
    st = lib._lib.slrf_batch_add(h, n, *[a.ctypes.data_as(C.c_void_p) for a in arrs], 1.0, 64, None, None,
                                 C.byref(pid))
    assert st == 3 and "arena" in lib._lib.slrf_batch_last_error(h).decode()
    st = lib._lib.slrf_batch_step(h, None)  # nothing to do: no device call
    assert st == 0
    assert lib._lib.slrf_batch_remove(h, 7) == 1
    lib._lib.slrf_batch_destroy(h)


def test_sgs_options_validated_on_the_host(lib):
    """The multicolour SGS preconditioner (4 point, 5 node blocks) runs with COCG
    only; the size query refuses it with BiCGStab and counts its colour tables."""
    n, nnz, L, N = 3000, 3000 * 27, 32, 4
    with pytest.raises(lib.SlrfError):
        lib.workspace_bytes(n, nnz, L, N, options=lib.default_options(solver=lib.SOLVER_BICGSTAB, precond=4))
    with pytest.raises(lib.SlrfError):
        lib.workspace_bytes(n, nnz, L, N, options=lib.default_options(solver=lib.SOLVER_COCG, precond=6))
    for bad in (-0.5, 2.0, 2.5, float("nan")):       # the SOR relaxation factor lies in (0, 2)
        with pytest.raises(lib.SlrfError):
            lib.workspace_bytes(n, nnz, L, N, options=lib.default_options(solver=lib.SOLVER_COCG, precond=4,
                                                                           sgs_omega=bad))
    assert lib.default_options().sgs_omega == 0.0                # by block size
    w07 = lib.workspace_bytes(n, nnz, L, N, options=lib.default_options(solver=lib.SOLVER_COCG, precond=4,
                                                                         sgs_omega=0.7))
    jac = lib.workspace_bytes(n, nnz, L, N, options=lib.default_options(solver=lib.SOLVER_COCG, precond=1))
    sgs = lib.workspace_bytes(n, nnz, L, N, options=lib.default_options(solver=lib.SOLVER_COCG, precond=4))
    # two coupling CSRs ((a, b) in FP64 and FP32, column index) within the merged pattern's
    # size, their row pointers, the colour tables, and R = sqrt(d) per (row, pole)
    assert 0 < sgs - jac < 2 * (nnz + 16) * 28 + 4 * (n + 1) * 4 + 1025 * 4 + n * N * 16 + 2 ** 16
    assert w07 == sgs                                # the relaxation changes values, not sizes
