"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle and
closed forms.  Sizes span several 256-row blocks and 64-column tiles with ragged
tails."""
import json
import os

import numpy as np
import pytest

import pencils
from closed_forms import closed_1d, closed_3d_cc
from oracle import dense, inertia, krylov
from oracle import filter as oflt

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def slrf(torch):
    import paper_2503_21618_amd as m
    return m


def say(*a):
    print(*a, flush=True)


def golden_poles(N, gamma):
    with open(os.path.join(GOLDEN, f"poles_N{N}_a1_b0.01.json")) as f:
        d = json.load(f)
    return ((np.array(d["sigma_re"]) + 1j * np.array(d["sigma_im"])) * gamma,
            (np.array(d["w_re"]) + 1j * np.array(d["w_im"])) * gamma)


@pytest.mark.parametrize("iters", [1, 3, 8])
def test_bicgstab_iterates_match_oracle(slrf, torch, iters):
    """After exactly `iters` BiCGStab iterations (tol 0) the filtered block equals the
    oracle's BiCGStab iterate pushed through the same filter sum."""
    q = pencils.scalar_q1(12, 3, 0.5, 21)           # n = 1331: 6 row blocks, ragged
    L = 40                                          # K = 80: 2 column tiles, ragged
    gamma = 300.0
    sig, w = golden_poles(4, gamma)
    sig, w = sig[:2], w[:2]
    X = pencils.start_block(q.n, L, 5)
    say(f"case iterates iters={iters} n={q.n} L={L} N=2")
    opt = slrf.default_options(inner_tol=0.0, inner_maxit=iters, check_every=1)
    s = slrf.Solver(q.A, q.B, max_L=L, max_poles=2, options=opt)
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    U = U.cpu().numpy()
    F = q.B @ X
    x, it, fl, _ = krylov.bicgstab(q.A, q.B, sig, F, 0.0, iters, fixed_iters=iters)
    Uo = sum(2.0 * np.real(w[j] * x[:, j * L:(j + 1) * L]) for j in range(2))
    err = np.abs(U - Uo).max() / np.abs(Uo).max()
    say(f"  rel err {err:.3e}, its max {st['max_iterations']}, n_maxit {st['n_maxit']}")
    assert st["max_iterations"] == iters and st["n_maxit"] == 2 * L
    # rounding-order differences grow through the data-dependent BiCGStab scalars
    assert err < max(1e-12, 1e-13 * 3.0 ** iters)


def test_filter_apply_converged_matches_exact_solve(slrf, torch):
    n = 2000
    p = pencils.c1_string()
    lam, _ = closed_1d(n)
    gamma = 0.5 * (lam[19] + lam[20])
    sig, w = golden_poles(4, gamma)
    X = pencils.start_block(n, 32, 1)
    say("case filter C1 converged")
    s = slrf.Solver(p.A, p.B, max_L=32, max_poles=4, options=slrf.default_options(inner_tol=1e-12))
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    Uo, _ = oflt.filter_apply(p.A, p.B, X, sig, w)
    err = np.abs(U.cpu().numpy() - Uo).max() / np.abs(Uo).max()
    say(f"  rel err {err:.3e}, mean its {st['mean_iterations']:.1f}, spmv {st['spmv']}")
    assert st["n_maxit"] == 0 and st["n_breakdown"] == 0
    assert st["max_relres"] <= 1e-12
    assert err < 1e-8


def test_filter_apply_closed_form_eigenvectors(slrf, torch):
    """Phi(A, B) x_k = Phi(lambda_k) x_k with closed-form 1D eigenvectors."""
    n = 777
    p = pencils.string_1d(n)
    lam, Xc = closed_1d(n)
    gamma = 0.5 * (lam[14] + lam[15])
    sig, w = golden_poles(4, gamma)
    ks = list(range(0, 70))                          # 70 columns: 2 tiles, ragged
    X = Xc[:, ks]
    say("case filter closed form")
    s = slrf.Solver(p.A, p.B, max_L=70, max_poles=4, options=slrf.default_options(inner_tol=1e-12))
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    phi = (2.0 * np.real(w[None, :] / (lam[ks][:, None] - sig[None, :]))).sum(1)
    err = np.abs(U.cpu().numpy() - X * phi[None, :]).max() / np.abs(X).max()
    say(f"  abs err / max|x| {err:.3e}")
    assert err < 1e-9


def test_filter_zero_column(slrf, torch):
    q = pencils.scalar_q1(8, 3, 0.5, 2)
    X = pencils.start_block(q.n, 8, 3)
    X[:, 3] = 0.0
    sig, w = golden_poles(4, 200.0)
    say("case zero column")
    s = slrf.Solver(q.A, q.B, max_L=8, max_poles=4)
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    U = U.cpu().numpy()
    assert np.all(np.isfinite(U)) and np.all(U[:, 3] == 0.0)


def test_filter_rejects_bad_poles(slrf, torch):
    q = pencils.scalar_q1(6, 3)
    s = slrf.Solver(q.A, q.B, max_L=4, max_poles=2)
    X = torch.zeros((q.n, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(slrf.SlrfError):
        s.filter_apply(X, np.array([10.0 - 5j]), np.array([1.0 + 0j]))    # lower half plane
    with pytest.raises(slrf.SlrfError):
        s.filter_apply(X, np.array([1 + 1j, 2 + 2j, 3 + 3j]), np.ones(3))  # more than max_poles


def test_solve_c1_closed_form(slrf, torch):
    n = 2000
    p = pencils.c1_string()
    lam, _ = closed_1d(n)
    gamma = 0.5 * (lam[19] + lam[20])
    sig, w = golden_poles(4, gamma)
    V0 = pencils.start_block(n, 32, 1)
    say("case solve C1")
    s = slrf.Solver(p.A, p.B, max_L=32, max_poles=4)
    r = s.solve_interval(gamma, 32, sig, w, V0=torch.from_numpy(V0).cuda())
    nf = r.n_found
    X = r.evecs.cpu().numpy()[:, :nf]
    rel = np.abs(r.evals[:nf] / lam[:nf] - 1).max()
    orth = np.abs(X.T @ (p.B @ X) - np.eye(nf)).max()
    say(f"  found {nf}, rel eig err {rel:.3e}, max rho {r.resid[:nf].max():.3e}, orth {orth:.2e}, "
        f"outer {r.stats['outer_iterations']}, spmv {r.stats['spmv_total']}")
    assert r.status == 0
    assert nf == 20 == inertia.sturm_count_tridiagonal(p.A, p.B, gamma)
    assert rel < 1e-10
    assert r.resid[:nf].max() <= 1e-8
    assert orth < 1e-10
    # residuals recomputed on the host from the returned pairs
    rho = np.linalg.norm(p.A @ X - (p.B @ X) * r.evals[:nf], axis=0) / (
        r.evals[:nf] * np.linalg.norm(p.B @ X, axis=0))
    assert rho.max() <= 1.01e-8


def test_solve_3d_lognormal_vs_dense_oracle(slrf, torch):
    q = pencils.scalar_q1(12, 3, 0.5, 31)            # n = 1331
    ev, Xd = dense.all_eigenpairs(q.A, q.B)
    gamma = 0.5 * (ev[29] + ev[30])
    L = 40
    say("case solve 3D log-normal small")
    s = slrf.Solver(q.A, q.B, max_L=L, max_poles=4)
    r = s.solve_interval(gamma, L, V0=torch.from_numpy(pencils.start_block(q.n, L, 4)).cuda())
    nf = r.n_found
    X = r.evecs.cpu().numpy()[:, :nf]
    rel = np.abs(r.evals[:nf] / ev[:nf] - 1).max()
    say(f"  found {nf}, rel eig err {rel:.3e}, max rho {r.resid[:nf].max():.3e}")
    assert r.status == 0 and nf == 30 == inertia.sparse_ldl_count(q.A, q.B, gamma)
    assert rel < 1e-10
    # eigenvectors: sign-invariant overlap for well-separated eigenvalues
    gaps = np.minimum(np.diff(ev[:31])[:-1], np.diff(ev[:31])[1:]) / ev[1:30]
    simple = np.concatenate([[True], gaps > 1e-3])[:nf]
    ov = np.abs(np.sum(X * (q.B @ Xd[:, :nf]), axis=0))
    assert np.abs(ov[simple] - 1).max() < 1e-7


def test_solve_3d_constant_coefficient_closed_form(slrf, torch):
    m = 16                                           # n = 3375
    q = pencils.scalar_q1(m, 3)
    lam = closed_3d_cc(m)
    # gamma in the middle of a gap of the closed-form spectrum above ~40 eigenvalues
    gaps = np.where(np.diff(lam[:60]) / lam[1:60] > 0.02)[0]
    k = gaps[np.argmin(np.abs(gaps - 40))]
    gamma = 0.5 * (lam[k] + lam[k + 1])
    nev = k + 1
    L = int(np.ceil(1.3 * nev / 8) * 8)
    say(f"case solve 3D cc m={m} nev={nev} L={L}")
    s = slrf.Solver(q.A, q.B, max_L=L, max_poles=4)
    r = s.solve_interval(gamma, L)                   # seeded start block on the device
    nf = r.n_found
    rel = np.abs(r.evals[:nf] / lam[:nf] - 1).max()
    say(f"  found {nf}, rel eig err {rel:.3e}, max rho {r.resid[:nf].max():.3e}")
    assert r.status == 0 and nf == nev
    assert rel < 1e-10


@pytest.mark.parametrize("n,L", [(1000, 40), (3001, 128), (777, 200)])
def test_mfma_gram_kernel(slrf, torch, n, L):
    rng = np.random.default_rng(n + L)
    U, WA, WB = (rng.standard_normal((n, L)) for _ in range(3))
    say(f"case gram n={n} L={L}")
    GA, GB = slrf.test_gram(*(torch.from_numpy(x).cuda() for x in (U, WA, WB)))
    ea = np.abs(GA.cpu().numpy() - U.T @ WA).max()
    eb = np.abs(GB.cpu().numpy() - U.T @ WB).max()
    say(f"  err {ea:.2e} {eb:.2e}")
    assert ea < 1e-11 * n and eb < 1e-11 * n


@pytest.mark.parametrize("n,L,r", [(1000, 40, 40), (3001, 128, 128), (777, 200, 136)])
def test_mfma_gemm_kernel(slrf, torch, n, L, r):
    rng = np.random.default_rng(n + L + r)
    X = rng.standard_normal((n, L))
    Z = rng.standard_normal((L, r))
    say(f"case gemm n={n} L={L} r={r}")
    Y = slrf.test_gemm(torch.from_numpy(X).cuda(), torch.from_numpy(Z).cuda())
    e = np.abs(Y.cpu().numpy() - X @ Z).max()
    say(f"  err {e:.2e}")
    assert e < 1e-12 * L * 10


@pytest.mark.parametrize("n,L", [(1000, 40), (3001, 128), (777, 200)])
def test_mfma_gram_kernel_f32(slrf, torch, n, L):
    """The FP32 MFMA Gram (first projection of a mixed-precision outer
    iteration): the products of the inputs rounded to FP32, with the error of
    FP32 accumulation, |err| <= 1e-5 (|U|^T |W|) elementwise.  A wrong
    accumulator layout would misplace whole 16 x 16 tiles."""
    rng = np.random.default_rng(n + L + 1)
    U, WA, WB = (rng.standard_normal((n, L)) for _ in range(3))
    say(f"case gram fp32 n={n} L={L}")
    GA, GB = slrf.test_gram(*(torch.from_numpy(x).cuda() for x in (U, WA, WB)), f32=True)
    r = lambda a: a.astype(np.float32).astype(np.float64)
    for G, W in ((GA, WA), (GB, WB)):
        ref = r(U).T @ r(W)
        bound = 1e-5 * (np.abs(U).T @ np.abs(W))
        err = np.abs(G.cpu().numpy() - ref)
        say(f"  max err / bound {(err / bound).max():.3f}")
        assert np.all(err <= bound)


@pytest.mark.parametrize("iters", [1, 2, 5])
def test_bicgstab_ilu0_iterates_match_oracle(slrf, torch, iters):
    """ILU(0)-preconditioned iterates (narrow pattern) against the oracle's."""
    n, L = 517, 40
    p = pencils.string_1d(n)
    lam, _ = closed_1d(n)
    sig, w = golden_poles(4, 0.5 * (lam[9] + lam[10]))
    sig, w = sig[:3], w[:3]
    X = pencils.start_block(n, L, 8)
    # bands at +-3 (nnz <= 5 n): ILU(0) drops the fill at +-2, so it is not exact
    import scipy.sparse as sp
    A = (p.A + sp.diags([np.full(n - 3, 0.02 * (n + 1))] * 2, [-3, 3])).tocsr()
    say(f"case ilu0 iterates iters={iters}")
    opt = slrf.default_options(inner_tol=0.0, inner_maxit=iters, check_every=1, precond=2)
    s = slrf.Solver(A, p.B, max_L=L, max_poles=3, options=opt)
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    x, it, fl, _ = krylov.bicgstab(A, p.B, sig, p.B @ X, 0.0, iters, fixed_iters=iters, precond="ilu0")
    Uo = sum(2.0 * np.real(w[j] * x[:, j * L:(j + 1) * L]) for j in range(3))
    err = np.abs(U.cpu().numpy() - Uo).max() / np.abs(Uo).max()
    say(f"  rel err {err:.3e}, its {st['max_iterations']}")
    assert st["max_iterations"] == iters
    assert err < max(1e-11, 1e-13 * 3.0 ** iters)
