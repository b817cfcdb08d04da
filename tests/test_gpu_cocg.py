"""GPU parity of the COCG inner solver (options.solver = 1, point or node block
Jacobi) against the oracle's COCG (iterates after a fixed number of steps), the
direct solve of the shifted systems (converged filter, FP64 and mixed), and the
dense FP64 oracle with the inertia count (complete interval solves)."""
import json
import os

import numpy as np
import pytest

import pencils
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
def test_cocg_iterates_match_oracle(slrf, torch, iters):
    """After exactly `iters` COCG steps (tol 0) the filtered block equals the
    oracle's COCG iterate pushed through the same filter sum."""
    q = pencils.scalar_q1(12, 3, 0.5, 21)           # n = 1331: several row blocks, ragged
    L = 40                                          # K = 80 per pole pair: ragged tiles
    sig, w = golden_poles(4, 300.0)
    sig, w = sig[:2], w[:2]
    X = pencils.start_block(q.n, L, 5)
    say(f"case COCG iterates iters={iters} n={q.n} L={L} N=2")
    opt = slrf.default_options(inner_tol=0.0, inner_maxit=iters, check_every=1, solver=slrf.SOLVER_COCG)
    s = slrf.Solver(q.A, q.B, max_L=L, max_poles=2, options=opt)
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    U = U.cpu().numpy()
    x, it, fl, _ = krylov.cocg(q.A, q.B, sig, q.B @ X, 0.0, iters, fixed_iters=iters)
    Uo = sum(2.0 * np.real(w[j] * x[:, j * L:(j + 1) * L]) for j in range(2))
    err = np.abs(U - Uo).max() / np.abs(Uo).max()
    say(f"  rel err {err:.3e}, its max {st['max_iterations']}, spmv {st['spmv']}")
    assert st["max_iterations"] == iters and st["n_maxit"] == 2 * L
    assert st["spmv"] == iters * 2 * L             # one product per COCG step
    assert err < max(1e-12, 1e-13 * 3.0 ** iters)


@pytest.mark.parametrize("prec", [0, 1])
def test_cocg_filter_matches_exact_solve(slrf, torch, prec):
    p = pencils.scalar_q1(13, 3, 0.5, 41)            # n = 1728
    gamma, L = 300.0, 48
    sig, w = golden_poles(4, gamma)
    X = pencils.start_block(p.n, L, 3)
    say(f"case COCG filter prec={prec}")
    opt = slrf.default_options(precision=prec, inner_tol=1e-11, solver=slrf.SOLVER_COCG)
    s = slrf.Solver(p.A, p.B, max_L=L, max_poles=4, options=opt)
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    Uo, _ = oflt.filter_apply(p.A, p.B, X, sig, w)
    err = np.abs(U.cpu().numpy() - Uo).max() / np.abs(Uo).max()
    say(f"  rel err {err:.3e}, mean its {st['mean_iterations']:.1f}, max relres {st['max_relres']:.2e}, "
        f"breakdowns {st['n_breakdown']}")
    assert st["n_breakdown"] == 0 and st["n_maxit"] == 0
    assert err < 1e-8


@pytest.mark.parametrize("prec", [0, 1])
def test_cocg_solve_3d_lognormal_vs_dense(slrf, torch, prec):
    q = pencils.scalar_q1(12, 3, 0.5, 31)            # n = 1331
    ev, _ = dense.all_eigenpairs(q.A, q.B)
    gamma = 0.5 * (ev[29] + ev[30])
    L = 40
    say(f"case COCG solve prec={prec}")
    opt = slrf.default_options(precision=prec, solver=slrf.SOLVER_COCG)
    s = slrf.Solver(q.A, q.B, max_L=L, max_poles=4, options=opt)
    r = s.solve_interval(gamma, L, V0=torch.from_numpy(pencils.start_block(q.n, L, 4)).cuda())
    nf = r.n_found
    X = r.evecs.cpu().numpy()[:, :nf]
    rel = np.abs(r.evals[:nf] / ev[:nf] - 1).max()
    orth = np.abs(X.T @ (q.B @ X) - np.eye(nf)).max()
    say(f"  found {nf}, rel eig err {rel:.3e}, max rho {r.resid[:nf].max():.3e}, orth {orth:.1e}, "
        f"outer {r.stats['outer_iterations']}")
    assert r.status == 0 and nf == 30 == inertia.sparse_ldl_count(q.A, q.B, gamma)
    assert rel < (1e-10 if prec == 0 else 1e-8)
    assert r.resid[:nf].max() <= 1e-8
    assert orth < 1e-10


def test_cocg_rejects_ilu0(slrf, torch):
    p = pencils.scalar_q1(6, 3, 0.0, 0)
    with pytest.raises(slrf.SlrfError):
        slrf.Solver(p.A, p.B, max_L=8, max_poles=2,
                    options=slrf.default_options(solver=slrf.SOLVER_COCG, precond=slrf.PRECOND_ILU0))


def elastic():
    """7 x 6 x 6 hexes (343 free nodes, n = 1029), log-normal Young's modulus,
    clamped face: node triples in the sparse product, node block Jacobi."""
    return pencils.elasticity_q1(7, 6, 6, 1.0 / 7, 0.7, 0.3, (0.8, 1.2), 3)


@pytest.mark.parametrize("iters", [1, 3])
def test_cocg_block_jacobi_iterates_match_oracle(slrf, torch, iters):
    e = elastic()
    ev, _ = dense.all_eigenpairs(e.A, e.B)
    sig, w = golden_poles(4, 0.5 * (ev[19] + ev[20]))
    sig, w = sig[:3], w[:3]
    L = 40
    X = pencils.start_block(e.n, L, 6)
    say(f"case COCG block-Jacobi iterates iters={iters} n={e.n}")
    opt = slrf.default_options(inner_tol=0.0, inner_maxit=iters, check_every=1, precond=slrf.PRECOND_BLOCK3,
                               solver=slrf.SOLVER_COCG)
    s = slrf.Solver(e.A, e.B, max_L=L, max_poles=3, options=opt)
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    x, it, fl, _ = krylov.cocg(e.A, e.B, sig, e.B @ X, 0.0, iters, fixed_iters=iters, precond="bjac3")
    Uo = sum(2.0 * np.real(w[j] * x[:, j * L:(j + 1) * L]) for j in range(3))
    err = np.abs(U.cpu().numpy() - Uo).max() / np.abs(Uo).max()
    say(f"  rel err {err:.3e}, its {st['max_iterations']}")
    assert st["max_iterations"] == iters
    assert err < max(1e-12, 1e-13 * 3.0 ** iters)


@pytest.mark.parametrize("prec", [0, 1])
def test_cocg_elasticity_solve_block_jacobi_vs_dense(slrf, torch, prec):
    e = elastic()
    ev, _ = dense.all_eigenpairs(e.A, e.B)
    k = 24
    while (ev[k] - ev[k - 1]) / ev[k] < 1e-3:
        k += 1
    gamma = 0.5 * (ev[k - 1] + ev[k])
    L = int(np.ceil(1.3 * k / 8) * 8)
    say(f"case COCG elasticity solve prec={prec} n={e.n} nev={k} L={L}")
    opt = slrf.default_options(precision=prec, precond=slrf.PRECOND_BLOCK3, solver=slrf.SOLVER_COCG)
    s = slrf.Solver(e.A, e.B, max_L=L, max_poles=4, options=opt)
    r = s.solve_interval(gamma, L, V0=torch.from_numpy(pencils.start_block(e.n, L, 9)).cuda())
    nf = r.n_found
    rel = np.abs(r.evals[:nf] / ev[:nf] - 1).max()
    X = r.evecs.cpu().numpy()[:, :nf]
    orth = np.abs(X.T @ (e.B @ X) - np.eye(nf)).max()
    say(f"  found {nf}, rel eig err {rel:.2e}, max rho {r.resid[:nf].max():.2e}, orth {orth:.1e}, "
        f"outer {r.stats['outer_iterations']}, inner its {r.stats['inner_iterations']:.1f}")
    assert r.status == 0 and nf == k == inertia.sparse_ldl_count(e.A, e.B, gamma)
    assert rel < (1e-10 if prec == 0 else 1e-8)
    assert r.resid[:nf].max() <= 1e-8
    assert orth < 1e-10
