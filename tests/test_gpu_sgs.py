"""GPU parity of COCG with the multicolour symmetric Gauss-Seidel preconditioner
(options.precond 4: point, 5: 3x3 node blocks).

The library runs COCG on the split system M_L^{-1} S M_L^{-T} y' = M_L^{-1} f
with one backward and one forward colour sweep per iteration; in exact
arithmetic its iterates, mapped back by y = M_L^{-T} y', are those of COCG
preconditioned with M = M_L M_L^T = (D + L) D^{-1} (D + U), which the oracle
computes plainly (oracle.krylov.cocg with precond "mcsgs" / "mcsgs3").

* Iterates after a fixed number of steps against the oracle's, pushed through
  the same filter sum (FP64 kernels).
* Converged filter against the oracle's exact filter (FP64 and mixed).
* Complete interval solves against the dense oracle and the inertia count, and
  fewer inner iterations than point / node block Jacobi on the same solve.
"""
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


def scalar():
    return pencils.scalar_q1(12, 3, 0.5, 21)                              # n = 1331, 8 colours


def elastic():
    return pencils.elasticity_q1(7, 6, 6, 1.0 / 7, 0.7, 0.3, (0.8, 1.2), 5)   # n = 1029, 8 node colours


CASES = [("point", scalar, 4, "mcsgs", 300.0), ("node", elastic, 5, "mcsgs3", 60.0)]


@pytest.mark.parametrize("omega", [1.0, 0.7])
@pytest.mark.parametrize("iters", [1, 3, 8])
@pytest.mark.parametrize("kind,make,pc,opc,gamma", CASES)
def test_sgs_iterates_match_oracle(slrf, torch, kind, make, pc, opc, gamma, iters, omega):
    """FP64 iterates after a fixed number of iterations against the oracle's COCG
    with the same multicolour SGS (omega = 1) or its symmetric SOR form."""
    q = make()
    L = 40                                           # K = 80: a ragged tile
    sig, w = golden_poles(4, gamma)
    sig, w = sig[:2], w[:2]
    X = pencils.start_block(q.n, L, 5)
    say(f"case SGS-COCG iterates {kind} iters={iters} omega={omega} n={q.n} L={L} N=2")
    opt = slrf.default_options(inner_tol=0.0, inner_maxit=iters, check_every=1, solver=slrf.SOLVER_COCG,
                               precond=pc, sgs_omega=omega)
    s = slrf.Solver(q.A, q.B, max_L=L, max_poles=2, options=opt)
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    U = U.cpu().numpy()
    s.close()
    x, it, fl, _ = krylov.cocg(q.A, q.B, sig, q.B @ X, 0.0, iters, fixed_iters=iters, precond=opc, omega=omega)
    Uo = sum(2.0 * np.real(w[j] * x[:, j * L:(j + 1) * L]) for j in range(2))
    err = np.abs(U - Uo).max() / np.abs(Uo).max()
    say(f"  rel err {err:.3e}, its max {st['max_iterations']}, spmv {st['spmv']}")
    assert st["max_iterations"] == iters and st["n_maxit"] == 2 * L
    assert err < max(1e-12, 1e-13 * 3.0 ** iters)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,make,pc,opc,gamma", CASES)
def test_sgs_filter_matches_exact_solve(slrf, torch, kind, make, pc, opc, gamma, prec):
    p = make()
    L = 48
    sig, w = golden_poles(4, gamma)
    X = pencils.start_block(p.n, L, 3)
    say(f"case SGS-COCG filter {kind} prec={prec}")
    its = {}
    for name, pcv in (("sgs", pc), ("jacobi", 1 if pc == 4 else 3)):
        opt = slrf.default_options(precision=prec, inner_tol=1e-11, solver=slrf.SOLVER_COCG, precond=pcv)
        s = slrf.Solver(p.A, p.B, max_L=L, max_poles=4, options=opt)
        U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
        U = U.cpu().numpy()
        s.close()
        its[name] = st["mean_iterations"]
        if name == "sgs":
            Uo, _ = oflt.filter_apply(p.A, p.B, X, sig, w)
            err = np.abs(U - Uo).max() / np.abs(Uo).max()
            say(f"  rel err {err:.3e}, mean its {st['mean_iterations']:.1f}, breakdowns {st['n_breakdown']}")
            assert st["n_breakdown"] == 0 and st["n_maxit"] == 0
            assert err < 1e-8
    say(f"  mean inner iterations: SGS {its['sgs']:.1f}, Jacobi {its['jacobi']:.1f}")
    assert its["sgs"] < 0.8 * its["jacobi"]


@pytest.mark.parametrize("prec,recycle,omega", [(0, 0, 1.0), (1, 0, 1.0), (1, 1, 1.0), (0, 0, 0.7), (1, 1, 0.7)])
@pytest.mark.parametrize("kind,make,pc,opc,gamma", CASES)
def test_sgs_solve_vs_dense(slrf, torch, kind, make, pc, opc, gamma, prec, recycle, omega):
    q = make()
    ev, _ = dense.all_eigenpairs(q.A, q.B)
    k = 24
    g = 0.5 * (ev[k - 1] + ev[k])
    L = 40
    sig, w = golden_poles(6, g)
    say(f"case SGS-COCG interval solve {kind} prec={prec} recycle={recycle} omega={omega} n={q.n} NEV={k}")
    opt = slrf.default_options(precision=prec, solver=slrf.SOLVER_COCG, precond=pc, recycle=recycle,
                               sgs_omega=omega)
    s = slrf.Solver(q.A, q.B, max_L=L, max_poles=6, options=opt)
    r = s.solve_interval(g, L, sig, w, V0=torch.from_numpy(pencils.start_block(q.n, L, 7)).cuda())
    s.close()
    cnt = inertia.dense_ldl_count(q.A, q.B, g)
    nf = r.n_found
    rel = np.abs(r.evals[:nf] / ev[:nf] - 1).max()
    X = r.evecs.cpu().numpy()[:, :nf]
    orth = np.abs(X.T @ (q.B @ X) - np.eye(nf)).max()
    say(f"  found {nf} (inertia {cnt}), max rel eig err {rel:.2e}, orth {orth:.1e}, "
        f"outer {r.stats['outer_iterations']}, inner its {r.stats['inner_iterations']:.1f}")
    assert r.status == 0 and nf == cnt == k
    assert rel <= (1e-10 if prec == 0 else 1e-8)
    assert orth < 1e-10
    assert r.resid[:nf].max() <= 1e-8


def test_sgs_rejected_with_bicgstab_and_node_fallback(slrf, torch):
    q = scalar()
    with pytest.raises(slrf.SlrfError):
        slrf.Solver(q.A, q.B, max_L=8, max_poles=2,
                    options=slrf.default_options(solver=slrf.SOLVER_BICGSTAB, precond=4))
    # node blocks where the pencil has none (n not divisible by 3): the point form
    p = pencils.string_1d(100)
    s = slrf.Solver(p.A, p.B, max_L=8, max_poles=2,
                    options=slrf.default_options(solver=slrf.SOLVER_COCG, precond=5))
    s.close()


def test_sgs_node_and_point_pencils_in_one_batch(slrf, torch):
    """precond 5 takes node blocks for the elasticity pencil and the point form
    for the scalar one; one batch holds both (one sweep launch per block size
    and colour).  The scalar pencil gives bitwise its solve alone (n >= 8192 and
    stencil rows: the same Krylov grid and row blocks) and its precond-4 solve;
    the elasticity pencil runs on the scalar pencil's row blocks in the batch
    (16 rows instead of its own 24), which reorders sums, so its found
    eigenvalues agree with its solve alone to 1e-9.  Every pencil's eigenvalues
    agree with the Lanczos reference (shift-invert, SciPy) to 1e-8."""
    import scipy.sparse.linalg as sla
    cases = []
    for q, nev in ((pencils.scalar_q1(22, 3, 0.5, 12), 24),
                   (pencils.elasticity_q1(14, 13, 13, 1.0 / 14, 0.7, 0.3, (0.8, 1.2), 5), 24)):
        ev = np.sort(sla.eigsh(q.A.tocsc(), k=nev + 8, M=q.B.tocsc(), sigma=0.0, which="LM",
                               return_eigenvectors=False))
        k = nev
        while (ev[k] - ev[k - 1]) / ev[k] < 1e-3:
            k += 1
        cases.append((q, 0.5 * (ev[k - 1] + ev[k]), 40, k, ev[:k]))
    N = 6
    opt = slrf.default_options(precision=slrf.MIXED, solver=slrf.SOLVER_COCG, precond=slrf.PRECOND_SGS3, recycle=1)
    alone = []
    for i, (q, g, L, k, ev) in enumerate(cases):
        sig, w, _ = slrf.design_poles(N, 1.0, 0.01, g)
        say(f"case SGS precond 5 alone: pencil {i} n={q.n} NEV={k}")
        s = slrf.Solver(q.A, q.B, max_L=L, max_poles=N, options=opt)
        r = s.solve_interval(g, L, sig, w, V0=torch.from_numpy(pencils.start_block(q.n, L, 50 + i)).cuda())
        s.close()
        rel = np.abs(r.evals[:r.n_found] / ev - 1).max() if r.n_found == k else np.inf
        say(f"  found {r.n_found}, rel eig err {rel:.2e}, outer {r.stats['outer_iterations']}")
        assert r.status == 0 and r.n_found == k and rel <= 1e-8
        alone.append(r)
    # the scalar pencil under precond 4 (the point form precond 5 falls back to)
    q, g, L, k, _ = cases[0]
    sig, w, _ = slrf.design_poles(N, 1.0, 0.01, g)
    s = slrf.Solver(q.A, q.B, max_L=L, max_poles=N,
                    options=slrf.default_options(precision=slrf.MIXED, solver=slrf.SOLVER_COCG,
                                                 precond=slrf.PRECOND_SGS, recycle=1))
    r4 = s.solve_interval(g, L, sig, w, V0=torch.from_numpy(pencils.start_block(q.n, L, 50)).cuda())
    s.close()
    assert np.array_equal(r4.evals, alone[0].evals) and torch.equal(r4.evecs, alone[0].evecs)
    pers = trans = 0
    for q, _, L, _, _ in cases:
        a, t = slrf.batch_footprint(q.n, int((abs(q.A) + abs(q.B)).nnz), L, N, options=opt)
        pers += a + 4096
        trans += t
    b = slrf.Batch(pers + trans + (1 << 20), trans, max_poles=N, options=opt)
    ids = []
    for i, (q, g, L, _, _) in enumerate(cases):
        sig, w, _ = slrf.design_poles(N, 1.0, 0.01, g)
        ids.append(b.add(q.A, q.B, g, L, sig, w, V0=pencils.start_block(q.n, L, 50 + i)))
    steps = 0
    while b.step() > 0:
        steps += 1
        assert steps < 60
    for i, pid in enumerate(ids):
        r = b.result(pid)
        say(f"  batch pencil {i}: found {r.n_found}, outer {r.stats['outer_iterations']} "
            f"(alone {alone[i].stats['outer_iterations']})")
        nf = r.n_found
        assert r.status == 0 and nf == alone[i].n_found == cases[i][3]
        assert np.abs(r.evals[:nf] / cases[i][4] - 1).max() <= 1e-8
        if i == 0:
            assert np.array_equal(r.evals, alone[i].evals)
            assert torch.equal(r.evecs, alone[i].evecs)
        else:
            assert np.abs(r.evals[:nf] / alone[i].evals[:nf] - 1).max() <= 1e-9
    b.close()
