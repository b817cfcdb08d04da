"""GPU parity of the node block-Jacobi preconditioner (three unknowns per node) on
elasticity pencils: BiCGStab iterates against the oracle's, and complete interval
solves against the dense FP64 oracle and the inertia count."""
import json
import os

import numpy as np
import pytest

import pencils
from oracle import dense, inertia, krylov

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


def elastic():
    """7 x 6 x 6 hexes (343 free nodes, n = 1029: five 256-row blocks, ragged),
    log-normal Young's modulus (sigma 0.7), density in [0.8, 1.2], clamped face."""
    return pencils.elasticity_q1(7, 6, 6, 1.0 / 7, 0.7, 0.3, (0.8, 1.2), 3)


@pytest.mark.parametrize("iters", [1, 3])
def test_bicgstab_block_jacobi_iterates_match_oracle(slrf, torch, iters):
    e = elastic()
    ev, _ = dense.all_eigenpairs(e.A, e.B)
    sig, w = golden_poles(4, 0.5 * (ev[19] + ev[20]))
    sig, w = sig[:3], w[:3]
    L = 40                                           # K = 120: two tiles, ragged
    X = pencils.start_block(e.n, L, 6)
    say(f"case block-Jacobi iterates iters={iters} n={e.n}")
    opt = slrf.default_options(inner_tol=0.0, inner_maxit=iters, check_every=1, precond=3)
    s = slrf.Solver(e.A, e.B, max_L=L, max_poles=3, options=opt)
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    x, it, fl, _ = krylov.bicgstab(e.A, e.B, sig, e.B @ X, 0.0, iters, fixed_iters=iters, precond="bjac3")
    Uo = sum(2.0 * np.real(w[j] * x[:, j * L:(j + 1) * L]) for j in range(3))
    err = np.abs(U.cpu().numpy() - Uo).max() / np.abs(Uo).max()
    say(f"  rel err {err:.3e}, its {st['max_iterations']}")
    assert st["max_iterations"] == iters
    assert err < max(1e-11, 1e-13 * 3.0 ** iters)


@pytest.mark.parametrize("prec", [0, 1])
def test_elasticity_solve_block_jacobi_vs_dense(slrf, torch, prec):
    e = elastic()
    ev, Xd = dense.all_eigenpairs(e.A, e.B)
    k = 24
    while (ev[k] - ev[k - 1]) / ev[k] < 1e-3:
        k += 1
    gamma = 0.5 * (ev[k - 1] + ev[k])
    L = int(np.ceil(1.3 * k / 8) * 8)
    say(f"case elasticity solve prec={prec} n={e.n} nev={k} L={L}")
    opt = slrf.default_options(precision=prec, precond=3)
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


def test_block_jacobi_rejects_bad_sizes(slrf, torch):
    p = pencils.string_1d(100)            # n not divisible by 3
    with pytest.raises(slrf.SlrfError):
        slrf.Solver(p.A, p.B, max_L=8, max_poles=2, options=slrf.default_options(precond=3))
