"""GPU parity at the full size of the elasticity workload: 3D linear elasticity
on trilinear hexahedra, 48^3 free nodes x 3 unknowns (n = 331,776, 81-entry
rows), L = 256, N = 8, in the configuration the benchmark times (mixed
precision, COCG with the multicolour node-block symmetric Gauss-Seidel
preconditioner, warm starts across outer iterations, default tiling).

* COCG iterates (FP64 kernels, fixed iteration count) of sampled columns
  against the oracle's COCG with its multicolour SGS on those columns alone.
  The two round differently: the library applies the preconditioner in split
  form with precomputed inverses of the 3x3 node blocks, the oracle applies
  M^{-1} with a solve per block.  This computation is sensitive: a relative
  perturbation of 1e-16 in the right-hand sides moves the oracle's own result
  by about 1.3e-12 (an amplification of 1e4 over three iterations), and every
  rounding step of either side enters with a similar gain, so the bound is
  2e-10 relative (observed 4.6e-11).  A wrong colour order, a dropped coupling
  or a wrong pole changes the iterates in the first digits.
* The complete interval solve against the oracle's eigenvalues of this pencil
  (shift-invert subspace iteration with a banded Cholesky factor, stored by
  tests/golden/make_golden.py, which also placed gamma in the middle of a gap of
  relative width 7e-3 with 199 eigenvalues below it): all 199 found, each
  within 1e-8 relative, residuals recomputed on the host <= 1e-8, B-orthonormal.
"""
import json
import os

import numpy as np
import pytest

import pencils
from oracle import krylov

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
L, N = 256, 8


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


@pytest.fixture(scope="module")
def c3():
    return pencils.c3_elasticity()


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(GOLDEN, "eig_elast3d_48_s3.json")) as f:
        return json.load(f)


def say(*a):
    print(*a, flush=True)


def test_c3_full_sgs_cocg_sampled_columns(slrf, torch, c3, golden):
    p = c3
    iters = 3
    sig, w, _ = slrf.design_poles(N, 1.0, 0.01, golden["gamma"])
    X = pencils.start_block(p.n, L, 1)
    say(f"case full-size FP64 SGS-COCG iterates n={p.n} L={L} N={N} iters={iters}")
    opt = slrf.default_options(precision=0, inner_tol=0.0, inner_maxit=iters, check_every=iters,
                               solver=slrf.SOLVER_COCG, precond=slrf.PRECOND_SGS3)
    s = slrf.Solver(p.A, p.B, max_L=L, max_poles=N, options=opt)
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    U = U.cpu().numpy()
    s.close()
    assert st["max_iterations"] == iters
    # columns on both sides of a 128-column tile boundary, a middle one, the last one
    cols = np.array([0, 127, 128, 201, L - 1])
    # the library's default relaxation of node blocks (sgs_omega 0: 0.7)
    x, _, _, _ = krylov.cocg(p.A, p.B, sig, p.B @ X[:, cols], 0.0, iters, fixed_iters=iters, precond="mcsgs3",
                             omega=0.7)
    m = len(cols)
    Uo = sum(2.0 * np.real(w[j] * x[:, j * m:(j + 1) * m]) for j in range(N))
    err = np.abs(U[:, cols] - Uo).max() / np.abs(Uo).max()
    say(f"  sampled columns {cols.tolist()}: rel err {err:.3e}")
    assert err < 2e-10


def test_c3_full_solve_matches_oracle(slrf, torch, c3, golden):
    p = c3
    gamma = golden["gamma"]
    ev = np.array(golden["eigenvalues"])
    sig, w, _ = slrf.design_poles(N, 1.0, 0.01, gamma)
    say(f"case full-size elasticity solve n={p.n} L={L} N={N} gamma={gamma:.6g} (oracle: {len(ev)})")
    opt = slrf.default_options(precision=slrf.MIXED, solver=slrf.SOLVER_COCG, precond=slrf.PRECOND_SGS3,
                               recycle=1)
    s = slrf.Solver(p.A, p.B, max_L=L, max_poles=N, options=opt)
    r = s.solve_interval(gamma, L, sig, w, V0=torch.from_numpy(pencils.start_block(p.n, L, 1)).cuda())
    s.close()
    nf = r.n_found
    th = r.evals[:nf]
    X = r.evecs.cpu().numpy()[:, :nf]
    BX = p.B @ X
    rho = np.linalg.norm(p.A @ X - BX * th, axis=0) / (th * np.linalg.norm(BX, axis=0))
    orth = np.abs(X.T @ BX - np.eye(nf)).max()
    rel = np.abs(th / ev - 1).max() if nf == len(ev) else np.inf
    say(f"  found {nf}, max rel eig err {rel:.2e}, max rho {rho.max():.2e} (reported {r.resid[:nf].max():.2e}), "
        f"orth {orth:.1e}, outer {r.stats['outer_iterations']}, inner its {r.stats['inner_iterations']:.1f}, "
        f"{r.stats['seconds']:.1f} s")
    assert r.status == 0
    assert nf == len(ev) == golden["count"]
    assert np.all(th > 0) and np.all(th <= gamma)
    assert rel <= 1e-8
    assert rho.max() <= 1.01e-8
    assert orth < 1e-10
