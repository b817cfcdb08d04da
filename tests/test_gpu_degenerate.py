"""Degenerate cases of the interval solve (Algorithm 1) on the GPU.

* A diagonal pencil: every shifted system A - sigma_j B is diagonal, so the
  point preconditioners (ILU(0), Jacobi, multicolour SGS with one colour) solve
  it exactly.  Its eigenpairs are known in closed form: lambda_i = a_i / b_i with
  x_i = e_i / sqrt(b_i).
* An empty interval: gamma below the smallest eigenvalue.  Nothing is found and
  the solve still ends with status OK.
* A subspace no larger than the number of eigenvalues in (0, gamma]: every Ritz
  value lies in the interval, which the solve reports as
  SLRF_E_SUBSPACE_TOO_SMALL instead of returning an unverifiable count.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import pencils
from closed_forms import closed_1d

pytestmark = pytest.mark.gpu


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


def diagonal_pencil(n, seed):
    """A = diag(a) with a a seeded permutation of 1..n, B = diag(b), b ~ U[0.5, 1.5]."""
    g = np.random.default_rng(seed)
    a = g.permutation(n).astype(np.float64) + 1.0
    b = 0.5 + g.random(n)
    return sp.diags(a, 0, format="csr"), sp.diags(b, 0, format="csr"), a, b


# (precision, solver, precond, recycle): the library default, COCG with point
# Jacobi, and the benchmark's configuration with the multicolour SGS
CONFIGS = [(0, 0, 0, 0), (1, 1, 1, 0), (1, 1, 4, 1)]


@pytest.mark.parametrize("prec,solver,pc,recycle", CONFIGS)
def test_diagonal_pencil_closed_form(slrf, torch, prec, solver, pc, recycle):
    n, L = 500, 24
    A, B, a, b = diagonal_pencil(n, 7)
    lam = np.sort(a / b)
    gamma = 0.5 * (lam[11] + lam[12])
    opt = slrf.default_options(precision=prec, solver=solver, precond=pc, recycle=recycle)
    say(f"case diagonal n={n} L={L} prec={prec} solver={solver} precond={pc} recycle={recycle}")
    s = slrf.Solver(A, B, max_L=L, max_poles=4, options=opt)
    r = s.solve_interval(gamma, L, V0=torch.from_numpy(pencils.start_block(n, L, 3)).cuda())
    s.close()
    nf = r.n_found
    X = r.evecs.cpu().numpy()[:, :nf]
    rel = np.abs(r.evals[:nf] / lam[:nf] - 1).max() if nf else np.inf
    orth = np.abs(X.T @ (B @ X) - np.eye(nf)).max()
    # x_i = +-e_k / sqrt(b_k) for the index k with a_k / b_k = lambda_i
    k = np.argmax(np.abs(X), axis=0)
    shape = np.abs(np.abs(X[k, np.arange(nf)]) * np.sqrt(b[k]) - 1).max()
    say(f"  found {nf}, rel eig err {rel:.1e}, orth {orth:.1e}, eigenvector shape {shape:.1e}, "
        f"outer {r.stats['outer_iterations']}, mean inner {r.stats['inner_iterations']:.1f}")
    assert r.status == 0 and nf == 12
    assert rel < 1e-10 and orth < 1e-10 and shape < 1e-8
    assert np.allclose(a[k] / b[k], r.evals[:nf], rtol=1e-10, atol=0)
    assert r.resid[:nf].max() <= 1e-8


@pytest.mark.parametrize("prec", [0, 1])
def test_empty_interval_finds_nothing(slrf, torch, prec):
    n, L = 400, 16
    p = pencils.string_1d(n)
    lam, _ = closed_1d(n)
    gamma = 0.5 * lam[0]
    say(f"case empty interval n={n} L={L} prec={prec} gamma={gamma:.4g} < lambda_1={lam[0]:.4g}")
    s = slrf.Solver(p.A, p.B, max_L=L, max_poles=4, options=slrf.default_options(precision=prec))
    r = s.solve_interval(gamma, L, V0=torch.from_numpy(pencils.start_block(n, L, 5)).cuda())
    s.close()
    say(f"  status {r.status}, found {r.n_found}, outer {r.stats['outer_iterations']}")
    assert r.status == 0 and r.n_found == 0
    assert np.all((r.evals <= 0) | (r.evals > gamma))


def test_subspace_too_small_is_reported(slrf, torch):
    n, L = 400, 8
    p = pencils.string_1d(n)
    lam, _ = closed_1d(n)
    gamma = 0.5 * (lam[9] + lam[10])       # ten eigenvalues in (0, gamma], subspace of eight
    say(f"case subspace too small n={n} L={L}, 10 eigenvalues below gamma")
    s = slrf.Solver(p.A, p.B, max_L=L, max_poles=4)
    r = s.solve_interval(gamma, L, V0=torch.from_numpy(pencils.start_block(n, L, 9)).cuda(),
                         raise_on_error=False)
    s.close()
    say(f"  status {r.status} ({r.message}), outer {r.stats['outer_iterations']}")
    assert r.status == 6
    assert "increase L" in r.message
