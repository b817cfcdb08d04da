"""GPU parity at the full size of the timed workload: the 64^3 scalar vibration
pencil (n = 250047, 27-point rows), L = 128, N = 6, in the launch configuration
the benchmark times (default tiling, banded row order, stencil-group sparse
products).

* BiCGStab iterates (FP64 kernels, fixed iteration count) of sampled columns
  against the oracle's BiCGStab run on those columns alone: the columns of a
  block are independent, so the oracle computes them one by one.
* Complete interval solves (mixed and FP64): properties that hold at any size,
  checked on the host in FP64 against the oracle's count.  The number of pairs
  found equals the Sylvester inertia count stored by tests/golden/make_golden.py
  (oracle only); every returned pair has relative residual <= 1e-8 recomputed
  from A and B; the pairs are B-orthonormal; every eigenvalue lies in (0, gamma].
  Together these fix the eigenpairs of (0, gamma] to the residual bound.
* The same solves against the oracle's eigenvalues of this pencil (shift-invert
  subspace iteration with a banded Cholesky factor, stored by
  tests/golden/make_golden.py): relative error <= 1e-8 (mixed) and <= 1e-10
  (FP64), the tolerances the path states.
* The constant-coefficient 64^3 pencil, whose spectrum is a Kronecker sum of the
  1D linear-element eigenvalues: exactly 102 eigenvalues lie below 421 (in
  multiplets of 1, 3 and 6).  Every eigenvalue against its closed form, and every
  multiplet's eigenspace against the closed-form tensor-product sines through the
  principal angles between the two subspaces (rotation invariant).
"""
import json
import os

import numpy as np
import pytest

import pencils
from oracle import krylov

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GAMMA = 421.0
L, N = 128, 6


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
def c2():
    return pencils.c2_scalar3d()


def say(*a):
    print(*a, flush=True)


def golden_poles(N, gamma):
    with open(os.path.join(GOLDEN, f"poles_N{N}_a1_b0.01.json")) as f:
        d = json.load(f)
    return ((np.array(d["sigma_re"]) + 1j * np.array(d["sigma_im"])) * gamma,
            (np.array(d["w_re"]) + 1j * np.array(d["w_im"])) * gamma)


def golden_count():
    with open(os.path.join(GOLDEN, "count_scalar3d_m64_ln0.5_s2_g421.json")) as f:
        return json.load(f)["count_below_gamma"]


def golden_eigs():
    with open(os.path.join(GOLDEN, "eig_scalar3d_m64_ln0.5_s2_g421.json")) as f:
        return np.array(json.load(f)["eigenvalues"])


def test_c2_full_bicgstab_sampled_columns(slrf, torch, c2):
    p = c2
    iters = 3
    sig, w = golden_poles(N, GAMMA)
    X = pencils.start_block(p.n, L, 1)
    say(f"case full-size FP64 BiCGStab iterates n={p.n} L={L} N={N} iters={iters}")
    opt = slrf.default_options(precision=0, inner_tol=0.0, inner_maxit=iters, check_every=iters)
    s = slrf.Solver(p.A, p.B, max_L=L, max_poles=N, options=opt)
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    U = U.cpu().numpy()
    s.close()
    assert st["max_iterations"] == iters
    # columns on both sides of a 64-column tile boundary, a middle one, the last one
    cols = np.array([0, 63, 64, 101, L - 1])
    x, _, _, _ = krylov.bicgstab(p.A, p.B, sig, p.B @ X[:, cols], 0.0, iters, fixed_iters=iters)
    m = len(cols)
    Uo = sum(2.0 * np.real(w[j] * x[:, j * m:(j + 1) * m]) for j in range(N))
    err = np.abs(U[:, cols] - Uo).max() / np.abs(Uo).max()
    say(f"  sampled columns {cols.tolist()}: rel err {err:.3e}")
    assert err < 1e-11


@pytest.mark.parametrize("prec,solver,recycle", [(1, 0, 0), (0, 0, 0), (1, 1, 1)])
def test_c2_full_solve_properties(slrf, torch, c2, prec, solver, recycle):
    """(1, 1, 1) is the benchmark's configuration: mixed precision, COCG, warm starts."""
    p = c2
    sig, w = golden_poles(N, GAMMA)
    say(f"case full-size interval solve prec={prec} solver={solver} recycle={recycle} n={p.n} L={L} N={N}")
    s = slrf.Solver(p.A, p.B, max_L=L, max_poles=N,
                    options=slrf.default_options(precision=prec, solver=solver, recycle=recycle))
    r = s.solve_interval(GAMMA, L, sig, w, V0=torch.from_numpy(pencils.start_block(p.n, L, 1)).cuda())
    s.close()
    nf = r.n_found
    X = r.evecs.cpu().numpy()[:, :nf]
    th = r.evals[:nf]
    BX = p.B @ X
    rho = np.linalg.norm(p.A @ X - BX * th, axis=0) / (th * np.linalg.norm(BX, axis=0))
    orth = np.abs(X.T @ BX - np.eye(nf)).max()
    say(f"  found {nf} (count {golden_count()}), max rho {rho.max():.2e} (reported "
        f"{r.resid[:nf].max():.2e}), orth {orth:.1e}, outer {r.stats['outer_iterations']}")
    ev = golden_eigs()
    rel = np.abs(th / ev[:nf] - 1).max() if nf == len(ev) else np.inf
    say(f"  eigenvalues vs oracle: max rel err {rel:.2e}")
    assert r.status == 0
    assert nf == golden_count() == len(ev)
    assert np.all(th > 0) and np.all(th <= GAMMA)
    assert rho.max() <= 1.01e-8
    assert orth < 1e-10
    assert rel <= (1e-8 if prec == 1 else 1e-10)


def closed_form_cc(m, gamma):
    """Eigenvalues below gamma of the constant-coefficient pencil with m elements
    per side (Kronecker sums of the 1D eigenvalues) with their index triples."""
    h = 1.0 / m
    k = np.arange(1, m)
    mu = (6.0 / h ** 2) * 2.0 * np.sin(0.5 * k * np.pi * h) ** 2 / (2.0 + np.cos(k * np.pi * h))
    lam = mu[:, None, None] + mu[None, :, None] + mu[None, None, :]
    idx = np.argwhere(lam < gamma)
    vals = lam[lam < gamma]
    order = np.argsort(vals, kind="stable")
    return vals[order], idx[order], mu


def sine_vector(m, a, b, c):
    """B-normalised eigenvector of the constant-coefficient pencil for 1D modes
    (a, b, c) along (z, y, x), lexicographic order with x fastest: the tensor
    product of the B-normalised 1D sines."""
    n1 = m - 1
    h = 1.0 / m
    i = np.arange(1, m)

    def s(k):
        return np.sin(k * np.pi * i * h) / np.sqrt((h / 6) * (4 + 2 * np.cos(k * np.pi * h)) * m / 2)
    return np.einsum("k,j,i->kji", s(a + 1), s(b + 1), s(c + 1)).reshape(n1 ** 3)


@pytest.mark.parametrize("prec,solver,recycle", [(1, 1, 1), (0, 1, 0)])
def test_c2cc_full_closed_form(slrf, torch, prec, solver, recycle):
    """(1, 1, 1): the benchmark's configuration; (0, 1, 0): the FP64 form it is
    compared with."""
    m = 64
    p = pencils.scalar_q1(m, 3)
    lam, idx, _ = closed_form_cc(m, GAMMA)
    assert len(lam) == 102
    sig, w = golden_poles(N, GAMMA)
    say(f"case constant-coefficient 64^3 solve prec={prec} solver={solver} recycle={recycle}")
    s = slrf.Solver(p.A, p.B, max_L=L, max_poles=N,
                    options=slrf.default_options(precision=prec, solver=solver, recycle=recycle))
    r = s.solve_interval(GAMMA, L, sig, w, V0=torch.from_numpy(pencils.start_block(p.n, L, 1)).cuda())
    s.close()
    nf = r.n_found
    th = r.evals[:nf]
    X = r.evecs.cpu().numpy()[:, :nf]
    rel = np.abs(th / lam - 1).max() if nf == len(lam) else np.inf
    # multiplets: closed-form values equal to rounding
    groups, start = [], 0
    for i in range(1, len(lam) + 1):
        if i == len(lam) or lam[i] > lam[start] * (1 + 1e-12):
            groups.append((start, i))
            start = i
    worst = 0.0
    if nf == len(lam):
        BX = p.B @ X
        for a, b in groups:
            Xo = np.stack([sine_vector(m, *idx[t]) for t in range(a, b)], axis=1)
            cos = np.linalg.svd(Xo.T @ BX[:, a:b], compute_uv=False)
            worst = max(worst, float(np.sqrt(max(0.0, 1.0 - cos.min() ** 2))))
    say(f"  found {nf} (closed form 102), max rel eig err {rel:.2e}, {len(groups)} multiplets, "
        f"largest sin of principal angle {worst:.2e}, outer {r.stats['outer_iterations']}")
    assert r.status == 0 and nf == 102
    assert rel <= (1e-8 if prec == 1 else 1e-10)
    assert worst <= 1e-5
