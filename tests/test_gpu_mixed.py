"""GPU parity of the mixed-precision path (complex FP32 inner solves with FP64
defect correction, FP64 Rayleigh-Ritz) against the FP64 oracle and closed forms."""
import json
import os

import numpy as np
import pytest

import pencils
from closed_forms import closed_1d, closed_3d_cc
from oracle import dense, inertia
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


@pytest.mark.parametrize("case", ["3d", "1d"])
def test_mixed_filter_matches_exact_solve(slrf, torch, case):
    if case == "3d":
        p = pencils.scalar_q1(13, 3, 0.5, 41)        # n = 1728
        gamma, L = 300.0, 48
    else:
        p = pencils.string_1d(1500)                  # ILU(0) path
        lam, _ = closed_1d(1500)
        gamma, L = 0.5 * (lam[11] + lam[12]), 24
    sig, w = golden_poles(4, gamma)
    X = pencils.start_block(p.n, L, 3)
    say(f"case mixed filter {case}")
    opt = slrf.default_options(precision=slrf.MIXED, inner_tol=1e-11)
    s = slrf.Solver(p.A, p.B, max_L=L, max_poles=4, options=opt)
    U, st = s.filter_apply(torch.from_numpy(X).cuda(), sig, w)
    Uo, _ = oflt.filter_apply(p.A, p.B, X, sig, w)
    err = np.abs(U.cpu().numpy() - Uo).max() / np.abs(Uo).max()
    say(f"  rel err {err:.3e}, rounds {st['refinements']}, max relres {st['max_relres']:.2e}")
    assert st["max_relres"] <= 1e-11
    assert st["refinements"] >= 2        # FP32 alone cannot reach 1e-11
    assert err < 1e-8


def test_mixed_solve_3d_lognormal_vs_dense(slrf, torch):
    q = pencils.scalar_q1(12, 3, 0.5, 31)
    ev, _ = dense.all_eigenpairs(q.A, q.B)
    gamma = 0.5 * (ev[29] + ev[30])
    L = 40
    say("case mixed solve 3D log-normal small")
    opt = slrf.default_options(precision=slrf.MIXED)
    s = slrf.Solver(q.A, q.B, max_L=L, max_poles=4, options=opt)
    r = s.solve_interval(gamma, L, V0=torch.from_numpy(pencils.start_block(q.n, L, 4)).cuda())
    nf = r.n_found
    rel = np.abs(r.evals[:nf] / ev[:nf] - 1).max()
    X = r.evecs.cpu().numpy()[:, :nf]
    orth = np.abs(X.T @ (q.B @ X) - np.eye(nf)).max()
    say(f"  found {nf}, rel eig err {rel:.3e}, max rho {r.resid[:nf].max():.3e}, orth {orth:.1e}, "
        f"outer {r.stats['outer_iterations']}")
    assert r.status == 0 and nf == 30 == inertia.sparse_ldl_count(q.A, q.B, gamma)
    assert rel < 1e-8 and r.resid[:nf].max() <= 1e-8 and orth < 1e-10


def test_mixed_solve_1d_closed_form(slrf, torch):
    n = 2000
    p = pencils.c1_string()
    lam, _ = closed_1d(n)
    gamma = 0.5 * (lam[19] + lam[20])
    say("case mixed solve C1")
    opt = slrf.default_options(precision=slrf.MIXED)
    s = slrf.Solver(p.A, p.B, max_L=32, max_poles=4, options=opt)
    r = s.solve_interval(gamma, 32, V0=torch.from_numpy(pencils.start_block(n, 32, 1)).cuda())
    nf = r.n_found
    rel = np.abs(r.evals[:nf] / lam[:nf] - 1).max()
    say(f"  found {nf}, rel eig err {rel:.3e}, max rho {r.resid[:nf].max():.3e}")
    assert r.status == 0 and nf == 20 and rel < 1e-8


def test_mixed_solve_3d_cc_closed_form(slrf, torch):
    m = 16
    q = pencils.scalar_q1(m, 3)
    lam = closed_3d_cc(m)
    gaps = np.where(np.diff(lam[:60]) / lam[1:60] > 0.02)[0]
    k = gaps[np.argmin(np.abs(gaps - 40))]
    gamma = 0.5 * (lam[k] + lam[k + 1])
    nev = k + 1
    L = int(np.ceil(1.3 * nev / 8) * 8)
    say(f"case mixed solve 3D cc nev={nev}")
    opt = slrf.default_options(precision=slrf.MIXED)
    s = slrf.Solver(q.A, q.B, max_L=L, max_poles=4, options=opt)
    r = s.solve_interval(gamma, L)
    nf = r.n_found
    rel = np.abs(r.evals[:nf] / lam[:nf] - 1).max()
    say(f"  found {nf}, rel eig err {rel:.3e}, max rho {r.resid[:nf].max():.3e}")
    assert r.status == 0 and nf == nev and rel < 1e-8
