"""The library's results do not depend on what its workspace held before.

Every buffer a kernel reads is written first in the same call (or is a table
the context built), so a workspace filled with 0xFF bytes (a NaN in FP32 and
FP64 alike) must give bit for bit the result of a zero-filled one.  The colour
sweeps of the multicolour SGS gather from a vector whose own rows are still
being written; the chunked gathers pad a row with zero coefficients, and the
padded values must not be read as 0 * (leftover bits).  The default tiling is
fixed (no autotuning), so both runs do the same arithmetic in the same order.
"""
import json
import os

import numpy as np
import pytest

import pencils

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
    return pencils.scalar_q1(12, 3, 0.5, 21)


def elastic():
    return pencils.elasticity_q1(7, 6, 6, 1.0 / 7, 0.7, 0.3, (0.8, 1.2), 5)


# (name, pencil, gamma, solver, precond)
CASES = [
    ("bicgstab-jacobi", scalar, 300.0, 0, 1),
    ("cocg-jacobi", scalar, 300.0, 1, 1),
    ("cocg-sgs-point", scalar, 300.0, 1, 4),
    ("cocg-node-jacobi", elastic, 60.0, 1, 3),
    ("cocg-sgs-node", elastic, 60.0, 1, 5),
]


def filled(torch, nbytes, byte):
    return torch.full((nbytes,), byte, dtype=torch.uint8, device="cuda:0")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name,make,gamma,solver,pc", CASES)
def test_filter_independent_of_workspace_contents(slrf, torch, name, make, gamma, solver, pc, prec):
    p = make()
    L = 47                                      # K = 188: a ragged last tile
    sig, w = golden_poles(4, gamma)
    X = torch.from_numpy(pencils.start_block(p.n, L, 11)).cuda()
    opt = slrf.default_options(precision=prec, inner_tol=1e-10, solver=solver, precond=pc)
    say(f"case workspace contents {name} prec={prec} n={p.n} L={L}")
    s = slrf.Solver(p.A, p.B, max_L=L, max_poles=4, options=opt)
    nbytes = s.ws_bytes
    s.close()
    out = []
    for byte in (0, 0xFF):
        s = slrf.Solver(p.A, p.B, max_L=L, max_poles=4, options=opt, workspace=filled(torch, nbytes, byte))
        U, st = s.filter_apply(X, sig, w)
        s.close()
        out.append((U.cpu().numpy(), st))
        say(f"  fill 0x{byte:02x}: mean its {st['mean_iterations']:.1f}, breakdowns {st['n_breakdown']}, "
            f"finite {np.isfinite(out[-1][0]).all()}")
    (U0, s0), (U1, s1) = out
    assert np.isfinite(U0).all() and np.isfinite(U1).all()
    assert s0["n_breakdown"] == 0 and s1["n_breakdown"] == 0
    assert np.array_equal(U0, U1)
    assert s0["mean_iterations"] == s1["mean_iterations"]


@pytest.mark.parametrize("name,make,gamma,solver,pc", [CASES[2], CASES[4]])
def test_recycled_solve_independent_of_workspace_contents(slrf, torch, name, make, gamma, solver, pc):
    """Mixed precision with warm starts across outer iterations (the buffers
    that carry Y and B X from one outer iteration to the next included)."""
    from oracle import dense
    q = make()
    ev, _ = dense.all_eigenpairs(q.A, q.B)
    g = 0.5 * (ev[23] + ev[24])
    L = 40
    sig, w = golden_poles(6, g)
    V0 = torch.from_numpy(pencils.start_block(q.n, L, 7)).cuda()
    opt = slrf.default_options(precision=1, solver=solver, precond=pc, recycle=1)
    say(f"case workspace contents, recycled solve {name} n={q.n}")
    s = slrf.Solver(q.A, q.B, max_L=L, max_poles=6, options=opt)
    nbytes = s.ws_bytes
    s.close()
    res = []
    for byte in (0, 0xFF):
        s = slrf.Solver(q.A, q.B, max_L=L, max_poles=6, options=opt, workspace=filled(torch, nbytes, byte))
        r = s.solve_interval(g, L, sig, w, V0=V0)
        s.close()
        say(f"  fill 0x{byte:02x}: status {r.status}, found {r.n_found}, outer {r.stats['outer_iterations']}")
        res.append(r)
    assert res[0].status == 0 and res[1].status == 0
    assert res[0].n_found == res[1].n_found == 24
    assert np.array_equal(res[0].evals, res[1].evals)
