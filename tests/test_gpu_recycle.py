"""GPU checks of the warm start across outer iterations (options.recycle = 1,
mixed precision): complete interval solves agree with the dense FP64 oracle and
the inertia count, alone and in a batch, and need fewer sparse products than
cold starts."""
import numpy as np
import pytest

import pencils
from oracle import dense, inertia

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


@pytest.mark.parametrize("solver", [0, 1])
def test_recycle_solve_matches_dense(slrf, torch, solver):
    q = pencils.scalar_q1(12, 3, 0.5, 31)            # n = 1331
    ev, _ = dense.all_eigenpairs(q.A, q.B)
    gamma = 0.5 * (ev[29] + ev[30])
    L = 40
    V0 = torch.from_numpy(pencils.start_block(q.n, L, 4)).cuda()
    res = {}
    for rec in (0, 1):
        opt = slrf.default_options(precision=slrf.MIXED, solver=solver, recycle=rec)
        s = slrf.Solver(q.A, q.B, max_L=L, max_poles=4, options=opt)
        r = s.solve_interval(gamma, L, V0=V0)
        s.close()
        nf = r.n_found
        X = r.evecs.cpu().numpy()[:, :nf]
        rel = np.abs(r.evals[:nf] / ev[:nf] - 1).max()
        orth = np.abs(X.T @ (q.B @ X) - np.eye(nf)).max()
        say(f"case solver={solver} recycle={rec}: found {nf}, rel eig err {rel:.2e}, max rho "
            f"{r.resid[:nf].max():.2e}, outer {r.stats['outer_iterations']}, spmv {r.stats['spmv_total']}")
        assert r.status == 0 and nf == 30 == inertia.sparse_ldl_count(q.A, q.B, gamma)
        assert rel < 1e-8 and r.resid[:nf].max() <= 1e-8 and orth < 1e-10
        res[rec] = r.stats["spmv_total"]
    assert res[1] < res[0]


def test_recycle_batch_matches_dense(slrf, torch):
    cases = []
    for (m, dim, ln, seed, k, L) in [(30, 2, 0.5, 3, 15, 24), (12, 3, 0.5, 31, 30, 40), (11, 3, 0.5, 8, 20, 32)]:
        p = pencils.scalar_q1(m, dim, ln, seed)
        ev, _ = dense.all_eigenpairs(p.A, p.B)
        cases.append((p, 0.5 * (ev[k - 1] + ev[k]), L, k, ev))
    pers = trans = 0
    for p, g, L, k, _ in cases:
        a, b = slrf.batch_footprint(p.n, int((abs(p.A) + abs(p.B)).nnz), L, 4, slrf.MIXED)
        pers += a + 4096
        trans += b
    say("case batch recycle")
    b = slrf.Batch(pers + trans + (1 << 20), trans, max_poles=4,
                   options=slrf.default_options(precision=slrf.MIXED, solver=slrf.SOLVER_COCG, recycle=1))
    ids = [b.add(p.A, p.B, g, L) for p, g, L, _, _ in cases]
    steps = 0
    while b.step() > 0:
        steps += 1
        assert steps < 60
    for pid, (p, g, L, k, ev) in zip(ids, cases):
        r = b.result(pid)
        nf = r.n_found
        rel = np.abs(r.evals[:nf] / ev[:nf] - 1).max()
        say(f"  n={p.n}: found {nf} of {k}, rel eig err {rel:.2e}, max rho {r.resid[:nf].max():.2e}, "
            f"outer {r.stats['outer_iterations']}")
        assert r.status == 0 and nf == k == inertia.sparse_ldl_count(p.A, p.B, g)
        assert rel < 1e-8 and r.resid[:nf].max() <= 1e-8
    b.close()
