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


def test_recycle_batch_bitwise_equals_alone(slrf, torch):
    """Warm starts in a batch whose pencils arrive at different steps and are
    removed as they finish: each pencil warm-starts from its own previous
    step, as it would alone, so every result is bitwise the solve alone and
    takes the same number of sparse products (fixed tiling: the autotuner may
    pick another row-block size for the batch than for a pencil alone, which
    rounds differently).  The last pencil joins after the first step: its first
    filter application runs from Y = 0 inside an application that warm-starts
    the others, which computes what its cold start computes."""
    from test_gpu_batch import big_cases, ws_for
    cases = big_cases()
    opt = slrf.default_options(precision=slrf.MIXED, solver=slrf.SOLVER_COCG, recycle=1)
    alone = []
    for i, (p, gamma, L, k) in enumerate(cases):
        say(f"case recycle alone pencil {i} n={p.n} L={L} nev={k}")
        s = slrf.Solver(p.A, p.B, max_L=L, max_poles=4, options=opt)
        r = s.solve_interval(gamma, L, V0=torch.from_numpy(pencils.start_block(p.n, L, 40 + i)).cuda())
        assert r.status == 0 and r.n_found == k
        alone.append(r)
        s.close()
    ws, arena = ws_for(slrf, cases, slrf.MIXED)
    say(f"case recycle batch: {len(cases)} pencils, the last one joining after the first step")
    b = slrf.Batch(ws, arena, max_poles=4, options=opt)

    def add(i):
        p, gamma, L, _ = cases[i]
        return b.add(p.A, p.B, gamma, L, V0=pencils.start_block(p.n, L, 40 + i))

    ids = {i: add(i) for i in range(len(cases) - 1)}
    out, steps = {}, 0
    while len(out) < len(cases):
        b.step()
        steps += 1
        assert steps < 60
        if steps == 1:
            ids[len(cases) - 1] = add(len(cases) - 1)
        for i, pid in ids.items():
            if i not in out and b.query(pid)[0]:
                out[i] = b.result(pid)
                b.remove(pid)
    assert len({out[i].stats["outer_iterations"] for i in out}) > 1   # pencils left at different steps
    for i, a in enumerate(alone):
        r = out[i]
        nf = r.n_found
        say(f"  pencil {i}: found {nf} outer {r.stats['outer_iterations']} "
            f"(alone {a.stats['outer_iterations']}), spmv {r.stats['spmv_total']} (alone {a.stats['spmv_total']})")
        assert r.status == 0 and nf == a.n_found
        assert r.stats["outer_iterations"] == a.stats["outer_iterations"]
        assert r.stats["spmv_total"] == a.stats["spmv_total"]
        assert np.array_equal(r.evals, a.evals)
        assert np.array_equal(r.resid, a.resid)
        assert torch.equal(r.evecs, a.evecs)
    b.close()


def test_recycle_autotune_same_work(slrf, torch):
    """With warm starts, the tile autotuner must leave the first correction
    round solving for the warm start's defect: the autotuned solve takes about
    the sparse products of the default tiling (the tilings round differently,
    so the counts need not match exactly) and finds the same eigenvalues."""
    from test_gpu_batch import big_cases
    p, gamma, L, k = big_cases()[0]
    V0 = torch.from_numpy(pencils.start_block(p.n, L, 40)).cuda()
    out = {}
    for tune in (0, 1):
        opt = slrf.default_options(precision=slrf.MIXED, solver=slrf.SOLVER_COCG, recycle=1, tune=tune)
        s = slrf.Solver(p.A, p.B, max_L=L, max_poles=4, options=opt)
        r = s.solve_interval(gamma, L, V0=V0)
        s.close()
        say(f"case recycle tune={tune}: found {r.n_found}, outer {r.stats['outer_iterations']}, "
            f"spmv {r.stats['spmv_total']}")
        assert r.status == 0 and r.n_found == k
        out[tune] = r
    assert abs(out[1].stats["spmv_total"] / out[0].stats["spmv_total"] - 1) < 0.15
    assert np.abs(out[1].evals[:k] / out[0].evals[:k] - 1).max() < 1e-9
