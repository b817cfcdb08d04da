"""GPU tests of the batch API: many pencils in one batched Krylov launch per step.

* A pencil gives bitwise the same eigenpairs alone (slrf_solve_interval) and
  inside a batch, when the Krylov grid is the same (every pencil here has
  n >= 8192, which fills the 1024-workgroup grid): the per-column reductions do
  not mix pencils and converged columns are frozen.
* Small pencils of different kinds (ILU(0) and Jacobi preconditioned in the same
  launch, different sizes, L and gamma) agree with the dense FP64 oracle.
* Continuous batching: admission by footprint, pencils joining between steps and
  leaving when done, results unchanged.
* hipGraph replay of the iteration chunks gives bitwise the eager result.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import pencils
from closed_forms import closed_1d
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


def gap_gamma(ev, k):
    """gamma halfway between the k-th and (k+1)-th eigenvalue (1-based k)."""
    return 0.5 * (ev[k - 1] + ev[k])


def smallest_eigs(p, k):
    vals = sla.eigsh(p.A.tocsc(), k=k, M=p.B.tocsc(), sigma=0.0, which="LM",
                     return_eigenvectors=False)
    return np.sort(vals)


def big_cases():
    """Three pencils with n >= 8192 (full Krylov grid), different kinds and sizes."""
    out = []
    for (m, dim, ln, seed, nev) in [(92, 2, 0.5, 11, 18), (22, 3, 0.5, 12, 24), (22, 3, 0.0, 0, 12)]:
        p = pencils.scalar_q1(m, dim, ln, seed)
        ev = smallest_eigs(p, nev + 8)
        # a gamma in a relative gap of at least 1e-3 near nev
        k = nev
        while (ev[k] - ev[k - 1]) / ev[k] < 1e-3:
            k += 1
        L = int(np.ceil(1.25 * k / 8) * 8)
        out.append((p, gap_gamma(ev, k), L, k))
    return out


def ws_for(slrf, cases, prec):
    pers = trans = 0
    for p, _, L, _ in cases:
        nnz = int((abs(p.A) + abs(p.B)).nnz)
        a, b = slrf.batch_footprint(p.n, nnz, L, 4, prec)
        pers += a + 4096
        trans += b
    return pers + trans + (1 << 20), trans


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_bitwise_equals_alone(slrf, torch, prec):
    cases = big_cases()
    opt = slrf.default_options(precision=prec)
    alone = []
    for i, (p, gamma, L, k) in enumerate(cases):
        say(f"case alone prec={prec} pencil {i} n={p.n} L={L} nev={k}")
        s = slrf.Solver(p.A, p.B, max_L=L, max_poles=4, options=opt)
        r = s.solve_interval(gamma, L, V0=torch.from_numpy(pencils.start_block(p.n, L, 40 + i)).cuda())
        assert r.status == 0 and r.n_found == k
        alone.append(r)
        s.close()
    ws, arena = ws_for(slrf, cases, prec)
    say(f"case batch prec={prec}: {len(cases)} pencils, workspace {ws / 2**20:.1f} MiB")
    b = slrf.Batch(ws, arena, max_poles=4, options=opt)
    ids = [b.add(p.A, p.B, gamma, L, V0=pencils.start_block(p.n, L, 40 + i))
           for i, (p, gamma, L, _) in enumerate(cases)]
    steps = 0
    while b.step() > 0:
        steps += 1
        assert steps < 60
    for i, pid in enumerate(ids):
        r = b.result(pid)
        a = alone[i]
        say(f"  pencil {i}: found {r.n_found} outer {r.stats['outer_iterations']} "
            f"(alone {a.stats['outer_iterations']})")
        assert r.status == 0 and r.n_found == a.n_found
        assert r.stats["outer_iterations"] == a.stats["outer_iterations"]
        assert np.array_equal(r.evals, a.evals)
        assert np.array_equal(r.resid, a.resid)
        assert torch.equal(r.evecs, a.evecs)
    b.close()


def small_cases():
    """Pencils below the full grid: a 1D string (ILU(0)), a 2D and a 3D
    log-normal pencil (Jacobi), different n, L and gamma."""
    out = []
    lam, _ = closed_1d(2000)
    out.append((pencils.c1_string(), gap_gamma(lam, 12), 24, 12, lam))
    for (m, dim, ln, seed, k, L) in [(30, 2, 0.5, 3, 15, 24), (12, 3, 0.5, 31, 30, 40)]:
        p = pencils.scalar_q1(m, dim, ln, seed)
        ev, _ = dense.all_eigenpairs(p.A, p.B)
        out.append((p, gap_gamma(ev, k), L, k, ev))
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_mixed_kinds_match_oracle(slrf, torch, prec):
    cases = small_cases()
    ws, arena = ws_for(slrf, [(p, g, L, k) for p, g, L, k, _ in cases], prec)
    say(f"case batch small kinds prec={prec}")
    b = slrf.Batch(ws, arena, max_poles=4, options=slrf.default_options(precision=prec))
    ids = [b.add(p.A, p.B, gamma, L) for p, gamma, L, _, _ in cases]
    while b.step() > 0:
        pass
    for pid, (p, gamma, L, k, ev) in zip(ids, cases):
        r = b.result(pid)
        nf = r.n_found
        rel = np.abs(r.evals[:nf] / ev[:nf] - 1).max()
        X = r.evecs.cpu().numpy()[:, :nf]
        orth = np.abs(X.T @ (p.B @ X) - np.eye(nf)).max()
        say(f"  n={p.n}: found {nf} of {k}, rel eig err {rel:.2e}, max rho {r.resid[:nf].max():.2e}, "
            f"orth {orth:.1e}")
        assert r.status == 0 and nf == k == inertia.sparse_ldl_count(p.A, p.B, gamma)
        assert rel < 1e-10
        assert r.resid[:nf].max() <= 1e-8
        assert orth < 1e-10
    b.close()


def test_batch_continuous_admission(slrf, torch):
    """Arena for two pencils: the third is refused until one finishes; results
    are those of the pencils solved alone in a batch of their own."""
    cases = small_cases()
    prec = 0
    nnz = [int((abs(p.A) + abs(p.B)).nnz) for p, *_ in cases]
    fp = [slrf.batch_footprint(p.n, z, L, 4, prec) for (p, _, L, _, _), z in zip(cases, nnz)]
    # order: the largest transient first so that the others fit once it leaves
    order = sorted(range(3), key=lambda i: -fp[i][1])
    arena = fp[order[0]][1] + fp[order[1]][1]
    assert fp[order[2]][1] <= fp[order[0]][1]
    ws = sum(a for a, _ in fp) + 3 * 4096 + arena + (1 << 20)
    say("case continuous admission")
    b = slrf.Batch(ws, arena, max_poles=4, options=slrf.default_options(precision=prec))
    ids = {}
    for i in order[:2]:
        p, g, L, _, _ = cases[i]
        ids[i] = b.add(p.A, p.B, g, L)
    p, g, L, _, _ = cases[order[2]]
    assert b.add(p.A, p.B, g, L, must_fit=False) is None
    pending = order[2]
    finished = {}
    for _ in range(80):
        act = b.step()
        for i, pid in list(ids.items()):
            done, _ = b.query(pid)
            if done and i not in finished:
                finished[i] = b.result(pid)
                b.remove(pid)
                del ids[i]
        if pending is not None:
            p, g, L, _, _ = cases[pending]
            pid = b.add(p.A, p.B, g, L, must_fit=False)
            if pid is not None:
                ids[pending] = pid
                pending = None
        if act == 0 and not ids and pending is None:
            break
    assert len(finished) == 3
    for i, (p, gamma, L, k, ev) in enumerate(cases):
        r = finished[i]
        nf = r.n_found
        say(f"  pencil {i} n={p.n}: found {nf}, outer {r.stats['outer_iterations']}")
        assert r.status == 0 and nf == k
        assert np.abs(r.evals[:nf] / ev[:nf] - 1).max() < 1e-10
    b.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replay_bitwise_equals_eager(slrf, torch, prec):
    cases = small_cases()
    ws, arena = ws_for(slrf, [(p, g, L, k) for p, g, L, k, _ in cases], prec)
    results = []
    for graph in (0, 1):
        stream = torch.cuda.Stream()
        say(f"case graph={graph} prec={prec}")
        b = slrf.Batch(ws, arena, max_poles=4,
                       options=slrf.default_options(precision=prec, graph=graph), stream=stream)
        ids = [b.add(p.A, p.B, g, L) for p, g, L, _, _ in cases]
        while b.step() > 0:
            pass
        results.append([b.result(pid) for pid in ids])
        torch.cuda.synchronize()
        b.close()
    for e, g in zip(*results):
        assert e.status == 0 and g.status == 0
        assert np.array_equal(e.evals, g.evals)
        assert torch.equal(e.evecs, g.evecs)


def test_batched_workload_recipe_with_autotune_and_graph(slrf, torch):
    """Eight instances of the batched workload's recipe (sizes cut to 2e3..1.5e4
    rows so the oracle stays quick), mixed precision, autotuned tiles, graph
    replay: every instance finds the oracle's count and eigenvalues (stored by
    tests/golden/make_golden.py from its shift-invert subspace iteration) and
    agrees with its FP64 solve alone."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "eig_batch8_n2e3_1.5e4.json")) as f:
        gold = json.load(f)
    insts = [pencils.batch_instance(i, n_range=tuple(gold["n_range"])) for i in range(8)]
    cases = [(p, g, L, k) for p, g, L, k in insts]
    ws, arena = ws_for(slrf, cases, 1)
    stream = torch.cuda.Stream()
    opt = slrf.default_options(precision=1, tune=1, graph=1)
    say("case batched recipe, 8 instances, mixed + tune + graph")
    b = slrf.Batch(ws, arena, max_poles=4, options=opt, stream=stream)
    ids = [b.add(p.A, p.B, g, L) for p, g, L, _ in cases]
    while b.step() > 0:
        pass
    res = [b.result(pid) for pid in ids]
    torch.cuda.synchronize()
    b.close()
    for (p, gamma, L, nev), r, g in zip(cases, res, gold["instances"]):
        s = slrf.Solver(p.A, p.B, max_L=L, max_poles=4)
        a = s.solve_interval(gamma, L)
        s.close()
        nf = r.n_found
        cnt = inertia.sparse_ldl_count(p.A, p.B, gamma)
        rel = np.abs(r.evals[:nf] / a.evals[:nf] - 1).max()
        ev_o = np.array(g["eigenvalues"])
        assert g["n"] == p.n and g["gamma"] == gamma and g["count"] == len(ev_o)
        rel_o = np.abs(r.evals[:nf] / ev_o[:nf] - 1).max() if nf == len(ev_o) else np.inf
        say(f"  n={p.n} dim={p.meta['dim']} nev~{nev} L={L}: found {nf} (count {cnt}, oracle {len(ev_o)}), "
            f"outer {r.stats['outer_iterations']}, rel vs FP64 alone {rel:.1e}, vs oracle {rel_o:.1e}")
        assert r.status == 0 and nf == cnt == a.n_found == len(ev_o)
        assert rel < 1e-9 and rel_o < 1e-9
        assert r.resid[:nf].max() <= 1e-8


def test_batched_workload_full_size_instances_match_oracle(slrf, torch):
    """The batched workload's first four pencils at full size (n = 101,124 2D,
    11,664 2D, 19,683 3D, 24,389 3D) in its configuration: one batch, mixed
    precision, COCG with the multicolour SGS, warm starts, autotuned tiles,
    graph replay, N = 6 designed poles each.  Every pencil finds the oracle's
    count and eigenvalues (tests/golden/eig_batch_full4.json) with residuals
    <= 1e-8."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "eig_batch_full4.json")) as f:
        gold = json.load(f)
    N = 6
    opt = slrf.default_options(precision=1, solver=slrf.SOLVER_COCG, precond=slrf.PRECOND_SGS3, recycle=1,
                               graph=1, profile=0, tune=1)
    insts = [pencils.batch_instance(g["index"], n_range=tuple(gold["n_range"])) for g in gold["instances"]]
    pers = trans = 0
    for (p, _, L, _), g in zip(insts, gold["instances"]):
        assert p.n == g["n"] and L == g["L"]
        a, b = slrf.batch_footprint(p.n, int((abs(p.A) + abs(p.B)).nnz), L, N, options=opt)
        pers += a + 4096
        trans += b
    say("case batched workload, first four instances at full size")
    bt = slrf.Batch(pers + trans + (1 << 24), trans, max_poles=N, options=opt, stream=torch.cuda.Stream())
    ids = []
    for p, gamma, L, _ in insts:
        sig, w, _ = slrf.design_poles(N, 1.0, 0.01, gamma)
        ids.append(bt.add(p.A, p.B, gamma, L, sig, w))
    steps = 0
    while bt.step() > 0:
        steps += 1
        assert steps < 60
    res = [bt.result(pid) for pid in ids]
    torch.cuda.synchronize()
    bt.close()
    for (p, gamma, L, _), r, g in zip(insts, res, gold["instances"]):
        nf = r.n_found
        ev_o = np.array(g["eigenvalues"])
        rel_o = np.abs(r.evals[:nf] / ev_o[:nf] - 1).max() if nf == len(ev_o) else np.inf
        say(f"  n={p.n} dim={p.meta['dim']} L={L}: found {nf} (oracle {len(ev_o)}), rel vs oracle {rel_o:.1e}, "
            f"max rho {r.resid[:nf].max():.1e}, outer {r.stats['outer_iterations']}")
        assert r.status == 0 and nf == len(ev_o) == g["count"]
        assert rel_o < 1e-9
        assert r.resid[:nf].max() <= 1e-8
