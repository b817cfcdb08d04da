"""GPU check of Section 3.2's filter comparison on a small 2D pencil: per-pole mean
BiCGStab iterations of the library's FP64 solves against the oracle's BiCGStab
on the same systems, for the SLRF design and the three quadrature-rule filters
(N = 3), and the comparison's findings as properties: the middle pole is shared
by the three rules and costs them the same; the Gauss-Chebyshev pole nearest the
real axis is the most expensive of all; the SLRF poles cost about the same."""
import numpy as np
import pytest

import pencils
from oracle import dense, krylov

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


def test_filter_comparison_inner_iterations(slrf, torch):
    p = pencils.scalar_q1(40, 2, 0.5, 7)               # n = 1521
    ev, _ = dense.all_eigenpairs(p.A, p.B)
    gamma = 0.5 * (ev[19] + ev[20])
    L = 24
    X = pencils.start_block(p.n, L, 1)
    Xd = torch.from_numpy(X).cuda()
    F = p.B @ X
    filters = {"SLRF": slrf.design_poles(3, 0.5, 0.01, gamma)[:2]}
    for rule, name in ((0, "midpoint"), (1, "gauss-legendre"), (2, "gauss-chebyshev")):
        filters[name] = slrf.quadrature_poles(rule, 3, gamma)
    its = {}
    for name, (sig, w) in filters.items():
        gpu, orc = [], []
        for j in range(3):
            opt = slrf.default_options(precision=slrf.FP64, inner_tol=1e-10)
            s = slrf.Solver(p.A, p.B, max_L=L, max_poles=1, options=opt)
            _, st = s.filter_apply(Xd, sig[j:j + 1], w[j:j + 1])
            s.close()
            _, it, _, _ = krylov.bicgstab(p.A, p.B, sig[j:j + 1], F, 1e-10, 1000)
            orc.append(np.mean(it))                      # a half-step exit counts its iteration in both
            gpu.append(st["mean_iterations"])
        print(f"{name}: GPU {np.round(gpu, 2)} oracle {np.round(orc, 2)}", flush=True)
        its[name] = np.array(gpu)
        # with a few hundred point-Jacobi iterations, rounding-order differences
        # move a column's exit by a few iterations (the iterates themselves are
        # compared at fixed iteration counts in test_gpu_parity.py)
        assert np.all(np.abs(np.array(gpu) - np.array(orc)) <= np.maximum(2.0, 0.05 * np.array(orc)))
    mid = [its[r][1] for r in ("midpoint", "gauss-legendre", "gauss-chebyshev")]
    assert max(mid) - min(mid) <= 1.0
    allq = np.concatenate([its[r] for r in ("midpoint", "gauss-legendre", "gauss-chebyshev")])
    assert its["gauss-chebyshev"][2] == allq.max()
    assert its["SLRF"].max() / its["SLRF"].min() < its["gauss-chebyshev"].max() / its["gauss-chebyshev"].min()
