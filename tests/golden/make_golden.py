"""Writes the stored expected values under tests/golden/ using only ``oracle/``
and the shared input generator ``pencils``.

    python tests/golden/make_golden.py poles     # SLRF pole tables, N = 4, 6, 8
    python tests/golden/make_golden.py count_c2  # inertia count of the 64^3 scalar pencil
    python tests/golden/make_golden.py eig_c2    # eigenvalues of the 64^3 scalar pencil in (0, 421]
    python tests/golden/make_golden.py eig_c3    # eigenvalues of the 48^3-node elasticity pencil
    python tests/golden/make_golden.py count_c3  # inertia count of that pencil at its gamma
    python tests/golden/make_golden.py eig_batch # eigenvalues of eight batched-recipe pencils
    python tests/golden/make_golden.py eig_serve # eigenvalues of the serving test's six requests
    python tests/golden/make_golden.py eig_batch_full  # the batched workload's first four pencils
    python tests/golden/make_golden.py eig_serve_mix   # the served-mix test's four requests

Pole tables: the oracle's SLRF design (ridge-regularised least squares, see
oracle/poles.py) at gamma = 1, alpha = 1, beta = 0.01 (the paper's Section 4.2
setting).  Count: Sylvester inertia of A - gamma B for the 64^3 log-normal
scalar pencil at gamma = 421 (sparse symmetric factorisation; several minutes).
Eigenvalues: shift-invert subspace iteration with one banded Cholesky factor of
A (oracle/shift_invert.py; minutes for the 64^3 pencil, about an hour for the
elasticity pencil), with the Sylvester count of A - gamma B by banded block
elimination at three block sizes beside it.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import pencils  # noqa: E402
from oracle import banded, inertia, poles, shift_invert  # noqa: E402


def make_poles():
    for N in (4, 6, 8):
        t = time.time()
        s, w, J = poles.design(N, 1.0, 0.01, 1.0)
        out = {"N": N, "alpha": 1.0, "beta": 0.01, "gamma": 1.0, "eta": poles.ETA,
               "sigma_re": s.real.tolist(), "sigma_im": s.imag.tolist(),
               "w_re": w.real.tolist(), "w_im": w.imag.tolist(), "J_fit": J,
               "separation_factor": poles.separation_factor(s, w, 1.0),
               "source": "oracle.poles.design (paper Section 3.1)"}
        with open(os.path.join(HERE, f"poles_N{N}_a1_b0.01.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(f"N={N} done in {time.time() - t:.1f}s", flush=True)


def make_count_c2():
    p = pencils.c2_scalar3d()
    t = time.time()
    c = inertia.sparse_ldl_count(p.A, p.B, 421.0)
    out = {"pencil": p.name, "n": p.n, "gamma": 421.0, "count_below_gamma": c,
           "source": "oracle.inertia.sparse_ldl_count (Sylvester inertia)",
           "seconds": time.time() - t}
    with open(os.path.join(HERE, "count_scalar3d_m64_ln0.5_s2_g421.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out, flush=True)


def _log(msg):
    print(time.strftime("%H:%M:%S"), msg, flush=True)


def _block_counts(p, gamma):
    """Sylvester counts at three block sizes; unpivoted elimination of an
    indefinite matrix can lose accuracy, so disagreeing counts are recorded as
    such rather than trusted."""
    out = {}
    for nb in (512, 1024, 1536):
        try:
            out[str(nb)] = banded.inertia_count(p.A, p.B, gamma, nb=nb)
        except RuntimeError as e:
            out[str(nb)] = str(e)
        _log(f"inertia nb={nb}: {out[str(nb)]}")
    return out


def _large_eigs(p, gamma_run, nsub, seed, tol):
    t = time.time()
    F = banded.band_cholesky(p.A)
    _log(f"banded Cholesky of A: n={p.n}, kd={F.kd}, {time.time() - t:.0f} s")
    V0 = pencils.start_block(p.n, nsub, seed)
    r = shift_invert.subspace_iteration(p.A, p.B, gamma_run, V0, tol=tol, factor=F, log=_log)
    return r, time.time() - t


def make_eig_c2():
    """All eigenvalues of the 64^3 log-normal scalar pencil in (0, 421]."""
    p = pencils.c2_scalar3d()
    gamma = 421.0
    r, secs = _large_eigs(p, gamma, 240, 11, 1e-10)
    out = {"pencil": p.name, "n": p.n, "gamma": gamma, "count": len(r.theta),
           "eigenvalues": r.theta.tolist(), "max_rho": float(r.rho.max()),
           "next_ritz_value": float(r.theta_all[len(r.theta)]),
           "subspace": 240, "iterations": r.iterations, "converged": bool(r.converged),
           "inertia_counts": _block_counts(p, gamma),
           "source": "oracle.shift_invert.subspace_iteration (shift 0, banded Cholesky)",
           "seconds": secs}
    with open(os.path.join(HERE, "eig_scalar3d_m64_ln0.5_s2_g421.json"), "w") as f:
        json.dump(out, f, indent=1)
    _log(f"c2: {out['count']} eigenvalues, max rho {out['max_rho']:.2e}")


def make_count_c3():
    """Sylvester count of A - gamma B for the elasticity pencil at the gamma that
    make_eig_c3 stored (sparse symmetric factorisation)."""
    p = pencils.c3_elasticity()
    path = os.path.join(HERE, "eig_elast3d_48_s3.json")
    with open(path) as f:
        d = json.load(f)
    t = time.time()
    c = inertia.sparse_ldl_count(p.A, p.B, d["gamma"])
    d["sparse_ldl_count"] = c
    d["sparse_ldl_seconds"] = time.time() - t
    with open(path, "w") as f:
        json.dump(d, f, indent=1)
    _log(f"c3 count at gamma {d['gamma']}: {c} (eigenvalues stored: {d['count']})")


def make_eig_c3():
    """Eigenvalues of the elasticity pencil below 112, then gamma in the middle of
    the widest gap (relative width >= 1e-4) that leaves 195..205 below it."""
    p = pencils.c3_elasticity()
    r, secs = _large_eigs(p, 112.0, 520, 13, 1e-10)
    th = r.theta
    best = None
    for k in range(195, min(206, len(th))):
        gap = (th[k] - th[k - 1]) / th[k]
        if best is None or gap > best[1]:
            best = (k, gap)
    k, gap = best
    gamma = float(0.5 * (th[k - 1] + th[k]))
    out = {"pencil": p.name, "n": p.n, "gamma": gamma, "count": k,
           "relative_gap": gap, "eigenvalues": th[:k].tolist(),
           "next_eigenvalue": float(th[k]), "max_rho": float(r.rho[:k].max()),
           "subspace": 520, "iterations": r.iterations, "converged": bool(r.converged),
           "source": "oracle.shift_invert.subspace_iteration (shift 0, banded Cholesky)",
           "seconds": secs}
    with open(os.path.join(HERE, "eig_elast3d_48_s3.json"), "w") as f:
        json.dump(out, f, indent=1)
    _log(f"c3: gamma {gamma}, {k} eigenvalues, gap {gap:.2e}, max rho {out['max_rho']:.2e}")


BATCH_N_RANGE = (2e3, 1.5e4)
SERVE_TEST_INSTANCES = [1, 6, 8, 34, 42, 51]


def make_eig_batch(indices=range(8), n_range=BATCH_N_RANGE, name="eig_batch8_n2e3_1.5e4.json"):
    """Eigenvalues in (0, gamma] of instances of the batched workload's recipe
    (pencils.batch_instance; by default the first eight with sizes cut to
    2e3..1.5e4 rows), by shift-invert subspace iteration, with their Sylvester
    counts beside them."""
    out = {"n_range": list(n_range), "instances": [],
           "source": "oracle.shift_invert.subspace_iteration (shift 0, banded Cholesky); "
                     "oracle.inertia.sparse_ldl_count"}
    for i in indices:
        p, gamma, L, nev = pencils.batch_instance(i, n_range=n_range)
        t = time.time()
        F = banded.band_cholesky(p.A)
        V0 = pencils.start_block(p.n, max(2 * nev, L + 16), 100 + i)
        r = shift_invert.subspace_iteration(p.A, p.B, gamma, V0, tol=1e-11, factor=F)
        cnt = inertia.sparse_ldl_count(p.A, p.B, gamma)
        if not r.converged or cnt != len(r.theta):
            raise RuntimeError(f"instance {i}: converged {r.converged}, {len(r.theta)} values, count {cnt}")
        out["instances"].append({
            "index": i, "pencil": p.name, "n": p.n, "gamma": gamma, "L": L, "count": cnt,
            "eigenvalues": r.theta.tolist(), "next_ritz_value": float(r.theta_all[len(r.theta)]),
            "max_rho": float(r.rho.max()), "iterations": r.iterations, "seconds": time.time() - t})
        _log(f"batch instance {i}: n={p.n}, {cnt} eigenvalues, max rho {r.rho.max():.1e}")
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)


SERVE_MIX = [("scalar", 1), ("elasticity", (10, 7101)), ("scalar", 8), ("elasticity", (12, 7103))]


def make_eig_serve_mix():
    """The requests of the served-mix GPU test: two scalar pencils of the batched
    recipe (their own gamma) and two small elasticity pencils of the serving
    recipe (nodes^3 free nodes x 3, log-normal Young's modulus sigma 0.7, nu 0.3,
    density U[0.8, 1.2]) with gamma in the middle of the widest relative gap
    that leaves 25..40 eigenvalues below it."""
    out = {"requests": [], "source": "oracle.shift_invert.subspace_iteration (shift 0, banded Cholesky); "
                                     "oracle.inertia.sparse_ldl_count"}
    for kind, arg in SERVE_MIX:
        t = time.time()
        if kind == "scalar":
            p, gamma, L, _ = pencils.batch_instance(arg)
            rec = {"kind": kind, "index": arg}
        else:
            nodes, seed = arg
            p = pencils.elasticity_q1(nodes, nodes - 1, nodes - 1, 1.0 / nodes, 0.7, 0.3, (0.8, 1.2), seed)
            F = banded.band_cholesky(p.A)
            ca, cp = pencils.ELASTICITY_SPECTRUM
            lo = shift_invert.subspace_iteration(p.A, p.B, ca * 50.0 ** cp, pencils.start_block(p.n, 96, seed),
                                                 tol=1e-11, factor=F)
            th = lo.theta
            k = max(range(25, min(41, len(th))), key=lambda k: (th[k] - th[k - 1]) / th[k])
            gamma = float(0.5 * (th[k - 1] + th[k]))
            L = int(np.ceil(np.ceil(1.2 * k) / 8.0) * 8)
            rec = {"kind": kind, "nodes": nodes, "seed": seed,
                   "relative_gap": float((th[k] - th[k - 1]) / th[k])}
        F = banded.band_cholesky(p.A)
        V0 = pencils.start_block(p.n, L + 24, 200 + len(out["requests"]))
        r = shift_invert.subspace_iteration(p.A, p.B, gamma, V0, tol=1e-11, factor=F)
        cnt = inertia.sparse_ldl_count(p.A, p.B, gamma)
        if not r.converged or cnt != len(r.theta):
            raise RuntimeError(f"{kind} {arg}: converged {r.converged}, {len(r.theta)} values, count {cnt}")
        rec.update({"pencil": p.name, "n": p.n, "gamma": gamma, "L": L, "count": cnt,
                    "eigenvalues": r.theta.tolist(), "next_ritz_value": float(r.theta_all[len(r.theta)]),
                    "max_rho": float(r.rho.max()), "seconds": time.time() - t})
        out["requests"].append(rec)
        _log(f"serve mix {kind} {arg}: n={p.n}, gamma {gamma:.6g}, {cnt} eigenvalues")
    with open(os.path.join(HERE, "eig_serve_mix4.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    what = sys.argv[1:] or ["poles", "count_c2"]
    if "poles" in what:
        make_poles()
    if "count_c2" in what:
        make_count_c2()
    if "eig_c2" in what:
        make_eig_c2()
    if "eig_c3" in what:
        make_eig_c3()
    if "count_c3" in what:
        make_count_c3()
    if "eig_batch" in what:
        make_eig_batch()
    if "eig_batch_full" in what:   # the first instances of the batched workload at full size
        make_eig_batch(range(4), (5e3, 2e5), "eig_batch_full4.json")
    if "eig_serve_mix" in what:
        make_eig_serve_mix()
    if "eig_serve" in what:   # the requests of the serving loop's GPU test
        make_eig_batch(SERVE_TEST_INSTANCES, (5e3, 2e5), "eig_serve6.json")
