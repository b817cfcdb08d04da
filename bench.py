"""Benchmark: eigenpairs/s of the SLRF interval eigensolver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c1]
                    [--precision both|mixed|fp64] [--no-cpu-baseline] [--calibrate-copy]

A step is one complete slrf_solve_interval (filter application with the shifted
BiCGStab solves over all poles and columns, filter sum, B-orthonormalising
Rayleigh-Ritz and residuals, repeated until every Ritz pair in (0, gamma] has
relative residual <= 1e-8) on synthetic, seeded input resident in HBM.

Workload c2 (default): 3D scalar vibration pencil, trilinear hexahedra on a
64^3 grid of the unit cube with Dirichlet boundary (n = 250047, 27 nnz/row),
log-normal coefficient (sigma 0.5, seed 2), consistent mass; gamma = 421
(87 eigenvalues below it, Sylvester count from the oracle); L = 128, N = 6 SLRF
poles (alpha 1, beta 0.01).  `value` is the mixed-precision form (complex FP32
BiCGStab with FP64 defect correction, FP64 Rayleigh-Ritz and residuals); the
plain FP64 form (complex FP64 BiCGStab, point Jacobi, inner tolerance 1e-10) is
timed in the same run and reported under "fp64" for the comparison.

Prints one JSON line.  `roofline` is measured live: HIP events around every
launch of the dominant kernel (the complex-shifted sparse product) during the
timed steps, against its algorithmic bytes (each processed column tile reads its
input block and writes its output block once, the merged CSR once per launch).
`cpu_baseline` times the FP64 oracle's BiCGStab on a bounded sample of the same
workload on the host and scales it to the whole solve.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "eigenpairs/s at rel. residual 1e-8, mixed vs FP64; HBM GB/s; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    import pencils
    if name == "c2":
        p = pencils.c2_scalar3d()
        return dict(pencil=p, gamma=421.0, L=128, N=6, expect=87,
                    desc=("3D scalar vibration, trilinear hex 64^3 unit cube, Dirichlet, "
                          "log-normal coefficient sigma=0.5 seed 2, consistent mass "
                          f"(n={p.n}, nnz={p.A.nnz}); gamma=421 (87 eigenvalues); L=128; "
                          "N=6 SLRF poles alpha=1 beta=0.01; point-Jacobi BiCGStab"))
    if name == "c1":
        import numpy as np
        p = pencils.c1_string()
        n = p.n
        h = 1.0 / (n + 1)
        k = np.arange(20, 22)
        lam = (6 / h ** 2) * 2 * np.sin(0.5 * k * np.pi * h) ** 2 / (2 + np.cos(k * np.pi * h))
        return dict(pencil=p, gamma=0.5 * (lam[0] + lam[1]), L=32, N=4, expect=20,
                    desc="1D linear-FE string n=2000, 20 eigenvalues; L=32; N=4; ILU(0) BiCGStab")
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(wl, sig, solve_stats):
    """Oracle BiCGStab (point Jacobi, FP64) on 1 pole x 4 columns for a fixed number
    of iterations, single thread; scaled by the column-iterations of the GPU solve."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import pencils
    from oracle import krylov
    p = wl["pencil"]
    cols, iters = 4, 20 if p.n > 100000 else 200
    F = p.B @ pencils.start_block(p.n, cols, 77)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        krylov.bicgstab(p.A, p.B, sig[:1], F, 0.0, iters, fixed_iters=iters)
        dt = time.perf_counter() - t0
    per_col_it = dt / (cols * iters)
    col_its = solve_stats["spmv_total"] / 2.0
    est = per_col_it * col_its
    return {"value": solve_stats["n_found"] / est, "unit": "eigenpairs/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"oracle.krylov.bicgstab (FP64, point Jacobi) on 1 pole x {cols} columns for "
                       f"{iters} iterations took {dt:.1f} s on 1 host thread; scaled to the "
                       f"{col_its:.0f} column-iterations of one GPU solve (Rayleigh-Ritz excluded)"),
            "seconds_per_column_iteration": per_col_it}


def run_form(slrf, wl, precision, steps, warmup, sig, w, V0):
    import torch
    p = wl["pencil"]
    L, N, gamma = wl["L"], wl["N"], wl["gamma"]
    opt = slrf.default_options(profile=1, precision=precision)
    solver = slrf.Solver(p.A, p.B, max_L=L, max_poles=N, options=opt)
    tag = "mixed" if precision == slrf.MIXED else "fp64"
    log(f"{tag}: n={p.n} L={L} N={N} workspace {solver.ws_bytes / 2**30:.2f} GiB")

    def step():
        r = solver.solve_interval(gamma, L, sig, w, V0=V0)
        if r.status != 0 or r.n_found != wl["expect"]:
            raise SystemExit(f"{tag} solve failed: status {r.status} found {r.n_found} ({r.message})")
        return r

    for i in range(warmup):
        r = step()
        log(f"{tag} warmup {i}: {r.stats['seconds']:.2f} s, outer {r.stats['outer_iterations']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    found, results = 0, []
    for i in range(steps):
        r = step()
        found += r.n_found
        results.append(r)
        log(f"{tag} step {i}: {r.stats['seconds']:.2f} s, outer {r.stats['outer_iterations']}, "
            f"found {r.n_found}, max rho {r.stats['max_resid']:.2e}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del solver
    torch.cuda.empty_cache()
    ks = {k: sum(r.stats["kernels"][k] for r in results) for k in
          ("spmm_seconds", "spmm_launches", "spmm_bytes", "update_seconds", "update_launches",
           "update_bytes")}
    return dict(value=found / dt, dt=dt, results=results, ks=ks)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="both", choices=["both", "mixed", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB elementwise copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the pole-sharded "
              "multi-GPU form is not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2503_21618_amd as slrf
    import pencils

    if args.calibrate_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.neg(a, out=b)          # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b
    wl = workload(args.workload)
    p = wl["pencil"]
    sig, w, _ = slrf.design_poles(wl["N"], 1.0, 0.01, wl["gamma"])
    V0 = torch.from_numpy(pencils.start_block(p.n, wl["L"], 1)).cuda()
    forms = {}
    if args.precision in ("both", "mixed"):
        forms["mixed"] = run_form(slrf, wl, slrf.MIXED, args.steps, args.warmup, sig, w, V0)
    if args.precision in ("both", "fp64"):
        fp_steps, fp_warm = (1, 0) if args.precision == "both" else (args.steps, args.warmup)
        forms["fp64"] = run_form(slrf, wl, slrf.FP64, fp_steps, fp_warm, sig, w, V0)
    main_form = "mixed" if "mixed" in forms else "fp64"
    m = forms[main_form]
    ks = m["ks"]
    spmm_gbs = ks["spmm_bytes"] / ks["spmm_seconds"] / 1e9
    upd_gbs = ks["update_bytes"] / ks["update_seconds"] / 1e9
    prec = "complex FP32 inner solves + FP64 defect correction and Rayleigh-Ritz" if main_form == "mixed" \
        else "complex FP64 inner solves"
    out = {
        "metric": METRIC, "value": m["value"], "unit": "eigenpairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * m["dt"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if main_form == "mixed" else "f64",
        "data": "synthetic", "config": {"workload": wl["desc"] + "; " + prec},
        "roofline": {"bound": "hbm", "achieved": spmm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": spmm_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"k_spmm_v / k_spmm_t <{'float' if main_form == 'mixed' else 'double'}> "
                               "(complex-shifted sparse product)",
                     "launches": ks["spmm_launches"],
                     "avg_launch_ms": 1e3 * ks["spmm_seconds"] / max(1, ks["spmm_launches"])},
        "vector_updates": {"achieved_GBs": upd_gbs, "frac": upd_gbs / HBM_PEAK_GBS,
                           "avg_launch_ms": 1e3 * ks["update_seconds"] / max(1, ks["update_launches"])},
        "solve": {k: m["results"][-1].stats[k] for k in ("outer_iterations", "spmv_total", "n_found",
                                                         "max_resid", "inner_iterations",
                                                         "filter_seconds")},
    }
    if "fp64" in forms and main_form != "fp64":
        f = forms["fp64"]
        fk = f["ks"]
        out["fp64"] = {"value": f["value"], "ms_per_step": 1e3 * f["dt"],
                       "spmm_GBs": fk["spmm_bytes"] / fk["spmm_seconds"] / 1e9,
                       "update_GBs": fk["update_bytes"] / fk["update_seconds"] / 1e9,
                       "outer_iterations": f["results"][-1].stats["outer_iterations"],
                       "max_resid": f["results"][-1].stats["max_resid"]}
        out["mixed_over_fp64"] = m["value"] / f["value"]
    if not args.no_cpu_baseline:
        log("cpu baseline sample...")
        ref = forms.get("fp64", m)
        out["cpu_baseline"] = cpu_baseline(wl, sig, ref["results"][-1].stats)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
