"""Benchmark: eigenpairs/s of the SLRF interval eigensolver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c1|batched|served|filters]
                    [--precond sgs|jacobi] [--no-c2] [--no-cpu-baseline]
    python bench.py --counters-probe [--workload c3] | --summarize-pmc FETCH_CSV WRITE_CSV PROBE_LOG
    python bench.py --mfma-probe | --summarize-mfma PMC_CSV TRACE_CSV

Default workload c3: 3D linear elasticity on trilinear hexahedra, 48^3 free
nodes x 3 unknowns (n = 331776, 81 nnz/row, clamped x = 0 face, log-normal
Young's modulus sigma 0.7 seed 3, nu 0.3, density U[0.8, 1.2]), consistent mass;
gamma from the oracle's eigenvalues (mid-gap, 199 below it); L = 256, N = 8 SLRF
poles (alpha 1, beta 0.01); mixed precision (complex FP32 COCG with FP64 defect
correction, FP64 Rayleigh-Ritz and residuals), the multicolour node-block
symmetric Gauss-Seidel preconditioner, warm starts across outer iterations.

A step is one outer iteration of Algorithm 1 on the workload (filter
application, filter sum, Rayleigh-Ritz, residuals); complete solves run back to
back and each is checked against the oracle's eigenvalues.  `value` counts the
eigenpairs of the solves that ran entirely inside the K timed steps over the
time of their steps.  Beside it, the 64^3 scalar pencil (C2) is solved once in
the mixed and once in the FP64 form ("c2_64cube").

Prints one JSON line.  `roofline` is measured live: HIP events around every
launch of the dominant kernel (the COCG iteration's colour sweeps, which carry
the product with A - sigma B) during the timed steps, against its algorithmic
bytes.  `roofline.traffic` is the bytes per launch from the rocprofv3
FETCH_SIZE and WRITE_SIZE passes summarised in profiles/spmm_c3_pmc.txt (each
scaled by what the counter reads for a copy kernel of known size), scaled to the
launches of the timed steps; it is null when the kernel sources differ from the
ones the counters were taken with.  `cpu_baseline` times the FP64 oracle on a
bounded sample of the same workload on the host's cores and scales it to one
solve.

Counter collection (the probe runs full-width launches of the products):
    rocprofv3 --pmc FETCH_SIZE --kernel-include-regex "k_spmm|k_cocg_spmm|k_sgs_sweep|elementwise" \
        --output-format csv -d <dir> -o run -- python3 bench.py --counters-probe --workload c3
    (again with WRITE_SIZE)
    python bench.py --summarize-pmc <fetch csv> <write csv> <probe log> --workload c3 > profiles/spmm_c3_pmc.txt
"""
import argparse
import csv
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "eigenpairs/s at rel. residual 1e-8, mixed vs FP64; HBM GB/s; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# FP32 FMA without packed (two-wide) instructions, which the HIP sources are compiled not to emit:
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz; FP64 FMA runs at the same rate
FP32_NONPACKED_TFS = 78.6
FP64_TFS = 78.6
def pmc_summary_path(wl_key):
    return os.path.join(ROOT, "profiles", f"spmm_{wl_key}_pmc.txt")
KERNEL_SOURCES = ["krylov.hip", "device_util.h", "kernels.h"]
COPY_BYTES = 1 << 30      # the calibration copy reads and writes 1 GiB


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name, probe=False):
    import pencils
    if name == "c2":
        p = pencils.c2_scalar3d()
        return dict(pencil=p, gamma=421.0, L=128, N=6, expect=87,
                    desc=("3D scalar vibration, trilinear hex 64^3 unit cube, Dirichlet, "
                          "log-normal coefficient sigma=0.5 seed 2, consistent mass "
                          f"(n={p.n}, nnz={p.A.nnz}); gamma=421 (87 eigenvalues); L=128; "
                          "N=6 SLRF poles alpha=1 beta=0.01; point Jacobi"))
    if name == "c3":
        p = pencils.c3_elasticity()
        g = c3_golden(required=not probe)
        return dict(pencil=p, gamma=g["gamma"], L=256, N=8, expect=g["count"], precond=3,
                    eigs=g["eigenvalues"],
                    desc=("3D linear elasticity, trilinear hex, 48^3 free nodes x 3 dofs, clamped x=0 face, "
                          "Young's modulus log-normal sigma=0.7 seed 3, nu=0.3, density U[0.8,1.2] "
                          f"(n={p.n}, nnz={p.A.nnz}); gamma={g['gamma']:.6g} ({g['count']} eigenvalues by "
                          "the oracle, mid-gap); L=256; N=8 SLRF poles alpha=1 beta=0.01"))
    if name == "c1":
        import numpy as np
        p = pencils.c1_string()
        n = p.n
        h = 1.0 / (n + 1)
        k = np.arange(20, 22)
        lam = (6 / h ** 2) * 2 * np.sin(0.5 * k * np.pi * h) ** 2 / (2 + np.cos(k * np.pi * h))
        return dict(pencil=p, gamma=0.5 * (lam[0] + lam[1]), L=32, N=4, expect=20,
                    desc="1D linear-FE string n=2000, 20 eigenvalues; L=32; N=4; ILU(0)")
    raise SystemExit(f"unknown workload {name}")


def c3_golden(required=True):
    """gamma, count and eigenvalues of the elasticity pencil stored by
    tests/golden/make_golden.py (the oracle's shift-invert subspace iteration).
    The counter probe, which checks no result, may run without them."""
    path = os.path.join(ROOT, "tests", "golden", "eig_elast3d_48_s3.json")
    if not os.path.exists(path) and not required:
        return {"gamma": 101.0, "count": None, "eigenvalues": []}
    with open(path) as f:
        return json.load(f)


def c2_golden():
    with open(os.path.join(ROOT, "tests", "golden", "eig_scalar3d_m64_ln0.5_s2_g421.json")) as f:
        return json.load(f)


_SAMPLE = {}


def _sample_worker(task):
    """One oracle sample in a forked worker (the pencil is inherited): COCG or
    BiCGStab iterations on a few columns, or B-orthonormalisation projections,
    or residual products.  Returns the seconds it took."""
    import numpy as np

    import pencils
    from oracle import krylov, subspace
    from threadpoolctl import threadpool_limits
    wl, sig = _SAMPLE["wl"], _SAMPLE["sig"]
    p = wl["pencil"]
    kind, k = task
    with threadpool_limits(1):
        t0 = time.perf_counter()
        if kind in ("inner", "setup"):
            # "setup": the same call with no iteration (the preconditioner set-up and
            # the start), which the iteration samples subtract
            pc = {3: "bjac3", 4: "mcsgs", 5: "mcsgs3"}.get(wl.get("precond", 0), "jacobi")
            F = p.B @ pencils.start_block(p.n, _SAMPLE["cols"], 77 + k)
            solve = krylov.cocg if wl.get("solver", 0) == 1 else krylov.bicgstab
            its = _SAMPLE["iters"] if kind == "inner" else 0
            # node-block SGS at the library's default relaxation (sgs_omega 0: 0.7 for node blocks)
            kw = {"omega": 0.7} if pc == "mcsgs3" else {}
            solve(p.A, p.B, sig[k % len(sig):k % len(sig) + 1], F, 0.0, its, fixed_iters=its, precond=pc, **kw)
        elif kind == "mgs":
            subspace.mgs_b(pencils.start_block(p.n, _SAMPLE["mgs_cols"], 99 + k), p.B)
        else:
            X = pencils.start_block(p.n, _SAMPLE["res_cols"], 55 + k)
            subspace.relative_residuals(p.A, p.B, X, np.ones(X.shape[1]))
        return time.perf_counter() - t0


def cpu_sample(wl, sig):
    """Times a bounded sample of the FP64 oracle on the host's cores before the GPU
    is touched (the workers are forked from this process): P workers, each
    running the oracle's inner solver (the workload's preconditioner) on one pole
    x `cols` columns for `iters` iterations, then the oracle's B-orthonormalising
    Gram-Schmidt on a few columns and its residual products.  The oracle is
    single-threaded per call (SciPy sparse products), so the host's cores are
    used by running the independent samples side by side."""
    import multiprocessing as mp
    import platform
    ncpu = os.cpu_count() or 1
    P = max(2, min(ncpu, 16))     # one worker times the set-up, the others the iterations
    big = wl["pencil"].A.nnz > 1e7
    _SAMPLE.update(wl=wl, sig=sig, cols=4, iters=4 if big else 12, mgs_cols=6, res_cols=16)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        model = platform.processor()
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(P) as pool:
        timed = pool.map(_sample_worker, [("setup", 0)] + [("inner", k) for k in range(1, P)])
        mgs = pool.map(_sample_worker, [("mgs", k) for k in range(P)])
        res = pool.map(_sample_worker, [("res", k) for k in range(P)])
    wall = time.perf_counter() - t0
    c, it, m, rc = _SAMPLE["cols"], _SAMPLE["iters"], _SAMPLE["mgs_cols"], _SAMPLE["res_cols"]
    # per unit of work, with P workers sharing the host: seconds of wall time per unit
    setup = timed[0]
    inner = [max(0.0, t - setup) for t in timed[1:]] or [0.0]
    return {"workers": P, "host_cpus": ncpu, "cpu_model": model, "wall_seconds": wall,
            "s_per_column_iteration": max(inner) / (max(1, P - 1) * c * it),
            "s_setup_per_pole": setup,
            # mgs_b on m columns: 2 passes of m (m - 1) / 2 projections and 2 m norms,
            # each one product with B: m (m + 3) products
            "s_per_b_product": max(mgs) / (P * m * (m + 3)),
            "s_per_residual_column": max(res) / (P * rc),
            "sample": (f"{P} forked workers on {ncpu} host CPUs ({model}): oracle inner solver on 1 pole x {c} "
                       f"columns x {it} iterations in {P - 1} of them, its set-up alone in the other, "
                       f"oracle.subspace.mgs_b on {m} columns each, "
                       f"oracle.subspace.relative_residuals on {rc} columns each; {wall:.1f} s wall")}


def cpu_baseline(smp, solve_stats, L, N):
    """Scales the oracle sample to one complete solve of the workload: the GPU
    solve's column-iterations (products with A - sigma B), the preconditioner
    set-up of the N poles once, plus per outer iteration the oracle's two-pass
    B-Gram-Schmidt of the L filtered columns (L (L + 3) products with B) and its
    residuals of the L Ritz pairs."""
    outer = solve_stats["outer_iterations"]
    col_its = solve_stats["spmv_total"]
    est = (col_its * smp["s_per_column_iteration"] + N * smp["s_setup_per_pole"]
           + outer * L * (L + 3) * smp["s_per_b_product"] + outer * L * smp["s_per_residual_column"])
    return {"value": solve_stats["n_found"] / est, "unit": "eigenpairs/s", "cores": smp["workers"],
            "kind": "oracle", "host_cpus": smp["host_cpus"], "cpu_model": smp["cpu_model"],
            "sample": smp["sample"] + (f"; scaled to one solve: {col_its} column-iterations, {outer} outer "
                                       f"iterations of Gram-Schmidt and residuals on L={L} columns"),
            "estimated_solve_seconds": est}


def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2503_21618_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_pmc_summary(wl_key):
    """key: value lines of the committed counter summary, or None."""
    path = pmc_summary_path(wl_key)
    if not os.path.exists(path):
        return None
    d = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            d[k.strip()] = v.strip()
    return d


def hbm_traffic(dtype, avg_alg_bytes, family="bicgstab", workload_key="c2"):
    """HBM bytes per launch of the sparse product from the counter summary, scaled
    from the probe's full-width launches to launches that average avg_alg_bytes
    algorithmic bytes (converged tiles are skipped); None if the summary is
    missing or the kernel sources changed since it was taken."""
    d = read_pmc_summary(workload_key)
    if not d or d.get("source_sha256") != kernel_source_hash():
        return None, "no counter summary for the current kernel sources"
    key = dtype if family == "bicgstab" else f"{family} {dtype}"
    if f"full_launch_traffic_bytes {key}" not in d:
        return None, f"no counter summary for the {family} sparse product"
    full_traffic = float(d[f"full_launch_traffic_bytes {key}"])
    full_alg = float(d[f"full_launch_algorithmic_bytes {key}"])
    return full_traffic * avg_alg_bytes / full_alg, (
        f"profiles/{os.path.basename(pmc_summary_path(workload_key))}: FETCH_SIZE + WRITE_SIZE per "
        f"full-width launch {full_traffic / 1e9:.3f} GB vs algorithmic {full_alg / 1e9:.3f} GB, "
        "scaled by the timed launches' mean algorithmic bytes")


def counters_probe(wl_key):
    """Short run for the rocprofv3 counter passes: a 1 GiB copy kernel (reads and
    writes COPY_BYTES) and full-width launches of the sparse product on the
    workload (fixed inner iterations, no column converges): BiCGStab and COCG in
    both precisions on the 64^3 scalar pencil, COCG in FP32 (the benchmark's
    form) on the elasticity pencil."""
    import torch

    import paper_2503_21618_amd as slrf
    import pencils
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b
    log("copy kernel done")
    wl = workload(wl_key, probe=True)
    p = wl["pencil"]
    sig, w, _ = slrf.design_poles(wl["N"], 1.0, 0.01, wl["gamma"])
    X = torch.from_numpy(pencils.start_block(p.n, wl["L"], 1)).cuda()
    sgs_pc = slrf.PRECOND_SGS if wl_key == "c2" else slrf.PRECOND_SGS3
    forms = ([(slrf.SOLVER_BICGSTAB, "bicgstab", slrf.MIXED, "float"), (slrf.SOLVER_BICGSTAB, "bicgstab", slrf.FP64, "double"),
              (slrf.SOLVER_COCG, "cocg", slrf.MIXED, "float"), (slrf.SOLVER_COCG, "cocg", slrf.FP64, "double")]
             if wl_key == "c2" else [(slrf.SOLVER_COCG, "cocg", slrf.MIXED, "float")])
    forms.append((slrf.SOLVER_COCG, "sgs", slrf.MIXED, "float"))
    for solver, family, prec, dtype in forms:
        opt = slrf.default_options(profile=1, precision=prec, inner_tol=0.0, inner_maxit=3, check_every=3,
                                   solver=solver, precond=sgs_pc if family == "sgs" else wl.get("precond", 0))
        s = slrf.Solver(p.A, p.B, max_L=wl["L"], max_poles=wl["N"], options=opt)
        U, st = s.filter_apply(X, sig, w)
        torch.cuda.synchronize()
        print(json.dumps({"family": family, "dtype": dtype, "spmm_launches": st["spmm_launches"],
                          "full_launch_algorithmic_bytes": st["spmm_bytes"] / st["spmm_launches"]}),
              flush=True)
        s.close()
        del s, U
        torch.cuda.empty_cache()


def summarize_pmc(fetch_csv, write_csv, probe_log, wl_key="c2"):
    """Prints the counter summary (key: value lines) from the two rocprofv3 CSVs
    and the probe's own output (algorithmic bytes per full launch)."""
    def per_kernel(path, counter):
        acc = {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] != counter:
                    continue
                name = row["Kernel_Name"]
                m = re.search(r"k_spmm_([vt])<(float|double)", name)
                mc = re.search(r"k_cocg_spmm<(float|double)", name)
                ms = re.search(r"k_sgs_sweep<(float|double), \d+, (\d+)>", name)
                key = ("copy" if "elementwise" in name and "neg" in name else
                       f"k_spmm_{m.group(1)}<{m.group(2)}>" if m else
                       f"k_cocg_spmm<{mc.group(1)}>" if mc else
                       f"k_sgs_sweep<{ms.group(1)}>" if ms and ms.group(2) in ("0", "2") else None)
                if key:
                    acc.setdefault(key, []).append(float(row["Counter_Value"]))
        return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}
    fe = per_kernel(fetch_csv, "FETCH_SIZE")
    wr = per_kernel(write_csv, "WRITE_SIZE")
    alg = {}
    with open(probe_log) as f:
        for line in f:
            if line.startswith("{"):
                d = json.loads(line)
                alg[(d.get("family", "bicgstab"), d["dtype"])] = d["full_launch_algorithmic_bytes"]
    kib = COPY_BYTES / 1024.0
    ff = fe["copy"][0] / kib
    fw = wr["copy"][0] / kib
    what = ("3D scalar vibration pencil 64^3 (n=250047, 27 nnz/row), L=128, N=6 (K=768)" if wl_key == "c2" else
            "3D elasticity pencil 48^3 nodes x 3 (n=331776, 81 nnz/row), L=256, N=8 (K=2048)")
    print("# Memory traffic of the complex-shifted sparse products (BiCGStab: k_spmm_v, k_spmm_t; COCG:")
    print("# k_cocg_spmm; multicolour SGS: the iteration sweeps k_sgs_sweep, backward and forward),")
    print(f"# {what}, full-width launches.  FETCH_SIZE and WRITE_SIZE count the L2's")
    print("# traffic to the memory fabric (served by the MALL or by HBM).")
    print("# Commands (repository root R, run from /tmp with TMPDIR=/tmp):")
    print("#   rocprofv3 --pmc FETCH_SIZE --kernel-include-regex \"k_spmm|k_cocg_spmm|k_sgs_sweep|elementwise\" --output-format csv "
          f"-d R/gpurun_out/pmc_fetch -o run -- python3 R/bench.py --counters-probe --workload {wl_key}")
    print("#   rocprofv3 --pmc WRITE_SIZE --kernel-include-regex \"k_spmm|k_cocg_spmm|k_sgs_sweep|elementwise\" --output-format csv "
          f"-d R/gpurun_out/pmc_write -o run -- python3 R/bench.py --counters-probe --workload {wl_key}")
    print("#   python3 bench.py --summarize-pmc R/gpurun_out/pmc_fetch/run_counter_collection.csv "
          f"R/gpurun_out/pmc_write/run_counter_collection.csv <probe stdout> --workload {wl_key}")
    print("# Counter values are KiB per dispatch; each is divided by the value the same counter")
    print("# reads for a copy kernel that reads and writes 1 GiB (torch.neg on 2^27 doubles).")
    print(f"source_sha256: {kernel_source_hash()}")
    print(f"copy FETCH_SIZE KiB: {fe['copy'][0]:.0f}")
    print(f"copy WRITE_SIZE KiB: {wr['copy'][0]:.0f}")
    print(f"copy_fetch_factor: {ff:.4f}")
    print(f"copy_write_factor: {fw:.4f}")
    for family, kerns in (("bicgstab", ("k_spmm_v<{}>", "k_spmm_t<{}>")), ("cocg", ("k_cocg_spmm<{}>",)),
                          ("sgs", ("k_sgs_sweep<{}>",))):
        for dtype in ("float", "double"):
            if (family, dtype) not in alg or any(k.format(dtype) not in fe for k in kerns):
                continue
            tot = 0.0
            for kern in (k.format(dtype) for k in kerns):
                fk, nf = fe[kern]
                wk, nw = wr[kern]
                fb, wb = fk * 1024 / ff, wk * 1024 / fw
                tot += fb + wb
                print(f"{kern} dispatches: {nf}")
                print(f"{kern} FETCH_SIZE KiB: {fk:.0f}")
                print(f"{kern} WRITE_SIZE KiB: {wk:.0f}")
                print(f"{kern} fetch bytes (calibrated): {fb:.4e}")
                print(f"{kern} write bytes (calibrated): {wb:.4e}")
            key = dtype if family == "bicgstab" else f"{family} {dtype}"
            a = alg[(family, dtype)]
            print(f"full_launch_traffic_bytes {key}: {tot / len(kerns):.6e}")
            print(f"full_launch_algorithmic_bytes {key}: {a:.6e}")
            print(f"traffic_over_algorithmic {key}: {tot / len(kerns) / a:.3f}")


def summarize_tcc(csv_path, wl_key="c3"):
    """Prints the L2 (TCC) hit rate per kernel from one rocprofv3 pass with the
    TCC_HIT_sum and TCC_MISS_sum counters over the counter probe."""
    acc = {}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            name = row["Kernel_Name"]
            ms = re.search(r"k_sgs_sweep<(float|double), (\d+), (\d+)>", name)
            mc = re.search(r"k_cocg_spmm<(float|double)", name)
            key = ("copy" if "elementwise" in name and "neg" in name else
                   f"k_sgs_sweep<{ms.group(1)}, {ms.group(2)}, {ms.group(3)}>" if ms else
                   f"k_cocg_spmm<{mc.group(1)}>" if mc else None)
            if key:
                acc.setdefault(key, {}).setdefault(row["Counter_Name"], []).append(float(row["Counter_Value"]))
    what = ("3D scalar vibration pencil 64^3 (n=250047, 27 nnz/row), L=128, N=6 (K=768)" if wl_key == "c2" else
            "3D elasticity pencil 48^3 nodes x 3 (n=331776, 81 nnz/row), L=256, N=8 (K=2048)")
    print("# L2 (TCC) hits and misses of the complex-shifted sparse products and colour sweeps,")
    print(f"# {what}, full-width launches of the counter probe (fixed inner iterations).")
    print("# k_sgs_sweep<R, B, M>: B block size (3 node), M 0 backward iteration, 2 forward")
    print("# iteration, 3 forward start, 1 backward final; k_cocg_spmm: the node-triple product of")
    print("# the block Jacobi form.  Requests per dispatch, averaged over the kernel's dispatches.")
    print("# Commands (repository root R, run from /tmp with TMPDIR=/tmp):")
    print("#   rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum --kernel-include-regex \"k_cocg_spmm|k_sgs_sweep|elementwise\" "
          f"--output-format csv -d <out>/pmc_tcc -o run -- python3 R/bench.py --counters-probe --workload {wl_key}")
    print("#   python3 bench.py --summarize-tcc <out>/pmc_tcc/run_counter_collection.csv "
          f"--workload {wl_key}")
    print(f"source_sha256: {kernel_source_hash()}")
    for key in sorted(acc):
        d = acc[key]
        if "TCC_HIT_sum" not in d or "TCC_MISS_sum" not in d:
            continue
        hit = sum(d["TCC_HIT_sum"]) / len(d["TCC_HIT_sum"])
        miss = sum(d["TCC_MISS_sum"]) / len(d["TCC_MISS_sum"])
        print(f"{key} dispatches: {len(d['TCC_HIT_sum'])}")
        print(f"{key} TCC_HIT per dispatch: {hit:.4e}")
        print(f"{key} TCC_MISS per dispatch: {miss:.4e}")
        print(f"{key} hit_rate: {hit / max(hit + miss, 1.0):.3f}")


MFMA_COUNTERS = ["SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_VALU_MFMA_BUSY_CYCLES",
                 "SQ_BUSY_CU_CYCLES", "GRBM_GUI_ACTIVE"]
MFMA_SHAPE = (331776, 256)        # the elasticity workload's n and L


def mfma_probe():
    """Short run for the MFMA counter pass: the Rayleigh-Ritz Gram kernel (FP64 and
    the FP32 first-pass variant) and the Ritz update at the elasticity workload's
    size, three launches each, through the kernel-level hooks."""
    import torch

    import paper_2503_21618_amd as slrf
    n, L = MFMA_SHAPE
    g = torch.Generator(device="cuda").manual_seed(3)
    U, WA, WB = (torch.randn((n, L), dtype=torch.float64, device="cuda", generator=g) for _ in range(3))
    Z = torch.randn((L, L), dtype=torch.float64, device="cuda", generator=g)
    for _ in range(3):
        slrf.test_gram(U, WA, WB)
        slrf.test_gram(U, WA, WB, f32=True)
        slrf.test_gemm(U, Z)
    torch.cuda.synchronize()
    print(json.dumps({"n": n, "L": L, "gram_flops": 4.0 * n * L * L, "gemm_flops": 2.0 * n * L * L}), flush=True)


def summarize_mfma(pmc_csv, trace_csv):
    """MFMA use of k_gram / k_gemm_nz from one rocprofv3 --pmc pass (MFMA_COUNTERS)
    and the kernel durations of a --kernel-trace run of the same probe."""
    vals, durs = {}, {}
    with open(pmc_csv) as f:
        for row in csv.DictReader(f):
            m = re.search(r"(k_gram<(true|false)>|k_gemm_nz)", row["Kernel_Name"])
            if m and row["Counter_Name"] in MFMA_COUNTERS:
                key = m.group(1)
                vals.setdefault(key, {}).setdefault(row["Counter_Name"], []).append(float(row["Counter_Value"]))
    with open(trace_csv) as f:
        for row in csv.DictReader(f):
            m = re.search(r"(k_gram<(true|false)>|k_gemm_nz)", row["Kernel_Name"])
            if m:
                durs.setdefault(m.group(1), []).append(
                    (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-9)
    n, L = MFMA_SHAPE
    alg = {"k_gram<false>": 4.0 * n * L * L, "k_gram<true>": 4.0 * n * L * L, "k_gemm_nz": 2.0 * n * L * L}
    peak = {"k_gram<false>": 78.6e12, "k_gram<true>": 157.3e12, "k_gemm_nz": 78.6e12}
    print(f"# MFMA use of the Rayleigh-Ritz kernels at n={n}, L={L} (three launches each).")
    print("# Commands (repository root R, run from /tmp with TMPDIR=/tmp):")
    print(f"#   rocprofv3 --pmc {' '.join(MFMA_COUNTERS)} --kernel-include-regex \"k_gram|k_gemm_nz\" "
          "--output-format csv -d R/gpurun_out/pmc_mfma -o run -- python3 R/bench.py --mfma-probe")
    print("#   rocprofv3 --kernel-trace --kernel-include-regex \"k_gram|k_gemm_nz\" --output-format csv "
          "-d R/gpurun_out/trace_mfma -o run -- python3 R/bench.py --mfma-probe")
    print("#   python3 bench.py --summarize-mfma <pmc csv> <kernel trace csv>")
    print("# MOPS counters count MFMA work in units of 512 flops; busy fraction = MFMA busy cycles /")
    print("# (GRBM_GUI_ACTIVE / 8 XCDs x 256 CUs x 4 SIMDs); achieved = algorithmic flops / mean")
    print("# duration (kernel trace), against the dense MFMA peak of the instruction's type.")
    for key in ("k_gram<false>", "k_gram<true>", "k_gemm_nz"):
        if key not in vals or key not in durs:
            continue
        v = {c: sum(x) / len(x) for c, x in vals[key].items()}
        d = sum(durs[key]) / len(durs[key])
        mops = v.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) + v.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0)
        # GRBM_GUI_ACTIVE is summed over the 8 XCDs; the busy cycles over the SIMDs
        busy = v.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / max(1.0, v.get("GRBM_GUI_ACTIVE", 0.0) / 8 * 256 * 4)
        print(f"{key} mean duration ms: {1e3 * d:.3f}")
        for c in MFMA_COUNTERS:
            if c in v:
                print(f"{key} {c}: {v[c]:.4e}")
        print(f"{key} MFMA flops from MOPS: {512 * mops:.4e} (algorithmic {alg[key]:.4e})")
        print(f"{key} MFMA busy fraction: {busy:.3f}")
        print(f"{key} achieved TFLOP/s: {alg[key] / d / 1e12:.2f} of {peak[key] / 1e12:.1f} "
              f"({alg[key] / d / peak[key]:.3f})")


def union_nnz(p):
    return int((abs(p.A) + abs(p.B)).nnz)


def batch_kernel_stats(results):
    """Batch-wide kernel statistics: every pencil's stats hold the batch launches of
    the steps it took part in, so the pencil that ran longest holds them all."""
    last = max(results, key=lambda r: r.stats["outer_iterations"])
    return last.stats["kernels"]


def many_options(slrf, args, precision, **kw):
    """Options of the batched, served and serial runs: COCG unless --solver
    bicgstab, with the multicolour SGS preconditioner (--precond sgs, the
    default: node blocks for node-structured pencils, points for the others) or
    point Jacobi;
    with --graph (the default) the Krylov iteration chunks replay as hipGraphs
    and the per-launch kernel timers are off; with --no-graph the kernels are
    timed (roofline fields)."""
    kw.setdefault("solver", slrf.SOLVER_BICGSTAB if args.solver == "bicgstab" else slrf.SOLVER_COCG)
    kw.setdefault("precond", slrf.PRECOND_SGS3 if args.precond == "sgs" and kw["solver"] == slrf.SOLVER_COCG
                  else slrf.PRECOND_AUTO)
    kw.setdefault("recycle", 1 if args.recycle == "1" or (args.recycle == "auto" and kw["solver"] == 1) else 0)
    if args.graph:
        return slrf.default_options(precision=precision, graph=1, profile=0, **kw)
    return slrf.default_options(precision=precision, profile=1, **kw)


def serial_solves(slrf, args, items, precision, limit_s=float("inf")):
    """The same pencils solved one at a time (create and pole design excluded),
    in order, until limit_s seconds of solve time have been spent; same graph
    setting as the batch."""
    import torch
    found, secs, done, not_ok = 0, 0.0, 0, 0
    stream = torch.cuda.Stream()
    for p, gamma, L in items:
        if secs >= limit_s:
            break
        s = slrf.Solver(p.A, p.B, max_L=L, max_poles=6, options=many_options(slrf, args, precision),
                        stream=stream)
        sig, w, _ = slrf.design_poles(6, 1.0, 0.01, gamma)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve_interval(gamma, L, sig, w, raise_on_error=False)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        found += r.n_found
        done += 1
        not_ok += r.status != 0
        log(f"serial {done}: n={p.n} found {r.n_found} status {r.status} "
            f"outer {r.stats['outer_iterations']}, total {secs:.1f} s")
        s.close()
        del s
        torch.cuda.empty_cache()
    return {"precision": "mixed" if precision == slrf.MIXED else "fp64",
            "value": found / secs if secs > 0 else 0.0, "seconds": secs, "found": found,
            "pencils": done, "pencils_not_converged": not_ok}


def run_batched(slrf, args):
    """64 independent 2D/3D scalar pencils (pencils.batch_instance) solved together:
    mixed precision, N = 6, autotuned tiles; one batched launch per Krylov step."""
    import torch

    import pencils
    t0 = time.perf_counter()
    insts = [pencils.batch_instance(i, n_range=(args.batch_n_min, args.batch_n_max)) for i in range(args.instances)]
    log(f"built {len(insts)} pencils in {time.perf_counter() - t0:.1f} s, "
        f"sum n = {sum(p.n for p, *_ in insts)}")
    N = 6
    opt = many_options(slrf, args, slrf.MIXED, tune=1)
    pers = trans = 0
    for p, g, L, _ in insts:
        a, b = slrf.batch_footprint(p.n, union_nnz(p), L, N, options=opt)
        pers += a + 4096
        trans += b
    ws = pers + trans + (1 << 24)
    log(f"workspace {ws / 2**30:.1f} GiB (filter arena {trans / 2**30:.1f} GiB)")
    b = slrf.Batch(ws, trans, max_poles=N, options=opt, stream=torch.cuda.Stream())
    ids = []
    for p, g, L, _ in insts:
        sig, w, _ = slrf.design_poles(N, 1.0, 0.01, g)
        ids.append(b.add(p.A, p.B, g, L, sig, w))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    while True:
        act = b.step()
        steps += 1
        log(f"batched step {steps}: {act} unfinished, {time.perf_counter() - t0:.1f} s")
        if act == 0:
            break
    res = [b.result(pid) for pid in ids]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.close()
    del b
    torch.cuda.empty_cache()
    bad = [i for i, r in enumerate(res) if r.status != 0]
    found = sum(r.n_found for r in res)
    ks = batch_kernel_stats(res)
    out = {"value": found / dt, "seconds": dt, "found": found, "steps": steps,
           "statuses_not_ok": bad, "max_resid": max(r.stats["max_resid"] for r in res), "ks": ks}
    if not args.no_serial:
        items = [(p, g, L) for p, g, L, _ in insts]
        for tag, prec in (("mixed", slrf.MIXED), ("fp64", slrf.FP64)):
            if args.serial_precision in (tag, "both"):
                log(f"serial solves ({tag})...")
                key = "serial" if args.serial_precision != "both" or tag == "mixed" else "serial_fp64"
                out[key] = serial_solves(slrf, args, items, prec, args.serial_limit)
    return out, insts


def run_served(slrf, args):
    """Poisson stream of interval eigensolves through the continuous-batching
    server: requests over a pool of --structures pencils (pencils.serve_structure:
    3D scalar and 3D elasticity alternating, n log-uniform on [--n-min, --n-max]),
    each with its own NEV (log-uniform on [20, --nev-max]) and gamma
    (pencils.serve_request_mix).  The arrival rate is 0.7 x the throughput of a
    closed calibration batch of the first requests; requests arrive for
    --duration seconds (at most --requests of them)."""
    import torch

    import numpy as np

    import paper_2503_21618_amd.serve as serve
    import pencils
    t0 = time.perf_counter()
    structures = {}
    for sid in range(args.structures):
        structures[sid] = pencils.serve_structure(sid, n_range=(args.n_min, args.n_max))
        log(f"structure {sid}: {structures[sid][1]} n={structures[sid][0].n} ({time.perf_counter() - t0:.0f} s)")
    R = args.requests
    specs = [pencils.serve_request_mix(r, structures, nev_range=(20, args.nev_max)) for r in range(R)]
    N = 6
    opt = many_options(slrf, args, slrf.MIXED)
    nnz = {sid: union_nnz(p) for sid, (p, _, _) in structures.items()}
    fps = [slrf.batch_footprint(structures[sid][0].n, nnz[sid], L, N, options=opt) for sid, g, L, _ in specs]
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.9 * free)
    big_t = max(t for _, t in fps)
    big_p = max(a for a, _ in fps)
    arena = min(max(int(args.arena_gb * 2**30), int(1.3 * big_t)), budget - 2 * big_p)
    pool = budget - arena
    log(f"{R} request specs; largest transient {big_t / 2**30:.1f} GiB, persistent {big_p / 2**30:.1f} GiB; "
        f"arena {arena / 2**30:.1f} GiB, pool {pool / 2**30:.1f} GiB")
    if big_t > arena or big_p > pool:
        raise SystemExit("a request does not fit the arena or pool")
    if args.serial_only:
        # the comparison alone: the first --requests requests one at a time
        items = [(structures[specs[i][0]][0], specs[i][1], specs[i][2]) for i in range(R)]
        ser = serial_solves(slrf, args, items, slrf.MIXED if args.serial_precision == "mixed" else slrf.FP64,
                            args.serial_limit)
        return {"value": ser["value"], "seconds": ser["seconds"], "found": ser["found"], "serial": ser,
                "ks": {"spmm_seconds": 0}}, [structures[specs[i][0]][0] for i in range(ser["pencils"])]
    stream = torch.cuda.Stream()

    def make(i, arrival):
        sid, g, L, _ = specs[i]
        p = structures[sid][0]
        sig, w, _ = slrf.design_poles(N, 1.0, 0.01, g)
        return serve.Request(i, p.A, p.B, g, L, sig, w, arrival=arrival)

    # calibration: the first C requests at once
    C = min(args.calibrate, R)
    srv = serve.Server(pool + arena, arena, max_poles=N, options=opt, stream=stream)
    for i in range(C):
        srv.submit(make(i, 0.0))
    t0 = time.perf_counter()
    while not srv.idle():
        srv.pump()
        log(f"calibration: {len(srv.done)}/{C} done, {time.perf_counter() - t0:.0f} s")
    mu = C / (time.perf_counter() - t0)
    rate = 0.7 * mu
    log(f"calibration: {C} requests in {C / mu:.1f} s -> rate {rate:.3f} requests/s")
    srv.close()
    del srv
    torch.cuda.empty_cache()
    arr = pencils.arrival_times(R, rate)
    count = max(1, int(np.searchsorted(arr - arr[0], args.duration, side="right")))
    log(f"{count} requests arrive within {args.duration:.0f} s")
    srv = serve.Server(pool + arena, arena, max_poles=N, options=opt, stream=stream)
    pending = [make(i, float(arr[i])) for i in range(count)]
    t0 = time.perf_counter()
    srv.clock = lambda: time.perf_counter() - t0
    last_log = 0.0
    while pending or not srv.idle():
        now = srv.clock()
        while pending and pending[0].arrival <= now:
            srv.submit(pending.pop(0))
        if srv.idle():
            time.sleep(min(0.05, max(0.0, pending[0].arrival - now)))
            continue
        srv.pump()
        if srv.clock() - last_log > 10:
            last_log = srv.clock()
            log(f"served {len(srv.done)}/{count}, active {len(srv.active)}, queued {len(srv.queue)}, "
                f"t {last_log:.0f} s")
    makespan = max(c.finished for c in srv.done) - float(arr[0])
    res = [c.result for c in srv.done]
    found = sum(r.n_found for r in res)
    lat = serve.latency_stats(srv.done)
    ks = batch_kernel_stats(res)
    kinds = [structures[specs[c.rid][0]][1] for c in srv.done]
    out = {"value": found / makespan, "seconds": makespan, "requests": count, "found": found, "latency_s": lat,
           "rate_per_s": rate, "peak_active": srv.peak_active, "steps": srv.steps,
           "elasticity_requests": kinds.count("elasticity"), "scalar_requests": kinds.count("scalar"),
           "statuses_not_ok": [c.rid for c in srv.done if c.result.status != 0],
           "max_resid": max(r.stats["max_resid"] for r in res), "ks": ks}
    srv.close()
    del srv
    torch.cuda.empty_cache()
    if not args.no_serial:
        log("serial solves...")
        items = [(structures[specs[i][0]][0], specs[i][1], specs[i][2]) for i in range(count)]
        out["serial"] = serial_solves(slrf, args, items,
                                      slrf.MIXED if args.serial_precision == "mixed" else slrf.FP64,
                                      args.serial_limit)
    return out, [structures[specs[i][0]][0] for i in range(count)]


def run_filters(slrf, args):
    """Section 3.2's filter comparison on a synthetic stand-in for its 2D model:
    N = 3 poles from the SLRF design (alpha = 0.5, beta = 0.01) and from the
    midpoint, Gauss-Legendre and Gauss-Chebyshev rules, on a 2D scalar pencil
    with gamma between its 20th and 21st eigenvalues.  Per pole: mean inner
    iterations of the FP64 solves (tol 1e-10, at most 5000 iterations, L = 24
    columns) with BiCGStab and
    with COCG; per filter: a complete mixed-precision interval solve (COCG)."""
    import numpy as np
    import scipy.sparse.linalg as sla
    import torch

    import pencils
    p = pencils.scalar_q1(100, 2, 0.5, 7)
    ev = np.sort(sla.eigsh(p.A.tocsc(), k=22, M=p.B.tocsc(), sigma=0.0, which="LM",
                           return_eigenvectors=False))
    gamma = 0.5 * (ev[19] + ev[20])
    L = 24
    X = torch.from_numpy(pencils.start_block(p.n, L, 1)).cuda()
    filters = {"SLRF": slrf.design_poles(3, 0.5, 0.01, gamma)[:2]}
    for rule, name in ((slrf.QUAD_MIDPOINT, "midpoint"), (slrf.QUAD_GAUSS_LEGENDRE, "gauss-legendre"),
                       (slrf.QUAD_GAUSS_CHEBYSHEV, "gauss-chebyshev")):
        filters[name] = slrf.quadrature_poles(rule, 3, gamma)
    log(f"2D pencil n={p.n}, gamma={gamma:.4f} (20 eigenvalues below)")
    out = {"pencil": f"2D scalar Q1 99^2 (n={p.n}), log-normal sigma=0.5 seed 7, gamma={gamma:.6g}",
           "inner": {}, "solve": {}}
    for fname, (sig, w) in filters.items():
        row = {"poles": [[float(z.real), float(z.imag)] for z in sig]}
        for solver, sname in ((slrf.SOLVER_BICGSTAB, "bicgstab"), (slrf.SOLVER_COCG, "cocg")):
            its = []
            for j in range(len(sig)):
                opt = slrf.default_options(precision=slrf.FP64, inner_tol=1e-10, inner_maxit=5000, solver=solver)
                s = slrf.Solver(p.A, p.B, max_L=L, max_poles=1, options=opt)
                _, st = s.filter_apply(X, sig[j:j + 1], w[j:j + 1])
                its.append(st["mean_iterations"])
                s.close()
            row[sname] = [round(v, 1) for v in its]
        out["inner"][fname] = row
        s = slrf.Solver(p.A, p.B, max_L=L, max_poles=3,
                        options=slrf.default_options(precision=slrf.MIXED, inner_maxit=5000,
                                                     solver=slrf.SOLVER_COCG))
        t0 = time.perf_counter()
        r = s.solve_interval(gamma, L, sig, w, V0=X, raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.close()
        out["solve"][fname] = {"status": r.status, "found": r.n_found, "outer": r.stats["outer_iterations"],
                               "spmv_total": r.stats["spmv_total"], "seconds": dt,
                               "max_resid": r.stats["max_resid"]}
        log(f"{fname}: inner its BiCGStab {row['bicgstab']}, COCG {row['cocg']}; solve found {r.n_found}, "
            f"outer {r.stats['outer_iterations']}, spmv {r.stats['spmv_total']}")
    return out


def many_line(args, kind, out, desc):
    ks = out.pop("ks")
    line = {"metric": METRIC, "value": out["value"], "unit": "eigenpairs/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": 1e3 * out["seconds"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": desc, "graph": bool(args.graph)}}
    if ks["spmm_seconds"] > 0:
        spmm_gbs = ks["spmm_bytes"] / ks["spmm_seconds"] / 1e9
        line["roofline"] = {"bound": "hbm", "achieved": spmm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": spmm_gbs / HBM_PEAK_GBS, "traffic": None,
                            "kernel": "the complex-shifted sparse product or the SGS sweeps <float>",
                            "launches": ks["spmm_launches"],
                            "avg_launch_ms": 1e3 * ks["spmm_seconds"] / max(1, ks["spmm_launches"]),
                            "traffic_note": "counters are taken on the 64^3 scalar workload only"}
        line["vector_updates"] = {"achieved_GBs": ks["update_bytes"] / ks["update_seconds"] / 1e9}
    else:
        line["roofline"] = None
        line["roofline_note"] = ("hipGraph replay with kernel timers off; bench.py --no-graph times the "
                                 "kernels of this workload")
    line[kind] = out
    for key in ("serial", "serial_fp64"):
        ser = out.get(key)
        if ser and ser["value"] > 0:
            line[f"over_serial_{ser['precision']}"] = out["value"] / ser["value"]
    return line


def check_against_oracle(wl, evals, n_found, tol):
    """The eigenvalues a solve returned against the oracle's (tests/golden):
    count and largest relative error; raises if either is off."""
    import numpy as np
    ev = np.asarray(wl.get("eigs") or [])
    if not len(ev):
        return None
    if n_found != len(ev):
        raise SystemExit(f"found {n_found} eigenpairs, the oracle has {len(ev)}")
    rel = float(np.abs(np.asarray(evals[:n_found]) / ev - 1).max())
    if rel > tol:
        raise SystemExit(f"eigenvalues differ from the oracle's by {rel:.2e} (> {tol:.0e})")
    return rel


def run_outer_steps(slrf, wl, precision, steps, warmup, sig, w, V0):
    """A step is one outer iteration of Algorithm 1 on the workload: the filter
    application (every shifted solve of the N poles x L columns, in the mixed
    form with its FP64 defect corrections), the filter sum, Rayleigh-Ritz and the
    residuals (slrf_batch_step on a one-pencil batch).  Solves run back to back:
    when one converges its eigenvalues are checked against the oracle's and the
    next starts from the same start block (slrf_batch_restart; the pencil's
    upload happens once, before the first step).  Each step is bracketed by
    device synchronisations; `value` counts the eigenpairs of the solves that
    ran entirely inside the K timed steps, over the time of their steps."""
    import torch
    p = wl["pencil"]
    L, N, gamma = wl["L"], wl["N"], wl["gamma"]
    tag = "mixed" if precision == slrf.MIXED else "fp64"
    opt = slrf.default_options(profile=1, precision=precision, precond=wl.get("precond", 0),
                               solver=wl.get("solver", 0), recycle=wl.get("recycle", 0))
    pers, trans = slrf.batch_footprint(p.n, union_nnz(p), L, N, options=opt)
    ws = pers + trans + (1 << 24)
    log(f"{tag}: n={p.n} L={L} N={N} workspace {ws / 2**30:.2f} GiB (one-pencil batch)")
    b = slrf.Batch(ws, trans, max_poles=N, options=opt)
    pid = b.add(p.A, p.B, gamma, L, sig, w, V0=V0)
    torch.cuda.synchronize()
    times, solves, cur = [], [], []
    ks_keys = ("spmm_seconds", "spmm_launches", "spmm_bytes", "spmm_columns", "update_seconds",
               "update_launches", "update_bytes")
    for k in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        act = b.step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        timed = k >= warmup
        times.append(dt if timed else None)
        cur.append(k)
        log(f"{tag} {'step' if timed else 'warmup'} {k - warmup if timed else k}: {dt:.2f} s, "
            f"solve {len(solves)} outer {len(cur)}")
        if act == 0:
            r = b.result(pid)
            if r.status != 0 or (wl["expect"] is not None and r.n_found != wl["expect"]):
                raise SystemExit(f"{tag} solve failed: status {r.status} found {r.n_found} ({r.message})")
            rel = check_against_oracle(wl, r.evals, r.n_found, 1e-8 if precision == slrf.MIXED else 1e-10)
            solves.append(dict(steps=cur, result=r, rel=rel))
            log(f"{tag} solve {len(solves)} done: {r.n_found} pairs, outer {r.stats['outer_iterations']}, "
                f"max rho {r.stats['max_resid']:.2e}, max rel eig err vs oracle {rel}")
            cur = []
            b.restart(pid, V0)
    torch.cuda.synchronize()
    b.close()
    del b
    torch.cuda.empty_cache()
    full = [sv for sv in solves if all(times[i] is not None for i in sv["steps"])]
    if not full:
        raise SystemExit(f"no complete solve inside the {steps} timed steps: raise --steps")
    t_full = sum(times[i] for sv in full for i in sv["steps"])
    found = sum(sv["result"].n_found for sv in full)
    ks = {k: sum(sv["result"].stats["kernels"][k] for sv in full) for k in ks_keys}
    t_all = sum(t for t in times if t is not None)
    return dict(value=found / t_full, dt=t_all, results=[sv["result"] for sv in full], ks=ks,
                solve_seconds=t_full / len(full), complete_solves=len(full),
                max_rel_eig_err=max(sv["rel"] for sv in full))


def run_form_stepwise(slrf, wl, precision, steps, warmup, sig, w, V0):
    """As run_form, through the batch API with the one pencil, so that every outer
    iteration reports (a solve of the elasticity workload takes minutes)."""
    import torch
    p = wl["pencil"]
    L, N, gamma = wl["L"], wl["N"], wl["gamma"]
    tag = "mixed" if precision == slrf.MIXED else "fp64"
    opt = slrf.default_options(profile=1, precision=precision, precond=wl.get("precond", 0),
                               solver=wl.get("solver", 0), recycle=wl.get("recycle", 0))
    pers, trans = slrf.batch_footprint(p.n, union_nnz(p), L, N, options=opt)
    ws = pers + trans + (1 << 24)
    log(f"{tag}: n={p.n} L={L} N={N} workspace {ws / 2**30:.2f} GiB (one-pencil batch)")

    def solve():
        b = slrf.Batch(ws, trans, max_poles=N, options=opt)
        pid = b.add(p.A, p.B, gamma, L, sig, w, V0=V0)
        t0, k = time.perf_counter(), 0
        while b.step() > 0:
            k += 1
            done, outer = b.query(pid)
            log(f"{tag} outer step {k}: {time.perf_counter() - t0:.1f} s")
        r = b.result(pid)
        b.close()
        if r.status != 0 or (wl["expect"] is not None and r.n_found != wl["expect"]):
            raise SystemExit(f"{tag} solve failed: status {r.status} found {r.n_found} ({r.message})")
        return r

    for i in range(warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    found, results = 0, []
    for i in range(steps):
        r = solve()
        found += r.n_found
        results.append(r)
        log(f"{tag} step {i}: outer {r.stats['outer_iterations']}, found {r.n_found}, "
            f"max rho {r.stats['max_resid']:.2e}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    torch.cuda.empty_cache()
    ks = {k: sum(r.stats["kernels"][k] for r in results) for k in
          ("spmm_seconds", "spmm_launches", "spmm_bytes", "update_seconds", "update_launches",
           "update_bytes")}
    return dict(value=found / dt, dt=dt, results=results, ks=ks)


def run_form(slrf, wl, precision, steps, warmup, sig, w, V0):
    import torch
    if wl.get("stepwise"):
        return run_form_stepwise(slrf, wl, precision, steps, warmup, sig, w, V0)
    p = wl["pencil"]
    L, N, gamma = wl["L"], wl["N"], wl["gamma"]
    opt = slrf.default_options(profile=1, precision=precision, precond=wl.get("precond", 0),
                               solver=wl.get("solver", 0), recycle=wl.get("recycle", 0))
    solver = slrf.Solver(p.A, p.B, max_L=L, max_poles=N, options=opt)
    tag = "mixed" if precision == slrf.MIXED else "fp64"
    log(f"{tag}: n={p.n} L={L} N={N} workspace {solver.ws_bytes / 2**30:.2f} GiB")

    def step():
        r = solver.solve_interval(gamma, L, sig, w, V0=V0)
        if r.status != 0 or (wl["expect"] is not None and r.n_found != wl["expect"]):
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


def roofline_fields(ks, kname, kdtype, spmm_flops):
    """The dominant kernel's rates from the timed launches: algorithmic HBM bytes
    and flops per second.  The bound is the roof the kernel is closer to."""
    secs = max(ks["spmm_seconds"], 1e-30)
    gbs = ks["spmm_bytes"] / secs / 1e9
    tfs = spmm_flops / secs / 1e12
    peak_tf = FP32_NONPACKED_TFS if kdtype == "float" else FP64_TFS
    out = {"achieved_GBs": gbs, "frac_hbm": gbs / HBM_PEAK_GBS,
           "achieved_TFLOPs": tfs, "frac_alu": tfs / peak_tf, "alu_peak_TFLOPs": peak_tf,
           "kernel": f"{kname} <{kdtype}> (complex-shifted sparse product)",
           "launches": ks["spmm_launches"],
           "avg_launch_ms": 1e3 * ks["spmm_seconds"] / max(1, ks["spmm_launches"]),
           "algorithmic_bytes_per_launch": ks["spmm_bytes"] / max(1, ks["spmm_launches"]),
           "algorithmic_flops_per_launch": spmm_flops / max(1, ks["spmm_launches"])}
    if out["frac_alu"] >= out["frac_hbm"]:
        out.update(bound="alu", achieved=tfs, peak=peak_tf, unit="TFLOP/s", frac=tfs / peak_tf)
    else:
        out.update(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS)
    return out


def spmm_flops_per_column(p):
    """Algorithmic flops of the complex-shifted product (A - sigma B) x for one
    complex column over all rows: 4 flops per stored nonzero of A and of B (a
    real coefficient times a complex value, accumulated) and 8 per row for
    a - sigma b."""
    import numpy as np
    return 4.0 * (np.count_nonzero(p.A.data) + np.count_nonzero(p.B.data)) + 8.0 * p.n


def main_c3(slrf, args):
    """The default line: the elasticity workload (the largest single pencil, the
    mixed-precision configuration), a step per outer iteration; the 64^3 scalar
    workload's mixed and FP64 solves beside it."""
    import numpy as np
    import pencils
    steps = 20 if args.steps is None else args.steps
    warmup = 5 if args.warmup is None else args.warmup
    wl = workload("c3")
    wl["solver"] = 0 if args.solver == "bicgstab" else 1
    wl["recycle"] = 0 if args.recycle == "0" or wl["solver"] == 0 else 1
    if wl["solver"] == 1 and args.precond == "sgs":
        wl["precond"] = slrf.PRECOND_SGS3
    p = wl["pencil"]
    sig, w, _ = slrf.design_poles(wl["N"], 1.0, 0.01, wl["gamma"])
    smp = None
    if not args.no_cpu_baseline:
        log("cpu baseline sample (before the GPU is used)...")
        smp = cpu_sample(wl, sig)
        log(smp["sample"])
    import torch
    V0 = torch.from_numpy(pencils.start_block(p.n, wl["L"], 1)).cuda()
    m = run_outer_steps(slrf, wl, slrf.MIXED, steps, warmup, sig, w, V0)
    del V0
    ks = m["ks"]
    res = m["results"]
    sgs = wl.get("precond") == slrf.PRECOND_SGS3
    kname = ("k_sgs_sweep (backward + forward colour sweeps: the product with S of an iteration)" if sgs else
             "k_cocg_spmm" if wl["solver"] == 1 else "k_spmm_v / k_spmm_t")
    spmm_flops = spmm_flops_per_column(p) * ks["spmm_columns"]
    roof = roofline_fields(ks, kname, "float", spmm_flops)
    traffic, note = hbm_traffic("float", roof["algorithmic_bytes_per_launch"],
                                "sgs" if sgs else "cocg" if wl["solver"] == 1 else "bicgstab", workload_key="c3")
    roof["traffic"] = traffic
    roof["traffic_note"] = note
    upd_gbs = ks["update_bytes"] / ks["update_seconds"] / 1e9
    last = res[-1].stats
    pcname = {3: "node 3x3 block Jacobi", 5: "multicolour node-block symmetric Gauss-Seidel"}[wl["precond"]]
    prec = ("complex FP32 inner solves + FP64 defect correction and Rayleigh-Ritz; inner solver "
            + ("COCG, warm starts across outer iterations" if wl["solver"] == 1 else "BiCGStab")
            + "; preconditioner " + pcname)
    out = {
        "metric": METRIC, "value": m["value"], "unit": "eigenpairs/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * m["dt"] / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl["desc"] + "; " + prec,
                   "step": "one outer iteration of Algorithm 1; value from the complete solves inside the "
                           "timed steps"},
        "roofline": roof,
        "vector_updates": {"achieved_GBs": upd_gbs, "frac": upd_gbs / HBM_PEAK_GBS,
                           "avg_launch_ms": 1e3 * ks["update_seconds"] / max(1, ks["update_launches"])},
        "solve": {"seconds": m["solve_seconds"], "complete_solves_timed": m["complete_solves"],
                  "max_rel_eig_err_vs_oracle": m["max_rel_eig_err"],
                  **{k: last[k] for k in ("outer_iterations", "spmv_total", "n_found", "max_resid",
                                          "inner_iterations", "filter_seconds")}},
    }
    if not args.no_c2:
        c2 = workload("c2")
        c2["eigs"] = c2_golden()["eigenvalues"]
        c2["solver"], c2["recycle"] = 1, 1
        c2["precond"] = slrf.PRECOND_SGS if args.precond == "sgs" else slrf.PRECOND_JACOBI
        s2, w2, _ = slrf.design_poles(c2["N"], 1.0, 0.01, c2["gamma"])
        V2 = torch.from_numpy(pencils.start_block(c2["pencil"].n, c2["L"], 1)).cuda()
        legs = {}
        for tag, prec2, st2, wu2 in (("mixed", slrf.MIXED, 1, 1), ("fp64", slrf.FP64, 1, 0)):
            f = run_form(slrf, dict(c2, recycle=1 if prec2 == slrf.MIXED else 0), prec2, st2, wu2, s2, w2, V2)
            r = f["results"][-1]
            rel = check_against_oracle(c2, r.evals, r.n_found, 1e-8 if prec2 == slrf.MIXED else 1e-10)
            fk = f["ks"]
            legs[tag] = {"value": f["value"], "seconds": f["dt"], "outer_iterations": r.stats["outer_iterations"],
                         "n_found": r.n_found, "max_resid": r.stats["max_resid"], "max_rel_eig_err_vs_oracle": rel,
                         "spmm_GBs": fk["spmm_bytes"] / fk["spmm_seconds"] / 1e9,
                         "update_GBs": fk["update_bytes"] / fk["update_seconds"] / 1e9}
        out["c2_64cube"] = {"workload": c2["desc"].replace("; point Jacobi", "") + "; COCG; " +
                            ("multicolour symmetric Gauss-Seidel" if args.precond == "sgs" else "point Jacobi"), **legs,
                            "mixed_over_fp64": legs["mixed"]["value"] / legs["fp64"]["value"]}
    if smp is not None:
        out["cpu_baseline"] = cpu_baseline(smp, last, wl["L"], wl["N"])
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20 outer iterations for c3, 1 solve otherwise)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default: 5 for c3, 1 otherwise)")
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-c2", action="store_true", help="c3: skip the 64^3 mixed and FP64 legs")
    ap.add_argument("--precond", default="sgs", choices=["sgs", "jacobi"],
                    help="shifted-operator preconditioner of the COCG workloads: multicolour symmetric "
                         "Gauss-Seidel (point, or node blocks for elasticity) or (node block) Jacobi")
    ap.add_argument("--precision", default="both", choices=["both", "mixed", "fp64"])
    ap.add_argument("--recycle", default="auto", choices=["auto", "0", "1"],
                    help="warm starts across outer iterations (mixed precision); auto: with COCG")
    ap.add_argument("--solver", default="auto", choices=["auto", "bicgstab", "cocg"],
                    help="inner solver of the shifted systems; auto: COCG (BiCGStab timed beside it on "
                         "the 64^3 workload), BiCGStab for the ILU(0) string")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--instances", type=int, default=64, help="batched workload: number of pencils")
    ap.add_argument("--batch-n-min", type=float, default=5e3, help="batched workload: smallest pencil")
    ap.add_argument("--batch-n-max", type=float, default=2e5, help="batched workload: largest pencil")
    ap.add_argument("--requests", type=int, default=2000, help="served workload: most requests")
    ap.add_argument("--duration", type=float, default=600.0, help="served workload: seconds of arrivals")
    ap.add_argument("--structures", type=int, default=16, help="served workload: distinct pencils")
    ap.add_argument("--serial-only", action="store_true",
                    help="served workload: only the one-at-a-time solves of the first --requests requests")
    ap.add_argument("--n-min", type=float, default=1e4, help="served workload: smallest pencil")
    ap.add_argument("--n-max", type=float, default=5e5, help="served workload: largest pencil")
    ap.add_argument("--nev-max", type=int, default=300, help="served workload: largest NEV")
    ap.add_argument("--calibrate", type=int, default=6, help="served workload: calibration batch")
    ap.add_argument("--arena-gb", type=float, default=64.0)
    ap.add_argument("--pool-gb", type=float, default=32.0)
    ap.add_argument("--no-serial", action="store_true", help="skip the one-pencil-at-a-time comparison")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="batched/served: time every kernel launch instead of replaying hipGraphs")
    ap.add_argument("--serial-limit", type=float, default=float("inf"),
                    help="stop the serial comparison after this many seconds of solves")
    ap.add_argument("--serial-precision", default="fp64", choices=["fp64", "mixed", "both"],
                    help="precision of the one-pencil-at-a-time comparison")
    ap.add_argument("--counters-probe", action="store_true",
                    help="short run for the rocprofv3 counter passes (see the module docstring)")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "PROBE_LOG"),
                    help="print the counter summary from two rocprofv3 CSVs")
    ap.add_argument("--summarize-tcc", metavar="TCC_CSV",
                    help="print the L2 hit rates from a TCC_HIT_sum / TCC_MISS_sum counter pass")
    ap.add_argument("--mfma-probe", action="store_true",
                    help="short run of the Rayleigh-Ritz MFMA kernels for the MFMA counter pass")
    ap.add_argument("--summarize-mfma", nargs=2, metavar=("PMC_CSV", "TRACE_CSV"),
                    help="print the MFMA summary from the counter pass and a kernel trace")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, wl_key=args.workload)
        return
    if args.summarize_tcc:
        summarize_tcc(args.summarize_tcc, wl_key=args.workload)
        return
    if args.summarize_mfma:
        summarize_mfma(*args.summarize_mfma)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the pole-sharded "
              "multi-GPU form is not built", file=sys.stderr)
        sys.exit(2)

    if args.counters_probe:
        counters_probe(args.workload)
        return
    if args.mfma_probe:
        mfma_probe()
        return

    import torch

    import paper_2503_21618_amd as slrf
    import pencils

    if args.workload == "batched":
        out, insts = run_batched(slrf, args)
        desc = (f"{len(insts)} independent 2D/3D scalar vibration pencils (bilinear/trilinear FE, "
                f"log-normal coefficient sigma=0.5, seeds 1000+i), n log-uniform {args.batch_n_min:.0e}..{args.batch_n_max:.0e} "
                f"(sum {sum(p.n for p, *_ in insts)}), NEV 10..80 each with its own gamma, "
                "L = ceil(1.2 NEV) to a multiple of 8, N=6; one batch, mixed precision, autotuned tiles; "
                f"inner solver {'BiCGStab' if args.solver == 'bicgstab' else 'COCG'}"
                f"{', warm starts' if args.recycle != '0' and args.solver != 'bicgstab' else ''}")
        print(json.dumps(many_line(args, "batched", out, desc)), flush=True)
        return
    if args.workload == "filters":
        print(json.dumps({"metric": "mean inner iterations per pole (Section 3.2 filter comparison)",
                          "data": "synthetic", "filters": run_filters(slrf, args)}), flush=True)
        return
    if args.workload == "served":
        out, reqs = run_served(slrf, args)
        desc = (f"{len(reqs)} Poisson-arriving requests in {args.duration:.0f} s (rate 0.7 x calibrated "
                f"capacity) over {args.structures} pencils, 3D scalar vibration and 3D elasticity alternating, "
                f"n log-uniform {args.n_min:.0e}..{args.n_max:.0e}, NEV log-uniform 20..{args.nev_max}, "
                "L = ceil(1.2 NEV) to a multiple of 8, N=6; continuous batching, admission by HBM footprint, "
                f"mixed precision; inner solver {'BiCGStab' if args.solver == 'bicgstab' else 'COCG'}"
                f"{', warm starts' if args.recycle != '0' and args.solver != 'bicgstab' else ''}"
                f"{', multicolour SGS (node blocks for elasticity)' if args.precond == 'sgs' else ''}")
        print(json.dumps(many_line(args, "served", out, desc)), flush=True)
        return
    if args.workload == "c3":
        main_c3(slrf, args)
        return
    if args.steps is None:
        args.steps = 1
    if args.warmup is None:
        args.warmup = 1
    wl = workload(args.workload)
    symmetric = args.workload != "c1"          # C1 runs ILU(0), which COCG does not take
    wl["solver"] = 1 if args.solver == "cocg" or (args.solver == "auto" and symmetric) else 0
    wl["recycle"] = 1 if args.recycle == "1" or (args.recycle == "auto" and wl["solver"] == 1) else 0
    p = wl["pencil"]
    sig, w, _ = slrf.design_poles(wl["N"], 1.0, 0.01, wl["gamma"])
    smp = None
    if not args.no_cpu_baseline:
        log("cpu baseline sample (before the GPU is used)...")
        smp = cpu_sample(wl, sig)
        log(smp["sample"])
    V0 = torch.from_numpy(pencils.start_block(p.n, wl["L"], 1)).cuda()
    forms = {}
    if args.precision in ("both", "mixed"):
        forms["mixed"] = run_form(slrf, wl, slrf.MIXED, args.steps, args.warmup, sig, w, V0)
    if args.precision in ("both", "fp64"):
        fp_steps, fp_warm = (1, 0) if args.precision == "both" else (args.steps, args.warmup)
        forms["fp64"] = run_form(slrf, wl, slrf.FP64, fp_steps, fp_warm, sig, w, V0)
    if (args.solver == "auto" and wl["solver"] == 1 and args.precision in ("both", "mixed")
            and not wl.get("stepwise")):
        # the paper's inner solver on the same workload, for comparison
        forms["bicgstab"] = run_form(slrf, dict(wl, solver=0, recycle=0), slrf.MIXED, 1, 0, sig, w, V0)
    main_form = "mixed" if "mixed" in forms else "fp64"
    m = forms[main_form]
    ks = m["ks"]
    spmm_gbs = ks["spmm_bytes"] / ks["spmm_seconds"] / 1e9
    upd_gbs = ks["update_bytes"] / ks["update_seconds"] / 1e9
    prec = "complex FP32 inner solves + FP64 defect correction and Rayleigh-Ritz" if main_form == "mixed" \
        else "complex FP64 inner solves"
    prec += "; inner solver " + ("COCG" if wl["solver"] == 1 else "BiCGStab")
    if wl["recycle"] and main_form == "mixed":
        prec += ", warm starts across outer iterations"
    kdtype = "float" if main_form == "mixed" else "double"
    if args.workload == "c2":
        traffic, traffic_note = hbm_traffic(kdtype, ks["spmm_bytes"] / max(1, ks["spmm_launches"]),
                                            "cocg" if wl["solver"] == 1 else "bicgstab")
    else:
        traffic, traffic_note = None, "counters are taken on the 64^3 scalar workload only"
    kname = "k_cocg_spmm" if wl["solver"] == 1 else "k_spmm_v / k_spmm_t"
    out = {
        "metric": METRIC, "value": m["value"], "unit": "eigenpairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * m["dt"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if main_form == "mixed" else "f64",
        "data": "synthetic", "config": {"workload": wl["desc"] + "; " + prec},
        "roofline": {"bound": "hbm", "achieved": spmm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": spmm_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"{kname} <{kdtype}> (complex-shifted sparse product)",
                     "launches": ks["spmm_launches"],
                     "avg_launch_ms": 1e3 * ks["spmm_seconds"] / max(1, ks["spmm_launches"]),
                     "algorithmic_bytes_per_launch": ks["spmm_bytes"] / max(1, ks["spmm_launches"]),
                     "traffic_note": traffic_note},
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
    if "bicgstab" in forms:
        f = forms["bicgstab"]
        fk = f["ks"]
        out["bicgstab_mixed"] = {"value": f["value"], "ms_per_step": 1e3 * f["dt"],
                                 "spmm_GBs": fk["spmm_bytes"] / fk["spmm_seconds"] / 1e9,
                                 "update_GBs": fk["update_bytes"] / fk["update_seconds"] / 1e9,
                                 "outer_iterations": f["results"][-1].stats["outer_iterations"],
                                 "spmv_total": f["results"][-1].stats["spmv_total"],
                                 "max_resid": f["results"][-1].stats["max_resid"]}
        out["cocg_over_bicgstab"] = m["value"] / f["value"]
    if smp is not None:
        ref = forms.get("fp64", m)      # the oracle is FP64: scale by the FP64 solve's work when it ran
        out["cpu_baseline"] = cpu_baseline(smp, ref["results"][-1].stats, wl["L"], wl["N"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
