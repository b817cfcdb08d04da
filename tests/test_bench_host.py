"""Host-side logic of bench.py (no GPU): the one-GPU guard and the counter
summary that turns rocprofv3 FETCH_SIZE / WRITE_SIZE values into bytes per
launch through the copy-kernel calibration."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def write_csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (kernel, value) in enumerate(rows):
            f.write(f'{i},"{kernel}",{counter},{value}\n')


def test_counter_summary_calibration(tmp_path):
    """A copy of 1 GiB that FETCH_SIZE reads as half its bytes and WRITE_SIZE as
    all of them gives factors 0.5 and 1.0; a sweep launch's counters are divided
    by them, averaged over its dispatches, and compared with the probe's
    algorithmic bytes."""
    copy = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda>(int)"
    back = "void slrf::k_sgs_sweep<float, 3, 0>(slrf::Batch, slrf::KrylovState<float>, int, int, int, int*)"
    fwd = "void slrf::k_sgs_sweep<float, 3, 2>(slrf::Batch, slrf::KrylovState<float>, int, int, int, int*)"
    final = "void slrf::k_sgs_sweep<float, 3, 1>(slrf::Batch, slrf::KrylovState<float>, int, int, int, int*)"
    kib = (1 << 30) / 1024
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    # the final sweep (mode 1) is not an iteration sweep and must be left out
    write_csv(fetch, "FETCH_SIZE", [(copy, 0.5 * kib), (back, 4e6), (fwd, 6e6), (final, 9e9)])
    write_csv(write, "WRITE_SIZE", [(copy, kib), (back, 1e6), (fwd, 1e6), (final, 9e9)])
    probe = tmp_path / "probe.log"
    probe.write_text('# probe\n{"family": "sgs", "dtype": "float", "full_launch_algorithmic_bytes": 3.43e9}\n')
    r = run_bench("--summarize-pmc", str(fetch), str(write), str(probe), "--workload", "c3")
    assert r.returncode == 0, r.stderr
    out = {}
    for line in r.stdout.splitlines():
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.rsplit(":", 1)
        out[k.strip()] = v.strip()
    assert float(out["copy_fetch_factor"]) == 0.5
    assert float(out["copy_write_factor"]) == 1.0
    assert out["k_sgs_sweep<float> dispatches"] == "2"
    expect = 5e6 * 1024 / 0.5 + 1e6 * 1024 / 1.0
    assert abs(float(out["full_launch_traffic_bytes sgs float"]) / expect - 1) < 1e-6
    assert abs(float(out["traffic_over_algorithmic sgs float"]) - expect / 3.43e9) < 1e-3


def test_l2_summary_hit_rate(tmp_path):
    """Hit rate = hits / (hits + misses), averaged per dispatch, per sweep mode."""
    back = "void slrf::k_sgs_sweep<float, 3, 0>(slrf::Batch, slrf::KrylovState<float>, int, int, int, int*)"
    fwd = "void slrf::k_sgs_sweep<float, 3, 2>(slrf::Batch, slrf::KrylovState<float>, int, int, int, int*)"
    path = tmp_path / "tcc.csv"
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (k, h, m) in enumerate([(back, 10, 30), (back, 30, 50), (fwd, 3, 1)]):
            f.write(f'{i},"{k}",TCC_HIT_sum,{h}\n{i},"{k}",TCC_MISS_sum,{m}\n')
    r = run_bench("--summarize-tcc", str(path), "--workload", "c3")
    assert r.returncode == 0, r.stderr
    lines = dict(l.rsplit(":", 1) for l in r.stdout.splitlines() if not l.startswith("#") and ":" in l)
    assert lines["k_sgs_sweep<float, 3, 0> dispatches"].strip() == "2"
    assert float(lines["k_sgs_sweep<float, 3, 0> hit_rate"]) == 0.333
    assert float(lines["k_sgs_sweep<float, 3, 2> hit_rate"]) == 0.75


def load_bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_roofline_fields_pick_the_nearer_roof():
    """The dominant kernel's line: algorithmic bytes and flops over the timed
    launches' seconds, each against its peak; the bound is the roof with the
    larger fraction, and frac = achieved / peak in the bound's unit."""
    b = load_bench()
    ks = {"spmm_seconds": 2.0, "spmm_bytes": 4.0e12, "spmm_launches": 1000}
    r = b.roofline_fields(ks, "k", "float", 2.0e13)          # 2 TB/s = 0.25 of HBM; 10 TF/s
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["achieved"] - 2000.0) < 1e-9 and r["peak"] == b.HBM_PEAK_GBS
    assert abs(r["frac"] - 0.25) < 1e-12
    assert abs(r["avg_launch_ms"] - 2.0) < 1e-12 and r["algorithmic_bytes_per_launch"] == 4.0e9
    r = b.roofline_fields(ks, "k", "double", 1.2e14)         # 60 TF/s of 78.6: the ALU roof is nearer
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert abs(r["frac"] - 60.0 / b.FP64_TFS) < 1e-12


def test_cpu_baseline_scaling():
    """The oracle sample scaled to one solve: column-iterations, the set-up of
    the N poles, and per outer iteration L (L + 3) B-products and L residuals."""
    b = load_bench()
    smp = {"s_per_column_iteration": 1e-3, "s_setup_per_pole": 2.0, "s_per_b_product": 1e-4,
           "s_per_residual_column": 1e-2, "workers": 16, "host_cpus": 32, "cpu_model": "x", "sample": "s"}
    stats = {"outer_iterations": 5, "spmv_total": 10000, "n_found": 50}
    out = b.cpu_baseline(smp, stats, 64, 8)
    est = 10000 * 1e-3 + 8 * 2.0 + 5 * 64 * 67 * 1e-4 + 5 * 64 * 1e-2
    assert abs(out["estimated_solve_seconds"] - est) < 1e-12
    assert abs(out["value"] - 50 / est) < 1e-12
    assert out["cores"] == 16 and out["kind"] == "oracle" and out["unit"] == "eigenpairs/s"
