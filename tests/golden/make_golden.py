"""Writes the stored expected values under tests/golden/ using only ``oracle/``
and the shared input generator ``pencils``.

    python tests/golden/make_golden.py poles     # SLRF pole tables, N = 4, 6, 8
    python tests/golden/make_golden.py count_c2  # inertia count of the 64^3 scalar pencil

Pole tables: the oracle's SLRF design (ridge-regularised least squares, see
oracle/poles.py) at gamma = 1, alpha = 1, beta = 0.01 (the paper's Section 4.2
setting).  Count: Sylvester inertia of A - gamma B for the 64^3 log-normal
scalar pencil at gamma = 421 (sparse symmetric factorisation; several minutes).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import pencils  # noqa: E402
from oracle import inertia, poles  # noqa: E402


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


if __name__ == "__main__":
    what = sys.argv[1:] or ["poles", "count_c2"]
    if "poles" in what:
        make_poles()
    if "count_c2" in what:
        make_count_c2()
