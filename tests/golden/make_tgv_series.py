#!/usr/bin/env python3
"""Write the FP64 oracle's Taylor-Green reference series for the mixed-tier
error metrics (Sec. 4.2: e_E(t), e_Omega(t) and their maxima are taken
against a double-precision run of the same case).

This script calls only the oracle package (plain FP64 CPU code).  It writes
one JSON file per workload into this folder: the workload parameters and, for
the initial condition and every step, t, KE, enstrophy, max|div u| and the
solver iteration counts.

Workloads (periodic box [-pi, pi]^3, Re 1600, the Sec. 3 initial condition,
BDF3/EXT3, collocated convection, absolute tolerances 1e-6 velocity / 1e-4
pressure as in Sec. 3, GMRES(30) with the three-level hybrid Schwarz
multigrid pressure preconditioner, no projection space):
  tgv32_n7  32^3 elements, N = 7, dt = 5e-4, 205 steps
  tgv16_n11 16^3 elements, N = 11, dt = 2.5e-4, 400 steps

Usage: python tests/golden/make_tgv_series.py tgv32_n7 [--steps K]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    "tgv32_n7": dict(nel=32, N=7, dt=5e-4, steps=205),
    "tgv16_n11": dict(nel=16, N=11, dt=2.5e-4, steps=400),
}
RE, VTOL, PTOL, RESTART = 1600.0, 1e-6, 1e-4, 30


def series_path(name):
    return os.path.join(HERE, "oracle_series_%s.json" % name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=None)
    a = ap.parse_args()
    from oracle import OracleMesh, OracleFluid, num_threads
    from oracle.oracle import INIT_TGV3D
    w = dict(WORKLOADS[a.workload])
    if a.steps:
        w["steps"] = a.steps
    nel = (w["nel"],) * 3
    m = OracleMesh(nel, w["N"])
    f = OracleFluid(m, 1.0 / RE, w["dt"], torder=3, vtol=VTOL, ptol=PTOL, restart=RESTART, init=INIT_TGV3D,
                    hsmg=True)
    d0 = m.diagnostics(f.velocity())
    rows = [{"step": 0, "t": 0.0, "ke": d0[0], "enst": d0[1], "maxdiv": d0[2], "vit": [0, 0, 0], "pit": 0}]
    out = {"workload": a.workload, "nel": w["nel"], "N": w["N"], "re": RE, "dt": w["dt"], "vel_tol": VTOL,
           "pres_tol": PTOL, "gmres_restart": RESTART, "pressure_preconditioner": "hsmg", "convection": "collocated",
           "torder": 3, "threads": num_threads(), "series": rows}
    t0 = time.time()
    for k in range(1, w["steps"] + 1):
        o = f.step()
        rows.append({"step": k, "t": o["t"], "ke": o["ke"], "enst": o["enst"], "maxdiv": o["maxdiv"],
                     "vit": o["vit"], "pit": o["pit"]})
        print("step %d t=%.5f ke=%.15f enst=%.15f maxdiv=%.3e its v=%s p=%d (%.1f s)"
              % (k, o["t"], o["ke"], o["enst"], o["maxdiv"], o["vit"], o["pit"], time.time() - t0), flush=True)
        if k % 10 == 0 or k == w["steps"]:
            tmp = series_path(a.workload) + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(out, fh, indent=0)
            os.replace(tmp, series_path(a.workload))


if __name__ == "__main__":
    main()
