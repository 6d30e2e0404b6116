#!/usr/bin/env python3
"""Error report of the FP32-storage precision form (GPU).

FP32 storage of the stage states, metrics and fluxes with FP64 Q^n, stage
accumulation and reductions, against
  (a) the plain FP64 GPU path on the 800 x 400 x 320 jet mesh (102.4 M
      points), 50 RK5 steps, and
  (b) the FP64 CPU oracle on the 160 x 100 x 128 jet mesh (2.05 M points),
      a shorter run (the oracle's cost), with the FP64 GPU path beside it.
Per result: the residual R(Q0), the state after N steps, and the mean and
rms fields of (rho, u, v, w, p) over the azimuth and the N steps,
    <phi>(i, j) = mean over k and n = 1..N,  rms = sqrt(<phi^2> - <phi>^2).
Errors are relative max-norms, max|a - b| / max|b|, per variable (rms: per
variable, normalised by the max of the reference rms).  Both runs use the
same fixed dt (the CFL step of the FP64 initial state), so the differences
are those of the precision alone.

Usage: python tests/precision_report.py [--steps 50] [--oracle-steps 10]
Prints a Markdown table.
"""
import argparse
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from cases import problems  # noqa: E402

NAMES = ("rho", "u", "v", "w", "p")
CONS = ("rho", "rho u", "rho v", "rho w", "E")


def rel(a, b):
    return [float(np.abs(a[c] - b[c]).max() / max(np.abs(b[c]).max(), 1e-300)) for c in range(5)]


def mean_rms(s1, s2, count):
    m = s1 / count
    return m, np.sqrt(np.maximum(s2 / count - m * m, 0.0))


def gpu_run(solver_cls, pb, precision, dt, steps):
    """R(Q0), Q^N and the mean/rms fields of an N-step run on the GPU."""
    s = solver_cls(pb["params"], pb["xyz"], pb["inflow"], precision=precision)
    Qn = s.field(5, dtype=torch.float64, fill=0.0)
    s.interior(Qn).copy_(pb["Q"])
    Qs = s.field(5, fill=0.0)
    s.interior(Qs).copy_(pb["Q"])
    R = s.interior(s.residual(Qs)).double().cpu().numpy()
    st = s.new_stats()
    for _ in range(steps):
        s.rk5_step(Qn, 1, dt)
        s.diagnostics(Qn, st)
    nth = s.shape[2]
    m, r = mean_rms(st[0].cpu().numpy(), st[1].cpu().numpy(), nth * steps)
    Q = s.interior(Qn).cpu().numpy()
    s.close()
    return R, Q, m, r


def oracle_run(pb, dt, steps):
    from oracle import les
    prm = pb["params"]
    geo = les.geometry(pb["xyz"].numpy(), prm)
    Q = pb["Q"].numpy()
    inflow = pb["inflow"].numpy()
    R = les.evaluate(Q, geo, prm, inflow)
    nth = Q.shape[1]
    s1 = np.zeros((5,) + Q.shape[2:])
    s2 = np.zeros_like(s1)
    for n in range(steps):
        Q, _ = les.rk5_step(Q, geo, prm, inflow, dt=dt)
        print(f"[report] oracle step {n + 1}/{steps}", file=sys.stderr, flush=True)
        f = np.stack(les.primitives(Q, prm["gamma"]))
        s1 += f.sum(axis=1)
        s2 += (f * f).sum(axis=1)
    m, r = mean_rms(s1, s2, nth * steps)
    return R, Q, m, r


def row(label, errs):
    return "| " + label + " | " + " | ".join("%.2e" % e for e in errs) + " |"


def report(name, pairs, steps):
    print(f"\n### {name}, {steps} steps\n")
    print("| result | " + " | ".join(f"{a}/{b}" for a, b in zip(CONS, NAMES)) + " |")
    print("|---|" + "---|" * 5)
    for label, (a, b) in pairs:
        R1, Q1, m1, r1 = a
        R2, Q2, m2, r2 = b
        print(row(f"{label}: residual R(Q0)", rel(R1, R2)))
        print(row(f"{label}: state Q^N", rel(Q1, Q2)))
        print(row(f"{label}: mean fields", rel(m1, m2)))
        print(row(f"{label}: rms fields", rel(r1, r2)))
    sys.stdout.flush()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--oracle-steps", type=int, default=10)
    ap.add_argument("--skip-large", action="store_true")
    a = ap.parse_args()
    from paper_2301_00817_amd.solver import Solver
    from paper_2301_00817_amd import adjoint as A

    def fixed_dt(pb):
        s = Solver(pb["params"], pb["xyz"], pb["inflow"])
        Q = s.field(5, dtype=torch.float64, fill=0.0)
        s.interior(Q).copy_(pb["Q"])
        dt = A.cfl_dt(s, Q)
        s.close()
        return dt

    if not a.skip_large:
        cfg = problems.CONFIGS["prec102M"]
        pb = problems.jet_problem(*cfg["shape"], seed=cfg["seed"], device="cuda")
        t0 = time.time()
        dt = fixed_dt(pb)
        g64 = gpu_run(Solver, pb, "fp64", dt, a.steps)
        g32 = gpu_run(Solver, pb, "fp32", dt, a.steps)
        print(f"[report] 102M runs done in {time.time() - t0:.1f} s, dt {dt:.4e}",
              file=sys.stderr, flush=True)
        report("jet 800x400x320, FP32 form vs plain FP64 GPU", [("FP32 vs FP64", (g32, g64))],
               a.steps)
        del pb, g64, g32
        torch.cuda.empty_cache()

    cfg = problems.CONFIGS["adj2M"]
    pb = problems.jet_problem(*cfg["shape"], seed=cfg["seed"])
    dt = fixed_dt(pb)
    g64 = gpu_run(Solver, pb, "fp64", dt, a.oracle_steps)
    g32 = gpu_run(Solver, pb, "fp32", dt, a.oracle_steps)
    t0 = time.time()
    print("[report] oracle run on 160x100x128", file=sys.stderr, flush=True)
    orc = oracle_run(pb, dt, a.oracle_steps)
    print(f"[report] oracle done in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    report("jet 160x100x128 against the FP64 oracle",
           [("FP32 form vs oracle", (g32, orc)), ("FP64 GPU vs oracle", (g64, orc))],
           a.oracle_steps)


if __name__ == "__main__":
    main()
