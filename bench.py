#!/usr/bin/env python3
"""Throughput of the explicit LES RK5 step on one MI355X.

One step = one Jameson five-stage Runge-Kutta step over the whole mesh
(ghost fill, residual and stage update five times, plus the CFL time-step
reduction).  The metric is grid-point RK-stage updates per second:
    value = N_interior * 5 * steps / wall time   [Mpoint-RK-stage updates/s]
with the state resident in HBM before the timed region starts.

Default workload: the 288 x 160 x 128 (5.9 M points) supersonic jet mesh in
plain FP64, CFL 0.5, synthetic seeded inputs (cases/).

The JSON line also carries
  roofline     the dominant kernel's algorithmic HBM bytes per launch divided
               by its average launch time (HIP events on the launch stream,
               over the timed region), against the 8 TB/s HBM peak; `traffic`
               is the HBM bytes per launch measured by rocprofv3 FETCH_SIZE +
               WRITE_SIZE (profiles/traffic.json) when those counters were
               taken on the current kernel sources, else null;
  cpu_baseline the CPU oracle (plain NumPy FP64, single thread) timed on a
               bounded sample of the same workload: one RK stage (ghost fill,
               residual, update) over the whole mesh.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2301_00817_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

# Algorithmic HBM bytes per interior point of one launch of the fused RK
# stage kernel (k_fused): read the stage state Q^(l-1) (5 values) and the
# metrics (10), read Q^(0) (5 FP64), write Q^(l) (5).  FP64: 200 B.  FP32
# storage: 20 + 40 + 40 + 20 = 120 B, plus 40 B for the FP64 Q^(n+1) in the
# last stage, i.e. 128 B averaged over the five stages.
STAGE_BYTES = {"fp64": (5 + 10 + 5 + 5) * 8, "fp32": (5 + 10 + 5) * 4 + 5 * 8 + 5 * 8 / 5}
DOMINANT_KERNEL = "k_fused"


def source_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def make_workload(name, device):
    import torch
    from cases import flow, mesh, problems
    cfg = problems.CONFIGS[name]
    if cfg["kind"] == "box":
        pb = problems.box_problem(cfg["n"], seed=cfg["seed"])
        return pb["params"], pb["xyz"].to(device), pb["Q"].to(device), None
    nx, nr, nth = cfg["shape"]
    X, R, TH = problems.jet_grid(nx, nr, nth)
    xyz = mesh.cylindrical_coords(X, R, TH, device=device)
    Q = flow.jet_state(X, R, TH, seed=cfg["seed"], device=device)
    inflow = flow.jet_inflow(R, TH, seed=cfg["seed"], device=device)
    return problems.jet_params(), xyz, Q, inflow


def cpu_baseline(name):
    """The oracle on one RK stage of the same workload (single thread)."""
    import numpy as np
    from cases import problems
    from oracle import les
    cfg = problems.CONFIGS[name]
    if cfg["kind"] == "box":
        pb = problems.box_problem(cfg["n"], seed=cfg["seed"])
    else:
        pb = problems.jet_problem(*cfg["shape"], seed=cfg["seed"])
    xyz, Q = pb["xyz"].numpy(), pb["Q"].numpy()
    inflow = pb["inflow"].numpy() if pb["inflow"] is not None else None
    prm = pb["params"]
    geo = les.geometry(xyz, prm)
    dt = les.time_step(Q, geo, prm)
    t0 = time.perf_counter()
    R = les.evaluate(Q, geo, prm, inflow)
    Q1 = Q - prm["rk_alpha"][0] * dt * R
    t = time.perf_counter() - t0
    assert np.isfinite(Q1).all()
    n = Q.shape[1] * Q.shape[2] * Q.shape[3]
    return {"value": n / t / 1e6, "unit": "Mpoint-RK-stage updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"one RK stage (ghost fill + residual + update) over the whole "
                      f"{Q.shape[3]}x{Q.shape[2]}x{Q.shape[1]} mesh, NumPy FP64, 1 thread, "
                      f"{t:.1f} s"}


def traffic_for(kernel, workload, launches_bytes):
    """HBM bytes per launch from committed rocprofv3 counters, if current."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = t.get(kernel, {}).get(workload)
    if not rec or rec.get("source_sha") != source_hash():
        return None
    return rec["bytes_per_launch"]


def copy_probe(gib, dev, reps=5):
    """Time a plain device copy of a known size (reads and writes `gib` GiB
    per launch); its FETCH_SIZE/WRITE_SIZE counters calibrate the traffic
    numbers and its bandwidth is the achievable streaming rate."""
    import torch
    n = int(gib * 2 ** 30) // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        b.copy_(a)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # a plain elementwise streaming kernel (dword loads/stores, like the
    # solver's kernels): reads a, writes b
    e0.record(st)
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    e1.record(st)
    torch.cuda.synchronize()
    ms2 = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_probe": {"bytes_read": n * 8, "bytes_written": n * 8,
                                     "copy_ms": ms, "copy_GBps": 2 * n * 8 / ms / 1e6,
                                     "elementwise_ms": ms2,
                                     "elementwise_GBps": 2 * n * 8 / ms2 / 1e6}}), flush=True)


def rocprof_summary(csv_dir, out_path, command, kernel=DOMINANT_KERNEL):
    """Short text summary of a rocprofv3 --kernel-trace --stats CSV run."""
    import csv
    stats = os.path.join(csv_dir, [f for f in os.listdir(csv_dir) if f.endswith("kernel_stats.csv")][0])
    rows = list(csv.DictReader(open(stats)))
    lines = [f"command: {command}", "",
             f"{'kernel':40s} {'calls':>7s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}"]
    for r in rows[:15]:
        lines.append(f"{r['Name'][:40]:40s} {int(r['Calls']):7d} {float(r['AverageNs'])/1e3:10.1f} "
                     f"{float(r['MinNs'])/1e3:10.1f} {float(r['MaxNs'])/1e3:10.1f} {float(r['Percentage']):6.2f}")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return out_path


def _counter_rows(csv_dir):
    import csv
    f = [x for x in os.listdir(csv_dir) if x.endswith("counter_collection.csv")][0]
    return list(csv.DictReader(open(os.path.join(csv_dir, f))))


def _median_counter(rows, kernel_prefix, counter):
    vals = sorted(float(r["Counter_Value"]) for r in rows
                  if r["Kernel_Name"].startswith(kernel_prefix) and r["Counter_Name"] == counter)
    return vals[len(vals) // 2] if vals else None, len(vals)


def traffic_record(fetch_dir, write_dir, cfetch_dir, cwrite_dir, workload, known_bytes):
    """Stage-kernel HBM bytes per launch from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled by the ratio known / counted bytes of a plain
    elementwise streaming kernel; written into profiles/traffic.json."""
    f, nf = _median_counter(_counter_rows(fetch_dir), DOMINANT_KERNEL, "FETCH_SIZE")
    w, nw = _median_counter(_counter_rows(write_dir), DOMINANT_KERNEL, "WRITE_SIZE")
    cf, _ = _median_counter(_counter_rows(cfetch_dir), "vectorized_elementwise", "FETCH_SIZE")
    cw, _ = _median_counter(_counter_rows(cwrite_dir), "vectorized_elementwise", "WRITE_SIZE")
    kf = known_bytes / (cf * 1024.0)
    kw = known_bytes / (cw * 1024.0)
    rec = {"fetch_kib": f, "write_kib": w, "dispatches": [nf, nw],
           "calib_fetch_factor": kf, "calib_write_factor": kw,
           "bytes_per_launch": f * 1024.0 * kf + w * 1024.0 * kw,
           "source_sha": source_hash()}
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        t = {}
    t.setdefault(DOMINANT_KERNEL, {})[workload] = rec
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1, sort_keys=True)
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="jet5.9M")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="GIB",
                    help="only time a device copy of this many GiB (counter calibration)")
    ap.add_argument("--rocprof-summary", nargs=3, metavar=("CSV_DIR", "OUT", "COMMAND"),
                    help="write a text summary of a rocprofv3 kernel-stats CSV and exit")
    ap.add_argument("--traffic-from", nargs=6,
                    metavar=("FETCH_DIR", "WRITE_DIR", "CAL_FETCH_DIR", "CAL_WRITE_DIR", "WORKLOAD",
                             "CAL_BYTES"),
                    help="record stage-kernel HBM traffic from rocprofv3 counter CSVs and exit")
    args = ap.parse_args()
    if args.traffic_from:
        a = args.traffic_from
        print(json.dumps(traffic_record(a[0], a[1], a[2], a[3], a[4], float(a[5]))))
        return
    if args.rocprof_summary:
        print(rocprof_summary(*args.rocprof_summary))
        return

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is a design note, not code.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2301_00817_amd.solver import Solver

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        copy_probe(args.copy_probe, dev)
        return
    from cases import problems
    kind = problems.CONFIGS[args.config]["kind"]
    prm, xyz, Q, inflow = make_workload(args.config, dev)
    s = Solver(prm, xyz, inflow, precision=args.precision, device=dev)
    del xyz
    nx, nr, nth = s.shape
    npts = nx * nr * nth
    Qn = s.pad(Q, dtype=torch.float64)
    del Q
    torch.cuda.synchronize()
    print(f"[bench] {args.config} {nx}x{nr}x{nth} {args.precision}: warmup {args.warmup}",
          file=sys.stderr, flush=True)
    if args.warmup:
        s.rk5_step(Qn, args.warmup)
    torch.cuda.synchronize()

    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    s.profile(True)
    s.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dts = s.rk5_step(Qn, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, kms = s.profile_read()
    s.profile(False)
    assert bool(torch.isfinite(s.interior(Qn)).all()), "state is not finite"

    value = npts * 5 * args.steps / wall / 1e6
    bytes_launch = STAGE_BYTES[args.precision] * npts
    avg_ms = kms / max(launches, 1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    workload = f"{args.config}-{args.precision}"
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic_for(DOMINANT_KERNEL, workload, bytes_launch),
            "kernel": DOMINANT_KERNEL, "avg_launch_ms": round(avg_ms, 4),
            "launches": launches, "algorithmic_bytes_per_launch": bytes_launch}

    out = {
        "metric": "Mpoint-RK-stage updates/s",
        "value": round(value, 2),
        "unit": "Mpoint-RK-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-storage/f64-accumulate",
        "data": "synthetic",
        "config": {"workload": f"jet mesh {nx}x{nr}x{nth} ({npts} points), {args.precision}, "
                               f"CFL {prm['cfl']}, RK5 steps" if kind == "jet" else
                               f"periodic box {nx}^3, {args.precision}, CFL {prm['cfl']}",
                   "points": npts, "precision": args.precision,
                   "dt_last": float(dts[-1])},
        "roofline": roof,
    }
    s.close()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.config)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
