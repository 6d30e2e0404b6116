#!/usr/bin/env python3
"""Throughput of the explicit LES RK5 step on one MI355X.

One step = one Jameson five-stage Runge-Kutta step over the whole mesh
(ghost fill, residual and stage update five times, plus the CFL time-step
reduction).  The metric is grid-point RK-stage updates per second:
    value = N_interior * 5 * steps / wall time   [Mpoint-RK-stage updates/s]
with the state resident in HBM before the timed region starts.

Default workload: the largest single-GPU jet mesh, 1250 x 640 x 1250
(1.0e9 points, the size of the paper's largest mesh), built on the device
from its 1-D axial, radial and azimuthal maps; the timed line is the plain
FP64 form, CFL 0.5, synthetic seeded inputs (cases/).

The JSON line also carries
  roofline     algorithmic HBM bytes per launch of the stage kernel divided
               by its average launch time (HIP events on the launch stream,
               over the timed region), against the 8 TB/s HBM peak.  The
               bytes are those the method moves per interior point and RK
               stage taken as its two steps, residual (read the stage state
               and the metrics, write R) and update (read Q^(0) and R, write
               the new stage state): FP64 280 B, FP32 storage 168 B averaged
               over the five stages.  `fused` gives the same kernel against
               the bytes it moves itself (R never leaves the chip: 200 B,
               FP32 storage 128 B).  `traffic` is the HBM bytes per launch
               measured by rocprofv3 FETCH_SIZE + WRITE_SIZE
               (profiles/traffic.json) when those counters were taken on the
               current kernel sources and on this workload, else null;
               `stream_GBs` the rate of a plain elementwise streaming kernel
               (4 GiB read and written) measured in the same run, the
               achievable bandwidth beside the nominal peak;
  cpu_baseline the CPU oracle (plain NumPy FP64, one thread) on bounded
               samples: one residual and one RK5 step of the 160 x 100 x 128
               and 288 x 160 x 128 jet meshes, median of three runs each;
               `value` is the RK5-step rate on 288 x 160 x 128;
  precision_forms  the same workload and step count in the other precision
               form (FP32 storage with FP64 accumulation, or plain FP64);
  adjoint      residual-adjoint calls per second (les_residual_vjp) on the
               160 x 100 x 128 jet mesh, and their time over that of
               les_residual on the same state (median of three alternating
               blocks of 20 calls of each).
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
VJP_BYTES_PER_POINT = 200
CSRC = os.path.join(ROOT, "paper_2301_00817_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
DEFAULT_CONFIG = "big1B"
# The metric this line reports: `value` is the point-update rate; the HBM
# fraction is `roofline`, FP32 against FP64 `precision_forms`, the adjoint's
# calls per second `adjoint`.
METRIC = "Mpoint-RK-stage updates/s + HBM GB/s % of peak, FP32 vs FP64; adjoint VJP/s"

# Algorithmic HBM bytes per interior point and RK stage, the method taken as
# residual + update: residual reads the stage state (5 values) and the
# metrics (10) and writes R (5); the update reads Q^(0) (5, FP64), R (5) and
# writes the stage state (5).  FP64: 160 + 120 = 280 B.  FP32 storage: 80 B
# residual; the update reads Q^(0) 40 + R 20, writes 20, and in the last
# stage also the FP64 Q^(n+1) (40): 88 B averaged; 168 B in all.
METHOD_STAGE_BYTES = {"fp64": 280.0, "fp32": 168.0}
# The fused stage kernel (k_fused) moves per interior point: read the stage
# state (5) and the metrics (10), read Q^(0) (5 FP64), write the stage state
# (5).  FP64: 200 B.  FP32 storage: 20 + 40 + 40 + 20 = 120 B, plus 40 B for
# the FP64 Q^(n+1) in the last stage, i.e. 128 B averaged over the stages.
FUSED_STAGE_BYTES = {"fp64": (5 + 10 + 5 + 5) * 8.0, "fp32": (5 + 10 + 5) * 4 + 5 * 8 + 5 * 8 / 5}
# The per-step update schedule (viscosities held from stage 1) adds two
# values per point: written by the first stage, read by the four others.
HELD_VISC_BYTES = {"fp64": 2 * 8, "fp32": 2 * 4}
DOMINANT_KERNEL = "k_fused"


# the sources the stage kernel is compiled from and its compiler flags (its
# traffic record is tied to them)
STAGE_SOURCES = ("common.hpp", "physics.hpp", "plane_io.hpp", "fused_stage.hpp",
                 "residual_fused.hip", "residual_fused32.hip")


def source_hash():
    from paper_2301_00817_amd import build
    h = hashlib.sha256()
    for f in STAGE_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    flags = list(build.CFLAGS)
    for f in STAGE_SOURCES:
        flags += list(build.SOURCE_FLAGS.get(f, []))
    h.update(" ".join(f for f in flags if not f.startswith("/")).encode())
    return h.hexdigest()[:16]


def make_workload(name, device, chunk_points=64 * 2 ** 20):
    """(params, mesh, fill, inflow) of a named workload on `device`: mesh is
    {"xyz": coordinates} (box) or {"grid": (X, R, TH)} (jet, the 1-D maps the
    library builds the mesh from); fill(Qi) writes the initial state into the
    interior view Qi (5, nth, nr, nx) in azimuthal chunks, so meshes of 1e9
    points need no full-size temporaries."""
    from cases import flow, problems
    cfg = problems.CONFIGS[name]
    if cfg["kind"] == "box":
        pb = problems.box_problem(cfg["n"], seed=cfg["seed"])
        Q = pb["Q"].to(device)
        return pb["params"], {"xyz": pb["xyz"]}, (lambda Qi: Qi.copy_(Q)), None
    nx, nr, nth = cfg["shape"]
    X, R, TH = problems.jet_grid(nx, nr, nth)
    kc = max(1, chunk_points // (nx * nr))

    def fill(Qi):
        for k0 in range(0, nth, kc):
            k1 = min(nth, k0 + kc)
            Qi[:, k0:k1] = flow.jet_state(X, R, TH, seed=cfg["seed"], k0=k0, k1=k1, device=device)

    inflow = flow.jet_inflow(R, TH, seed=cfg["seed"], device=device)
    prm = problems.jet_params() if cfg.get("sgs", True) else problems.jet_params(sgs_model=0)
    return prm, {"grid": (X, R, TH)}, fill, inflow


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(reps=3):
    """The oracle (NumPy FP64, one thread) on bounded samples: one residual
    (ghost fill + residual) and one RK5 step (CFL dt + five stages) of the
    160 x 100 x 128 and 288 x 160 x 128 jet meshes, median of `reps` runs
    each.  `value` is the RK5-step rate on 288 x 160 x 128."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from cases import problems
    from oracle import les
    samples = {}
    with threadpool_limits(limits=1):
        for name in ("adj2M", "jet5.9M"):
            cfg = problems.CONFIGS[name]
            pb = problems.jet_problem(*cfg["shape"], seed=cfg["seed"])
            xyz, Q = pb["xyz"].numpy(), pb["Q"].numpy()
            inflow, prm = pb["inflow"].numpy(), pb["params"]
            geo = les.geometry(xyz, prm)
            n = Q.shape[1] * Q.shape[2] * Q.shape[3]
            tr, ts = [], []
            for _ in range(reps):
                t0 = time.perf_counter()
                R = les.evaluate(Q, geo, prm, inflow)
                tr.append(time.perf_counter() - t0)
                t0 = time.perf_counter()
                Q1, _ = les.rk5_step(Q, geo, prm, inflow)
                ts.append(time.perf_counter() - t0)
                assert np.isfinite(R).all() and np.isfinite(Q1).all()
            mr, ms = float(np.median(tr)), float(np.median(ts))
            nx, nr, nth = cfg["shape"]
            samples[f"jet{nx}x{nr}x{nth}"] = {
                "points": n,
                "residual_s": round(mr, 3), "residual_Mpoint_per_s": round(n / mr / 1e6, 4),
                "rk5_step_s": round(ms, 3),
                "rk5_Mpoint_stage_per_s": round(5 * n / ms / 1e6, 4),
                "runs_s": {"residual": [round(t, 3) for t in tr],
                           "rk5_step": [round(t, 3) for t in ts]}}
            del geo, Q, xyz, pb
    head = samples["jet288x160x128"]
    return {"value": head["rk5_Mpoint_stage_per_s"], "unit": "Mpoint-RK-stage updates/s",
            "cores": 1, "kind": "oracle",
            "sample": "one RK5 step (CFL dt, 5 x (ghost fill + residual + update)) of the "
                      "288x160x128 jet mesh, NumPy FP64, 1 thread, median of 3; also one "
                      "residual and one step of the 160x100x128 mesh (samples)",
            "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(),
            "samples": samples}


def traffic_for(kernel, workload):
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
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_read": n * 8, "bytes_written": n * 8, "copy_ms": ms,
            "copy_GBps": 2 * n * 8 / ms / 1e6, "elementwise_ms": ms2,
            "elementwise_GBps": 2 * n * 8 / ms2 / 1e6}


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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default=DEFAULT_CONFIG)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--sgs", default=None, choices=["none", "smagorinsky", "vreman", "dynamic"],
                    help="subgrid model (default: the workload's own)")
    ap.add_argument("--schedule", default="stage", choices=["stage", "step"],
                    help="update viscosities and boundary values every stage (default) or "
                         "once per step, as the paper's solver does")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other-precision run and the adjoint timing")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only time les_residual_vjp against les_residual (160x100x128 jet)")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="only time the CPU oracle samples (no GPU needed)")
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
    if args.cpu_baseline_only:
        print(json.dumps({"cpu_baseline": cpu_baseline()}), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is a design note, not code.", file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        print(json.dumps({"copy_probe": copy_probe(args.copy_probe, dev)}), flush=True)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": time_adjoint("adj2M", dev)}), flush=True)
        return
    from cases import problems
    kind = problems.CONFIGS[args.config]["kind"]
    r = time_rk(args.config, args.precision, args.steps, args.warmup, dev, args.schedule, args.sgs)
    nx, nr, nth = r["shape"]
    npts = nx * nr * nth
    prm = r["params"]
    value = npts * 5 * args.steps / r["wall"] / 1e6
    workload = f"{args.config}-{args.precision}" + ("-step" if args.schedule == "step" else "")
    roof = roofline(args.precision, args.schedule == "step" and prm["visc_coef"] != 0.0, npts,
                    r, workload)

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mpoint-RK-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["wall"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-storage/f64-accumulate",
        "data": "synthetic",
        "config": {"workload": f"jet mesh {nx}x{nr}x{nth} ({npts} points), {args.precision}, "
                               f"CFL {prm['cfl']}, RK5 steps"
                               + {0: ", no SGS model", 1: "", 2: ", Vreman SGS model",
                                  3: ", dynamic SGS model"}[prm.get("sgs_model", 1)]
                               + (", viscosities and boundary values updated once per step"
                                  if args.schedule == "step" else "")
                               if kind == "jet" else
                               f"periodic box {nx}^3, {args.precision}, CFL {prm['cfl']}",
                   "points": npts, "precision": args.precision,
                   "dt_last": r["dt_last"], "hbm_footprint_gb": r["hbm_gb"],
                   "device_used_gb": r["device_used_gb"],
                   "device_total_gb": r["device_total_gb"]},
        "roofline": roof,
    }
    if not args.no_extras:
        other = "fp32" if args.precision == "fp64" else "fp64"
        print(f"[bench] same workload in {other}", file=sys.stderr, flush=True)
        r2 = time_rk(args.config, other, args.steps, args.warmup, dev, args.schedule, args.sgs)
        v2 = npts * 5 * args.steps / r2["wall"] / 1e6
        fp32_v, fp64_v = (v2, value) if other == "fp32" else (value, v2)
        roof2 = roofline(other, args.schedule == "step" and prm["visc_coef"] != 0.0, npts, r2,
                         f"{args.config}-{other}" + ("-step" if args.schedule == "step" else ""))
        out["precision_forms"] = {"fp64": round(fp64_v, 2), "fp32": round(fp32_v, 2),
                                  "fp32_over_fp64": round(fp32_v / fp64_v, 3),
                                  "unit": "Mpoint-RK-stage updates/s",
                                  other + "_run": {
                                          "ms_per_step": round(r2["wall"] / args.steps * 1e3, 4),
                                          "hbm_footprint_gb": r2["hbm_gb"],
                                          "device_used_gb": r2["device_used_gb"],
                                          "roofline": roof2}}
        print("[bench] adjoint timing", file=sys.stderr, flush=True)
        out["adjoint"] = time_adjoint("adj2M", dev)
        # the achievable streaming rate on this machine: a plain elementwise
        # kernel reading and writing 4 GiB, beside the nominal 8 TB/s peak
        print("[bench] streaming probe", file=sys.stderr, flush=True)
        cp = copy_probe(4, dev)
        stream = round(cp["elementwise_GBps"], 1)
        for rf in (out["roofline"], out["precision_forms"][other + "_run"]["roofline"]):
            rf["stream_GBs"] = stream
            rf["frac_of_stream"] = round(rf["achieved"] / stream, 4)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def roofline(precision, held, npts, r, workload):
    """Roofline object of the stage kernel from a time_rk result."""
    avg_ms = r["kernel_ms"] / max(r["launches"], 1)
    extra = HELD_VISC_BYTES[precision] if held else 0
    method_bytes = (METHOD_STAGE_BYTES[precision] + extra) * npts
    fused_bytes = (FUSED_STAGE_BYTES[precision] + extra) * npts
    achieved = method_bytes / (avg_ms * 1e-3) / 1e9
    fused = fused_bytes / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic_for(DOMINANT_KERNEL, workload),
            "kernel": DOMINANT_KERNEL, "avg_launch_ms": round(avg_ms, 4),
            "launches": r["launches"],
            "algorithmic_bytes_per_point": METHOD_STAGE_BYTES[precision] + extra,
            "algorithmic_bytes_per_launch": method_bytes,
            "fused": {"bytes_per_point": FUSED_STAGE_BYTES[precision] + extra,
                      "achieved": round(fused, 1), "frac": round(fused / PEAK_HBM_GBS, 4)}}


SGS_MODELS = {"none": 0, "smagorinsky": 1, "vreman": 2, "dynamic": 3}


def time_rk(config, precision, steps, warmup, dev, schedule="stage", sgs=None):
    """Wall time of `steps` RK5 steps (CFL dt) of a workload resident in HBM,
    with the stage kernel's launches timed by HIP events on its stream."""
    import torch
    from paper_2301_00817_amd.solver import Solver
    t_setup = time.perf_counter()
    prm, mesh, fill, inflow = make_workload(config, dev)
    prm = dict(prm, schedule=schedule)
    if sgs is not None:
        prm["sgs_model"] = SGS_MODELS[sgs]
    s = Solver(prm, inflow=inflow, precision=precision, device=dev, **mesh)
    torch.cuda.empty_cache()
    nx, nr, nth = s.shape
    Qn = s.field(5, dtype=torch.float64, fill=0.0)
    fill(s.interior(Qn))
    torch.cuda.synchronize()
    hbm = torch.cuda.max_memory_allocated(dev) / 1e9
    _, _, held = s.query()
    print(f"[bench] device bytes held by the library {held / 1e9:.1f} GB, state "
          f"{Qn.numel() * 8 / 1e9:.1f} GB, torch peak {hbm:.1f} GB, set-up "
          f"{time.perf_counter() - t_setup:.1f} s", file=sys.stderr, flush=True)
    print(f"[bench] {config} {nx}x{nr}x{nth} {precision}: warmup {warmup}",
          file=sys.stderr, flush=True)
    if warmup:
        s.rk5_step(Qn, warmup)
    torch.cuda.synchronize()
    print(f"[bench] timing {steps} steps", file=sys.stderr, flush=True)
    s.profile(True)
    s.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dts = s.rk5_step(Qn, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launches, kms = s.profile_read()
    s.profile(False)
    assert bool(torch.isfinite(s.interior(Qn)).all()), "state is not finite"
    _, _, held = s.query()
    free, total = torch.cuda.mem_get_info(dev)
    r = {"shape": s.shape, "params": prm, "wall": wall, "launches": launches, "kernel_ms": kms,
         "dt_last": float(dts[-1]), "hbm_gb": round((held + Qn.numel() * 8) / 1e9, 2),
         "device_used_gb": round((total - free) / 1e9, 1), "device_total_gb": round(total / 1e9, 1)}
    print(f"[bench] {steps} steps in {wall:.3f} s, stage kernel {kms / max(launches, 1):.3f} ms "
          f"per launch", file=sys.stderr, flush=True)
    s.close()
    del Qn
    torch.cuda.empty_cache()
    return r


def time_adjoint(config, dev, reps=20, rounds=3):
    """Time of les_residual_vjp and of les_residual (ghost fill included in
    both) on one state, by HIP events on the call stream: the mean over
    `reps` calls, in `rounds` alternating blocks of each, the median block
    reported (a single block of the 0.2 ms residual varied by a few per cent
    between runs)."""
    import torch
    from cases import flow, problems
    from paper_2301_00817_amd.solver import Solver
    prm, mesh, fill, inflow = make_workload(config, dev)
    s = Solver(prm, inflow=inflow, precision="fp64", device=dev, **mesh)
    Qp = s.field(5, dtype=torch.float64, fill=0.0)
    fill(s.interior(Qp))
    nx, nr, nth = s.shape
    Rb = s.pad(problems.seeded_field((5, nth, nr, nx), 3, flow.FIELD_COTANGENT, device=dev),
               fill=0.0)
    Qb = s.field(5, dtype=torch.float64)
    R = s.field(5)
    ib = s.new_inflow_bar()
    for _ in range(3):
        s.residual(Qp, R)
        s.residual_vjp(Qp, Rb, Qb, ib)
    st = torch.cuda.current_stream(dev)
    trs, tvs = [], []
    for _ in range(rounds):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        torch.cuda.synchronize()
        ev[0].record(st)
        for _ in range(reps):
            s.residual(Qp, R)
        ev[1].record(st)
        for _ in range(reps):
            s.residual_vjp(Qp, Rb, Qb, ib)
        ev[2].record(st)
        torch.cuda.synchronize()
        trs.append(ev[0].elapsed_time(ev[1]) / reps)
        tvs.append(ev[1].elapsed_time(ev[2]) / reps)
    tr = sorted(trs)[rounds // 2]
    tv = sorted(tvs)[rounds // 2]
    nx, nr, nth = s.shape
    s.close()
    torch.cuda.empty_cache()
    # algorithmic bytes of one VJP per interior point: read Q 40, metrics 80,
    # Rbar 40; write Qbar 40
    gbs = VJP_BYTES_PER_POINT * nx * nr * nth / (tv * 1e-3) / 1e9
    return {"workload": f"jet mesh {nx}x{nr}x{nth}, fp64, seeded Gaussian cotangent",
            "vjp_per_s": round(1e3 / tv, 2), "vjp_ms": round(tv, 4),
            "residual_ms": round(tr, 4), "vjp_over_residual": round(tv / tr, 3),
            "timing": f"median of {rounds} alternating blocks of {reps} calls each",
            "hbm_algorithmic_GBs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)}


if __name__ == "__main__":
    main()
