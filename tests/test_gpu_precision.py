"""The FP32-storage precision form against FP64, with the bars of the
precision form asserted per result (the norms are described in _helpers):

  result                      bar     asserted norm
  residual R(Q0)              1e-3    per variable
  state Q^N                   1e-5    P1 (momentum over its magnitude)
  mean fields                 1e-5    P1 (velocity over its magnitude)
  rms fields                  1e-2    per variable

Mean and rms fields of phi = (rho, u, v, w, p) are taken over the azimuth
and the N steps, <phi>(i, j) = mean over k and n = 1..N,
rms = sqrt(<phi^2> - <phi>^2).  Both forms run with the same fixed dt (the
CFL step of the FP64 initial state), so the differences are those of the
precision alone.  Two comparisons:
  * the 160 x 100 x 128 jet (2.05 M points) against the FP64 CPU oracle,
    10 steps (the oracle's cost), with the plain FP64 GPU path beside it
    (per-variable bar 1e-11 on its state, as for every FP64 state);
  * the 800 x 400 x 320 jet (102.4 M points) against the plain FP64 GPU
    path, 50 steps.
Every norm of every result is printed."""
import numpy as np
import pytest
import torch

from _helpers import announce, per_variable_err, report, vector_err
from cases import problems

pytestmark = pytest.mark.gpu

BARS = {"residual": 1e-3, "state": 1e-5, "mean": 1e-5, "rms": 1e-2}


def _mean_rms(s1, s2, count):
    m = s1 / count
    return m, np.sqrt(np.maximum(s2 / count - m * m, 0.0))


def _fixed_dt(pb, grid=False):
    from paper_2301_00817_amd import adjoint as A
    from paper_2301_00817_amd.solver import Solver
    mesh = {"grid": pb["grid"]} if grid else {"xyz": pb["xyz"]}
    s = Solver(pb["params"], inflow=pb["inflow"], **mesh)
    Q = s.field(5, dtype=torch.float64, fill=0.0)
    s.interior(Q).copy_(pb["Q"])
    dt = A.cfl_dt(s, Q)
    s.close()
    return dt


def _gpu_run(pb, precision, dt, steps, grid=False):
    """R(Q0), Q^N and the mean/rms fields of an N-step run on the GPU."""
    from paper_2301_00817_amd.solver import Solver
    mesh = {"grid": pb["grid"]} if grid else {"xyz": pb["xyz"]}
    s = Solver(pb["params"], inflow=pb["inflow"], precision=precision, **mesh)
    Qn = s.field(5, dtype=torch.float64, fill=0.0)
    s.interior(Qn).copy_(pb["Q"])
    Qs = s.field(5, fill=0.0)
    s.interior(Qs).copy_(pb["Q"])
    R = s.interior(s.residual(Qs)).double().cpu().numpy()
    del Qs
    st = s.new_stats()
    for _ in range(steps):
        s.rk5_step(Qn, 1, dt)
        s.diagnostics(Qn, st)
    nth = s.shape[2]
    m, r = _mean_rms(st[0].cpu().numpy(), st[1].cpu().numpy(), nth * steps)
    Q = s.interior(Qn).cpu().numpy()
    s.close()
    return R, Q, m, r


def _oracle_run(pb, dt, steps):
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
        print(f"[precision] oracle step {n + 1}/{steps}", flush=True)
        f = np.stack(les.primitives(Q, prm["gamma"]))
        s1 += f.sum(axis=1)
        s2 += (f * f).sum(axis=1)
    m, r = _mean_rms(s1, s2, nth * steps)
    return R, Q, m, r


def _check(label, got, ref, bars=BARS):
    """Print every norm of the four results; return the asserted ones."""
    R1, Q1, m1, r1 = got
    R2, Q2, m2, r2 = ref
    out = {}
    for name, a, b in (("residual", R1, R2), ("state", Q1, Q2), ("mean", m1, m2),
                       ("rms", r1, r2)):
        pv = per_variable_err(a, b)
        vn = vector_err(a, b)
        report(f"{label} {name}", per_variable=pv, vector=vn)
        out[name] = float(pv.max()) if name in ("residual", "rms") else float(vn.max())
    for name, bar in bars.items():
        assert out[name] <= bar, (label, name, out[name], bar)
    return out


@pytest.mark.timeout(900)
def test_fp32_form_against_oracle_2M():
    announce("precision", "jet160x100x128 vs oracle, 10 steps")
    cfg = problems.CONFIGS["adj2M"]
    pb = problems.jet_problem(*cfg["shape"], seed=cfg["seed"])
    dt = _fixed_dt(pb)
    steps = 10
    g64 = _gpu_run(pb, "fp64", dt, steps)
    g32 = _gpu_run(pb, "fp32", dt, steps)
    orc = _oracle_run(pb, dt, steps)
    _check("jet160x100x128 FP32 vs oracle", g32, orc)
    # the plain form: state per variable within the FP64 bar
    pv = per_variable_err(g64[1], orc[1])
    _check("jet160x100x128 FP64 vs oracle", g64, orc,
           bars={"residual": 1e-12, "state": 1e-11, "mean": 1e-11, "rms": 1e-5})
    assert pv.max() <= 1e-11


@pytest.mark.timeout(600)
def test_fp32_form_against_fp64_102M():
    announce("precision", "jet800x400x320 FP32 vs FP64, 50 steps")
    cfg = problems.CONFIGS["prec102M"]
    pb = problems.jet_problem(*cfg["shape"], seed=cfg["seed"], device="cuda", with_xyz=False)
    dt = _fixed_dt(pb, grid=True)
    steps = 50
    g64 = _gpu_run(pb, "fp64", dt, steps, grid=True)
    torch.cuda.empty_cache()
    g32 = _gpu_run(pb, "fp32", dt, steps, grid=True)
    _check("jet800x400x320 FP32 vs FP64 GPU", g32, g64)
