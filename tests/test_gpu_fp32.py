"""FP32-storage form: stage states, metrics and fluxes in FP32, Q^n and the
stage accumulation Q^n - alpha dt R in FP64.  Its error against the FP64
oracle is a precision statement, not parity: FP32 rounding of O(1) fluxes
whose differences are O(h) smaller leaves a relative residual error of
order 1e-6 .. 1e-4, and a state error of order N * CFL * 6e-8.

Bars: residual 1e-3 per variable; state after 10 and after 50 steps 1e-5
in the vector norm (P1 of _helpers: momentum components over the largest
momentum magnitude; the per-variable errors of the noise-level rho v, rho w
are printed); free stream 1e-5 of the flux scale.  The full set of bars
(with mean and rms fields) is asserted in test_gpu_precision."""
import numpy as np
import pytest
import torch

from _helpers import announce, make_solver, per_variable_err, report, to_np, vector_err
from cases import flow, problems
from oracle import les

pytestmark = pytest.mark.gpu


def _oracle(pb):
    geo = les.geometry(pb["xyz"].numpy(), pb["params"])
    inflow = pb["inflow"].numpy() if pb.get("inflow") is not None else None
    return geo, inflow


@pytest.mark.parametrize("name", ["box32", "jet70x33x24"])
def test_fp32_residual_error(name):
    announce("fp32-residual", name)
    pb = problems.box_problem(32) if name == "box32" else problems.jet_problem(70, 33, 24)
    geo, inflow = _oracle(pb)
    R_ref = les.evaluate(pb["Q"].numpy(), geo, pb["params"], inflow)
    s = make_solver(pb, precision="fp32")
    Qp = s.pad(pb["Q"].cuda().float())
    R = to_np(s.interior(s.residual(Qp))).astype(np.float64)
    pv = per_variable_err(R, R_ref)
    report(f"{name} FP32 residual", per_variable=pv, vector=vector_err(R, R_ref))
    assert pv.max() <= 1e-3
    s.close()


@pytest.mark.parametrize("name,steps", [("box32", 10), ("jet70x33x24", 10), ("jet70x33x24", 50)])
def test_fp32_state_after_steps(name, steps):
    announce("fp32-rk5", name, steps)
    pb = problems.box_problem(32) if name == "box32" else problems.jet_problem(70, 33, 24)
    geo, inflow = _oracle(pb)
    Q_ref, dts = les.run(pb["Q"].numpy(), geo, pb["params"], inflow, steps=steps)
    s = make_solver(pb, precision="fp32")
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    dt = to_np(s.rk5_step(Qn, steps))
    Q = to_np(s.interior(Qn))
    vn = vector_err(Q, Q_ref)
    err = float(vn.max())
    report(f"{name} FP32-form state after {steps} steps", per_variable=per_variable_err(Q, Q_ref),
           vector=vn)
    print(f"dt rel {np.abs(dt / dts - 1).max():.2e}")
    assert np.abs(dt / np.asarray(dts) - 1).max() <= 1e-5
    assert err <= 1e-5
    s.close()


def test_fp32_free_stream():
    announce("fp32-free-stream", "jet96x64x32")
    prim = (1.0, 0.6, 0.3, -0.2, 1.0 / 1.4)
    pb = problems.jet_problem(96, 64, 32, noise=0.0)
    pb["params"] = dict(pb["params"], ref_prim=prim, p_exit=prim[4])
    pb["inflow"] = torch.tensor(prim, dtype=torch.float64).view(5, 1, 1).expand(5, 32, 64).contiguous()
    Q = flow.uniform_state((32, 64, 96), prim)
    s = make_solver(pb, precision="fp32", keep_metrics=True)
    R = s.interior(s.residual(s.pad(Q.cuda().float()))).double()
    V = s.interior(s.metrics64[9:10])
    VR = float((R * V).abs().max())
    fscale = float(s.interior(s.metrics64[:9]).abs().max()) * (0.6 ** 2 + prim[4])
    print(f"FP32 free stream: {VR / fscale:.3e}")
    assert VR <= 1e-5 * fscale
    s.close()
