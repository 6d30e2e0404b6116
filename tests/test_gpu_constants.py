"""GPU parity with every physical and numerical constant moved off its
default: gamma, Pr, Pr_sgs, the Sutherland constant, Cs, k2, k4, the
viscous coefficient, the CFL number and the five RK coefficients, on a jet
(every boundary kind) and a periodic box.  A constant written into a kernel
instead of taken from the parameters shows up here.  Bars as in the other
parity tests: residual 1e-12 (FP64) and 1e-3 (FP32 storage), state after
3 steps 1e-11, time steps 1e-12, directional VJP 1e-11."""
import numpy as np
import pytest
import torch

from _helpers import announce, grouped_rel_err, make_solver, to_np
from cases import flow, problems
from oracle import les

pytestmark = pytest.mark.gpu

H_CS = 1e-30
OVER = dict(gamma=1.3, Pr=0.7, Pr_sgs=0.85, suth_S=0.5, Cs=0.16, k2=0.3, k4=0.02,
            cfl=0.4, rk_alpha=(0.2, 0.25, 0.4, 0.55, 1.0))


def _case(name):
    if name.startswith("jet"):
        pb = problems.jet_problem(37, 22, 20, seed=9, thermo_noise=1e-2)
        over = dict(OVER, visc_coef=2e-3, ref_prim=(1.0, flow.JET_UCO, 0.0, 0.0, 1.0 / 1.3),
                    p_exit=1.0 / 1.3)
    else:
        pb = problems.box_problem(24, seed=4, noise=1e-3)
        over = dict(OVER, visc_coef=1e-3)
    if name.endswith("vreman"):
        over["sgs_model"] = 2
    pb["params"] = dict(pb["params"], **over)
    return pb


CASES = ["jet37x22x20", "jet37x22x20_vreman", "box24"]


def _oracle(pb):
    geo = les.geometry(pb["xyz"].numpy(), pb["params"])
    inflow = pb["inflow"].numpy() if pb.get("inflow") is not None else None
    return geo, inflow


@pytest.mark.parametrize("name", CASES)
def test_residual_and_steps(name):
    announce("constants", name)
    pb = _case(name)
    geo, inflow = _oracle(pb)
    R_ref = les.evaluate(pb["Q"].numpy(), geo, pb["params"], inflow)
    Q_ref, dts = les.run(pb["Q"].numpy(), geo, pb["params"], inflow, steps=3)
    s = make_solver(pb)
    R = to_np(s.interior(s.residual(s.pad(pb["Q"].cuda()))))
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    dt = to_np(s.rk5_step(Qn, 3))
    er, eq = grouped_rel_err(R, R_ref), grouped_rel_err(to_np(s.interior(Qn)), Q_ref)
    print(f"{name}: residual {er:.3e}, state after 3 steps {eq:.3e}")
    assert er <= 1e-12 and eq <= 1e-11
    assert np.allclose(dt, dts, rtol=1e-12, atol=0)
    s.close()
    s = make_solver(pb, precision="fp32")
    R32 = to_np(s.interior(s.residual(s.pad(pb["Q"].cuda().float())))).astype(np.float64)
    e32 = grouped_rel_err(R32, R_ref)
    print(f"{name}: FP32 residual {e32:.3e}")
    assert e32 <= 1e-3
    s.close()


@pytest.mark.parametrize("name", ["jet37x22x20", "jet37x22x20_vreman"])
def test_vjp_directional(name):
    announce("constants-vjp", name)
    pb = _case(name)
    geo, inflow = _oracle(pb)
    Q = pb["Q"].numpy()
    Rbar = problems.seeded_field(Q.shape, 3, flow.FIELD_COTANGENT).numpy()
    v = problems.seeded_field(Q.shape, 11, flow.FIELD_DIRECTION).numpy()
    Qc = Q.astype(np.complex128) + 1j * H_CS * v
    jv = np.imag(les.evaluate(Qc, geo, pb["params"], inflow.astype(np.complex128))) / H_CS
    s = make_solver(pb)
    Qb = to_np(s.interior(s.residual_vjp(s.pad(pb["Q"].cuda()),
                                         s.pad(torch.from_numpy(Rbar).cuda(), fill=0.0))))
    lhs, rhs = float(np.sum(Rbar * jv)), float(np.sum(Qb * v))
    rel = abs(rhs - lhs) / abs(lhs)
    print(f"{name}: <Rbar, J v> {lhs:.12e} <Qbar, v> {rhs:.12e} rel {rel:.2e}")
    assert rel <= 1e-11
    s.close()
