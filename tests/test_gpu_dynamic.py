"""GPU parity of the dynamic Smagorinsky model (LES_SGS_DYNAMIC) against the
oracle: the global coefficients C_I, C_ds, Pr_sgs, the residual (fused and
two-pass kernels), RK5 steps under both update schedules, and the FP32
storage form under both schedules.

Cases: multi-mode periodic boxes on which the averaged C_I and C_ds are
positive (the eddy viscosity and the isotropic stress both act), one where
C_ds is clipped to zero, and a jet where both are (clipping path; Pr_sgs
undefined).  Bars: coefficients 1e-9 relative (ratios of sums with
cancellation), residual 1e-12, state after the steps 1e-11; FP32 form 1e-3
and 1e-5."""
import math

import numpy as np
import pytest
import torch

from _helpers import announce, grouped_rel_err, make_solver, to_np
from cases import problems
from oracle import les

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "modes24_s2":
        return problems.modes_box_problem(24, seed=2)
    if name == "modes33_s3":
        return problems.modes_box_problem(33, seed=3)
    if name == "modes16_s1":
        return problems.modes_box_problem(16, seed=1)
    pb = problems.jet_problem(37, 22, 20, seed=3, thermo_noise=1e-2)
    pb["params"] = dict(pb["params"], visc_coef=1e-3, sgs_model=3)
    return pb


CASES = ["modes24_s2", "modes33_s3", "modes16_s1", "jet37x22x20"]


def _oracle(pb):
    geo = les.geometry(pb["xyz"].numpy(), pb["params"])
    inflow = pb["inflow"].numpy() if pb.get("inflow") is not None else None
    return geo, inflow


def _oracle_coefs(pb):
    geo, inflow = _oracle(pb)
    Qp = les.pad_state(pb["Q"].numpy())
    les.fill_ghosts(Qp, geo, pb["params"], inflow)
    with np.errstate(all="ignore"):
        return les.dynamic_coefficients(Qp, geo, pb["params"])


@pytest.mark.parametrize("name", CASES)
def test_coefficients_match_oracle(name):
    announce("dynamic-coefficients", name)
    pb = _case(name)
    d = _oracle_coefs(pb)
    s = make_solver(pb)
    c = s.dynamic_coefficients(s.pad(pb["Q"].cuda()))
    print(f"{name}: GPU {c} oracle {(d['C_I'], d['C_ds'], d['Pr_sgs'])}")
    for got, ref in ((c[0], d["C_I"]), (c[1], d["C_ds"])):
        assert abs(got - ref) <= 1e-9 * abs(ref) + 1e-15
    if math.isfinite(d["Pr_sgs"]) and d["C_ds_eff"] > 0.0:
        assert abs(c[2] - d["Pr_sgs"]) <= 1e-9 * abs(d["Pr_sgs"])
    assert c[3] == max(c[0], 0.0) or abs(c[3] - max(c[0], 0.0)) <= 1e-15 * abs(c[0])
    assert abs(c[4] - d["C_ds_eff"]) <= 1e-9 * abs(d["C_ds_eff"]) + 1e-15
    assert abs(c[5] - d["Pr_eff"]) <= 1e-9 * d["Pr_eff"]
    s.close()


def test_cases_cover_both_signs():
    """The case list exercises a positive C_ds and a clipped one."""
    signs = {_oracle_coefs(_case(n))["C_ds"] > 0.0 for n in ("modes24_s2", "modes16_s1")}
    assert signs == {True, False}


@pytest.mark.parametrize("name", CASES)
def test_residual_matches_oracle(name):
    announce("dynamic-residual", name)
    pb = _case(name)
    geo, inflow = _oracle(pb)
    with np.errstate(all="ignore"):
        R_ref = les.evaluate(pb["Q"].numpy(), geo, pb["params"], inflow)
    s = make_solver(pb)
    R = to_np(s.interior(s.residual(s.pad(pb["Q"].cuda()))))
    R2 = to_np(s.interior(s.residual_reference(s.pad(pb["Q"].cuda()))))
    e1, e2 = grouped_rel_err(R, R_ref), grouped_rel_err(R2, R_ref)
    print(f"{name}: residual fused {e1:.3e}, two-pass {e2:.3e}")
    assert np.isfinite(R).all() and e1 <= 1e-12 and e2 <= 1e-12
    s.close()


def test_model_terms_are_visible():
    """On the multi-mode box the dynamic residual differs from the one
    without SGS model by far more than the parity bar."""
    pb = _case("modes24_s2")
    geo, inflow = _oracle(pb)
    R3 = les.evaluate(pb["Q"].numpy(), geo, pb["params"], inflow)
    R0 = les.evaluate(pb["Q"].numpy(), geo, dict(pb["params"], sgs_model=0), inflow)
    assert grouped_rel_err(R3, R0) > 1e-6


@pytest.mark.parametrize("name,schedule", [("modes24_s2", "stage"), ("modes24_s2", "step"),
                                           ("jet37x22x20", "stage")])
def test_rk5_steps_match_oracle(name, schedule):
    announce("dynamic-rk5", name, schedule)
    pb = _case(name)
    pb["params"] = dict(pb["params"], schedule=schedule)
    geo, inflow = _oracle(pb)
    with np.errstate(all="ignore"):
        Q_ref, dts = les.run(pb["Q"].numpy(), geo, pb["params"], inflow, steps=3)
    s = make_solver(pb)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    dt = to_np(s.rk5_step(Qn, 3))
    err = grouped_rel_err(to_np(s.interior(Qn)), Q_ref)
    print(f"{name} {schedule}: state after 3 steps rel err {err:.3e}")
    assert np.allclose(dt, dts, rtol=1e-12, atol=0)
    assert err <= 1e-11
    s.close()


@pytest.mark.parametrize("schedule", ["stage", "step"])
def test_fp32_storage(schedule):
    announce("dynamic-fp32", "modes24_s2", schedule)
    pb = _case("modes24_s2")
    pb["params"] = dict(pb["params"], schedule=schedule)
    geo, inflow = _oracle(pb)
    R_ref = les.evaluate(pb["Q"].numpy(), geo, pb["params"], inflow)
    Q_ref, _ = les.run(pb["Q"].numpy(), geo, pb["params"], inflow, steps=3)
    s = make_solver(pb, precision="fp32")
    R = to_np(s.interior(s.residual(s.pad(pb["Q"].cuda().float())))).astype(np.float64)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    s.rk5_step(Qn, 3)
    er, eq = grouped_rel_err(R, R_ref), grouped_rel_err(to_np(s.interior(Qn)), Q_ref)
    print(f"FP32 dynamic ({schedule}): residual {er:.3e}, state after 3 steps {eq:.3e}")
    assert er <= 1e-3 and eq <= 1e-5
    s.close()


def test_adjoint_and_other_models_refused():
    from paper_2301_00817_amd import binding as B
    announce("dynamic-refusals")
    pb = _case("modes16_s1")
    s = make_solver(pb)
    Qp = s.pad(pb["Q"].cuda())
    with pytest.raises(B.LesError) as e:
        s.residual_vjp(Qp, torch.zeros_like(Qp))
    assert e.value.code == B.LES_EUNSUPPORTED
    s.close()
    pb2 = problems.box_problem(16)
    s = make_solver(pb2)
    with pytest.raises(B.LesError) as e:
        s.dynamic_coefficients(s.pad(pb2["Q"].cuda()))
    assert e.value.code == B.LES_EINVAL
    s.close()
