"""GPU parity of the per-step update schedule (LES_SCHEDULE_STEP: viscosities,
physical-face ghosts and the centerline row held from Q^n through the five
stages) against the oracle, FP64 and FP32-storage forms, on meshes spanning
several tiles with ragged tails, with k-chunks that make blocks share the
points whose viscosities they store.

Bars as for the per-stage schedule: state after the steps 1e-11 per group
(FP64), 1e-5 (FP32 form).  Each case also checks that the schedule changes
the result (the comparison is not with the per-stage step by accident)."""
import numpy as np
import pytest
import torch

from _helpers import announce, grouped_rel_err, make_solver, to_np
from cases import problems
from oracle import les

pytestmark = pytest.mark.gpu


def _perturbed(pb, seed, amp=0.02):
    Q = pb["Q"].clone()
    g = torch.Generator().manual_seed(seed)
    Q[1:4] += amp * torch.randn(Q[1:4].shape, generator=g, dtype=torch.float64)
    pb["Q"] = Q
    return pb


def _case(name):
    if name == "jet37x22x20_smagorinsky":
        pb = _perturbed(problems.jet_problem(37, 22, 20, seed=3, thermo_noise=1e-2), 3)
        pb["params"] = dict(pb["params"], visc_coef=1e-3, sgs_model=1)
    elif name == "jet37x22x20_inviscid":
        pb = _perturbed(problems.jet_problem(37, 22, 20, seed=4, thermo_noise=1e-2), 4)
        pb["params"] = dict(pb["params"], visc_coef=0.0, sgs_model=0)
    elif name == "axis20x9x16_vreman":
        pb = _perturbed(problems.jet_problem(20, 9, 16, seed=5, thermo_noise=1e-2,
                                             axis_node=True), 5)
        pb["params"] = dict(pb["params"], visc_coef=1e-3, sgs_model=2)
    else:   # box32_viscous
        pb = problems.box_problem(32)
        pb["params"] = dict(pb["params"], visc_coef=1e-2)
    pb["params"] = dict(pb["params"], schedule="step")
    return pb


CASES = ["jet37x22x20_smagorinsky", "jet37x22x20_inviscid", "axis20x9x16_vreman",
         "box32_viscous"]


def _oracle_steps(pb, steps, schedule="step"):
    prm = dict(pb["params"], schedule=schedule)
    geo = les.geometry(pb["xyz"].numpy(), prm)
    inflow = pb["inflow"].numpy() if pb.get("inflow") is not None else None
    return les.run(pb["Q"].numpy(), geo, prm, inflow, steps=steps)


def _rows(Q, pb):
    """Rows compared with the oracle (the axis row is derived data)."""
    return Q[:, :, 1:, :] if pb["params"]["bc"][2] == "axis_node" else Q


@pytest.mark.parametrize("name", CASES)
def test_steps_match_oracle(name):
    announce("schedule-step", name)
    pb = _case(name)
    steps = 3
    Q_ref, dts = _oracle_steps(pb, steps)
    Q_stage, _ = _oracle_steps(pb, steps, "stage")
    s = make_solver(pb)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    dt = to_np(s.rk5_step(Qn, steps))
    Q = to_np(s.interior(Qn))
    assert np.allclose(dt, dts, rtol=1e-12, atol=0)
    err = grouped_rel_err(_rows(Q, pb), _rows(Q_ref, pb))
    sep = grouped_rel_err(_rows(Q_stage, pb), _rows(Q_ref, pb))
    print(f"{name}: state after {steps} steps rel err {err:.3e} (schedules differ by {sep:.1e})")
    assert err <= 1e-11
    assert sep > 1e3 * max(err, 1e-16)
    s.close()


@pytest.mark.parametrize("kchunk", [1, 3])
def test_chunk_boundaries(kchunk, monkeypatch):
    announce("schedule-step-chunk", kchunk)
    monkeypatch.setenv("LESJET_KCHUNK", str(kchunk))
    pb = _case("jet37x22x20_smagorinsky")
    Q_ref, _ = _oracle_steps(pb, 2)
    s = make_solver(pb)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    s.rk5_step(Qn, 2)
    assert grouped_rel_err(to_np(s.interior(Qn)), Q_ref) <= 1e-11
    s.close()


@pytest.mark.parametrize("name", ["jet37x22x20_smagorinsky", "axis20x9x16_vreman"])
def test_fp32_storage_steps(name):
    announce("schedule-step-fp32", name)
    pb = _case(name)
    Q_ref, _ = _oracle_steps(pb, 3)
    s = make_solver(pb, precision="fp32")
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    s.rk5_step(Qn, 3)
    err = grouped_rel_err(_rows(to_np(s.interior(Qn)), pb), _rows(Q_ref, pb))
    print(f"{name}: FP32 state after 3 steps rel err {err:.3e}")
    assert err <= 1e-5
    s.close()


def test_step_adjoint_is_refused():
    from paper_2301_00817_amd import binding as B
    announce("schedule-step-adjoint-refused")
    pb = _case("jet37x22x20_smagorinsky")
    s = make_solver(pb)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    with pytest.raises(B.LesError) as e:
        s.rk5_step_vjp(Qn, 1e-4, torch.zeros_like(Qn))
    assert e.value.code == B.LES_EUNSUPPORTED
    s.close()
