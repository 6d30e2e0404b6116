"""Edge cases of the GPU path against the oracle: the smallest meshes the
library accepts (5 points per direction; even azimuthal counts where the
centerline needs them), meshes thinner than one tile in a direction, and a
call with no steps.  Bars as for the other parity tests."""
import numpy as np
import pytest
import torch

from _helpers import announce, grouped_rel_err, make_solver, to_np
from cases import problems
from oracle import les

pytestmark = pytest.mark.gpu


def _perturbed(pb, seed=4, amp=0.02):
    Q = pb["Q"].clone()
    g = torch.Generator().manual_seed(seed)
    Q[1:4] += amp * torch.randn(Q[1:4].shape, generator=g, dtype=torch.float64)
    pb["Q"] = Q
    return pb


CASES = {
    "box5": lambda: problems.box_problem(5),
    "jet5x5x6": lambda: _perturbed(problems.jet_problem(5, 5, 6, seed=3, thermo_noise=1e-2)),
    "axis5x5x6": lambda: _perturbed(problems.jet_problem(5, 5, 6, seed=3, thermo_noise=1e-2,
                                                          axis_node=True)),
    "jet300x5x6": lambda: _perturbed(problems.jet_problem(300, 5, 6, seed=5, thermo_noise=1e-2)),
    "jet5x40x6": lambda: _perturbed(problems.jet_problem(5, 40, 6, seed=6, thermo_noise=1e-2)),
}


def _oracle(pb):
    geo = les.geometry(pb["xyz"].numpy(), pb["params"])
    inflow = pb["inflow"].numpy() if pb.get("inflow") is not None else None
    return geo, inflow


def _rows(Q, pb):
    return Q[:, :, 1:, :] if pb["params"]["bc"][2] == "axis_node" else Q


@pytest.mark.parametrize("name", list(CASES))
def test_residual_and_steps(name):
    announce("edges", name)
    pb = CASES[name]()
    geo, inflow = _oracle(pb)
    R_ref = les.evaluate(pb["Q"].numpy(), geo, pb["params"], inflow)
    Q_ref, dts = les.run(pb["Q"].numpy(), geo, pb["params"], inflow, steps=2)
    s = make_solver(pb)
    R = to_np(s.interior(s.residual(s.pad(pb["Q"].cuda()))))
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    dt = to_np(s.rk5_step(Qn, 2))
    Q = to_np(s.interior(Qn))
    er = grouped_rel_err(R, R_ref)
    eq = grouped_rel_err(_rows(Q, pb), _rows(Q_ref, pb))
    print(f"{name}: residual {er:.3e}, state after 2 steps {eq:.3e}")
    assert er <= 1e-12 and eq <= 1e-11
    assert np.allclose(dt, dts, rtol=1e-12, atol=0)
    s.close()
    s = make_solver(pb, precision="fp32")
    R32 = to_np(s.interior(s.residual(s.pad(pb["Q"].cuda().float())))).astype(np.float64)
    assert grouped_rel_err(R32, R_ref) <= 1e-3
    s.close()


def test_zero_steps_leave_the_state_untouched():
    announce("edges", "zero steps")
    pb = CASES["jet5x5x6"]()
    s = make_solver(pb)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64, fill=0.0)
    before = Qn.clone()
    s.rk5_step(Qn, 0)
    torch.cuda.synchronize()
    assert torch.equal(Qn, before)
    s.close()
