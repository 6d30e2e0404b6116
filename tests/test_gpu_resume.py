"""Checkpoint and resume.  Q^n in FP64 is the whole state carried from one
RK5 step to the next (stage states, held viscosities, boundary values and
the CFL time step are formed again from it, in both precision forms and both
update schedules), so 5 steps, Q^n written to a .npz file, a fresh context
loading it and 5 more steps give bitwise the state and time steps of 10
uninterrupted steps.  The first step of a call takes its time step from
the separate maximum reduction over the state; the uninterrupted run from
the one in the last stage of the previous step: the two must agree
bitwise too."""
import numpy as np
import pytest
import torch

from _helpers import announce, make_solver
from cases import problems

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,schedule", [("fp64", "stage"), ("fp32", "stage"),
                                                ("fp64", "step")])
def test_resume_from_checkpoint_is_bitwise(precision, schedule, tmp_path):
    announce("resume", precision, schedule)
    pb = problems.jet_problem(48, 32, 24)
    prm = dict(pb["params"], schedule=schedule)

    s = make_solver(pb, precision=precision, params=prm)
    Q = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    dt_a = s.rk5_step(Q, 10).cpu().numpy()
    q_a = s.interior(Q).cpu().numpy().copy()
    s.close()
    del Q

    s = make_solver(pb, precision=precision, params=prm)
    Q = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    dt_1 = s.rk5_step(Q, 5).cpu().numpy()
    path = tmp_path / "checkpoint.npz"
    np.savez(path, Q=s.interior(Q).cpu().numpy(), step=5, t=float(dt_1.sum()))
    s.close()
    del Q

    ck = np.load(path)
    assert int(ck["step"]) == 5
    s = make_solver(pb, precision=precision, params=prm)
    Q = s.pad(torch.from_numpy(ck["Q"]).cuda(), dtype=torch.float64)
    dt_2 = s.rk5_step(Q, 5).cpu().numpy()
    q_b = s.interior(Q).cpu().numpy()
    s.close()

    assert np.isfinite(q_b).all()
    assert np.array_equal(dt_a, np.concatenate([dt_1, dt_2])), (dt_a, dt_1, dt_2)
    assert np.array_equal(q_a, q_b)
    assert float(ck["t"]) + float(dt_2.sum()) == pytest.approx(float(dt_a.sum()), rel=1e-15)
