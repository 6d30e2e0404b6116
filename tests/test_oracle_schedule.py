"""Pins of the oracle's per-step update schedule (schedule "step": viscosity,
SGS viscosity, physical-face ghosts and the centerline row evaluated from
Q^n once per step and held through the five stages; readings L1, L2 in the
oracle's header; the iteration loop of section "The JAZzY code").

  * the scalar brute-force oracle, written separately, gives the same step;
  * special cases where holding changes nothing: a single stage (the only
    evaluation is at Q^n), and an inviscid fully periodic box (nothing is
    held);
  * the two schedules differ by O(dt^2) over one step (the held values are
    O(dt) away from the stage values and enter multiplied by alpha dt): the
    difference shrinks fourfold when dt halves;
  * the ghosts of a stage state: held values on the physical faces, the
    standard copies on the periodic and cross-axis faces.
"""
import numpy as np
import pytest

from _helpers import grouped_rel_err
from cases import problems
from oracle import brute, les


def _jet(nx=8, nr=6, nth=8, axis_node=False, sgs_model=1, visc=1e-2, seed=3):
    pb = problems.jet_problem(nx, nr, nth, seed=seed, thermo_noise=1e-2, axis_node=axis_node)
    Q = pb["Q"].numpy().copy()
    rng = np.random.default_rng(seed)
    Q[1:4] += 0.05 * rng.standard_normal(Q[1:4].shape)
    pb["Q"] = Q
    pb["params"] = dict(pb["params"], visc_coef=visc, sgs_model=sgs_model)
    return pb


def _dt(pb):
    """The CFL time step of the state."""
    geo = les.geometry(pb["xyz"].numpy(), pb["params"])
    return les.time_step(np.asarray(pb["Q"]), geo, pb["params"])


def _step(pb, schedule, dt, alpha=None):
    prm = dict(pb["params"], schedule=schedule)
    if alpha is not None:
        prm["rk_alpha"] = alpha
    geo = les.geometry(pb["xyz"].numpy(), prm)
    inflow = pb["inflow"].numpy() if pb["inflow"] is not None else None
    Qn, _ = les.rk5_step(np.asarray(pb["Q"]), geo, prm, inflow, dt)
    return Qn


def _brute_step(pb, schedule, dt):
    prm = dict(pb["params"], schedule=schedule)
    inflow = pb["inflow"].numpy() if pb["inflow"] is not None else None
    B = brute.Brute(pb["xyz"].numpy(), prm, inflow)
    D = B.step(np.asarray(pb["Q"]), dt, schedule)
    out = np.zeros(np.asarray(pb["Q"]).shape)
    for (i, j, k), v in D.items():
        out[:, k, j, i] = v
    return out


@pytest.mark.parametrize("case", ["jet_smagorinsky", "jet_axis_node_vreman", "box_viscous"])
def test_brute_force_step_schedule(case):
    if case == "jet_smagorinsky":
        pb = _jet()
    elif case == "jet_axis_node_vreman":
        pb = _jet(axis_node=True, sgs_model=2)
    else:
        pb = problems.box_problem(5)
        pb["params"] = dict(pb["params"], visc_coef=1e-2)
        pb["Q"] = pb["Q"].numpy()
    dt = _dt(pb)
    Qv = _step(pb, "step", dt)
    Qb = _brute_step(pb, "step", dt)
    assert grouped_rel_err(Qv, Qb) <= 1e-13
    # and the schedule matters for these cases (the check above is not
    # vacuous): the per-stage schedule gives a different step
    Qs = _step(pb, "stage", dt)
    assert grouped_rel_err(Qv, Qs) > 1e-12


def test_single_stage_is_schedule_independent():
    pb = _jet()
    a = _step(pb, "step", _dt(pb), alpha=(1.0,))
    b = _step(pb, "stage", _dt(pb), alpha=(1.0,))
    assert np.array_equal(a, b)


def test_inviscid_periodic_box_is_schedule_independent():
    pb = problems.box_problem(8)
    pb["params"] = dict(pb["params"], visc_coef=0.0, sgs_model=0)
    pb["Q"] = pb["Q"].numpy()
    dt = _dt(pb)
    assert np.array_equal(_step(pb, "step", dt), _step(pb, "stage", dt))


@pytest.mark.parametrize("case", ["box_viscous", "jet"])
def test_schedule_difference_is_second_order_in_dt(case):
    """Box: only the held viscosities differ (asymptotic already at the CFL
    step); jet: mainly the held boundary values, asymptotic once dt lambda
    is small (steps of 1/16 .. 1/64 of the CFL step)."""
    if case == "box_viscous":
        pb = problems.box_problem(8)
        pb["params"] = dict(pb["params"], visc_coef=1e-2)
        pb["Q"] = pb["Q"].numpy()
        scales = [1.0, 0.5, 0.25]
    else:
        pb = _jet(12, 8, 8, visc=1e-4)
        scales = [1.0 / 16, 1.0 / 32, 1.0 / 64]
    diffs = []
    for dt in _dt(pb) * np.array(scales):
        d = _step(pb, "step", dt) - _step(pb, "stage", dt)
        diffs.append(np.abs(d).max())
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, diffs


@pytest.mark.parametrize("axis_node", [False, True])
def test_stage_ghosts_hold_physical_faces_and_copy_the_rest(axis_node):
    pb = _jet(axis_node=axis_node)
    prm = pb["params"]
    geo = les.geometry(pb["xyz"].numpy(), prm)
    inflow = pb["inflow"].numpy()
    Hp = les.pad_state(pb["Q"])
    les.fill_ghosts(Hp, geo, prm, inflow)
    rng = np.random.default_rng(9)
    q = pb["Q"] * (1.0 + 1e-2 * rng.standard_normal(pb["Q"].shape))
    Sp = les.pad_state(q)
    les.fill_ghosts(Sp, geo, prm, inflow, held=Hp)
    Fp = les.pad_state(q)
    les.fill_ghosts(Fp, geo, prm, inflow)
    g = les.NG
    nth, nr, nx = q.shape[1:]
    # physical faces (entrance i < 0, exit i >= nx, far field j >= nr): held
    assert np.array_equal(Sp[..., :g], Hp[..., :g])
    assert np.array_equal(Sp[..., g + nx:], Hp[..., g + nx:])
    assert np.array_equal(Sp[:, :, g + nr:, :], Hp[:, :, g + nr:, :])
    # away from those, ghosts are copies of the stage state (a full fill)
    inner = (slice(None), slice(None), slice(0, g + nr), slice(g, g + nx))
    if axis_node:    # the centerline row is held too
        assert np.array_equal(Sp[:, g:g + nth, g, g:g + nx], Hp[:, g:g + nth, g, g:g + nx])
        # mirror ghosts copy the stage rows j = 1, 2 (k + nth/2)
        for m in (1, 2):
            for k in range(nth):
                assert np.array_equal(Sp[:, g + k, g - m, g:g + nx],
                                      Sp[:, g + (k + nth // 2) % nth, g + m, g:g + nx])
    else:
        assert np.array_equal(Sp[inner], Fp[inner])
