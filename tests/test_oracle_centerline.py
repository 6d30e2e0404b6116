"""Pins of the oracle's centerline treatment on meshes with nodes on the
axis (subsection "Centerline Boundary Condition"; readings C1-C6 in the
oracle's header)."""
import numpy as np

from cases import flow, problems
from oracle import brute, les


def _pb(nx=8, nr=6, nth=8, seed=5, perturb=0.05):
    pb = problems.jet_problem(nx, nr, nth, seed=seed, axis_node=True, thermo_noise=1e-2)
    Q = pb["Q"].numpy().copy()
    rng = np.random.default_rng(seed)
    Q[1:4] += perturb * rng.standard_normal(Q[1:4].shape)
    pb["Q"] = Q
    return pb


def test_mesh_has_its_first_row_on_the_axis_and_zero_volume_there():
    pb = _pb()
    xyz = pb["xyz"].numpy()
    assert np.all(xyz[1:, :, 0, :] == 0.0)
    geo = les.geometry(xyz, pb["params"])
    V = les.interior(geo["V"])
    assert np.all(V[:, 0, :] == 0.0) and np.all(V[:, 1:, :] > 0.0)


def test_fill_sets_the_axis_row_to_the_azimuthal_mean_of_row_one():
    pb = _pb()
    geo = les.geometry(pb["xyz"].numpy(), pb["params"])
    Qp = les.pad_state(pb["Q"])
    les.fill_ghosts(Qp, geo, pb["params"], pb["inflow"].numpy())
    Q = les.interior(Qp)
    mean = pb["Q"][:, :, 1, :].mean(axis=1)
    for k in range(Q.shape[1]):
        assert np.abs(Q[:, k, 0, :] - mean).max() <= 1e-15 * np.abs(mean).max()
    # mirror ghosts across the axis node
    g = les.NG
    nth = Q.shape[1]
    for m in (1, 2):
        for k in range(nth):
            assert np.array_equal(Qp[:, g + k, g - m, g:-g], Qp[:, g + (k + nth // 2) % nth, g + m, g:-g])


def test_free_stream_is_preserved():
    """A uniform state equal to the entrance target and the far field: R = 0
    on every advanced point (the cross-product metrics satisfy the discrete
    metric identities at j = 1 with S^eta = 0 on the axis)."""
    pb = problems.jet_problem(10, 8, 8, axis_node=True)
    prm = pb["params"]
    ref = prm["ref_prim"]
    Q = flow.uniform_state((8, 8, 10), ref).numpy()
    inflow = np.broadcast_to(np.asarray(ref).reshape(5, 1, 1), (5, 8, 8)).copy()
    geo = les.geometry(pb["xyz"].numpy(), prm)
    R = les.evaluate(Q, geo, prm, inflow)
    flux_scale = abs(ref[4]) * np.abs(les.interior(geo["S"])).max() / np.abs(les.interior(geo["V"])[:, 1:, :]).min()
    assert np.abs(R).max() <= 1e-12 * flux_scale
    assert np.all(R[:, :, 0, :] == 0.0)


def test_axis_face_uses_the_three_point_fourth_difference():
    """The modified fourth difference at the axis face does not reach the
    ghost row j = -1: with k2 = 0 (the sensor then plays no part) and no
    viscous terms, changing that row leaves R unchanged on every advanced
    point (the standard five-point stencil would reach it through the axis
    face).  The brute-force oracle, written separately, checks the values."""
    pb = problems.jet_problem(8, 6, 8, axis_node=True)
    prm = dict(pb["params"], k2=0.0, visc_coef=0.0, sgs_model=0)
    geo = les.geometry(pb["xyz"].numpy(), prm)
    Qp = les.pad_state(pb["Q"].numpy())
    les.fill_ghosts(Qp, geo, prm, pb["inflow"].numpy())
    R1 = les.residual(Qp, geo, prm)
    Qp2 = Qp.copy()
    Qp2[0, :, les.NG - 1, :] *= 1.5                # density of the ghost row j = -1
    R2 = les.residual(Qp2, geo, prm)
    assert np.isfinite(R1).all()
    assert np.array_equal(R1, R2)


def test_brute_force_axis_node():
    pb = _pb()
    xyz, Q = pb["xyz"].numpy(), pb["Q"]
    geo = les.geometry(xyz, pb["params"])
    R = les.evaluate(Q, geo, pb["params"], pb["inflow"].numpy())
    Rb, _ = brute.Brute(xyz, pb["params"], pb["inflow"].numpy()).residual(Q)
    out = np.zeros(R.shape)
    for (i, j, k), r in Rb.items():
        out[:, k, j, i] = r
    assert np.isfinite(R).all()
    assert np.abs(R - out).max() / np.abs(R).max() <= 1e-13


def test_steps_stay_finite_and_the_time_step_skips_the_axis():
    pb = _pb(12, 8, 8, perturb=0.01)
    prm = pb["params"]
    geo = les.geometry(pb["xyz"].numpy(), prm)
    dt = les.time_step(pb["Q"], geo, prm)
    assert np.isfinite(dt) and dt > 0.0
    Q, dts = les.run(pb["Q"], geo, prm, pb["inflow"].numpy(), steps=3)
    assert np.isfinite(Q).all()
