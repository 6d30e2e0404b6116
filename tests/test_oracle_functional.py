"""Pins of the oracle's pressure functional (closed forms and invariants)."""
import math

import numpy as np

from cases import flow, problems
from oracle import functional as fun
from oracle import les


def test_trapezoid_weights_integrate_linear_functions_exactly():
    x = np.cumsum(np.linspace(0.1, 0.9, 17))          # nonuniform nodes
    w = fun.trapezoid_weights(x)
    assert abs(w.sum() - (x[-1] - x[0])) < 1e-14
    a, b = 0.7, -1.3
    exact = a * (x[-1] - x[0]) + 0.5 * b * (x[-1] ** 2 - x[0] ** 2)
    assert abs(np.sum(w * (a + b * x)) - exact) < 1e-12


def test_surface_term_of_a_uniform_pressure_offset_is_the_cylinder_area():
    """(p - p_inf) = delta everywhere: S = delta^2 * length * 2 pi r_s."""
    nx, nr, nth = 20, 16, 12
    X, R, TH = problems.jet_grid(nx, nr, nth)
    gamma = flow.GAMMA
    p_inf, delta = 1.0 / gamma, 3e-3
    Q = flow.uniform_state((nth, nr, nx), (1.0, 0.3, 0.1, -0.2, p_inf + delta)).numpy()
    surf = fun.surface(X.numpy(), R.numpy(), nth, 6.0)
    js, w, rs, dth = surf
    assert js == int(np.argmin(np.abs(R.numpy() - 6.0)))
    S = fun.surface_term(Q, surf, p_inf, gamma)
    area = (X[-1] - X[0]).item() * 2.0 * math.pi * rs
    assert abs(S - delta * delta * area) < 1e-12 * delta * delta * area


def test_rollout_functional_vanishes_on_a_free_stream():
    """A uniform state that matches the entrance target and the far field is
    preserved by the scheme on the product mesh, so p stays p_inf."""
    nx, nr, nth = 10, 8, 8
    pb = problems.jet_problem(nx, nr, nth)
    prm = pb["params"]
    ref = prm["ref_prim"]
    Q = flow.uniform_state((nth, nr, nx), ref).numpy()
    inflow = np.broadcast_to(np.asarray(ref).reshape(5, 1, 1), (5, nth, nr)).copy()
    geo = les.geometry(pb["xyz"].numpy(), prm)
    X, R, TH = pb["grid"]
    surf = fun.surface(X.numpy(), R.numpy(), nth, 0.5)
    J, QN = fun.rollout(Q, geo, prm, inflow, 1e-3, 3, surf, ref[4])
    assert abs(J) < 1e-26
    assert np.abs(QN - Q).max() < 1e-13


def test_rollout_functional_is_positive_and_additive():
    """J of N steps = J of the first k steps + J of the remaining N - k steps
    started from Q^k (the sum over steps); J > 0 for a disturbed jet."""
    pb = problems.jet_problem(12, 8, 8, seed=3)
    prm = pb["params"]
    geo = les.geometry(pb["xyz"].numpy(), prm)
    X, R, TH = pb["grid"]
    surf = fun.surface(X.numpy(), R.numpy(), 8, 0.5)
    Q0, inflow = pb["Q"].numpy(), pb["inflow"].numpy()
    dt = 5e-4
    J4, Q4 = fun.rollout(Q0, geo, prm, inflow, dt, 4, surf, prm["p_exit"])
    J1, Q1 = fun.rollout(Q0, geo, prm, inflow, dt, 1, surf, prm["p_exit"])
    J3, Q4b = fun.rollout(Q1, geo, prm, inflow, dt, 3, surf, prm["p_exit"])
    assert J4 > 0.0
    assert abs(J4 - (J1 + J3)) <= 1e-14 * J4
    assert np.array_equal(Q4, Q4b)
