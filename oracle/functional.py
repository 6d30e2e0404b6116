"""Oracle of the far-field pressure functional and its rollout (plain NumPy).

TEST INFRASTRUCTURE ONLY: used by the test suite to check the GPU gradient;
never imported by the GPU library, with which it shares no code.

The functional measures acoustic energy through a cylindrical surface r = r_s
around the jet over a rollout of N RK5 steps with a frozen dt:

  J = sum_{n=1}^{N} dt  sum_{i,k} w_i r_s dtheta (p^n_{i, j_s, k} - p_inf)^2

with j_s the radial index whose radius is closest to r_s, w_i the
trapezoid weights of the axial coordinates (so sum_i w_i f_i integrates f
along x exactly for linear f), dtheta = 2 pi / n_theta (the azimuth has
n_theta distinct points) and p = (gamma - 1)(E - rho |u|^2 / 2).  The
pressure of the state is the one of section "Governing Equations" (System I
energy closure).  Complex-safe: complex inputs give complex-step derivatives.
"""
import numpy as np

from . import les


def trapezoid_weights(x):
    """Weights w with sum_i w_i f(x_i) = the trapezoid rule on the nodes x."""
    x = np.asarray(x, dtype=np.float64)
    w = np.zeros_like(x)
    dx = np.diff(x)
    w[:-1] += 0.5 * dx
    w[1:] += 0.5 * dx
    return w


def surface(X, R, nth, r_target):
    """(j_s, w, r_s, dtheta) of the surface closest to radius r_target on a
    cylindrical product mesh with 1-D maps X (axial) and R (radial)."""
    R = np.asarray(R, dtype=np.float64)
    js = int(np.argmin(np.abs(R - r_target)))
    return js, trapezoid_weights(X), float(R[js]), 2.0 * np.pi / nth


def surface_term(Q, surf, p_inf, gamma):
    """sum_{i,k} w_i r_s dtheta (p_{i,j_s,k} - p_inf)^2 of the interior state
    Q (5, nth, nr, nx)."""
    js, w, rs, dth = surf
    rho, u, v, wv, p = les.primitives(Q[:, :, js, :], gamma)
    d = p - p_inf
    return np.sum(w[None, :] * d * d) * rs * dth


def rollout(Q0, geo, prm, inflow, dt, nsteps, surf, p_inf):
    """J of an N-step rollout from Q0 with the frozen step dt; returns
    (J, Q^N)."""
    Q = np.asarray(Q0)
    J = 0.0
    for _ in range(nsteps):
        Q, _ = les.rk5_step(Q, geo, prm, inflow, dt=dt)
        J = J + dt * surface_term(Q, surf, p_inf, prm["gamma"])
    return J, Q
