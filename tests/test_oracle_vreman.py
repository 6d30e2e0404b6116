"""Pins of the oracle's Vreman subgrid model (subsection "Vreman Model").

For a linear velocity field the central differences are exact, so the eddy
viscosity the oracle computes at every point can be compared with values
derived by hand from the model's definition:
  * uniform flow (alpha = 0): the model is defined as zero;
  * pure shear u = (s y, 0, 0): one gradient component, B_beta = 0, zero;
  * u = (a y, b x, 0): alpha_21 = a, alpha_12 = b, beta = Delta^2 diag(a^2,
    b^2, 0), B_beta = Delta^4 a^2 b^2, alpha.alpha = a^2 + b^2, so
    mu_sgs = rho c Delta^2 |a b| / sqrt(a^2 + b^2), c = 2.5 Cs^2;
  * rotating the field (gradient R A R^T) leaves mu_sgs unchanged, the
    model's invariance for isotropic filter widths;
and the brute-force scalar oracle agrees with the vectorised one.
"""
import math

import numpy as np

from cases import flow, mesh, problems
from oracle import brute, les

N = 8
H = 2.0 * math.pi / N


def _linear_field_mu(A, rho=1.2, p=0.7, base=(0.3, -0.1, 0.2), Cs=0.148):
    """mu_t (region one) of the velocity u = base + A x on an N^3 uniform
    Cartesian mesh, state filled on the whole padded box."""
    prm = problems.box_params(Cs=Cs, sgs_model=2)
    xyz = mesh.box_coords(N).numpy()
    geo = les.geometry(xyz, prm)
    g = les.NG
    idx = (np.arange(-g, N + g) * H)
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")     # (k, j, i)
    X = np.stack([x, y, z])
    u = [base[c] + sum(A[c][m] * X[m] for m in range(3)) for c in range(3)]
    Qp = np.stack([np.full_like(x, rho), rho * u[0], rho * u[1], rho * u[2],
                   p / (prm["gamma"] - 1.0) + 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)])
    pt = les.point_terms(Qp, geo, prm)
    return pt["mu_t"], prm


def test_uniform_flow_and_pure_shear_give_zero():
    mu, _ = _linear_field_mu(np.zeros((3, 3)))
    assert np.all(mu == 0.0)
    A = np.zeros((3, 3))
    A[0][1] = 0.7                      # u = s y
    mu, _ = _linear_field_mu(A)
    assert np.abs(mu).max() == 0.0


def test_two_component_shear_closed_form():
    a, b, rho, Cs = 0.9, -0.4, 1.2, 0.148
    A = np.zeros((3, 3))
    A[0][1] = a                        # d u / d y
    A[1][0] = b                        # d v / d x
    mu, prm = _linear_field_mu(A, rho=rho, Cs=Cs)
    c = 2.5 * Cs * Cs
    expected = rho * c * H * H * abs(a * b) / math.sqrt(a * a + b * b) / prm["visc_coef"]
    assert np.abs(mu - expected).max() <= 1e-12 * expected


def test_rotation_invariance():
    rng = np.random.default_rng(3)
    A = rng.uniform(-1.0, 1.0, (3, 3))
    th = 0.61
    Rz = np.array([[math.cos(th), -math.sin(th), 0.0], [math.sin(th), math.cos(th), 0.0],
                   [0.0, 0.0, 1.0]])
    ph = -0.37
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, math.cos(ph), -math.sin(ph)],
                   [0.0, math.sin(ph), math.cos(ph)]])
    R = Rz @ Rx
    mu1, _ = _linear_field_mu(A)
    mu2, _ = _linear_field_mu(R @ A @ R.T)
    ref = np.abs(mu1).max()
    assert ref > 0.0
    assert np.abs(mu1 - mu2).max() <= 1e-12 * ref


def test_vreman_differs_from_smagorinsky():
    """The two models give different eddy viscosities for a generic gradient
    (guards against a branch that silently falls back)."""
    rng = np.random.default_rng(4)
    A = rng.uniform(-1.0, 1.0, (3, 3))
    mu_v, prm = _linear_field_mu(A)
    prm_s = dict(prm, sgs_model=1)
    xyz = mesh.box_coords(N).numpy()
    geo = les.geometry(xyz, prm_s)
    g = les.NG
    idx = (np.arange(-g, N + g) * H)
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    X = np.stack([x, y, z])
    u = [0.3 + sum(A[0][m] * X[m] for m in range(3)),
         -0.1 + sum(A[1][m] * X[m] for m in range(3)),
         0.2 + sum(A[2][m] * X[m] for m in range(3))]
    rho, p = 1.2, 0.7
    Qp = np.stack([np.full_like(x, rho), rho * u[0], rho * u[1], rho * u[2],
                   p / 0.4 + 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)])
    mu_s = les.point_terms(Qp, geo, prm_s)["mu_t"]
    assert np.abs(mu_v - mu_s).max() > 1e-3 * np.abs(mu_s).max()


def _brute_rel(pb):
    xyz, Q = pb["xyz"].numpy(), pb["Q"].numpy()
    inflow = pb["inflow"].numpy() if pb["inflow"] is not None else None
    geo = les.geometry(xyz, pb["params"])
    R = les.evaluate(Q, geo, pb["params"], inflow)
    Rb, _ = brute.Brute(xyz, pb["params"], inflow).residual(Q)
    out = np.zeros(R.shape)
    for (i, j, k), r in Rb.items():
        out[:, k, j, i] = r
    return np.abs(R - out).max() / np.abs(R).max()


def test_brute_force_vreman():
    pb = problems.box_problem(6)
    pb["params"] = dict(pb["params"], sgs_model=2)
    assert _brute_rel(pb) <= 1e-13
    pb = problems.jet_problem(8, 6, 8, thermo_noise=1e-2)
    pb["params"] = dict(pb["params"], sgs_model=2)
    assert _brute_rel(pb) <= 1e-13
