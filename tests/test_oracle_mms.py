"""Method of manufactured solutions: the discrete residual R_h(Q(x)) must
converge at second order to the exact divergence of the continuous
Navier-Stokes fluxes, div F(Q(x)), derived symbolically here with sympy from
the governing equations (the paper's modified System I without SGS terms),
independent of the oracle's discretisation.  The heat flux is written
down-gradient, q = -(mu/Pr) grad T / (gamma - 1), and the viscous fluxes carry
the factor M/Re.  A wrong sign or a dropped term in any flux leaves an O(1)
error that does not converge."""
import math

import numpy as np
import pytest
import sympy as sp

from cases import mesh, problems
from oracle import les

G = 1.4
PR = 0.72
SUTH = 110.4 / 288.15
CV = 0.05


def _exact_fields():
    x, y, z = sp.symbols("x y z", real=True)
    X = (x, y, z)
    rho = 1 + sp.Rational(1, 10) * sp.sin(x) * sp.cos(y) + sp.Rational(1, 20) * sp.sin(z)
    u = [sp.Rational(2, 5) + sp.Rational(1, 10) * sp.cos(x) * sp.sin(z),
         -sp.Rational(3, 10) + sp.Rational(1, 10) * sp.sin(y) * sp.cos(x),
         sp.Rational(1, 5) + sp.Rational(1, 10) * sp.cos(y + z)]
    p = sp.Rational(4, 5) + sp.Rational(1, 20) * sp.sin(x) * sp.sin(y) * sp.cos(z)
    g = sp.Float(G)
    T = g * p / rho
    mu = T ** sp.Rational(3, 2) * (1 + SUTH) / (T + SUTH)
    E = p / (g - 1) + rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2) / 2
    gu = [[sp.diff(u[i], X[m]) for m in range(3)] for i in range(3)]
    div = gu[0][0] + gu[1][1] + gu[2][2]
    tau = [[mu * (gu[i][j] + gu[j][i] - (sp.Rational(2, 3) * div if i == j else 0))
            for j in range(3)] for i in range(3)]
    q = [-(mu / PR) / (g - 1) * sp.diff(T, X[j]) for j in range(3)]
    R = [0] * 5
    for j in range(3):
        F = [rho * u[j]]
        F += [rho * u[i] * u[j] + (p if i == j else 0) - CV * tau[i][j] for i in range(3)]
        F += [(E + p) * u[j] - CV * (sum(tau[i][j] * u[i] for i in range(3)) - q[j])]
        for c in range(5):
            R[c] = R[c] + sp.diff(F[c], X[j])
    state = [rho, rho * u[0], rho * u[1], rho * u[2], E]
    fQ = sp.lambdify(X, state, "numpy", cse=True)
    fR = sp.lambdify(X, R, "numpy", cse=True)
    return fQ, fR


@pytest.fixture(scope="module")
def exact():
    return _exact_fields()


def _error(exact, xyz, prm):
    fQ, fR = exact
    x, y, z = xyz
    Q = np.stack([np.broadcast_to(np.asarray(c, dtype=float), x.shape) for c in fQ(x, y, z)])
    Rex = np.stack([np.broadcast_to(np.asarray(c, dtype=float), x.shape) for c in fR(x, y, z)])
    geo = les.geometry(xyz, prm)
    R = les.evaluate(Q, geo, prm)
    return np.abs(R - Rex).max(axis=(1, 2, 3)) / np.abs(Rex).max()


def _orders(exact, make, prm, ns=(16, 32, 64)):
    errs = [_error(exact, make(n), prm) for n in ns]
    return errs, [np.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]


def test_mms_second_order_wavy_mesh_navier_stokes(exact):
    L = 2 * math.pi
    prm = problems.box_params(L, visc_coef=CV, k2=0.0, k4=0.0, Cs=0.0)
    errs, orders = _orders(exact, lambda n: mesh.wavy_coords(n, L, 0.1).numpy(), prm)
    for o in orders[-1]:
        assert 1.9 <= o <= 2.1, (errs, orders)


def test_mms_second_order_box_with_dissipation_and_sgs(exact):
    """Dissipation is O(h^3) for smooth fields and the SGS viscosity O(h^2),
    so the full scheme keeps second order."""
    L = 2 * math.pi
    prm = problems.box_params(L, visc_coef=CV)
    errs, orders = _orders(exact, lambda n: mesh.box_coords(n, L).numpy(), prm)
    for o in orders[-1]:
        assert 1.85 <= o <= 2.3, (errs, orders)
