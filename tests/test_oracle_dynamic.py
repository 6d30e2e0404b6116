"""Pins of the oracle's dynamic Smagorinsky model (subsection "Dynamic
Smagorinsky Model"; readings D1-D8 in the oracle's header).

  * the test filter keeps constants and linear functions and adds the
    filter variance h^2/2 per direction to x^2 (its second moment);
  * on a uniform Cartesian mesh with a linear velocity u = A x + c, uniform
    density and a linear temperature T = b.x + T0, every filtered quantity
    has a closed form: hat(f g) = f g + (h^2/2) grad f . grad g for linear
    f, g; S_hat = S; so
        C_I  = sum A^2 / (12 |S|^2),
        C_ds = [L:S - tr S L_ll/3 + C_I+ tr S 2 h^2 rho |S|^2 / 3]
               / [-6 h^2 rho |S| (S:S - (tr S)^2/3)],
        Pr   = C_ds+ (-3 h^2 rho |S| |b|^2) / (rho h^2/2 b.A b),
    with L = rho (h^2/2) A A^T and C+ = max(C, 0);
  * with its coefficients fixed to C_ds = Cs^2, C_I = 0 and the static
    Pr_sgs the model is the Smagorinsky model;
  * the isotropic stress alone (C_I > 0, C_ds = 0) on the linear field adds
    nothing to the momentum residual and p_sgs tr A to the energy residual
    (p_sgs = (2/3) C_I rho h^2 |S|^2 uniform, divergence of p_sgs u);
  * the seven volume sums against the brute-force oracle's scalar loops
    (explicit 27-point filter) on a curvilinear jet and a multi-mode box.
"""
import math

import numpy as np
import pytest

from cases import mesh, problems
from oracle import les

N = 8
H = 2.0 * math.pi / N
RHO = 1.1
T0 = 0.9


def _linear_state(A, b, c=(0.3, -0.2, 0.1)):
    """Padded box state (all points, ghosts included) of u = A x + c,
    T = b.x + T0, rho uniform; and the box geometry."""
    prm = problems.box_params(sgs_model=3, visc_coef=1e-3)
    geo = les.geometry(mesh.box_coords(N).numpy(), prm)
    g = les.NG
    idx = np.arange(-g, N + g) * H
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    X = (x, y, z)
    u = [c[i] + sum(A[i][m] * X[m] for m in range(3)) for i in range(3)]
    T = T0 + sum(b[m] * X[m] for m in range(3))
    gamma = prm["gamma"]
    p = RHO * T / gamma
    Qp = np.stack([np.full_like(x, RHO), RHO * u[0], RHO * u[1], RHO * u[2],
                   p / (gamma - 1.0) + 0.5 * RHO * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)])
    return Qp, geo, prm


def _closed_forms(A, b):
    A = np.asarray(A, dtype=float)
    b = np.asarray(b, dtype=float)
    S = 0.5 * (A + A.T)
    SS = float(np.sum(S * S))
    Smag = math.sqrt(2.0 * SS)
    trS = float(np.trace(S))
    h2 = H * H
    L = RHO * (h2 / 2.0) * A @ A.T
    Lll = float(np.trace(L))
    C_I = float(np.sum(A * A)) / (12.0 * Smag ** 2)
    C_Ip = max(C_I, 0.0)
    N_d = float(np.sum(L * S)) - trS * Lll / 3.0 + C_Ip * trS * 2.0 * h2 * RHO * Smag ** 2 / 3.0
    D_d = -6.0 * h2 * RHO * Smag * (SS - trS ** 2 / 3.0)
    C_ds = N_d / D_d
    bAb = float(b @ A @ b)
    Pr = (max(C_ds, 0.0) * (-3.0 * h2 * RHO * Smag * float(b @ b)) / (RHO * h2 / 2.0 * bAb)
          if bAb != 0.0 else float("nan"))
    return C_I, C_ds, Pr


def test_filter_moments():
    n = 9
    i = np.arange(n, dtype=float)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    assert np.allclose(les.test_filter(np.full((n, n, n), 2.5)), 2.5, rtol=0, atol=1e-15)
    lin = 0.3 * x - 1.2 * y + 0.7 * z + 4.0
    assert np.abs(les.test_filter(lin) - lin[1:-1, 1:-1, 1:-1]).max() <= 1e-13
    q = x * x
    # second moment of (1/4, 1/2, 1/4) at unit spacing: 1/2
    assert np.abs(les.test_filter(q) - (q[1:-1, 1:-1, 1:-1] + 0.5)).max() <= 1e-12
    xy = x * y                                        # separable: no cross term
    assert np.abs(les.test_filter(xy) - xy[1:-1, 1:-1, 1:-1]).max() <= 1e-12


@pytest.mark.parametrize("A,b", [
    ([[-0.5, 0.3, 0.1], [0.2, 0.4, -0.3], [0.1, -0.2, -0.6]], [0.2, -0.1, 0.3]),
    ([[0.7, 0.0, 0.2], [-0.3, -0.2, 0.1], [0.0, 0.4, 0.5]], [-0.3, 0.2, 0.1]),
    ([[0.0, 0.9, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]], [0.1, 0.0, 0.0]),
])
def test_linear_field_closed_forms(A, b):
    Qp, geo, prm = _linear_state(A, b)
    d = les.dynamic_coefficients(Qp, geo, prm)
    C_I, C_ds, Pr = _closed_forms(A, b)
    assert abs(d["C_I"] - C_I) <= 1e-11 * abs(C_I)
    assert abs(d["C_ds"] - C_ds) <= 1e-10 * abs(C_ds) + 1e-14   # C_ds = 0 for pure shear
    if C_ds > 0.0 and Pr > 0.0:
        assert abs(d["Pr_sgs"] - Pr) <= 1e-10 * abs(Pr)
        assert d["Pr_eff"] == d["Pr_sgs"]
    else:
        assert d["Pr_eff"] == prm["Pr_sgs"]
    assert d["C_I_eff"] == max(d["C_I"], 0.0) and d["C_ds_eff"] == max(d["C_ds"], 0.0)


def test_some_case_has_a_positive_dynamic_constant():
    """The closed-form cases above exercise both signs of C_ds (the clipped
    and the unclipped path)."""
    signs = set()
    for A in ([[-0.5, 0.3, 0.1], [0.2, 0.4, -0.3], [0.1, -0.2, -0.6]],
              [[0.7, 0.0, 0.2], [-0.3, -0.2, 0.1], [0.0, 0.4, 0.5]]):
        signs.add(_closed_forms(A, [0.2, -0.1, 0.3])[1] > 0.0)
    assert signs == {True, False}


def test_fixed_coefficients_reduce_to_smagorinsky():
    pb = problems.jet_problem(12, 8, 8, seed=3, thermo_noise=1e-2)
    prm = dict(pb["params"], visc_coef=1e-3)
    geo = les.geometry(pb["xyz"].numpy(), prm)
    Qp = les.pad_state(pb["Q"].numpy())
    les.fill_ghosts(Qp, geo, prm, pb["inflow"].numpy())
    Cs = prm["Cs"]
    dyn = dict(C_I_eff=0.0, C_ds_eff=Cs * Cs, Pr_eff=prm["Pr_sgs"])
    Rd = les.residual(Qp, geo, dict(prm, sgs_model=3), dyn=dyn)
    Rs = les.residual(Qp, geo, dict(prm, sgs_model=1))
    R0 = les.residual(Qp, geo, dict(prm, sgs_model=0))
    scale = np.abs(Rs).max()
    assert np.abs(Rd - Rs).max() <= 1e-13 * scale
    assert np.abs(Rs - R0).max() > 1e-9 * scale       # the SGS part is visible


def test_isotropic_stress_on_a_linear_field():
    A = [[-0.5, 0.3, 0.1], [0.2, 0.4, -0.3], [0.1, -0.2, -0.6]]
    Qp, geo, prm = _linear_state(A, [0.2, -0.1, 0.3])
    c = 0.07
    base = dict(C_I_eff=0.0, C_ds_eff=0.0, Pr_eff=prm["Pr_sgs"])
    with np.errstate(all="ignore"):
        R1 = les.residual(Qp, geo, prm, dyn=dict(base, C_I_eff=c))
        R0 = les.residual(Qp, geo, prm, dyn=base)
    S = 0.5 * (np.asarray(A) + np.asarray(A).T)
    p_sgs = (2.0 / 3.0) * c * RHO * H * H * 2.0 * float(np.sum(S * S))
    dR = R1 - R0
    assert np.abs(dR[1:4]).max() <= 1e-12 * p_sgs
    assert np.abs(dR[4] - p_sgs * float(np.trace(np.asarray(A)))).max() <= 1e-11 * p_sgs


def test_dynamic_step_is_finite_and_differs_from_smagorinsky():
    pb = problems.jet_problem(12, 8, 8, seed=3, thermo_noise=1e-2)
    prm = dict(pb["params"], visc_coef=1e-3, sgs_model=3)
    geo = les.geometry(pb["xyz"].numpy(), prm)
    Q1, _ = les.run(pb["Q"].numpy(), geo, prm, pb["inflow"].numpy(), steps=2)
    Q2, _ = les.run(pb["Q"].numpy(), geo, dict(prm, sgs_model=1), pb["inflow"].numpy(), steps=2)
    assert np.isfinite(Q1).all()
    assert np.abs(Q1 - Q2).max() > 0.0


@pytest.mark.parametrize("case", ["jet8x6x8", "modes_box8"])
def test_sums_match_brute_force(case):
    """The vectorised sums against the scalar loops of the brute-force
    oracle (explicit 27-point filter, point-by-point gradients) on a
    curvilinear jet (every boundary kind) and a multi-mode periodic box:
    each sum within 1e-12 of the sum of its terms' magnitudes."""
    from oracle import brute
    if case == "jet8x6x8":
        pb = problems.jet_problem(8, 6, 8, seed=5, thermo_noise=1e-2)
        Q = pb["Q"].numpy().copy()
        rng = np.random.default_rng(3)
        Q[1:4] += 0.05 * rng.standard_normal(Q[1:4].shape)
        pb["Q"] = Q
        prm = dict(pb["params"], sgs_model=3, visc_coef=1e-3)
    else:
        pb = problems.modes_box_problem(8, seed=1)
        Q = pb["Q"].numpy()
        prm = pb["params"]
    inflow = pb["inflow"].numpy() if pb.get("inflow") is not None else None
    xyz = pb["xyz"].numpy()
    geo = les.geometry(xyz, prm)
    Qp = les.pad_state(np.asarray(Q))
    les.fill_ghosts(Qp, geo, prm, inflow)
    ref = les.dynamic_coefficients(Qp, geo, prm)["sums"]
    sums, mags = brute.Brute(xyz, prm, inflow).dynamic_sums(np.asarray(Q))
    for k in sums:
        assert mags[k] > 0.0
        assert abs(sums[k] - ref[k]) <= 1e-12 * mags[k], (k, sums[k], ref[k], mags[k])
