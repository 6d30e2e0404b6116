"""Oracle pins: metrics against the exact discrete closed form, and ghost
values against the defining properties of each boundary condition."""
import math

import numpy as np
import pytest

from cases import flow, mesh, problems
from oracle import les


def _jet(nx=12, nr=10, nth=16, **kw):
    pb = problems.jet_problem(nx, nr, nth, **kw)
    return pb, pb["xyz"].numpy(), pb["params"]


# ---------------------------------------------------------------------------
# metrics
# ---------------------------------------------------------------------------
def test_metrics_closed_form_cylindrical_product_mesh():
    """On x = X_i, y = R_j cos(theta_k), z = R_j sin(theta_k) the central
    differences give V = x_xi R R_eta sin(dth), S^xi = (R R_eta sin(dth), 0, 0),
    S^eta = x_xi R sin(dth) (0, cos, sin), S^zeta = x_xi R_eta (0, -sin, cos),
    on the whole padded box.  The ghost coordinates are the extended 1-D maps:
    X and the far-field R linearly extrapolated, R_{-1-m} = -R_m across the
    axis, theta periodic."""
    nx, nr, nth = 12, 10, 16
    pb, xyz, prm = _jet(nx, nr, nth)
    X, R, TH = (t.numpy() for t in pb["grid"])
    geo = les.geometry(xyz, prm)
    g = 3
    Xe = np.concatenate([X[0] + np.arange(g, 0, -1) * (X[0] - X[1]), X,
                         X[-1] + np.arange(1, g + 1) * (X[-1] - X[-2])])
    Re = np.concatenate([-R[g - 1::-1], R, R[-1] + np.arange(1, g + 1) * (R[-1] - R[-2])])
    k = np.arange(-2, nth + 2)
    th = 2 * math.pi * k / nth
    dth = 2 * math.pi / nth
    x_xi = (Xe[2:] - Xe[:-2]) / 2           # at i = -2 .. nx+1
    R_c = Re[1:-1]                          # at j = -2 .. nr+1
    R_eta = (Re[2:] - Re[:-2]) / 2
    s = math.sin(dth)
    Vx = x_xi[None, None, :] * (R_c * R_eta)[None, :, None] * s * np.ones((nth + 4, 1, 1))
    assert np.allclose(geo["V"], Vx, rtol=1e-12, atol=0)
    S = geo["S"]
    scale = np.abs(S).max()
    exp = np.zeros_like(S)
    exp[0, 0] = ((R_c * R_eta)[None, :, None] * s) * np.ones((nth + 4, 1, nx + 4))
    exp[1, 1] = x_xi[None, None, :] * R_c[None, :, None] * s * np.cos(th)[:, None, None]
    exp[1, 2] = x_xi[None, None, :] * R_c[None, :, None] * s * np.sin(th)[:, None, None]
    exp[2, 1] = -x_xi[None, None, :] * R_eta[None, :, None] * np.sin(th)[:, None, None]
    exp[2, 2] = x_xi[None, None, :] * R_eta[None, :, None] * np.cos(th)[:, None, None]
    assert np.abs(S - exp).max() <= 1e-13 * scale
    # cross-axis ghost: V(j=-1) = -V(j=0), hence a zero face volume on the axis
    assert np.allclose(geo["V"][:, 1, :], -geo["V"][:, 2, :], rtol=1e-13)


def test_metrics_box():
    n = 8
    L = 2 * math.pi
    h = L / n
    prm = problems.box_params(L)
    geo = les.geometry(mesh.box_coords(n, L).numpy(), prm)
    assert np.allclose(geo["V"], h ** 3, rtol=1e-14)
    for d in range(3):
        for m in range(3):
            assert np.allclose(geo["S"][d, m], h * h if d == m else 0.0,
                               rtol=1e-14, atol=1e-15 * h * h)


def test_discrete_gcl_on_jet_mesh():
    """sum_d delta_d S^d = 0 (discrete geometric conservation) at every
    interior point of the product mesh: free stream is preserved exactly."""
    pb, xyz, prm = _jet(10, 8, 12)
    S = les.geometry(xyz, prm)["S"]
    g = 2
    tot = (S[0][..., g:-g, g:-g, g + 1:S.shape[-1] - g + 1] - S[0][..., g:-g, g:-g, g - 1:-g - 1]
           + S[1][..., g:-g, g + 1:S.shape[-2] - g + 1, g:-g] - S[1][..., g:-g, g - 1:-g - 1, g:-g]
           + S[2][..., g + 1:S.shape[-3] - g + 1, g:-g, g:-g] - S[2][..., g - 1:-g - 1, g:-g, g:-g])
    assert np.abs(tot).max() <= 1e-13 * np.abs(S).max()


# ---------------------------------------------------------------------------
# Riemann-invariant boundary state
# ---------------------------------------------------------------------------
def _invariants(prim, n, gamma):
    rho, u, v, w, p = prim
    a = np.sqrt(gamma * p / rho)
    q = u * n[0] + v * n[1] + w * n[2]
    tang = np.array([u - q * n[0], v - q * n[1], w - q * n[2]])
    return q + 2 * a / (gamma - 1), q - 2 * a / (gamma - 1), p / rho ** gamma, tang


@pytest.mark.parametrize("qn", [0.3, -0.3])
def test_riemann_state_characteristics(qn):
    """Subsonic branches: R+ of the boundary state equals R+ of the interior,
    R- equals R- of the outside state; entropy and tangential velocity come
    from the upwind side (interior for q >= 0, outside for q < 0)."""
    g = 1.4
    n = np.array([0.6, 0.0, 0.8])
    t = np.array([0.8, 0.0, -0.6])
    e = (1.1, *(qn * n + 0.2 * t), 0.75)
    r = (0.95, *(0.1 * n - 0.1 * t), 0.70)
    f, _ = les.riemann_state(tuple(np.asarray(c) for c in e), r, n, g)
    f = [float(c) for c in f]
    Rp_f, Rm_f, s_f, t_f = _invariants(f, n, g)
    Rp_e, _, s_e, t_e = _invariants(e, n, g)
    _, Rm_r, s_r, t_r = _invariants(r, n, g)
    assert abs(Rp_f - Rp_e) < 1e-14 and abs(Rm_f - Rm_r) < 1e-14
    if qn >= 0:
        assert abs(s_f - s_e) < 1e-14 and np.allclose(t_f, t_e, atol=1e-15)
    else:
        assert abs(s_f - s_r) < 1e-14 and np.allclose(t_f, t_r, atol=1e-15)


def test_riemann_uniform_state_reproduces_itself():
    g = 1.4
    n = np.array([0.0, 0.6, 0.8])
    for qn in (0.5, -0.5, 1.5, -1.5, 0.0):
        prim = (1.0, 0.1, qn * 0.6 - 0.8 * 0.2, qn * 0.8 + 0.6 * 0.2, 1 / g)
        f, _ = les.riemann_state(tuple(np.asarray(c) for c in prim), prim, n, g)
        assert np.allclose([float(c) for c in f], prim, rtol=1e-15, atol=1e-15)


def test_riemann_supersonic_branches_copy():
    g = 1.4
    n = np.array([1.0, 0.0, 0.0])
    e = (1.0, 2.0, 0.1, 0.0, 1 / g)       # M = 2 outward
    r = (1.2, -0.3, 0.0, 0.2, 0.8)
    f, _ = les.riemann_state(tuple(np.asarray(c) for c in e), r, n, g)
    assert [float(c) for c in f] == list(e)
    e2 = (1.0, -2.0, 0.1, 0.0, 1 / g)     # M = -2, inflow: outside state
    f, _ = les.riemann_state(tuple(np.asarray(c) for c in e2), r, n, g)
    assert [float(c) for c in f] == list(r)


# ---------------------------------------------------------------------------
# ghost fill
# ---------------------------------------------------------------------------
def test_ghost_fill_defines_every_padded_point_and_copies():
    pb, xyz, prm = _jet(8, 6, 8)
    geo = les.geometry(xyz, prm)
    Q = pb["Q"].numpy()
    Qp = les.pad_state(Q)
    les.fill_ghosts(Qp, geo, prm, pb["inflow"].numpy())
    assert np.isfinite(Qp).all()
    g = 2
    nth = Q.shape[1]
    # theta periodic wrap (bitwise), over all i, j
    assert np.array_equal(Qp[:, 0], Qp[:, nth]) and np.array_equal(Qp[:, 1], Qp[:, nth + 1])
    assert np.array_equal(Qp[:, nth + 2], Qp[:, 2]) and np.array_equal(Qp[:, nth + 3], Qp[:, 3])
    # cross-axis copy (bitwise): ghost j = -1-m equals (m, k + nth/2)
    for m in range(2):
        for k in range(nth):
            assert np.array_equal(Qp[:, g + k, g - 1 - m, :],
                                  Qp[:, g + (k + nth // 2) % nth, g + m, :])


def test_outflow_subsonic_takes_back_pressure():
    pb, xyz, prm = _jet(8, 6, 8)
    prm = dict(prm, p_exit=0.7)
    geo = les.geometry(xyz, prm)
    Qp = les.pad_state(pb["Q"].numpy())
    les.fill_ghosts(Qp, geo, prm, pb["inflow"].numpy())
    g = 2
    gh = Qp[:, g:-g, g:-g, -1]
    ins = Qp[:, g:-g, g:-g, -3]
    rho, u, v, w, p = les.primitives(gh, prm["gamma"])
    ri, ui, vi, wi, pi = les.primitives(ins, prm["gamma"])
    sub = ui / np.sqrt(1.4 * pi / ri) < 1.0           # axial normal on this mesh
    assert sub.any() and (~sub).any()
    assert np.allclose(p[sub], 0.7, rtol=1e-13)
    assert np.allclose(rho, ri, rtol=1e-15) and np.allclose(u, ui, rtol=1e-14)
    assert np.array_equal(gh[:, ~sub], ins[:, ~sub])    # supersonic exit: copy


def test_inflow_supersonic_target_is_imposed():
    """The jet core (Mach 1.4) receives the target state; the coflow (Mach
    0.05) goes through the Riemann-invariant branch."""
    pb, xyz, prm = _jet(8, 12, 8)
    geo = les.geometry(xyz, prm)
    Qp = les.pad_state(pb["Q"].numpy())
    tgt = pb["inflow"].numpy()
    les.fill_ghosts(Qp, geo, prm, tgt)
    g = 2
    gh = Qp[:, g:-g, g:-g, 1]                          # i = -1
    core = tgt[1] / np.sqrt(1.4 * tgt[4] / tgt[0]) >= 1.0
    assert core.any() and (~core).any()
    expect = les.conserved(*tgt, 1.4)
    assert np.array_equal(gh[:, core], expect[:, core])
    assert not np.allclose(gh[:, ~core], expect[:, ~core], rtol=1e-12, atol=0)
    assert np.array_equal(Qp[:, g:-g, g:-g, 0], gh)    # both layers


def test_farfield_ghost_has_invariants_of_riemann():
    pb, xyz, prm = _jet(8, 6, 8)
    geo = les.geometry(xyz, prm)
    Qp = les.pad_state(pb["Q"].numpy())
    les.fill_ghosts(Qp, geo, prm, pb["inflow"].numpy())
    g = 2
    gam = prm["gamma"]
    Se = geo["S"][1][:, g:-g, -3, :]                    # S^eta at j = nr-1
    n = Se / np.sqrt((Se ** 2).sum(axis=0))
    e = les.primitives(Qp[:, g:-g, -3, :], gam)
    f = les.primitives(Qp[:, g:-g, -2, :], gam)
    Rp_e, _, s_e, _ = _invariants(e, n, gam)
    Rp_f, Rm_f, s_f, _ = _invariants(f, n, gam)
    _, Rm_r, _, _ = _invariants(tuple(np.float64(c) for c in prm["ref_prim"]), n, gam)
    q = e[1] * n[0] + e[2] * n[1] + e[3] * n[2]
    assert np.abs(Rp_f - Rp_e).max() < 1e-13 and np.abs(Rm_f - Rm_r).max() < 1e-13
    out = q >= 0
    assert np.abs(s_f - s_e)[out].max() < 1e-13
