"""Oracle pins for the residual and the time step: invariants, closed forms
of the dissipation on checkerboard modes, exact special cases of the
viscous/SGS terms, brute force on tiny grids, and the RK5 polynomial."""
import math

import numpy as np
import pytest

from cases import flow, mesh, problems
from oracle import brute, les


def _box(n=8, **over):
    L = 2 * math.pi
    prm = problems.box_params(L, **over)
    xyz = mesh.box_coords(n, L).numpy()
    return xyz, prm, les.geometry(xyz, prm)


def _uniform_cons(shape, prim, g=1.4):
    return flow.uniform_state(shape, prim).numpy()


# ---------------------------------------------------------------------------
# free stream and conservation
# ---------------------------------------------------------------------------
def _free_stream_ratio(xyz, prm, prim, inflow=None):
    geo = les.geometry(xyz, prm)
    _, nth, nr, nx = xyz.shape
    Q = _uniform_cons((nth, nr, nx), prim)
    Qp = les.pad_state(Q)
    les.fill_ghosts(Qp, geo, prm, inflow)
    R = les.residual(Qp, geo, prm)
    VR = R * les.interior(geo["V"])
    pt = les.point_terms(Qp, geo, prm)
    fscale = max(np.abs(pt["G"][d]).max() for d in range(3))
    return np.abs(VR).max() / fscale


def test_free_stream_preserved_on_jet_mesh():
    """A uniform state with all three velocity components nonzero, with the
    boundary data equal to it, has zero residual to rounding: the metric
    identity holds exactly on the product mesh, including the cross-axis
    ghosts and the extrapolated ghost coordinates."""
    prim = (1.0, 0.6, 0.3, -0.2, 1.0 / 1.4)
    pb = problems.jet_problem(16, 12, 16)
    prm = dict(pb["params"], ref_prim=prim, p_exit=prim[4])
    inflow = np.broadcast_to(np.array(prim)[:, None, None], (5, 16, 12)).copy()
    assert _free_stream_ratio(pb["xyz"].numpy(), prm, prim, inflow) <= 1e-12


def test_free_stream_preserved_on_box_and_wavy_mesh():
    """Cartesian box, and the non-orthogonal periodic mesh
    x = xi + a sin(eta), y = eta + a sin(zeta), z = zeta + a sin(xi): every
    coordinate is a sum of single-index functions, for which the
    cross-product metrics satisfy the discrete identity exactly as well."""
    xyz, prm, _ = _box(8)
    prim = (1.0, 0.5, -0.25, 0.125, 0.8)
    assert _free_stream_ratio(xyz, prm, prim) <= 1e-13
    L = 2 * math.pi
    for n in (12, 16):
        w = mesh.wavy_coords(n, L, 0.1).numpy()
        assert _free_stream_ratio(w, problems.box_params(L), prim) <= 1e-13


def test_periodic_box_conservation():
    """Each face flux enters its two cells with opposite signs, so
    sum V R = 0 over a fully periodic mesh, and sum V Q is constant in time."""
    pb = problems.box_problem(12)
    xyz, prm, Q = pb["xyz"].numpy(), pb["params"], pb["Q"].numpy()
    geo = les.geometry(xyz, prm)
    R = les.evaluate(Q, geo, prm)
    V = les.interior(geo["V"])
    for c in range(5):
        VR = (V * R[c]).ravel()
        assert abs(math.fsum(VR)) <= 1e-13 * math.fsum(np.abs(VR))
    tot0 = [math.fsum((V * Q[c]).ravel()) for c in range(5)]
    Qn, _ = les.run(Q, geo, prm, steps=3)
    tot1 = [math.fsum((V * Qn[c]).ravel()) for c in range(5)]
    for c in (0, 1, 2, 4):
        assert abs(tot1[c] - tot0[c]) <= 1e-13 * abs(tot0[c])
    # the w-momentum total is near zero; compare with the momentum scale
    assert abs(tot1[3] - tot0[3]) <= 1e-13 * abs(tot0[1])


# ---------------------------------------------------------------------------
# artificial dissipation: closed forms on checkerboard modes
# ---------------------------------------------------------------------------
def _lam_bar_cartesian(u, a, h, d):
    lam = [(abs(u[e]) + a) / h for e in range(3)]
    o1, o2 = lam[(d + 1) % 3], lam[(d + 2) % 3]
    return lam[d] * (1 + math.sqrt(o1 / lam[d]) + math.sqrt(o2 / lam[d]))


@pytest.mark.parametrize("d", [0, 1, 2])
def test_fourth_difference_damps_density_checkerboard(d):
    """rho_i = rho0 (1 + eps (-1)^i) along direction d, uniform u and p: the
    central fluxes cancel, all central-difference gradients vanish and the
    sensor is zero, so only the k4 term acts.  With
    W_{i+2} - 3W_{i+1} + 3W_i - W_{i-1} = 8 A (-1)^i for a checkerboard of
    amplitude A:  R = 16 k4 lambda_f A (-1)^i, lambda_f the mean of the two
    lambda_bar values; A = rho0 eps (1, u, v, w, |u|^2/2) for W."""
    n = 8
    L = 2 * math.pi
    h = L / n
    xyz, prm, geo = _box(n, visc_coef=5e-3)
    g = 1.4
    rho0, eps, u, p0 = 1.2, 1e-3, (0.3, -0.2, 0.1), 0.9
    idx = np.arange(n)
    sgn = (-1.0) ** idx
    shape = [1, 1, 1]
    shape[2 - d] = n
    rho = rho0 * (1 + eps * sgn.reshape(shape)) * np.ones((n, n, n))
    Q = np.stack([rho, rho * u[0], rho * u[1], rho * u[2],
                  p0 / (g - 1) + 0.5 * rho * sum(c * c for c in u)])
    R = les.evaluate(Q, geo, prm)
    lam_f = 0.5 * (_lam_bar_cartesian(u, math.sqrt(g * p0 / (rho0 * (1 + eps))), h, d)
                   + _lam_bar_cartesian(u, math.sqrt(g * p0 / (rho0 * (1 - eps))), h, d))
    amp = rho0 * eps * np.array([1.0, u[0], u[1], u[2], 0.5 * sum(c * c for c in u)])
    expect = 16 * prm["k4"] * lam_f * amp[:, None, None, None] * sgn.reshape(shape)
    assert np.allclose(R, expect, rtol=1e-9, atol=1e-13 * np.abs(expect).max())


@pytest.mark.parametrize("eps", [0.01, 0.1])
def test_second_difference_and_sensor_on_pressure_checkerboard(eps):
    """p_i = p0 (1 + eps (-1)^i) along xi: sensor nu = |eps| exactly, so
    eps2 = k2 |eps|, eps4 = max(0, k4 - eps2); only W5 = E + p carries the
    mode, with amplitude gamma p0 eps/(gamma-1).  Then
    R_E = 4 lambda_f (eps2 + 4 eps4) A (-1)^i and the other components vanish.
    eps = 0.01 exercises both terms, eps = 0.1 switches the fourth difference
    off (eps2 > k4)."""
    n = 8
    L = 2 * math.pi
    h = L / n
    xyz, prm, geo = _box(n, visc_coef=5e-3)
    g = 1.4
    rho0, u = 1.0, (0.3, -0.2, 0.1)
    p0 = 1 / g
    sgn = (-1.0) ** np.arange(n)
    p = p0 * (1 + eps * sgn.reshape(1, 1, n)) * np.ones((n, n, n))
    Q = np.stack([np.full((n, n, n), rho0), *(np.full((n, n, n), rho0 * c) for c in u),
                  p / (g - 1) + 0.5 * rho0 * sum(c * c for c in u)])
    R = les.evaluate(Q, geo, prm)
    e2 = prm["k2"] * eps
    e4 = max(0.0, prm["k4"] - e2)
    lam_f = 0.5 * (_lam_bar_cartesian(u, math.sqrt(g * p0 * (1 + eps) / rho0), h, 0)
                   + _lam_bar_cartesian(u, math.sqrt(g * p0 * (1 - eps) / rho0), h, 0))
    A = g * p0 * eps / (g - 1)
    expect = 4 * lam_f * (e2 + 4 * e4) * A * sgn.reshape(1, 1, n) * np.ones((n, n, n))
    assert np.allclose(R[4], expect, rtol=1e-9)
    assert np.abs(R[:4]).max() <= 1e-12 * np.abs(expect).max()


def test_dissipation_sign_decays_energy():
    """Inviscid, at rest, a small odd-even pressure mode: the total
    perturbation energy must decrease over RK steps (a wrong sign of either
    dissipation term makes it grow)."""
    n = 8
    xyz, prm, geo = _box(n, visc_coef=0.0)
    g = 1.4
    rng = np.random.default_rng(3)
    p = 1 / g * (1 + 1e-3 * rng.standard_normal((n, n, n)))
    Q = np.stack([np.ones((n, n, n)), np.zeros((n, n, n)), np.zeros((n, n, n)),
                  np.zeros((n, n, n)), p / (g - 1)])
    def energy(q):
        return float(((q - q.mean(axis=(1, 2, 3), keepdims=True)) ** 2).sum())
    e0 = energy(Q)
    Qn, _ = les.run(Q, geo, prm, steps=5)
    assert energy(Qn) < 0.9 * e0


# ---------------------------------------------------------------------------
# viscous and SGS terms: exact special cases (central differences are exact
# on linear fields)
# ---------------------------------------------------------------------------
def _padded_linear_state(n, h, fields, g=1.4):
    """Padded state filled analytically (ghosts included) from functions of
    (x, y, z); returns Qp on the 2-ghost box of an n^3 Cartesian mesh."""
    s = (np.arange(-2, n + 2)) * h
    z, y, x = np.meshgrid(s, s, s, indexing="ij")
    rho, u, v, w, p = (f(x, y, z) * np.ones_like(x) for f in fields)
    return np.stack([rho, rho * u, rho * v, rho * w,
                     p / (g - 1) + 0.5 * rho * (u * u + v * v + w * w)])


def _cartesian_geo(n, h):
    Vb = np.full((n + 4,) * 3, h ** 3)
    S = np.zeros((3, 3) + (n + 4,) * 3)
    for d in range(3):
        S[d, d] = h * h
    return dict(S=S, V=Vb)


def test_smagorinsky_on_linear_shear_and_rotation():
    """u = gd * y: |S| = |gd| and mu_t = rho (Cs h)^2 |gd| / visc_coef.
    Solid-body rotation (u, v) = (-W y, W x): S = 0, so mu_t = 0."""
    n, h = 6, 0.2
    prm = problems.box_params(visc_coef=1e-3)
    geo = _cartesian_geo(n, h)
    gd = 0.7
    Qp = _padded_linear_state(n, h, (lambda x, y, z: 1.3, lambda x, y, z: gd * y,
                                     lambda x, y, z: 0.0, lambda x, y, z: 0.0,
                                     lambda x, y, z: 0.7))
    pt = les.point_terms(Qp, geo, prm)
    mt = pt["mu_t"][1:-1, 1:-1, 1:-1]
    assert np.allclose(mt, 1.3 * (prm["Cs"] * h) ** 2 * gd / prm["visc_coef"], rtol=1e-12)
    Om = 0.4
    Qp = _padded_linear_state(n, h, (lambda x, y, z: 1.0, lambda x, y, z: -Om * y,
                                     lambda x, y, z: Om * x, lambda x, y, z: 0.0,
                                     lambda x, y, z: 0.7))
    pt = les.point_terms(Qp, geo, prm)
    assert np.abs(pt["mu_t"][1:-1, 1:-1, 1:-1]).max() <= 1e-12


def test_viscous_flux_for_linear_shear():
    """Constant T and rho, u = gd*y: the only viscous stress is
    tau_xy = (mu + mu_t) gd with mu = 1 (Sutherland at T = 1), so the eta
    point flux of x-momentum is Fe - visc_coef h^2 tau_xy and its energy
    component carries tau_xy u."""
    n, h = 6, 0.2
    g = 1.4
    prm = problems.box_params(visc_coef=1e-3, Cs=0.0)
    geo = _cartesian_geo(n, h)
    gd = 0.5
    Qp = _padded_linear_state(n, h, (lambda x, y, z: 1.0, lambda x, y, z: gd * y,
                                     lambda x, y, z: 0.0, lambda x, y, z: 0.0,
                                     lambda x, y, z: 1.0 / g))
    pt = les.point_terms(Qp, geo, prm)
    G1 = pt["G"][1][:, 1:-1, 1:-1, 1:-1]           # eta point flux, interior
    s = (np.arange(n)) * h
    yv = s.reshape(1, n, 1) * np.ones((n, n, n))
    tau_xy = 1.0 * gd
    assert np.allclose(G1[1], -prm["visc_coef"] * h * h * tau_xy, rtol=1e-12)
    assert np.allclose(G1[4], -prm["visc_coef"] * h * h * tau_xy * gd * yv,
                       rtol=1e-12, atol=1e-18)


def test_heat_flux_is_down_gradient():
    """At rest with uniform pressure and a hot spot, energy must leave the
    hot spot: R_E > 0 (dE/dt < 0) at the temperature maximum."""
    n = 16
    xyz, prm, geo = _box(n, visc_coef=1e-2, k2=0.0, k4=0.0, Cs=0.0)
    g = 1.4
    s = np.arange(n) * (2 * math.pi / n)
    z, y, x = np.meshgrid(s, s, s, indexing="ij")
    T = 1.0 + 0.2 * np.exp(-((x - math.pi) ** 2 + (y - math.pi) ** 2 + (z - math.pi) ** 2))
    p = 1 / g
    rho = g * p / T
    Q = np.stack([rho, 0 * rho, 0 * rho, 0 * rho, np.full_like(rho, p / (g - 1))])
    R = les.evaluate(Q, geo, prm)
    c = n // 2
    assert R[4, c, c, c] > 0
    assert abs(R[0, c, c, c]) < 1e-12 and np.abs(R[1:4]).max() < 1e-6 * R[4, c, c, c]


# ---------------------------------------------------------------------------
# time step and RK5
# ---------------------------------------------------------------------------
def test_lambda_sum_cartesian_closed_form():
    n = 6
    L = 2 * math.pi
    h = L / n
    xyz, prm, geo = _box(n)
    prim = (1.1, 0.3, -0.4, 0.2, 0.8)
    Q = _uniform_cons((n, n, n), prim)
    a = math.sqrt(1.4 * prim[4] / prim[0])
    expect = sum(abs(c) + a for c in prim[1:4]) / h
    assert np.allclose(les.lambda_sum(les.pad_state(Q), geo, prm), expect, rtol=1e-14)
    assert abs(les.time_step(Q, geo, prm) - prm["cfl"] / expect) <= 1e-15 * prm["cfl"] / expect


def test_rk5_linear_amplification_polynomial():
    """For R(Q) = lam Q each stage multiplies: Q^(l) = 1 + alpha_l z Q^(l-1)
    with z = -lam dt, so one step is P(z) = 1 + z + z^2/2 + 3 z^3/16 + z^4/32
    + z^5/128 for alpha = (1/4, 1/6, 3/8, 1/2, 1) (second order)."""
    alpha = problems.RK_ALPHA
    for z in (-0.3, -1.7, 0.9, 2.2j, -0.5 + 1.5j):
        lam, dt = -z, 1.0
        q1 = les.jameson_rk(np.array([1.0 + 0j]), lambda q: lam * q, dt, alpha)[0]
        P = 1 + z + z ** 2 / 2 + 3 * z ** 3 / 16 + z ** 4 / 32 + z ** 5 / 128
        assert abs(q1 - P) <= 1e-14 * max(1.0, abs(P))
    # stability on the imaginary axis up to |y| = 2 sqrt(2) (the quoted CFL bound)
    for y in np.linspace(0, 2 * math.sqrt(2), 50):
        z = 1j * y
        P = 1 + z + z ** 2 / 2 + 3 * z ** 3 / 16 + z ** 4 / 32 + z ** 5 / 128
        assert abs(P) <= 1.0 + 1e-15


# ---------------------------------------------------------------------------
# brute force on tiny grids
# ---------------------------------------------------------------------------
def _brute_array(Rb, shape):
    out = np.zeros(shape)
    for (i, j, k), r in Rb.items():
        out[:, k, j, i] = r
    return out


def _compare_brute(xyz, Q, prm, inflow=None):
    geo = les.geometry(xyz, prm)
    R = les.evaluate(Q, geo, prm, inflow)
    Rb, _ = brute.Brute(xyz, prm, inflow).residual(Q)
    Rb = _brute_array(Rb, R.shape)
    return np.abs(R - Rb).max() / np.abs(R).max()


def test_brute_force_box():
    pb = problems.box_problem(6)
    assert _compare_brute(pb["xyz"].numpy(), pb["Q"].numpy(), pb["params"]) <= 1e-13


def test_brute_force_jet_all_boundary_kinds():
    """8 x 6 x 8 jet: entrance (supersonic core + Riemann coflow), exit,
    cross-axis ghosts, far field, periodic azimuth.  A radial outflow and a
    strong perturbation make the far field take several Riemann branches."""
    pb = problems.jet_problem(8, 6, 8)
    Q = pb["Q"].numpy().copy()
    rng = np.random.default_rng(5)
    Q[1:4] += 0.05 * rng.standard_normal(Q[1:4].shape)
    Q[2, :, -1, :] += 0.3 * np.cos(2 * math.pi * np.arange(8) / 8)[:, None]
    Q[3, :, -1, :] += 0.3 * np.sin(2 * math.pi * np.arange(8) / 8)[:, None]
    assert _compare_brute(pb["xyz"].numpy(), Q, pb["params"], pb["inflow"].numpy()) <= 1e-13
