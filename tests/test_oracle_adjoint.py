"""Pins of the oracle's derivatives, which the GPU adjoint is checked against.

The oracle is written dtype-generically so that a complex-step evaluation
R(Q + i h v) gives the directional derivative J v = Im R / h with no
subtractive cancellation.  That only holds if every operation on the path is
complex-analytic where the real function is smooth (abs, max and branch tests
acting on real parts).  These tests check the complex-step derivatives
against central finite differences of the real oracle, an independent route,
for the residual (state and entrance data), for an RK5 step, and on every
boundary kind.  A planted mistake (a conjugate where the real part was
meant) is shown to be caught.
"""
import numpy as np
import pytest

from cases import flow, problems
from oracle import les

H_CS = 1e-30


def _jet(nx=8, nr=6, nth=8, seed=5):
    pb = problems.jet_problem(nx, nr, nth, seed=seed, thermo_noise=1e-3)
    geo = les.geometry(pb["xyz"].numpy(), pb["params"])
    return pb, geo


def _box(n=8, seed=6):
    pb = problems.box_problem(n, seed=seed, noise=1e-3)
    geo = les.geometry(pb["xyz"].numpy(), pb["params"])
    return pb, geo


def _dirs(pb, seed=11):
    Q = pb["Q"].numpy()
    v = problems.seeded_field(Q.shape, seed, flow.FIELD_DIRECTION).numpy()
    # scale per variable so each perturbs its own variable comparably
    v = v * np.abs(Q).reshape(5, -1).max(axis=1).reshape(5, 1, 1, 1)
    vin = None
    if pb["inflow"] is not None:
        inf = pb["inflow"].numpy()
        vin = problems.seeded_field(inf.shape, seed, flow.FIELD_DIRECTION_IN).numpy()
        vin = vin * (np.abs(inf).reshape(5, -1).max(axis=1).reshape(5, 1, 1) + 0.1)
    return v, vin


def _complex_step(fn, Q, v, inflow=None, vin=None):
    Qc = Q.astype(np.complex128) + 1j * H_CS * v
    infc = None
    if inflow is not None:
        infc = inflow.astype(np.complex128)
        if vin is not None:
            infc = infc + 1j * H_CS * vin
    return np.imag(fn(Qc, infc)) / H_CS


def _central(fn, Q, v, inflow=None, vin=None, h=1e-7):
    # h small enough that no sensor or limiter kink of the box vortex lies
    # within +-h v of the state (at h = 1e-5 one does, and the two routes
    # then differ by 2e-3 while the complex step stays exact)
    def at(s):
        inf = None
        if inflow is not None:
            inf = inflow + (s * h * vin if vin is not None else 0.0)
        return fn(Q + s * h * v, inf)
    return (at(1.0) - at(-1.0)) / (2.0 * h)


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("case", ["jet", "box"])
def test_complex_step_matches_central_differences(case):
    pb, geo = _jet() if case == "jet" else _box()
    Q = pb["Q"].numpy()
    inflow = pb["inflow"].numpy() if pb["inflow"] is not None else None
    v, vin = _dirs(pb)

    def fn(q, inf):
        return les.evaluate(q, geo, pb["params"], inf)

    cs = _complex_step(fn, Q, v, inflow)
    fd = _central(fn, Q, v, inflow)
    assert _rel(cs, fd) < 1e-6
    if inflow is not None:       # entrance data direction alone
        cs = _complex_step(fn, Q, 0 * v, inflow, vin)
        fd = _central(fn, Q, 0 * v, inflow, vin)
        assert np.abs(cs).max() > 0.0
        assert _rel(cs, fd) < 1e-6


def test_complex_step_rk5_step():
    pb, geo = _jet()
    Q = pb["Q"].numpy()
    inflow = pb["inflow"].numpy()
    v, vin = _dirs(pb)
    dt = 1e-3

    def fn(q, inf):
        return les.rk5_step(q, geo, pb["params"], inf, dt=dt)[0]

    cs = _complex_step(fn, Q, v, inflow, vin)
    fd = _central(fn, Q, v, inflow, vin)
    assert _rel(cs, fd) < 1e-6


def test_every_boundary_kind_has_a_nonzero_ghost_derivative():
    """The tiny jet state exercises a Riemann (subsonic) branch at the
    entrance, far field and exit; the derivative of the boundary-adjacent
    residual with respect to the first interior point is nonzero there."""
    pb, geo = _jet()
    prm = pb["params"]
    Q = pb["Q"].numpy()
    inflow = pb["inflow"].numpy()
    nx, nr = Q.shape[3], Q.shape[2]
    for (j, i) in [(2, 0), (nr - 1, 3), (2, nx - 1), (0, 3)]:
        v = np.zeros_like(Q)
        v[:, 3, j, i] = 1.0
        cs = _complex_step(lambda q, inf: les.evaluate(q, geo, prm, inf), Q, v, inflow)
        assert np.abs(cs[:, 3, j, i]).max() > 0.0


def test_planted_conjugate_is_caught(monkeypatch):
    """A complex-unsafe abs (np.abs, the modulus) breaks the complex step;
    the comparison above must see it."""
    pb, geo = _jet()
    Q = pb["Q"].numpy()
    inflow = pb["inflow"].numpy()
    v, _ = _dirs(pb)

    def fn(q, inf):
        return les.evaluate(q, geo, pb["params"], inf)

    fd = _central(fn, Q, v, inflow)
    monkeypatch.setattr(les, "rabs", lambda x: np.abs(x).astype(np.asarray(x).dtype))
    cs = _complex_step(fn, Q, v, inflow)
    assert _rel(cs, fd) > 1e-3
