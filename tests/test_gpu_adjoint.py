"""GPU parity of the adjoint entry points against the oracle's derivatives.

The oracle's derivatives are complex-step evaluations of the plain residual
(exact to rounding; pinned against central differences in
test_oracle_adjoint.py).  Cases:
  * dense Jacobian on the 8x6x8 jet (every boundary kind): every row of
    dR/dQ and of dR/d(inflow data) from les_residual_vjp with unit
    cotangents, against the complex-step Jacobian, per row <= 1e-12;
  * directional checks <Rbar, J v> = <Qbar, v> on a periodic box and a
    24x12x16 jet with the Smagorinsky and with the Vreman model, on thin
    meshes (tile edges of the main pass), and on the full 160x100x128 jet
    mesh with a seeded Gaussian cotangent;
  * RK5-step adjoint against complex-step derivatives of the oracle's RK5
    step (fixed dt), including the entrance-data cotangent and in-place use;
  * central differences of the GPU's own forward residual (dot-product
    test) at <= 1e-6;
  * bitwise reproducibility, ghost entries of Qbar zero, FP32 refused.
States carry relative rho and p noise (thermo_noise) so that no pressure
sensor sits at its kink (a uniform pressure makes the sensor's numerator
vanish, where R is not differentiable).
"""
import numpy as np
import pytest
import torch

from cases import flow, problems
from oracle import les
from _helpers import announce, make_solver, to_np

pytestmark = pytest.mark.gpu

H_CS = 1e-30


def _jet(nx, nr, nth, seed=5):
    return problems.jet_problem(nx, nr, nth, seed=seed, thermo_noise=1e-3)


def _geo(pb):
    return les.geometry(pb["xyz"].numpy(), pb["params"])


def _oracle_jv(pb, geo, v, vin=None):
    """Complex-step J v (state direction v, entrance-data direction vin)."""
    Qc = pb["Q"].numpy().astype(np.complex128) + 1j * H_CS * v
    infc = None
    if pb["inflow"] is not None:
        infc = pb["inflow"].numpy().astype(np.complex128)
        if vin is not None:
            infc = infc + 1j * H_CS * vin
    return np.imag(les.evaluate(Qc, geo, pb["params"], infc)) / H_CS


def _oracle_rk_jv(pb, geo, v, vin, dt):
    Qc = pb["Q"].numpy().astype(np.complex128) + 1j * H_CS * v
    infc = pb["inflow"].numpy().astype(np.complex128) + 1j * H_CS * vin
    return np.imag(les.rk5_step(Qc, geo, pb["params"], infc, dt=dt)[0]) / H_CS


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def test_vjp_dense_jacobian_tiny_jet():
    pb = _jet(8, 6, 8)
    announce("vjp dense jacobian 8x6x8 jet")
    geo = _geo(pb)
    Q = pb["Q"].numpy()
    n = Q.size
    nin = pb["inflow"].numel()
    J = np.empty((n, n))
    for c in range(n):
        v = np.zeros(n)
        v[c] = 1.0
        J[:, c] = _oracle_jv(pb, geo, v.reshape(Q.shape)).ravel()
    Jin = np.empty((n, nin))
    for c in range(nin):
        vin = np.zeros(nin)
        vin[c] = 1.0
        Jin[:, c] = _oracle_jv(pb, geo, np.zeros_like(Q), vin.reshape(pb["inflow"].shape)).ravel()
    s = make_solver(pb)
    Qp = s.pad(pb["Q"].cuda())
    Rb = s.field(5, dtype=torch.float64, fill=0.0)
    Rb_int = s.interior(Rb)
    Qb = s.field(5, dtype=torch.float64)
    G = torch.empty((n, n), dtype=torch.float64, device="cuda")
    Gin = torch.empty((n, nin), dtype=torch.float64, device="cuda")
    ib = s.new_inflow_bar()
    for r in range(n):
        Rb.zero_()
        Rb_int[tuple(int(x) for x in np.unravel_index(r, Q.shape))] = 1.0
        ib.zero_()
        s.residual_vjp(Qp, Rb, Qb, ib)
        G[r] = s.interior(Qb).reshape(-1)
        Gin[r] = ib.reshape(-1)
        if r == 0:
            ghost = Qb.clone()
            s.interior(ghost).zero_()
            assert float(ghost.abs().max()) == 0.0
    G = to_np(G)
    Gin = to_np(Gin)
    rowmax = np.maximum(np.abs(J).max(axis=1), np.abs(Jin).max(axis=1))
    err = np.abs(G - J).max(axis=1) / rowmax
    err_in = np.abs(Gin - Jin).max(axis=1) / rowmax
    print("dense J rows: max rel err state %.3e inflow %.3e" % (err.max(), err_in.max()))
    assert np.abs(Jin).max() > 0.0
    assert err.max() <= 1e-12
    assert err_in.max() <= 1e-12


@pytest.mark.parametrize("case", ["box16", "jet24x12x16", "box16_vreman", "jet24x12x16_vreman"])
def test_vjp_directional(case):
    if case.startswith("box16"):
        pb = problems.box_problem(16, seed=7, noise=1e-3)
    else:
        pb = _jet(24, 12, 16, seed=8)
    if case.endswith("vreman"):
        pb["params"] = dict(pb["params"], sgs_model=2)
    announce("vjp directional", case)
    geo = _geo(pb)
    Q = pb["Q"].numpy()
    Rbar = problems.seeded_field(Q.shape, 3, flow.FIELD_COTANGENT).numpy()
    s = make_solver(pb)
    Qp = s.pad(pb["Q"].cuda())
    Rb = s.pad(torch.from_numpy(Rbar).cuda(), fill=0.0)
    ib = s.new_inflow_bar() if pb["inflow"] is not None else None
    Qb = to_np(s.interior(s.residual_vjp(Qp, Rb, inflow_bar=ib)))
    for seed in (11, 12):
        v = problems.seeded_field(Q.shape, seed, flow.FIELD_DIRECTION).numpy()
        lhs = float(np.sum(Rbar * _oracle_jv(pb, geo, v)))
        rhs = float(np.sum(Qb * v))
        print(case, seed, lhs, rhs, _rel(rhs, lhs))
        assert _rel(rhs, lhs) <= 1e-11
    if ib is not None:
        vin = problems.seeded_field(tuple(pb["inflow"].shape), 13, flow.FIELD_DIRECTION_IN).numpy()
        lhs = float(np.sum(Rbar * _oracle_jv(pb, geo, np.zeros_like(Q), vin)))
        rhs = float(np.sum(to_np(ib) * vin))
        print(case, "inflow", lhs, rhs, _rel(rhs, lhs))
        assert _rel(rhs, lhs) <= 1e-11


THIN = {
    # the main pass works on 32 x 8 tiles of the padded plane (nx + 4 by
    # nr + 4): many tiles along one direction and a part of one along the
    # other, exactly one tile along xi with one row in a third tile along
    # eta, exactly two tiles along xi, and the smallest box (one partial
    # tile)
    "jet300x5x6": lambda: _jet(300, 5, 6, seed=21),
    "jet5x40x6": lambda: _jet(5, 40, 6, seed=22),
    "jet28x13x8": lambda: _jet(28, 13, 8, seed=23),
    "jet60x5x6": lambda: _jet(60, 5, 6, seed=25),
    "box5": lambda: problems.box_problem(5, seed=24, noise=1e-3),
}


@pytest.mark.parametrize("case", list(THIN))
def test_vjp_directional_thin_meshes(case):
    pb = THIN[case]()
    announce("vjp thin mesh", case)
    geo = _geo(pb)
    Q = pb["Q"].numpy()
    Rbar = problems.seeded_field(Q.shape, 3, flow.FIELD_COTANGENT).numpy()
    s = make_solver(pb)
    Qp = s.pad(pb["Q"].cuda())
    Rb = s.pad(torch.from_numpy(Rbar).cuda(), fill=0.0)
    ib = s.new_inflow_bar() if pb["inflow"] is not None else None
    Qb = to_np(s.interior(s.residual_vjp(Qp, Rb, inflow_bar=ib)))
    v = problems.seeded_field(Q.shape, 11, flow.FIELD_DIRECTION).numpy()
    vin = None
    if ib is not None:
        vin = problems.seeded_field(tuple(pb["inflow"].shape), 13, flow.FIELD_DIRECTION_IN).numpy()
    lhs = float(np.sum(Rbar * _oracle_jv(pb, geo, v, vin)))
    rhs = float(np.sum(Qb * v)) + (float(np.sum(to_np(ib) * vin)) if ib is not None else 0.0)
    print(case, lhs, rhs, _rel(rhs, lhs))
    assert _rel(rhs, lhs) <= 1e-11
    s.close()


def test_vjp_full_jet_mesh():
    """160x100x128 jet (2.05M points), seeded Gaussian cotangent: <Qbar, v>
    against the oracle's complex-step <Rbar, J v> (state and entrance-data
    directions together); Qbar's ghost entries are zero."""
    nx, nr, nth = problems.CONFIGS["adj2M"]["shape"]
    pb = problems.jet_problem(nx, nr, nth, seed=problems.CONFIGS["adj2M"]["seed"],
                              thermo_noise=1e-3)
    announce("vjp full mesh", nx, nr, nth)
    geo = _geo(pb)
    Q = pb["Q"].numpy()
    Rbar = problems.seeded_field(Q.shape, 4, flow.FIELD_COTANGENT).numpy()
    v = problems.seeded_field(Q.shape, 14, flow.FIELD_DIRECTION).numpy()
    vin = problems.seeded_field(tuple(pb["inflow"].shape), 15, flow.FIELD_DIRECTION_IN).numpy()
    s = make_solver(pb)
    Qp = s.pad(pb["Q"].cuda())
    Rb = s.pad(torch.from_numpy(Rbar).cuda(), fill=0.0)
    ib = s.new_inflow_bar()
    Qb = s.residual_vjp(Qp, Rb, inflow_bar=ib)
    rhs = float(torch.sum(s.interior(Qb) * torch.from_numpy(v).cuda()))
    rhs += float(torch.sum(ib * torch.from_numpy(vin).cuda()))
    lhs = float(np.sum(Rbar * _oracle_jv(pb, geo, v, vin)))
    print("full mesh", lhs, rhs, _rel(rhs, lhs))
    assert _rel(rhs, lhs) <= 1e-10
    ghost = Qb.clone()
    s.interior(ghost).zero_()
    assert float(ghost.abs().max()) == 0.0


def test_vjp_matches_forward_differences():
    """Dot-product test against central differences of the GPU's own
    residual: <Rbar, (R(Q + h v) - R(Q - h v)) / 2h> = <Qbar, v>."""
    pb = _jet(24, 12, 16, seed=9)
    announce("vjp vs forward central differences 24x12x16")
    Q = pb["Q"].cuda()
    s = make_solver(pb)
    Rbar = problems.seeded_field(tuple(Q.shape), 5, flow.FIELD_COTANGENT).cuda()
    v = problems.seeded_field(tuple(Q.shape), 16, flow.FIELD_DIRECTION).cuda()
    v = v * Q.abs().reshape(5, -1).amax(dim=1).view(5, 1, 1, 1)
    Qb = s.residual_vjp(s.pad(Q), s.pad(Rbar, fill=0.0))
    rhs = float(torch.sum(s.interior(Qb) * v))
    best = None
    for h in (1e-6, 1e-7, 1e-8):
        Rp = s.interior(s.residual(s.pad(Q + h * v)))
        Rm = s.interior(s.residual(s.pad(Q - h * v)))
        lhs = float(torch.sum(Rbar * (Rp - Rm))) / (2.0 * h)
        e = _rel(rhs, lhs)
        print("h", h, lhs, rhs, e)
        best = e if best is None else min(best, e)
    assert best <= 1e-6


def test_rk5_step_vjp():
    pb = _jet(12, 8, 8, seed=10)
    announce("rk5 step vjp 12x8x8 jet")
    geo = _geo(pb)
    Q = pb["Q"].numpy()
    dt = 2e-3
    s = make_solver(pb)
    Qn = s.pad(pb["Q"].cuda())
    Qn0 = Qn.clone()
    Bn1 = problems.seeded_field(Q.shape, 6, flow.FIELD_COTANGENT).numpy()
    Bp = s.pad(torch.from_numpy(Bn1).cuda(), fill=7.0)   # ghosts must be ignored
    ib = s.new_inflow_bar()
    Bn = s.rk5_step_vjp(Qn, dt, Bp, inflow_bar=ib)
    assert torch.equal(s.interior(Qn), s.interior(Qn0))
    ghost = Bn.clone()
    s.interior(ghost).zero_()
    assert float(ghost.abs().max()) == 0.0
    Bn_np, ib_np = to_np(s.interior(Bn)), to_np(ib)
    for seed in (17, 18, 19):
        v = problems.seeded_field(Q.shape, seed, flow.FIELD_DIRECTION).numpy()
        vin = problems.seeded_field(tuple(pb["inflow"].shape), seed, flow.FIELD_DIRECTION_IN).numpy()
        lhs = float(np.sum(Bn1 * _oracle_rk_jv(pb, geo, v, vin, dt)))
        rhs = float(np.sum(Bn_np * v) + np.sum(ib_np * vin))
        print("rk5 vjp", seed, lhs, rhs, _rel(rhs, lhs))
        assert _rel(rhs, lhs) <= 1e-11
    # in place (Qbar_n aliases Qbar_np1) gives the same bits
    ib2 = s.new_inflow_bar()
    s.rk5_step_vjp(Qn, dt, Bp, Bp, inflow_bar=ib2)
    assert torch.equal(s.interior(Bp), s.interior(Bn))
    assert torch.equal(ib2, ib)


def test_vjp_bitwise_reproducible_and_fp32_refused():
    pb = _jet(24, 12, 16, seed=8)
    announce("vjp reproducibility")
    s = make_solver(pb)
    Qp = s.pad(pb["Q"].cuda())
    Rb = s.pad(problems.seeded_field(tuple(pb["Q"].shape), 3, flow.FIELD_COTANGENT).cuda(),
               fill=0.0)
    a = s.residual_vjp(Qp, Rb).clone()
    b = s.residual_vjp(Qp, Rb).clone()
    assert torch.equal(a, b)
    # Rbar and Qbar may alias
    s.residual_vjp(Qp, Rb, Rb)
    assert torch.equal(Rb, a)
    from paper_2301_00817_amd import binding as B
    s32 = make_solver(pb, precision="fp32")
    Q32 = s32.pad(pb["Q"].cuda(), dtype=torch.float64)
    with pytest.raises(B.LesError) as ei:
        s32.residual_vjp(Q32, a)
    assert ei.value.code == B.LES_EUNSUPPORTED


def test_vjp_and_step_with_poisoned_buffers(monkeypatch):
    """Every library buffer starts as NaN (LESJET_POISON=1): the residual,
    an RK5 step and both adjoints still match their values in a context
    whose buffers start as the allocator left them, bit for bit — no pass
    reads memory another pass has not written."""
    pb = _jet(24, 12, 16, seed=8)
    announce("poisoned buffers")
    Q = pb["Q"].cuda()
    Rb = problems.seeded_field(tuple(Q.shape), 3, flow.FIELD_COTANGENT).cuda()
    out = []
    for poison in ("0", "1"):
        monkeypatch.setenv("LESJET_POISON", poison)
        s = make_solver(pb)
        Qp = s.pad(Q)
        R = s.residual(Qp, s.field(5, fill=0.0)).clone()
        ib = s.new_inflow_bar()
        Qb = s.residual_vjp(Qp, s.pad(Rb, fill=0.0), inflow_bar=ib).clone()
        ib2 = s.new_inflow_bar()
        Qb2 = s.rk5_step_vjp(Qp, 1e-4, s.pad(Rb, fill=0.0), inflow_bar=ib2).clone()
        Q1 = s.pad(Q)
        s.rk5_step(Q1, 2)
        out.append([s.interior(R), s.interior(Qb), ib, s.interior(Qb2), ib2, s.interior(Q1)])
        s.close()
    for a, b in zip(*out):
        assert bool(torch.isfinite(b).all())
        assert torch.equal(a, b)
