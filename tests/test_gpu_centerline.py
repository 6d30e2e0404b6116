"""GPU parity of the centerline condition on meshes whose first row lies on
the axis (subsection "Centerline Boundary Condition"), against the oracle:
metrics, ghost fill (axis row = azimuthal mean of row 1, mirror ghosts),
residual (fused and two-pass kernels), time step, RK5 steps and the FP32
storage form, on meshes spanning several tiles with ragged tails.

Bars as for the other FP64 parity tests (residual 1e-12, state 1e-11 per
group), the FP32 form as in its own tests (residual 1e-3, state 1e-5).  The
axis row of a stepped state is derived data: the oracle leaves it as given
(R = 0 there), the solver returns the azimuthal mean of the returned row 1,
so steps are compared on rows j >= 1 and the axis row is checked against
that mean.  The adjoint entry points are checked against the oracle's
complex-step derivatives (dense Jacobian on the smallest case, directional
products, one RK5 step)."""
import numpy as np
import pytest
import torch

from _helpers import announce, grouped_rel_err, make_solver, to_np
from cases import flow, problems
from oracle import les

pytestmark = pytest.mark.gpu

R_BAR = 1e-12
Q_BAR = 1e-11


def _pb(nx, nr, nth, seed=5, perturb=0.02):
    pb = problems.jet_problem(nx, nr, nth, seed=seed, axis_node=True, thermo_noise=1e-2)
    Q = pb["Q"].clone()
    g = torch.Generator().manual_seed(seed)
    Q[1:4] += perturb * torch.randn(Q[1:4].shape, generator=g, dtype=torch.float64)
    pb["Q"] = Q
    return pb


SHAPES = {"axis37x22x20": (37, 22, 20), "axis20x9x16": (20, 9, 16), "axis8x6x8": (8, 6, 8)}


def _oracle(pb):
    geo = les.geometry(pb["xyz"].numpy(), pb["params"])
    return geo, pb["inflow"].numpy()


def _axis_mean_ok(Q):
    """Every axis point holds the azimuthal mean of row 1 (per i)."""
    mean = Q[:, :, 1, :].mean(axis=1)
    for k in range(Q.shape[1]):
        assert np.abs(Q[:, k, 0, :] - mean).max() <= 1e-14 * np.abs(mean).max()


def test_metrics_vanish_on_the_axis_and_match_oracle():
    announce("centerline-metrics", "axis37x22x20")
    pb = _pb(*SHAPES["axis37x22x20"])
    geo, _ = _oracle(pb)
    s = make_solver(pb, keep_metrics=True)
    M = to_np(s.metrics64)[..., :s.shape[0] + 4]
    S = geo["S"].reshape(9, *geo["V"].shape)
    assert np.abs(M[:9] - S).max() <= 1e-14 * np.abs(S).max()
    assert np.abs(M[9] - geo["V"]).max() <= 1e-14 * np.abs(geo["V"]).max()
    g = les.NG
    assert np.all(M[9][g:-g, g, g:-g] == 0.0)
    s.close()


@pytest.mark.parametrize("name", ["axis37x22x20", "axis8x6x8"])
def test_ghost_fill_matches_oracle(name):
    announce("centerline-ghosts", name)
    pb = _pb(*SHAPES[name])
    geo, inflow = _oracle(pb)
    Qp = les.pad_state(pb["Q"].numpy())
    les.fill_ghosts(Qp, geo, pb["params"], inflow)
    s = make_solver(pb)
    G = s.pad(pb["Q"].cuda())
    s.fill_ghosts(G)
    torch.cuda.synchronize()
    Gn = to_np(G)[..., :s.shape[0] + 4]
    assert np.isfinite(Gn).all()
    assert grouped_rel_err(Gn, Qp) <= 1e-14
    _axis_mean_ok(les.interior(Gn))
    s.close()


@pytest.mark.parametrize("name", list(SHAPES))
def test_residual_matches_oracle(name):
    announce("centerline-residual", name)
    pb = _pb(*SHAPES[name])
    geo, inflow = _oracle(pb)
    R_ref = les.evaluate(pb["Q"].numpy(), geo, pb["params"], inflow)
    assert np.isfinite(R_ref).all()
    s = make_solver(pb)
    R = to_np(s.interior(s.residual(s.pad(pb["Q"].cuda()))))
    R2 = to_np(s.interior(s.residual_reference(s.pad(pb["Q"].cuda()))))
    assert np.isfinite(R).all() and np.isfinite(R2).all()
    assert np.all(R[:, :, 0, :] == 0.0) and np.all(R2[:, :, 0, :] == 0.0)
    e1, e2 = grouped_rel_err(R, R_ref), grouped_rel_err(R2, R_ref)
    print(f"{name}: fused {e1:.3e}, two-pass {e2:.3e}")
    assert e1 <= R_BAR and e2 <= R_BAR
    s.close()


@pytest.mark.parametrize("kchunk", [1, 3])
def test_residual_chunk_boundaries(kchunk, monkeypatch):
    announce("centerline-chunk", kchunk)
    monkeypatch.setenv("LESJET_KCHUNK", str(kchunk))
    pb = _pb(*SHAPES["axis37x22x20"])
    geo, inflow = _oracle(pb)
    R_ref = les.evaluate(pb["Q"].numpy(), geo, pb["params"], inflow)
    s = make_solver(pb)
    R = to_np(s.interior(s.residual(s.pad(pb["Q"].cuda()))))
    assert grouped_rel_err(R, R_ref) <= R_BAR
    s.close()


@pytest.mark.parametrize("name,steps", [("axis37x22x20", 5), ("axis8x6x8", 3)])
def test_rk5_steps_match_oracle(name, steps):
    announce("centerline-rk5", name, steps)
    pb = _pb(*SHAPES[name])
    geo, inflow = _oracle(pb)
    Q_ref, dts = les.run(pb["Q"].numpy(), geo, pb["params"], inflow, steps=steps)
    s = make_solver(pb)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    dt = to_np(s.rk5_step(Qn, steps))
    Q = to_np(s.interior(Qn))
    assert np.allclose(dt, dts, rtol=1e-12, atol=0)
    err = grouped_rel_err(Q[:, :, 1:, :], Q_ref[:, :, 1:, :])
    print(f"{name}: Q after {steps} steps rel err {err:.3e}")
    assert err <= Q_BAR
    _axis_mean_ok(Q)
    s.close()


def test_fp32_storage_residual_and_steps():
    announce("centerline-fp32", "axis37x22x20")
    pb = _pb(*SHAPES["axis37x22x20"])
    geo, inflow = _oracle(pb)
    R_ref = les.evaluate(pb["Q"].numpy(), geo, pb["params"], inflow)
    Q_ref, _ = les.run(pb["Q"].numpy(), geo, pb["params"], inflow, steps=4)
    s = make_solver(pb, precision="fp32")
    R = to_np(s.interior(s.residual(s.pad(pb["Q"].cuda().float())))).astype(np.float64)
    assert np.isfinite(R).all() and np.all(R[:, :, 0, :] == 0.0)
    er = grouped_rel_err(R, R_ref)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    s.rk5_step(Qn, 4)
    Q = to_np(s.interior(Qn))
    eq = grouped_rel_err(Q[:, :, 1:, :], Q_ref[:, :, 1:, :])
    print(f"FP32 axis: residual {er:.3e}, state after 4 steps {eq:.3e}")
    assert er <= 1e-3 and eq <= 1e-5
    _axis_mean_ok(Q)
    s.close()


def test_free_stream_on_full_size_axis_mesh():
    """288 x 160 x 128 mesh with nodes on the axis, uniform state equal to the
    boundary data: R stays at rounding level on every advanced point."""
    announce("centerline-free-stream", "axis288x160x128")
    prim = (1.0, 0.6, 0.3, -0.2, 1.0 / 1.4)
    pb = problems.jet_problem(288, 160, 128, noise=0.0, axis_node=True)
    pb["params"] = dict(pb["params"], ref_prim=prim, p_exit=prim[4])
    pb["inflow"] = torch.tensor(prim, dtype=torch.float64).view(5, 1, 1).expand(5, 128, 160).contiguous()
    Q = flow.uniform_state((128, 160, 288), prim)
    s = make_solver(pb, keep_metrics=True)
    R = s.interior(s.residual(s.pad(Q.cuda())))
    V = s.interior(s.metrics64[9:10])
    VR = float((R * V).abs().max())
    Smax = float(s.interior(s.metrics64[:9]).abs().max())
    fscale = Smax * (prim[0] * 0.6 ** 2 + prim[4])
    assert torch.isfinite(R).all()
    assert VR <= 1e-12 * fscale
    s.close()


# ---- adjoint ------------------------------------------------------------
# Derivatives against the oracle's complex step on states with relative rho
# and p noise (no pressure sensor at its kink).  The residual does not depend
# on the input's axis row (it is replaced by the mean of row 1), so the GPU
# returns a zero cotangent there and the oracle a zero derivative.

H_CS = 1e-30


def _adj_pb(nx, nr, nth, seed):
    return problems.jet_problem(nx, nr, nth, seed=seed, thermo_noise=1e-3, axis_node=True)


def _cs_jv(pb, geo, v, vin=None):
    Qc = pb["Q"].numpy().astype(np.complex128) + 1j * H_CS * v
    infc = pb["inflow"].numpy().astype(np.complex128)
    if vin is not None:
        infc = infc + 1j * H_CS * vin
    with np.errstate(all="ignore"):
        return np.imag(les.evaluate(Qc, geo, pb["params"], infc)) / H_CS


def test_vjp_dense_jacobian_tiny_axis_mesh():
    """Every row of dR/dQ and dR/d(inflow data) on the 8 x 6 x 8 axis-node
    jet against the complex-step Jacobian, per row <= 1e-12."""
    announce("centerline-vjp-dense", "axis8x6x8")
    pb = _adj_pb(8, 6, 8, seed=6)
    geo, _ = _oracle(pb)
    Q = pb["Q"].numpy()
    n, nin = Q.size, pb["inflow"].numel()
    J = np.empty((n, n))
    for c in range(n):
        v = np.zeros(n)
        v[c] = 1.0
        J[:, c] = _cs_jv(pb, geo, v.reshape(Q.shape)).ravel()
    Jin = np.empty((n, nin))
    for c in range(nin):
        vin = np.zeros(nin)
        vin[c] = 1.0
        Jin[:, c] = _cs_jv(pb, geo, np.zeros_like(Q), vin.reshape(pb["inflow"].shape)).ravel()
    assert np.all(J.reshape(Q.shape + Q.shape)[..., :, :, 0, :] == 0.0)   # axis row of Q: no effect
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
    G, Gin = to_np(G), to_np(Gin)
    rowmax = np.maximum(np.abs(J).max(axis=1), np.abs(Jin).max(axis=1))
    live = rowmax > 0.0                                   # rows of the axis row are zero
    err = np.abs(G - J).max(axis=1)[live] / rowmax[live]
    err_in = np.abs(Gin - Jin).max(axis=1)[live] / rowmax[live]
    print("axis dense J rows: max rel err state %.3e inflow %.3e" % (err.max(), err_in.max()))
    assert np.all(G[~live] == 0.0) and np.all(Gin[~live] == 0.0)
    assert err.max() <= 1e-12 and err_in.max() <= 1e-12
    s.close()


@pytest.mark.parametrize("shape,seed", [((20, 9, 16), 7), ((37, 22, 20), 8)])
def test_vjp_directional_axis_mesh(shape, seed):
    announce("centerline-vjp-directional", shape)
    pb = _adj_pb(*shape, seed=seed)
    geo, _ = _oracle(pb)
    Q = pb["Q"].numpy()
    Rbar = problems.seeded_field(Q.shape, 3, flow.FIELD_COTANGENT).numpy()
    s = make_solver(pb)
    Qp = s.pad(pb["Q"].cuda())
    Rb = s.pad(torch.from_numpy(Rbar).cuda(), fill=0.0)
    ib = s.new_inflow_bar()
    Qb_full = s.residual_vjp(Qp, Rb, inflow_bar=ib)
    Qb = to_np(s.interior(Qb_full))
    assert np.all(Qb[:, :, 0, :] == 0.0)
    ghost = Qb_full.clone()
    s.interior(ghost).zero_()
    assert float(ghost.abs().max()) == 0.0
    v = problems.seeded_field(Q.shape, 11, flow.FIELD_DIRECTION).numpy()
    vin = problems.seeded_field(tuple(pb["inflow"].shape), 13, flow.FIELD_DIRECTION_IN).numpy()
    lhs = float(np.sum(Rbar * _cs_jv(pb, geo, v)))
    rhs = float(np.sum(Qb * v))
    lhs_in = float(np.sum(Rbar * _cs_jv(pb, geo, np.zeros_like(Q), vin)))
    rhs_in = float(np.sum(to_np(ib) * vin))
    e, e_in = abs(rhs - lhs) / abs(lhs), abs(rhs_in - lhs_in) / abs(lhs_in)
    print(f"{shape}: state {e:.3e}, inflow {e_in:.3e}")
    assert e <= 1e-11 and e_in <= 1e-11
    s.close()


def test_rk5_step_vjp_axis_mesh():
    """One step with a fixed dt: <Qbar_n, v> against <Qbar_np1, J v> of the
    oracle's step, cotangent and direction zero on the axis row (the oracle
    returns the input's axis row, the solver the mean of the returned row 1;
    on the other rows the two steps are the same map)."""
    announce("centerline-rk5-vjp", "axis12x8x8")
    pb = _adj_pb(12, 8, 8, seed=9)
    geo, _ = _oracle(pb)
    Q = pb["Q"].numpy()
    dt = 2e-3
    Qb1 = problems.seeded_field(Q.shape, 6, flow.FIELD_COTANGENT).numpy()
    Qb1[:, :, 0, :] = 0.0
    v = problems.seeded_field(Q.shape, 17, flow.FIELD_DIRECTION).numpy()
    v[:, :, 0, :] = 0.0
    vin = problems.seeded_field(tuple(pb["inflow"].shape), 18, flow.FIELD_DIRECTION_IN).numpy()
    Qc = Q.astype(np.complex128) + 1j * H_CS * v
    infc = pb["inflow"].numpy().astype(np.complex128) + 1j * H_CS * vin
    with np.errstate(all="ignore"):
        Jv = np.imag(les.rk5_step(Qc, geo, pb["params"], infc, dt=dt)[0]) / H_CS
    lhs = float(np.sum(Qb1 * Jv))
    s = make_solver(pb)
    Qn = s.pad(pb["Q"].cuda())
    ib = s.new_inflow_bar()
    Qbn = s.rk5_step_vjp(Qn, dt, s.pad(torch.from_numpy(Qb1).cuda(), fill=0.0), inflow_bar=ib)
    rhs = float(np.sum(to_np(s.interior(Qbn)) * v)) + float(np.sum(to_np(ib) * vin))
    e = abs(rhs - lhs) / abs(lhs)
    print(f"axis step vjp: {lhs} {rhs} {e:.3e}")
    assert e <= 1e-11
    s.close()
