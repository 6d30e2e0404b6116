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
that mean."""
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


def test_adjoint_is_refused():
    from paper_2301_00817_amd import binding as B
    announce("centerline-adjoint-refused")
    pb = _pb(*SHAPES["axis8x6x8"])
    s = make_solver(pb)
    Qp = s.pad(pb["Q"].cuda())
    with pytest.raises(B.LesError) as e:
        s.residual_vjp(Qp, torch.zeros_like(Qp))
    assert e.value.code == B.LES_EUNSUPPORTED
    s.close()
