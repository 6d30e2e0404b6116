"""GPU parity of the plain FP64 path against the CPU oracle, through the
C-ABI: metrics, ghost fill, residual, time step and RK5 steps, on grids that
span several tiles with ragged tails, plus properties at full size.

Bars (FP64; the norms are described in _helpers): metrics and copied ghosts
agree to rounding (1e-14 relative); the residual to 1e-13 of its flux scale
per variable (the face fluxes whose differences form it: rounding of a
difference is bounded relative to the terms, not to the difference) and to
1e-12 of its max (momentum over the vector's magnitude); the state after
10 RK5 steps to 1e-11 per variable, after 100 steps (the jet workload's run
length, on a mesh the oracle steps in seconds) to 1e-10: rounding
differences grow at most linearly with the number of steps.  The GPU
contracts multiply-adds and uses reciprocal multiplies where the oracle
divides, so agreement is to a few ulps of the flux scale.  Every test
prints the per-variable errors (relative to each variable's own max)."""
import math

import numpy as np
import pytest
import torch

from _helpers import (announce, flux_err, flux_scale, grouped_rel_err, make_solver,
                      per_variable_err, report, to_np, vector_err)
from cases import problems
from oracle import les

pytestmark = pytest.mark.gpu

R_BAR = 1e-12          # vector norm (P1) of the residual
R_FLUX_BAR = 1e-13     # residual over its flux scale (P2), per variable
Q_BAR = 1e-11          # per variable
Q_BAR_100 = 1e-10


def check_residual(label, R, R_ref, Q, geo, prm, inflow):
    """Assert the FP64 residual bars; print all three norms."""
    pv = per_variable_err(R, R_ref)
    vn = vector_err(R, R_ref)
    fx = flux_err(R, R_ref, flux_scale(Q, geo, prm, inflow))
    report(label + " residual", per_variable=pv, vector=vn, flux=fx)
    assert np.isfinite(R).all()
    assert fx.max() <= R_FLUX_BAR
    assert vn.max() <= R_BAR


def _oracle(pb):
    xyz = pb["xyz"].numpy()
    geo = les.geometry(xyz, pb["params"])
    inflow = pb["inflow"].numpy() if pb.get("inflow") is not None else None
    return geo, inflow


def _jet(nx, nr, nth, perturb=0.0, seed=2):
    pb = problems.jet_problem(nx, nr, nth, seed=seed)
    if perturb:
        Q = pb["Q"].clone()
        g = torch.Generator().manual_seed(7)
        Q[1:4] += perturb * torch.randn(Q[1:4].shape, generator=g, dtype=torch.float64)
        pb["Q"] = Q
    return pb


def _with(pb, **over):
    pb = dict(pb)
    pb["params"] = dict(pb["params"], **over)
    return pb


CASES = {
    "box32": lambda: problems.box_problem(32),
    "box_inviscid": lambda: _with(problems.box_problem(24), visc_coef=0.0, sgs_model=0),
    "jet37x22x20_nosgs": lambda: _with(_jet(37, 22, 20), sgs_model=0),
    "box32_vreman": lambda: _with(problems.box_problem(32), sgs_model=2),
    "jet37x22x20_vreman": lambda: _with(_jet(37, 22, 20, perturb=0.01), sgs_model=2),
    "box32_cs018": lambda: problems.box_problem(32, Cs=0.18),
    "box_ragged": lambda: problems.box_problem(17, shape=(17, 23, 9)),
    "jet8x6x8": lambda: _jet(8, 6, 8, perturb=0.05),
    "jet37x22x20": lambda: _jet(37, 22, 20),
    "jet70x33x24": lambda: _jet(70, 33, 24, perturb=0.01),
}


@pytest.mark.parametrize("name", ["box32", "jet37x22x20", "jet70x33x24"])
def test_metrics_match_oracle(name):
    announce("metrics", name)
    pb = CASES[name]()
    geo, _ = _oracle(pb)
    s = make_solver(pb, keep_metrics=True)
    M = to_np(s.metrics64)[..., :s.shape[0] + 4]
    S = geo["S"].reshape(9, *geo["V"].shape)
    assert np.abs(M[:9] - S).max() <= 1e-14 * np.abs(S).max()
    assert np.abs(M[9] - geo["V"]).max() <= 1e-14 * np.abs(geo["V"]).max()
    s.close()


@pytest.mark.parametrize("name", ["box_ragged", "jet8x6x8", "jet37x22x20"])
def test_ghost_fill_matches_oracle_and_defines_every_point(name):
    """Ghosts poisoned with NaN before the fill: every padded point must be
    finite afterwards; copies bitwise, Riemann states to rounding."""
    announce("ghosts", name)
    pb = CASES[name]()
    geo, inflow = _oracle(pb)
    Qp = les.pad_state(pb["Q"].numpy())
    les.fill_ghosts(Qp, geo, pb["params"], inflow)
    s = make_solver(pb)
    G = s.pad(pb["Q"].cuda())
    s.fill_ghosts(G)
    torch.cuda.synchronize()
    Gn = to_np(G)[..., :s.shape[0] + 4]
    assert np.isfinite(Gn).all()
    assert grouped_rel_err(Gn, Qp, label=f"{name} ghosts") <= 1e-14
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_residual_matches_oracle(name):
    announce("residual", name)
    pb = CASES[name]()
    geo, inflow = _oracle(pb)
    R_ref = les.evaluate(pb["Q"].numpy(), geo, pb["params"], inflow)
    s = make_solver(pb)
    Qp = s.pad(pb["Q"].cuda())
    R = to_np(s.interior(s.residual(Qp)))
    check_residual(name, R, R_ref, pb["Q"].numpy(), geo, pb["params"], inflow)
    s.close()


def test_time_step_matches_oracle():
    announce("dt", "jet37x22x20")
    pb = CASES["jet37x22x20"]()
    geo, inflow = _oracle(pb)
    dt_ref = les.time_step(pb["Q"].numpy(), geo, pb["params"])
    s = make_solver(pb)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    dt = float(s.rk5_step(Qn, 1)[0])
    assert abs(dt - dt_ref) <= 1e-14 * dt_ref
    s.close()


@pytest.mark.parametrize("name,steps", [("box32", 10), ("jet37x22x20", 10), ("jet8x6x8", 4),
                                        ("jet37x22x20", 100)])
def test_rk5_steps_match_oracle(name, steps):
    announce("rk5", name, steps)
    pb = CASES[name]()
    geo, inflow = _oracle(pb)
    Q_ref, dts = les.run(pb["Q"].numpy(), geo, pb["params"], inflow, steps=steps)
    s = make_solver(pb)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    dt = to_np(s.rk5_step(Qn, steps))
    Q = to_np(s.interior(Qn))
    assert np.allclose(dt, dts, rtol=1e-12, atol=0)
    pv = per_variable_err(Q, Q_ref)
    report(f"{name} Q after {steps} steps", per_variable=pv, vector=vector_err(Q, Q_ref))
    assert pv.max() <= (Q_BAR if steps <= 10 else Q_BAR_100)
    s.close()


def test_rk5_fixed_dt_and_reproducible():
    """Fixed dt is used as given; two runs from the same state are bitwise
    equal (no atomics on floats, fixed summation order)."""
    announce("rk5-repro", "jet37x22x20")
    pb = CASES["jet37x22x20"]()
    s = make_solver(pb)
    out = []
    for _ in range(2):
        Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
        dt = s.rk5_step(Qn, 3, dt=1e-4)
        out.append(to_np(s.interior(Qn)))
    assert np.all(to_np(dt) == 1e-4)
    assert np.array_equal(out[0], out[1])
    s.close()


def test_residual_2M_jet_matches_oracle():
    """The 160 x 100 x 128 jet mesh (2.05 M points), full comparison."""
    announce("residual", "jet160x100x128")
    pb = problems.jet_problem(160, 100, 128, seed=4)
    geo, inflow = _oracle(pb)
    R_ref = les.evaluate(pb["Q"].numpy(), geo, pb["params"], inflow)
    s = make_solver(pb)
    Qp = s.pad(pb["Q"].cuda())
    R = to_np(s.interior(s.residual(Qp)))
    check_residual("jet160x100x128", R, R_ref, pb["Q"].numpy(), geo, pb["params"], inflow)
    s.close()


def test_free_stream_on_5p9M_jet_mesh():
    """Full-size 288 x 160 x 128 mesh: a uniform state (boundary data equal
    to it) keeps a residual at rounding level, max |V R| / max |F| <= 1e-12."""
    announce("free-stream", "jet288x160x128")
    prim = (1.0, 0.6, 0.3, -0.2, 1.0 / 1.4)
    pb = problems.jet_problem(288, 160, 128, noise=0.0)
    pb["params"] = dict(pb["params"], ref_prim=prim, p_exit=prim[4])
    pb["inflow"] = torch.tensor(prim, dtype=torch.float64).view(5, 1, 1).expand(5, 128, 160).contiguous()
    from cases import flow
    Q = flow.uniform_state((128, 160, 288), prim)
    s = make_solver(pb, keep_metrics=True)
    Qp = s.pad(Q.cuda())
    R = s.interior(s.residual(Qp))
    V = s.interior(s.metrics64[9:10])
    VR = float((R * V).abs().max())
    Smax = float(s.interior(s.metrics64[:9]).abs().max())
    fscale = Smax * (prim[0] * 0.6 ** 2 + prim[4])
    assert VR <= 1e-12 * fscale
    s.close()


@pytest.mark.parametrize("kchunk", [1, 3, 7, 64])
def test_residual_chunk_boundaries(kchunk, monkeypatch):
    """The fused kernel marches over azimuthal chunks; every chunk length
    (including 1 and one longer than the mesh) gives the oracle's residual."""
    announce("residual-chunk", kchunk)
    monkeypatch.setenv("LESJET_KCHUNK", str(kchunk))
    pb = CASES["jet37x22x20"]()
    geo, inflow = _oracle(pb)
    R_ref = les.evaluate(pb["Q"].numpy(), geo, pb["params"], inflow)
    s = make_solver(pb)
    R = to_np(s.interior(s.residual(s.pad(pb["Q"].cuda()))))
    check_residual(f"jet37x22x20 kchunk {kchunk}", R, R_ref, pb["Q"].numpy(), geo, pb["params"],
                   inflow)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rk5_steps_chunk_boundaries(precision, monkeypatch):
    """Two RK5 steps under chunk lengths of 1, 3 and 7 planes.  The last
    stage of a step takes each output plane's metric terms for the next
    step's CFL sum from the previous plane of its chunk, so where chunks
    start must not change the time steps beyond rounding (taking a
    neighbouring plane's terms would change them by percents): they equal
    those of the automatic chunking to 1e-13 (FP64; FP32 form 1e-6), the
    states to 1e-14 (1e-6) of their maximum, and the time steps are the
    oracle's (FP64 1e-12; the FP32 form's, from FP32 metrics, 1e-5).  A
    chunk's first planes are formed by its prologue, compiled apart from
    the march, so they may round differently by an ulp."""
    announce("rk5-chunk", precision)
    pb = CASES["jet37x22x20"]()
    geo, inflow = _oracle(pb)
    _, dts = les.run(pb["Q"].numpy(), geo, pb["params"], inflow, steps=2)
    out = []
    for kchunk in (None, 1, 3, 7):
        if kchunk is None:
            monkeypatch.delenv("LESJET_KCHUNK", raising=False)
        else:
            monkeypatch.setenv("LESJET_KCHUNK", str(kchunk))
        s = make_solver(pb, precision=precision)
        Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
        dt = to_np(s.rk5_step(Qn, 2))
        out.append((kchunk, dt, to_np(s.interior(Qn))))
        s.close()
    dt_bar, q_bar = (1e-13, 1e-14) if precision == "fp64" else (1e-6, 1e-6)
    for kchunk, dt, Q in out[1:]:
        ddt = np.abs(dt / out[0][1] - 1).max()
        dq = np.abs(Q - out[0][2]).max() / np.abs(out[0][2]).max()
        print(f"{precision} kchunk {kchunk}: dt rel {ddt:.2e}, state rel {dq:.2e}")
        assert ddt <= dt_bar
        assert dq <= q_bar
    assert np.abs(out[0][1] / np.asarray(dts) - 1).max() <= (1e-12 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("shape", [(288, 160, 128), (401, 97, 64)])
def test_fused_matches_two_pass_reference(shape):
    """Consistency of the fused kernel with the two-pass reference kernels on
    full-size and ragged jet meshes.  Both are GPU code sharing the point and
    face formulas, so this is not parity evidence (the sampled oracle
    comparisons at these sizes are): it checks the tiling, the march and the
    halo handling of the fused kernel against plain indexing, to 1e-13 (the
    two are compiled with different multiply-add contraction)."""
    announce("fused-vs-ref", shape)
    pb = problems.jet_problem(*shape, seed=2)
    s = make_solver(pb)
    Qp = s.pad(pb["Q"].cuda())
    R1 = s.interior(s.residual(Qp)).clone()
    R2 = s.interior(s.residual_reference(Qp))
    torch.cuda.synchronize()
    err = grouped_rel_err(to_np(R1), to_np(R2), label=f"fused vs two-pass {shape}")
    print(f"{shape}: fused vs reference {err:.3e}")
    assert err <= 1e-13
    s.close()


def test_diagnostics_conservation_and_stats():
    """Totals of J^-1 Q match the oracle's sums and stay constant over RK5
    steps on the periodic box (telescoping fluxes); azimuthal sums match
    NumPy; two runs are bitwise identical."""
    announce("diagnostics", "box32")
    pb = problems.box_problem(32)
    geo, _ = _oracle(pb)
    Q = pb["Q"].numpy()
    V = les.interior(geo["V"])
    ref = [math.fsum((V * Q[c]).ravel()) for c in range(5)]
    s = make_solver(pb)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    st = s.new_stats()
    t0 = to_np(s.diagnostics(Qn, st))
    t0b = to_np(s.diagnostics(Qn))
    assert np.array_equal(t0, t0b)
    for c in range(5):
        assert abs(t0[c] - ref[c]) <= 1e-13 * max(abs(ref[c]), abs(ref[1]))
    rho, u, v, w, p = les.primitives(Q, 1.4)
    for c, f in enumerate((rho, u, v, w, p)):
        assert np.allclose(to_np(st[0][c]), f.sum(axis=0), rtol=1e-13, atol=1e-13)
        assert np.allclose(to_np(st[1][c]), (f * f).sum(axis=0), rtol=1e-13, atol=1e-13)
    s.rk5_step(Qn, 5)
    t1 = to_np(s.diagnostics(Qn))
    for c in range(5):
        assert abs(t1[c] - t0[c]) <= 1e-13 * max(abs(t0[c]), abs(t0[1]))
    s.close()
