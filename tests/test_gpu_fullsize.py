"""Parity at the measured sizes, in the configuration bench.py times (the
same workload generator — the mesh built by the library from its 1-D maps —
precision and launch shapes), on sampled outputs: the 288 x 160 x 128 jet,
the paper's mesh A shape 128 x 128 x 360 (no SGS model, as in the paper's
runs; 24-plane FP64 chunks) and the 1250 x 640 x 1250 jet.

The residual at an interior point depends only on the state and coordinates
within two points of it (point quantities at the neighbours need their
central differences, faces need W two points out); after one RK5 step the
state at a point depends on the initial data within ten points.  So the
oracle, run on a small block cut out around a sampled point (any boundary
kind: its ghosts never reach the centre), gives the exact full-mesh value
there.  The block's coordinates are formed on the host from the same 1-D
maps and the same C-library angle functions the library uses, so they are
the library's coordinates bitwise.  Points are sampled at least the block
half-width away from the physical boundaries (the azimuth wraps).

Norms (see _helpers; per-variable errors relative to the full field's max
are printed): FP64 residual 1e-13 of the flux scale at the sampled points
per variable and 1e-12 in the vector norm; FP32-storage residual 1e-3 per
variable; FP64 state after one step 1e-11 per variable, FP32-storage state
after one step 1e-5 in the vector norm."""
import numpy as np
import pytest
import torch

from _helpers import announce, make_solver, report
from cases import mesh, problems
from oracle import les

pytestmark = pytest.mark.gpu


def _workload(config, precision):
    import bench
    from paper_2301_00817_amd.solver import Solver
    dev = torch.device("cuda:0")
    prm, msh, fill, inflow = bench.make_workload(config, dev)
    s = Solver(prm, inflow=inflow, precision=precision, device=dev, **msh)
    Qn = s.field(5, dtype=torch.float64, fill=0.0)
    fill(s.interior(Qn))
    torch.cuda.synchronize()
    return prm, msh["grid"], s, Qn


def _samples(shape, n, h, seed):
    nx, nr, nth = shape
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(h, nx - h)), int(rng.integers(h, nr - h)), int(rng.integers(0, nth)))
            for _ in range(n)]


def _ks(k, h, nth):
    return [(k + d) % nth for d in range(-h, h + 1)]


def _block(A, p, h):
    """(c, 2h+1, 2h+1, 2h+1) block of an interior-indexed device array
    (c, nth, nr, nx) around p = (i, j, k), k wrapped; as NumPy FP64."""
    i, j, k = p
    ks = torch.tensor(_ks(k, h, A.shape[1]), device=A.device)
    B = A[:, :, j - h:j + h + 1, i - h:i + h + 1].index_select(1, ks)
    return B.to(torch.float64).cpu().numpy()


def _block_xyz(grid, p, h):
    """Coordinates of the block from the 1-D maps (host, C-library angles)."""
    X, R, TH = grid
    i, j, k = p
    th = TH[torch.tensor(_ks(k, h, TH.numel()))]
    return mesh.cylindrical_coords(X[i - h:i + h + 1], R[j - h:j + h + 1], th).numpy()


def _block_params(prm):
    """The block's own boundary kinds (periodic, no translation): its ghosts
    are never read by the centre values compared."""
    return dict(prm, bc=("periodic",) * 6, period=((0.0, 0.0, 0.0),) * 3)


def _oracle_at(prm, xyz_b, Q_b, h):
    """The oracle's residual at the block centre and the flux scale there,
    sum over its six faces of |F_v| / |J^-1|."""
    pb = _block_params(prm)
    with np.errstate(all="ignore"):
        geo = les.geometry(xyz_b, pb)
        Qp = les.pad_state(Q_b)
        les.fill_ghosts(Qp, geo, pb)
        pt = les.point_terms(Qp, geo, pb)
        R = les.residual(Qp, geo, pb)
        acc = np.zeros(5)
        for d in range(3):
            F = les.face_fluxes(pt, d, pb)      # faces -1/2 .. n-1/2 along the last axis
            Fc = np.moveaxis(F, -1, F.ndim - 1 - d)
            # the two faces of the centre along d: indices h and h + 1 of the face axis
            sl_lo = [slice(None), h, h, h]
            sl_hi = [slice(None), h, h, h]
            sl_lo[3 - d] = h
            sl_hi[3 - d] = h + 1
            acc += np.abs(Fc[tuple(sl_lo)]) + np.abs(Fc[tuple(sl_hi)])
        V = abs(float(les.interior(geo["V"])[h, h, h]))
    return R[:, h, h, h], acc / V


@pytest.mark.timeout(600)
@pytest.mark.parametrize("config,precision,nsamp", [("jet5.9M", "fp64", 48),
                                                    ("jet5.9M", "fp32", 48),
                                                    ("meshA", "fp64", 32),
                                                    ("meshA", "fp32", 32),
                                                    ("big1B", "fp64", 24),
                                                    ("big1B", "fp32", 24)])
def test_sampled_residual(config, precision, nsamp):
    announce("fullsize-residual", config, precision)
    prm, grid, s, Qn = _workload(config, precision)
    Qp = Qn if precision == "fp64" else Qn.to(torch.float32)
    if precision == "fp32":
        del Qn
        torch.cuda.empty_cache()
    R = s.residual(Qp)
    Ri = s.interior(R)
    vmax = np.array([float(Ri[v].abs().max()) for v in range(5)])
    mmag = float(torch.sqrt((Ri[1:4].double() ** 2).sum(dim=0)).max())
    Qi = s.interior(Qp)
    h = 2
    pts = _samples(s.shape, nsamp, h + 1, seed=7)
    got, ref, fsc = [], [], []
    for p in pts:
        i, j, k = p
        got.append(Ri[:, k, j, i].to(torch.float64).cpu().numpy())
        r, f = _oracle_at(prm, _block_xyz(grid, p, h), _block(Qi, p, h), h)
        ref.append(r)
        fsc.append(f)
    got, ref, fsc = np.array(got), np.array(ref), np.array(fsc)
    e = np.abs(got - ref).max(axis=0)
    pv = e / vmax
    vn = pv.copy()
    vn[1:4] = e[1:4] / mmag
    fx = e / fsc.max(axis=0)
    report(f"{config} {precision} sampled residual ({len(pts)} points)", per_variable=pv,
           vector=vn, flux=fx)
    assert np.isfinite(got).all()
    if precision == "fp64":
        assert fx.max() <= 1e-13
        assert vn.max() <= 1e-12
    else:
        assert pv.max() <= 1e-3
    s.close()
    del R, Ri, Qp, Qi
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("config,precision,nsamp", [("jet5.9M", "fp64", 4), ("meshA", "fp64", 3),
                                                    ("big1B", "fp64", 3), ("big1B", "fp32", 3)])
def test_sampled_rk5_step(config, precision, nsamp):
    """One CFL step of the workload bench.py times (its stage-kernel
    instances, chunking and launch shapes); the state at sampled points
    against the oracle's step of a 23^3 block with the same dt (one RK5 step
    reaches ten points).  FP64: 1e-11 per variable; FP32 storage: 1e-5 in
    the vector norm (P1)."""
    announce("fullsize-rk5", config, precision)
    prm, grid, s, Qn = _workload(config, precision)
    h = 11
    pts = _samples(s.shape, nsamp, h + 1, seed=8)
    Qi = s.interior(Qn)
    blocks = [_block(Qi, p, h) for p in pts]          # initial data, before the step
    dt = float(s.rk5_step(Qn, 1)[0])
    Q1 = s.interior(Qn)
    pb = _block_params(prm)
    got, ref = [], []
    for p, Qb0 in zip(pts, blocks):
        i, j, k = p
        got.append(Q1[:, k, j, i].cpu().numpy())
        with np.errstate(all="ignore"):
            geo = les.geometry(_block_xyz(grid, p, h), pb)
            Qb, _ = les.rk5_step(Qb0, geo, pb, None, dt)
        ref.append(Qb[:, h, h, h])
    got, ref = np.array(got), np.array(ref)
    e = np.abs(got - ref).max(axis=0)
    vmax = np.array([float(Q1[v].abs().max()) for v in range(5)])
    mmag = float(torch.sqrt((Q1[1:4] ** 2).sum(dim=0)).max())
    pv = e / vmax
    vn = pv.copy()
    vn[1:4] = e[1:4] / mmag
    # the increment Q^(n+1) - Q^n of the step (dt R, about 1e-5 of Q on the
    # 1.0e9-point mesh), which the state comparison alone barely resolves
    q0 = np.array([b[:, h, h, h] for b in blocks])
    dg, dr = got - q0, ref - q0
    di = np.abs(dg - dr).max(axis=0)
    dmax = np.abs(dr).max(axis=0)
    inc = di / np.where(dmax > 0, dmax, 1.0)
    inc[1:4] = di[1:4] / max(float(np.sqrt((dr[:, 1:4] ** 2).sum(axis=1)).max()), 1e-300)
    report(f"{config} {precision} sampled state after one step ({len(pts)} points)",
           per_variable=pv, vector=vn, increment=inc)
    assert np.isfinite(got).all()
    if precision == "fp64":
        assert pv.max() <= 1e-11
        # rounding of Q^(n+1) = Q^n - ... is a few ulps of Q: relative to the
        # increment that is u |Q| / |dQ|; 64 ulps of it, plus the residual's bar
        bar = 64 * np.finfo(np.float64).eps * float((np.abs(q0).max(axis=0) / dmax).max()) + 1e-12
        assert inc.max() <= bar, (inc, bar)
    else:
        assert vn.max() <= 1e-5
        assert inc.max() <= 1e-3          # the FP32-form residual's bar
    s.close()
    del Qn, Qi, Q1
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,bar", [("fp64", 1e-13), ("fp32", 1e-9)])
def test_periodic_box_conserves_at_scale(precision, bar):
    """A property of every point at a size the oracle cannot run: on the
    periodic 384^3 box (56.6 M points, many rounds of tiles and k-chunks)
    each face flux enters its two cells with opposite signs, across tiles,
    chunks and the periodic seams, so the totals of J^-1 Q stay constant
    over RK5 steps.  Bars: the rounding of the residual's flux differences
    summed over the box, 1e-13 of the totals in FP64; in the FP32-storage
    form the residual is rounded to FP32 per point (about 1e-7 of the flux
    scale), a random walk over 5.7e7 points that stays far below 1e-9."""
    announce("box-conservation", 384, precision)
    pb = problems.box_problem(384)
    s = make_solver(pb, precision=precision)
    Qn = s.pad(pb["Q"].cuda(), dtype=torch.float64)
    del pb
    t0 = s.diagnostics(Qn).cpu().numpy()
    s.rk5_step(Qn, 2)
    t1 = s.diagnostics(Qn).cpu().numpy()
    assert np.isfinite(t1).all()
    drift = [abs(t1[c] - t0[c]) / max(abs(t0[c]), abs(t0[1])) for c in range(5)]
    report(f"box384 {precision} conservation over 2 steps", relative_drift=np.array(drift))
    assert max(drift) <= bar
    s.close()
    del Qn
    torch.cuda.empty_cache()
