"""Named synthetic workloads: mesh + initial state + boundary data + constants.

A problem is a plain dict of inputs:
  xyz     (3, nth, nr, nx) float64 coordinates
  Q       (5, nth, nr, nx) float64 conserved state
  inflow  (5, nth, nr) float64 inflow target primitives, or None
  params  dict of scalar constants and boundary kinds (see `base_params`)
The solver (GPU library) and the CPU oracle each consume these inputs their
own way; nothing here computes any part of the residual.
"""
import math

import torch

from . import flow, mesh, rng

RK_ALPHA = (1.0 / 4.0, 1.0 / 6.0, 3.0 / 8.0, 1.0 / 2.0, 1.0)   # Jameson 5-stage


def base_params(**over):
    """Physical and numerical constants.

    gamma = 1.4, Pr = 0.72, Pr_sgs = 0.9 (static SGS models), k2 = 0.25,
    k4 = 0.016 (Turkel-Vatsa constants), Cs = 0.148 (Lilly),
    Sutherland S1 = 110.4 K over a 288.15 K reference temperature.
    visc_coef = M/Re multiplies the viscous fluxes.
    bc order: xi-, xi+, eta-, eta+, zeta-, zeta+.
    """
    p = dict(gamma=1.4, Pr=0.72, Pr_sgs=0.9, visc_coef=0.0,
             suth_S=110.4 / 288.15, Cs=0.148, k2=0.25, k4=0.016, cfl=0.5,
             rk_alpha=RK_ALPHA, ref_prim=(1.0, 0.0, 0.0, 0.0, 1.0 / 1.4),
             p_exit=1.0 / 1.4, sgs_model=1,
             bc=("periodic",) * 6,
             period=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0)))
    p.update(over)
    return p


def box_params(L=2.0 * math.pi, **over):
    p = base_params(visc_coef=0.5 / 1.0e4,
                    period=((L, 0.0, 0.0), (0.0, L, 0.0), (0.0, 0.0, L)))
    p.update(over)
    return p


def jet_params(**over):
    g = 1.4
    p = base_params(visc_coef=flow.JET_UJ / 1.5e6,
                    ref_prim=(1.0, flow.JET_UCO, 0.0, 0.0, 1.0 / g),
                    p_exit=1.0 / g,
                    bc=("inflow", "outflow", "axis", "farfield", "periodic", "periodic"))
    p.update(over)
    return p


def box_problem(n=32, seed=1, Cs=0.148, noise=1e-4, shape=None):
    """Periodic box, L = 2 pi, isentropic Mach-0.5 vortex plus noise."""
    L = 2.0 * math.pi
    xyz = mesh.box_coords(n, L, shape=shape)
    Q = flow.vortex_box_state(xyz, seed=seed, noise=noise)
    return dict(name=f"box{n}", xyz=xyz, Q=Q, inflow=None,
                params=box_params(L, Cs=Cs))


def modes_box_problem(n=32, seed=1, kmax=3, amp=0.1, visc_coef=1e-3):
    """Periodic box with the multi-mode velocity field and the dynamic SGS
    model (a state on which its averaged coefficients are positive)."""
    L = 2.0 * math.pi
    xyz = mesh.box_coords(n, L)
    Q = flow.modes_box_state(xyz, seed=seed, kmax=kmax, amp=amp)
    return dict(name=f"modes{n}", xyz=xyz, Q=Q, inflow=None,
                params=box_params(L, sgs_model=3, visc_coef=visc_coef))


def jet_grid(nx, nr, nth, axis_node=False):
    """1-D maps of the jet mesh; axis_node puts the radial row j = 0 on the
    axis (r = 0) instead of at r = 0.005 D."""
    R = mesh.jet_radial(nr, rmin=0.0) if axis_node else mesh.jet_radial(nr)
    return mesh.jet_axial(nx), R, mesh.azimuth(nth)


def jet_problem(nx, nr, nth, seed=2, coef=None, noise=1e-3 * flow.JET_UJ,
                with_xyz=True, device="cpu", thermo_noise=0.0, axis_node=False):
    """Cylindrical jet mesh with the Mach-1.4 parallel-jet state.  axis_node:
    mesh nodes on the axis with the centerline condition of the paper."""
    X, R, TH = jet_grid(nx, nr, nth, axis_node)
    xyz = mesh.cylindrical_coords(X, R, TH, device=device) if with_xyz else None
    Q = flow.jet_state(X, R, TH, seed=seed, coef=coef, noise=noise, device=device,
                       thermo_noise=thermo_noise)
    inflow = flow.jet_inflow(R, TH, seed=seed, coef=coef, noise=noise, device=device,
                             thermo_noise=thermo_noise)
    prm = jet_params()
    if axis_node:
        prm["bc"] = ("inflow", "outflow", "axis_node", "farfield", "periodic", "periodic")
    return dict(name=f"jet{nx}x{nr}x{nth}" + ("_axisnode" if axis_node else ""), xyz=xyz, Q=Q,
                inflow=inflow, params=prm, grid=(X, R, TH))


def seeded_field(shape, seed, field, kind="gaussian", device="cpu"):
    """A seeded random array of `shape` (cotangents and perturbation
    directions of derivative checks), indexed by the row-major position."""
    n = 1
    for s in shape:
        n *= s
    idx = torch.arange(n, dtype=torch.int64, device=device)
    draw = rng.gaussian if kind == "gaussian" else rng.symmetric
    return draw(seed, field, idx).view(*shape)


# the configurations the measurements and parity tests are run on
CONFIGS = {
    "box32": dict(kind="box", n=32, steps=10, seed=1),
    "jet5.9M": dict(kind="jet", shape=(288, 160, 128), steps=100, seed=2),
    "prec102M": dict(kind="jet", shape=(800, 400, 320), steps=50, seed=3),
    "adj2M": dict(kind="jet", shape=(160, 100, 128), steps=20, seed=4),
    "big1B": dict(kind="jet", shape=(1250, 640, 1250), steps=20, seed=2),
}

# The paper's mesh family A-I (axial x radial x azimuthal; its 361 azimuthal
# points repeat the periodic point, so 360 distinct ones here), run as the
# paper ran them: no subgrid model.
PAPER_MESHES = {
    "A": (128, 128), "B": (256, 128), "C": (256, 256), "D": (512, 256), "E": (512, 512),
    "F": (1024, 512), "G": (1024, 1024), "H": (2048, 1024), "I": (1700, 1700),
}
for _m, (_nx, _nr) in PAPER_MESHES.items():
    CONFIGS["mesh" + _m] = dict(kind="jet", shape=(_nx, _nr, 360), steps=10, seed=2, sgs=False)
