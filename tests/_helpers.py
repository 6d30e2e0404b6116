"""Shared helpers of the GPU tests (marshalling between the solver's padded
tensors and the oracle's NumPy arrays; error norms).

Error norms (all relative max-norms over the compared points):
  per-variable  max|a_v - b_v| / max|b_v| for each of the five variables,
                the norm of the tolerance table; always printed;
  vector (P1)   the scalars (rho, E; or rho, p) per variable, and the three
                components of the momentum (or velocity) vector each
                normalised by the largest magnitude of that vector,
                max|b_1..3|_2: the components form one vector, and on the jet
                the cross-stream ones are noise-level (about 1e-3 of the
                axial one), so their per-variable error measures rounding of
                small numbers against themselves.  This is the asserted
                norm of states, ghosts and statistics;
  flux (P2)     for a residual against the oracle: max|R_v - R_ref,v| over
                the flux scale max over points of (sum over the six faces of
                |F_v|) / |J^-1|, the magnitude of the terms whose differences
                form R.  Rounding of a flux difference is bounded relative
                to the fluxes, not to their difference, so this is the
                asserted norm of FP64 residuals.
"""
import sys

import numpy as np

VECTOR = (1, 2, 3)
NAMES_Q = ("rho", "rho u", "rho v", "rho w", "E")


def per_variable_err(a, b):
    """max|a_v - b_v| / max|b_v| per variable (5 numbers)."""
    a = np.asarray(a)
    b = np.asarray(b)
    out = []
    for v in range(a.shape[0]):
        s = float(np.abs(b[v]).max())
        out.append(float(np.abs(a[v] - b[v]).max()) / (s if s != 0.0 else 1.0))
    return np.array(out)


def vector_err(a, b):
    """Reading P1: scalars per variable; components 1..3 over the largest
    magnitude of the vector they form (5 numbers)."""
    a = np.asarray(a)
    b = np.asarray(b)
    out = per_variable_err(a, b)
    mag = float(np.sqrt(sum(np.asarray(b[c], dtype=np.float64) ** 2 for c in VECTOR)).max())
    for c in VECTOR:
        out[c] = float(np.abs(a[c] - b[c]).max()) / (mag if mag != 0.0 else 1.0)
    return out


def rel_err(a, b, label=None):
    """max over the variables of the P1 norm; prints both norms."""
    pv = per_variable_err(a, b)
    vn = vector_err(a, b)
    if label:
        report(label, per_variable=pv, vector=vn)
    return float(vn.max())


# the former name of rel_err (same norm for the scalars; the momentum
# components now over the vector's magnitude)
grouped_rel_err = rel_err


def flux_scale(Q, geo, prm, inflow=None):
    """Per-variable flux scale of the residual of the interior state Q:
    max over interior points of sum_faces |F_v| / |J^-1| (5 numbers), from
    the oracle's face fluxes."""
    from oracle import les
    Qp = les.pad_state(np.asarray(Q))
    les.fill_ghosts(Qp, geo, prm, inflow)
    with np.errstate(all="ignore"):
        pt = les.point_terms(Qp, geo, prm)
        acc = 0.0
        for d in range(3):
            F = np.abs(les.face_fluxes(pt, d, prm))
            s = F[..., 1:] + F[..., :-1]
            acc = acc + np.moveaxis(s, -1, s.ndim - 1 - d)
        V = np.abs(les.interior(geo["V"]))
        tot = acc / V
    if prm["bc"][2] == "axis_node":
        tot = tot.copy()
        tot[:, :, 0, :] = 0.0          # the axis row is not advanced (V = 0)
    return np.array([float(np.nanmax(tot[v])) for v in range(5)])


def flux_err(R, R_ref, scale):
    """Reading P2: max|R_v - R_ref,v| / scale_v per variable (5 numbers)."""
    R = np.asarray(R)
    R_ref = np.asarray(R_ref)
    return np.array([float(np.abs(R[v] - R_ref[v]).max()) / scale[v] for v in range(5)])


def report(label, **norms):
    parts = [f"{k} [" + " ".join(f"{x:.2e}" for x in v) + "]" for k, v in norms.items()]
    print(f"[parity] {label}: " + "; ".join(parts), flush=True)


def announce(*parts):
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()


def to_np(t):
    return t.detach().to("cpu").numpy()


def make_solver(pb, precision="fp64", keep_metrics=False, params=None):
    from paper_2301_00817_amd.solver import Solver
    return Solver(params or pb["params"], pb["xyz"], pb.get("inflow"), precision=precision,
                  keep_metrics=keep_metrics)
