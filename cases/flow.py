"""Synthetic initial states, inflow data and problem parameters.

Nondimensional scales follow the paper's "Dimensionless Formulation": speed
of sound, density and temperature of the jet at the inlet, and the jet
diameter D.  Hence rho_j = a_j = T_j = 1 and p_j = 1/gamma.  The jet is
isothermal and perfectly expanded, so the ambient state has the same rho, T
and p.

States are returned as conserved variables Q = (rho, rho u, rho v, rho w, E)
with E = p/(gamma-1) + rho |u|^2 / 2 (the System-I energy closure), shaped
(5, nth, nr, nx).  Everything here is an input to the solver; nothing here is
part of the residual.
"""
import math

import torch

from . import rng

GAMMA = 1.4

# random-field ids (top byte of the counter key); one per independent field
FIELD_BOX = {"rho": 1, "u": 2, "v": 3, "w": 4, "p": 5}
FIELD_JET_IC = {"u": 11, "v": 12, "w": 13, "rho": 14, "p": 15}
FIELD_JET_IN = {"u": 21, "v": 22, "w": 23, "rho": 24, "p": 25}
FIELD_COTANGENT = 31      # cotangents (output-side seeds of adjoint checks)
FIELD_DIRECTION = 32      # perturbation directions (input side)
FIELD_DIRECTION_IN = 33   # perturbation directions of the inflow data
FIELD_MODES = 41          # phases of the multi-mode box velocity


def conserved(rho, u, v, w, p, gamma=GAMMA):
    """Stack primitives into (rho, rho u, rho v, rho w, E)."""
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return torch.stack([rho, rho * u, rho * v, rho * w, E])


def interior_index(shape, k0=0, device="cpu"):
    """Linear interior index k*nr*nx + j*nx + i for planes k0.. of `shape`
    = (nth_chunk, nr, nx)."""
    nth, nr, nx = shape
    k = torch.arange(k0, k0 + nth, dtype=torch.int64, device=device).view(nth, 1, 1)
    j = torch.arange(nr, dtype=torch.int64, device=device).view(1, nr, 1)
    i = torch.arange(nx, dtype=torch.int64, device=device).view(1, 1, nx)
    return (k * nr + j) * nx + i


# ----------------------------------------------------------------------------
# periodic box with an isentropic vortex
# ----------------------------------------------------------------------------
def vortex_box_state(xyz, seed=1, mach=0.5, beta=5.0, radius=1.0,
                     center=(math.pi, math.pi), noise=1e-4, gamma=GAMMA):
    """Isentropic vortex (axis along z) convected at Mach `mach` along +x.

    Written in a_inf = 1 units: with r^2 = ((x-x0)^2 + (y-y0)^2)/radius^2,
      u = M - c (y - y0) e^{(1-r^2)/2},  v = c (x - x0) e^{(1-r^2)/2},
      c = beta / (2 pi sqrt(gamma)),  T = 1 - (gamma-1) beta^2/(8 gamma pi^2) e^{1-r^2},
      rho = T^{1/(gamma-1)},  p = rho T / gamma.
    Seeded uniform noise of amplitude `noise` is added to rho, u, v, w, p.
    """
    x, y = xyz[0], xyz[1]
    dx = (x - center[0]) / radius
    dy = (y - center[1]) / radius
    r2 = dx * dx + dy * dy
    c = beta / (2.0 * math.pi * math.sqrt(gamma))
    e = torch.exp(0.5 * (1.0 - r2))
    u = mach - c * dy * e
    v = c * dx * e
    w = torch.zeros_like(u)
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * e * e
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T / gamma
    if noise:
        idx = interior_index(tuple(x.shape), device=x.device)
        rho = rho + noise * rng.symmetric(seed, FIELD_BOX["rho"], idx)
        u = u + noise * rng.symmetric(seed, FIELD_BOX["u"], idx)
        v = v + noise * rng.symmetric(seed, FIELD_BOX["v"], idx)
        w = w + noise * rng.symmetric(seed, FIELD_BOX["w"], idx)
        p = p + noise * rng.symmetric(seed, FIELD_BOX["p"], idx)
    return conserved(rho, u, v, w, p, gamma)


# ----------------------------------------------------------------------------
# supersonic jet
# ----------------------------------------------------------------------------
JET_UJ = 1.4       # jet Mach number (u_j / a_j, a_j = 1)
JET_UCO = 0.05     # coflow Mach number
JET_THETA = 0.05   # momentum thickness / D
N_INFLOW_COEF = 64


def momentum_thickness(theta_k, coef=None, theta_m=JET_THETA):
    """theta_m(phi) = theta_m0 [1 + sum_{m=1}^{32} (c_{2m-2} cos m phi
    + c_{2m-1} sin m phi)]; coef=None means all coefficients zero."""
    if coef is None:
        return torch.full_like(theta_k, theta_m)
    nm = coef.numel() // 2
    m = torch.arange(1, nm + 1, dtype=theta_k.dtype, device=theta_k.device)
    ph = theta_k.view(-1, 1) * m.view(1, -1)
    s = (torch.cos(ph) * coef[0::2].view(1, -1)
         + torch.sin(ph) * coef[1::2].view(1, -1)).sum(dim=1)
    return theta_m * (1.0 + s)


def jet_axial_velocity(R, TH, coef=None):
    """u(r, theta) = U_co + (U_j - U_co)/2 [1 + tanh((0.5 - r)/(2 theta_m))],
    shaped (nth, nr)."""
    tm = momentum_thickness(TH, coef).view(-1, 1)
    r = R.view(1, -1)
    return JET_UCO + 0.5 * (JET_UJ - JET_UCO) * (1.0 + torch.tanh((0.5 - r) / (2.0 * tm)))


def jet_state(X, R, TH, seed=2, coef=None, noise=1e-3 * JET_UJ, k0=0, k1=None,
              gamma=GAMMA, device="cpu", thermo_noise=0.0):
    """Parallel-jet initial state: the inflow profile extended uniformly in x,
    rho = 1, p = 1/gamma, plus seeded velocity noise on u, v, w.

    thermo_noise > 0 also multiplies rho and p by 1 + thermo_noise U(-1, 1)
    (a state with no uniform-pressure degeneracy, for derivative checks).
    Planes k0..k1 only (for chunked generation of large meshes)."""
    nth_all = TH.numel()
    if k1 is None:
        k1 = nth_all
    X, R, TH = X.to(device), R.to(device), TH.to(device)
    if coef is not None:
        coef = coef.to(device)
    nx, nr = X.numel(), R.numel()
    nk = k1 - k0
    u2d = jet_axial_velocity(R, TH, coef)[k0:k1]           # (nk, nr)
    u = u2d.view(nk, nr, 1).expand(nk, nr, nx)
    v = torch.zeros((nk, nr, nx), dtype=torch.float64, device=device)
    w = torch.zeros_like(v)
    if noise:
        idx = interior_index((nk, nr, nx), k0, device=device)
        u = u + noise * rng.symmetric(seed, FIELD_JET_IC["u"], idx)
        v = v + noise * rng.symmetric(seed, FIELD_JET_IC["v"], idx)
        w = w + noise * rng.symmetric(seed, FIELD_JET_IC["w"], idx)
    rho = torch.ones_like(v)
    p = torch.full_like(v, 1.0 / gamma)
    if thermo_noise:
        idx = interior_index((nk, nr, nx), k0, device=device)
        rho = rho * (1.0 + thermo_noise * rng.symmetric(seed, FIELD_JET_IC["rho"], idx))
        p = p * (1.0 + thermo_noise * rng.symmetric(seed, FIELD_JET_IC["p"], idx))
    return conserved(rho, u, v, w, p, gamma)


def jet_inflow(R, TH, seed=2, coef=None, noise=1e-3 * JET_UJ, gamma=GAMMA,
               device="cpu", thermo_noise=0.0):
    """Inflow target primitives (rho, u, v, w, p) at the entrance plane,
    shaped (5, nth, nr): the jet profile plus a frozen seeded noise pattern
    (and relative rho, p noise when thermo_noise > 0)."""
    R, TH = R.to(device), TH.to(device)
    if coef is not None:
        coef = coef.to(device)
    nth, nr = TH.numel(), R.numel()
    u = jet_axial_velocity(R, TH, coef)
    v = torch.zeros_like(u)
    w = torch.zeros_like(u)
    if noise:
        k = torch.arange(nth, dtype=torch.int64, device=device).view(nth, 1)
        j = torch.arange(nr, dtype=torch.int64, device=device).view(1, nr)
        idx = k * nr + j
        u = u + noise * rng.symmetric(seed, FIELD_JET_IN["u"], idx)
        v = v + noise * rng.symmetric(seed, FIELD_JET_IN["v"], idx)
        w = w + noise * rng.symmetric(seed, FIELD_JET_IN["w"], idx)
    rho = torch.ones_like(u)
    p = torch.full_like(u, 1.0 / gamma)
    if thermo_noise:
        k = torch.arange(nth, dtype=torch.int64, device=device).view(nth, 1)
        j = torch.arange(nr, dtype=torch.int64, device=device).view(1, nr)
        idx = k * nr + j
        rho = rho * (1.0 + thermo_noise * rng.symmetric(seed, FIELD_JET_IN["rho"], idx))
        p = p * (1.0 + thermo_noise * rng.symmetric(seed, FIELD_JET_IN["p"], idx))
    return torch.stack([rho, u, v, w, p])


def uniform_state(shape, prim, gamma=GAMMA, device="cpu"):
    """A uniform state (free stream) with primitives prim = (rho,u,v,w,p)."""
    f = [torch.full(shape, float(c), dtype=torch.float64, device=device) for c in prim]
    return conserved(*f, gamma=gamma)


# ----------------------------------------------------------------------------
# periodic box with a multi-mode velocity field
# ----------------------------------------------------------------------------
def modes_box_state(xyz, seed=1, kmax=3, amp=0.1, slope=1.0, tamp=0.05, rho=1.0,
                    p=1.0 / GAMMA, gamma=GAMMA):
    """u_c = sum over integer wave vectors 0 < |k|_inf <= kmax of
    amp |k|^(-2 slope) cos(k . x + phi_{k,c}), seeded phases phi; uniform
    density; pressure p (1 + s), s the same sum with amplitude `tamp` and
    its own phases.  A field with an energy spectrum decaying with |k|
    (dynamic SGS-model checks: random single-scale noise makes the model's
    averages vanish)."""
    x, y, z = xyz[0], xyz[1], xyz[2]
    rng_idx = 0
    f = [torch.zeros_like(x) for _ in range(4)]
    ks = [(a, b, c) for a in range(-kmax, kmax + 1) for b in range(-kmax, kmax + 1)
          for c in range(-kmax, kmax + 1) if (a, b, c) != (0, 0, 0)]
    idx = torch.arange(4 * len(ks), dtype=torch.int64)
    phases = 2.0 * math.pi * rng.uniform(seed, FIELD_MODES, idx)
    for (a, b, c) in ks:
        k2 = a * a + b * b + c * c
        arg = a * x + b * y + c * z
        for comp in range(4):
            scale = amp if comp < 3 else tamp
            f[comp] = f[comp] + scale * k2 ** (-slope) * torch.cos(arg + float(phases[rng_idx]))
            rng_idx += 1
    r = torch.full_like(x, rho)
    return conserved(r, f[0], f[1], f[2], p * (1.0 + f[3]), gamma)
