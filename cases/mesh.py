"""Synthetic structured meshes (coordinates only; no metric arithmetic).

Index order follows the solver: xi = axial (i), eta = radial (j),
zeta = azimuthal (k).  Coordinate arrays are shaped (3, nth, nr, nx) with the
axial index fastest.

Jet mesh (the paper's cylindrical jet domain, section "Boundary Conditions"
and the mesh family of the performance study):
  * axial   X_0 = 0, X_{nx-1} = 30 D, spacing growing geometrically by 1.005;
  * radial  r in [0.005 D, 20 D], points clustered at the lip line r = 0.5 D
            by a point density 1 + A sech^2((r - 0.5)/w), A = 50, w = 0.2 D;
  * azimuth nth distinct points theta_k = 2 pi k / nth (periodic, no
            duplicated point).
"""
import math

import torch


def jet_axial(nx, length=30.0, ratio=1.005, dtype=torch.float64):
    """X_i, i = 0..nx-1, with dX_i = dX_0 * ratio**i and X_{nx-1} = length."""
    n = nx - 1
    dx0 = length * (ratio - 1.0) / (ratio ** n - 1.0)
    i = torch.arange(nx, dtype=dtype)
    x = dx0 * (ratio ** i - 1.0) / (ratio - 1.0)
    x[-1] = length
    return x


def _radial_arc(r, rmin, rc, amp, width):
    return (r - rmin) + amp * width * (torch.tanh((r - rc) / width)
                                       - math.tanh((rmin - rc) / width))


def jet_radial(nr, rmin=0.005, rmax=20.0, rc=0.5, amp=50.0, width=0.2,
               dtype=torch.float64):
    """R_j, j = 0..nr-1, uniform in the stretched coordinate s(r).

    s(r) = (r - rmin) + A w [tanh((r - rc)/w) - tanh((rmin - rc)/w)] is the
    integral of the point density 1 + A sech^2((r - rc)/w); s is inverted by
    bisection (monotone), so the clustering is exact to rounding.
    """
    smax = float(_radial_arc(torch.tensor(rmax, dtype=dtype), rmin, rc, amp, width))
    s = torch.linspace(0.0, smax, nr, dtype=dtype)
    lo = torch.full_like(s, rmin)
    hi = torch.full_like(s, rmax)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        f = _radial_arc(mid, rmin, rc, amp, width)
        left = f < s
        lo = torch.where(left, mid, lo)
        hi = torch.where(left, hi, mid)
    r = 0.5 * (lo + hi)
    r[0] = rmin
    r[-1] = rmax
    return r


def azimuth(nth, dtype=torch.float64):
    return 2.0 * math.pi * torch.arange(nth, dtype=dtype) / nth


def angle_tables(TH):
    """cos and sin of the angles by the host C library (math.cos, math.sin):
    the functions the GPU library's product-mesh set-up calls, so that
    coordinates formed here and there from the same maps agree bitwise."""
    th = [float(t) for t in TH.reshape(-1).tolist()]
    c = torch.tensor([math.cos(t) for t in th], dtype=torch.float64)
    s = torch.tensor([math.sin(t) for t in th], dtype=torch.float64)
    return c, s


def cylindrical_coords(X, R, TH, k0=0, k1=None, device="cpu"):
    """x = X_i, y = R_j cos(theta_k), z = R_j sin(theta_k) for k in [k0, k1)."""
    if k1 is None:
        k1 = TH.numel()
    X = X.to(device)
    R = R.to(device)
    ct, st = angle_tables(TH[k0:k1])
    ct, st = ct.to(device), st.to(device)
    nth, nr, nx = ct.numel(), R.numel(), X.numel()
    xyz = torch.empty((3, nth, nr, nx), dtype=torch.float64, device=device)
    xyz[0] = X.view(1, 1, nx)
    xyz[1] = (R.view(1, nr, 1) * ct.view(nth, 1, 1)).expand(nth, nr, nx)
    xyz[2] = (R.view(1, nr, 1) * st.view(nth, 1, 1)).expand(nth, nr, nx)
    return xyz


def box_coords(n, length=2.0 * math.pi, shape=None):
    """Uniform Cartesian box; x along i, y along j, z along k; spacing L/n."""
    nx, nr, nth = shape if shape is not None else (n, n, n)
    h = (length / nx, length / nr, length / nth)
    i = torch.arange(nx, dtype=torch.float64) * h[0]
    j = torch.arange(nr, dtype=torch.float64) * h[1]
    k = torch.arange(nth, dtype=torch.float64) * h[2]
    xyz = torch.empty((3, nth, nr, nx), dtype=torch.float64)
    xyz[0] = i.view(1, 1, nx)
    xyz[1] = j.view(1, nr, 1)
    xyz[2] = k.view(nth, 1, 1)
    return xyz


def wavy_coords(n, length=2.0 * math.pi, amp=0.1):
    """Non-orthogonal periodic mesh x = xi + a sin(eta), y = eta + a sin(zeta),
    z = zeta + a sin(xi), with (xi, eta, zeta) uniform on [0, L)^3."""
    h = length / n
    s = torch.arange(n, dtype=torch.float64) * h
    xi = s.view(1, 1, n)
    eta = s.view(1, n, 1)
    zeta = s.view(n, 1, 1)
    xyz = torch.empty((3, n, n, n), dtype=torch.float64)
    xyz[0] = xi + amp * torch.sin(eta)
    xyz[1] = eta + amp * torch.sin(zeta)
    xyz[2] = zeta + amp * torch.sin(xi)
    return xyz
