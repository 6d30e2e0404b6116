"""Plain, slow FP64 NumPy oracle of the explicit LES residual and RK5 step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg import this module; the GPU library never
calls it and shares no code with it.

What it computes, in the order of the paper (Junqueira-Junior et al., "A LES
solver for supersonic jet flows", arXiv 2301.00817):
  * metrics and Jacobian of the curvilinear transformation
    (section "Transformation of Coordinates", metric-term and Jacobian
    equations);
  * ghost values from the boundary conditions (section "Boundary Conditions":
    far field by Riemann invariants, entrance, exit, centerline, periodic);
  * the residual RHS/V of the semi-discrete system (section "Spatial
    Discretization", eq. spatial_discret and the RHS equation), built from
    centred inviscid point fluxes (eq. hat-flux-G), viscous and SGS point
    fluxes (eqs. hat-flux-Ev/Fv/Gv, q_mod, kappa_sgs, tau_mod, sutherland,
    Smagorinsky model), and the Turkel-Vatsa artificial dissipation
    (eqs. inv_flux_vec, dissip_term, eps_2_dissip, eps_4_dissip,
    p_grad_sensor, W_dissip, spectral radii);
  * the five-stage Runge-Kutta step (section "Time Marching Method",
    eq. localdt and the alpha coefficients).

Readings taken where the paper is silent, garbled or inconsistent (each is
also listed in the design notes):
  R1  the state is stored unhatted, Q = (rho, rho u, rho v, rho w, E); the
      dissipation vector is W = (rho, rho u, rho v, rho w, E + p) and the
      face factor J^-1 is the face average V_f = (V_L + V_R)/2.
  R2  the operator between the eps2 and eps4 terms of the dissipation is a
      minus sign (the standard, dissipative choice).
  R3  the pressure sensor denominator is p+ + 2p + p- (the printed
      p+ - 2p + p- would make the sensor identically 1).
  R4  lambda_d = |U_d| + a |grad xi_d| for d = xi, eta, zeta (the printed
      three rows are all labelled lambda_xi with one mixed norm).
  R5  the eta metric row is the cofactor grad eta = J (r_zeta x r_xi).
  R6  heat flux q = -(kappa + kappa_sgs) grad T (down-gradient).
  R7  Smagorinsky mu_sgs = rho (Cs Delta)^2 |S|; in units of the jet
      viscosity it is divided by visc_coef = M/Re.  The Vreman variant
      (sgs_model 2) uses the same width Delta in every direction and the
      same units: mu_sgs = rho c sqrt(B_beta / alpha_ij alpha_ij) / visc_coef.
  R9  filter width Delta = |V|^(1/3).
  R10 Sutherland mu = T^1.5 (1 + S)/(T + S), S = 110.4 K / 288.15 K.
  R11 viscous face flux = average of the two point viscous fluxes, with point
      gradients by central differences and the chain rule (R12).
  R13 mu and mu_sgs are recomputed from the state at every evaluation.
  R14 ghosts are refilled before every residual evaluation.
  R15 dissipation is zero on physical-boundary faces (entrance, exit, far
      field); periodic and cross-axis faces are internal.
  R18 one global time step dt = CFL / max(lambda_xi + lambda_eta + lambda_zeta)
      over the interior of Q^n, or a fixed dt.
  R19 periodic azimuth with n_theta distinct points (no duplicated point).
  R20 the mesh has no node on the axis; the ghosts across the axis are the
      points (i, m, k + n_theta/2), coordinates and state copied.
  R21 entrance: a supersonic target (normal Mach >= 1) is imposed; otherwise
      Riemann invariants with the outward normal -xi and the target as the
      outside state.
  R22 exit: subsonic -> rho, u, v, w from the last interior plane and
      p = p_exit; supersonic -> copy.
  R23 R+ = q_e + 2 a_e/(gamma-1), and the velocity is corrected along the
      unit normal.
  R24 branch ties: q/a >= 1 exit copy, q/a <= -1 outside state, q >= 0
      subsonic exit.
  Centerline through mesh nodes (eta- kind "axis_node", subsection
  "Centerline Boundary Condition"; the mesh has its j = 0 points on the
  axis):
  C1  before every residual the axis row takes the azimuthal mean of the
      conserved variables of the row j = 1 (extrapolated and averaged); it
      is not advanced by the scheme (R = 0 there);
  C2  ghosts across the axis are the mirror points (i, m, k + nth/2);
  C3  the eta point flux vanishes at the axis (S^eta = 0 there; the
      viscous terms, singular at V = 0, are not evaluated);
  C4  the dissipation at the axis face uses lambda_bar of the j = 1 point
      (the axis point has V = 0) and the modified fourth difference of the
      centerline subsection, (Delta w)_{-1/2} = -(Delta w)_{1/2}, i.e.
      W_{2} - 4 W_{1} + 3 W_{0} in place of W_{2} - 3 W_{1} + 3 W_{0} - W_{-1};
  C5  boundary normals of axis points (entrance, exit) are those of the
      j = 1 point (S^xi vanishes on the axis);
  C6  the time step maximum runs over j >= 1.
  Dynamic Smagorinsky model (sgs_model 3, subsection "Dynamic Smagorinsky
  Model"; the isotropic SGS stress enters the momentum and energy fluxes as
  in the modified System I equations):
  D1  test filter: the separable three-point filter (1/4, 1/2, 1/4) along
      each index direction (27 points), test width Delta_hat = 2 Delta;
  D2  <.> is the volume average over the interior points (weights J^-1);
      each coefficient is the ratio of two such averages;
  D3  Delta stays outside the hats (the local width of the averaging
      point); hat(sigma_ll) = 2 C_I Delta^2 hat(rho |S|^2);
  D4  T_ll is the trace of L_ij = hat(rho u_i u_j) - hat(rho u_i)
      hat(rho u_j) / hat(rho); S_ij in the contractions is the resolved
      strain at the point, S_hat_ij the strain of u_hat = hat(rho u)/hat(rho);
  D5  mu_sgs = rho C_ds Delta^2 |S| (the printed square of rho C_ds Delta
      read as for the static model, R7), in jet-viscosity units; C_ds and
      C_I below 0 are taken as 0 (a negative eddy viscosity or isotropic
      stress is not used);
  D6  Pr_sgs = C_ds <Delta^2 hat(rho |S| dT/dx_j) dT/dx_j - Delta_hat^2
      rho_hat |S_hat| dT_hat/dx_j dT/dx_j> / <(hat(rho u_j T) - hat(rho u_j)
      hat(rho T)/hat(rho)) dT/dx_j>, T_hat = hat(rho T)/hat(rho); the static
      0.9 where that is not a positive finite number;
  D7  the isotropic stress sigma_kk = 2 C_I rho Delta^2 |S|^2 adds
      sigma_kk / 3 to the pressure of the momentum and energy point fluxes
      (not to W or the spectral radii);
  D8  the coefficients are evaluated with the viscosities: from every stage
      state (schedule "stage"), or from Q^n and held (schedule "step"; the
      isotropic stress then uses the held C_I and the stage |S|).
  Update schedule (prm["schedule"]; section "The JAZzY code", the iteration
  loop: viscosity, SGS viscosity and boundary conditions are updated once
  per iteration, after the time marching):
  L1  "stage" (default): R13/R14, everything recomputed for every stage;
      "step": mu and mu_t are evaluated once per step from Q^n (equal to
      the paper's end-of-iteration update of the previous step) and held
      through the five stages;
  L2  "step": ghost values of physical faces (entrance, exit, far field) and
      the centerline average are evaluated once per step from Q^n and held;
      periodic and cross-axis ghosts are copies of the stage state (the
      paper's data exchanges, done for every stage); edge ghosts that copy
      a physical-face ghost take the held value.

The code is dtype-generic: complex128 arrays give complex-step derivatives
(abs, max and branch tests act on real parts).
"""
import numpy as np

NG = 2      # ghost layers of the state and metric arrays
NGC = 3     # ghost layers of the coordinate array

PHYSICAL_FACE_KINDS = ("inflow", "outflow", "farfield")


# ---------------------------------------------------------------------------
# complex-safe elementary operations
# ---------------------------------------------------------------------------
def rabs(x):
    """|x| acting on the real part (identity derivative sign for x >= 0)."""
    return np.where(np.real(x) < 0, -x, x)


def rmax(a, b):
    return np.where(np.real(a) >= np.real(b), a, b)


# ---------------------------------------------------------------------------
# layout helpers: arrays are (..., zeta, eta, xi) with xi fastest
# ---------------------------------------------------------------------------
def _axis(A, d):
    """Array axis of spatial direction d (0 = xi, 1 = eta, 2 = zeta)."""
    return A.ndim - 1 - d


def _fill_region(A, d, g):
    """View of A with direction d last, restricted in the other directions to
    what is defined when direction d is filled (fill order xi, eta, zeta):
    xi is filled on the interior of eta and zeta, eta on the interior of
    zeta (all xi), zeta everywhere."""
    sl = [slice(None)] * A.ndim
    if d == 0:
        sl[_axis(A, 1)] = slice(g, -g)
        sl[_axis(A, 2)] = slice(g, -g)
    elif d == 1:
        sl[_axis(A, 2)] = slice(g, -g)
    return np.moveaxis(A[tuple(sl)], _axis(A, d), -1)


# ---------------------------------------------------------------------------
# geometry: coordinate ghosts and metrics
# ---------------------------------------------------------------------------
def pad_coords(xyz, prm):
    """Coordinates (3, nth, nr, nx) -> padded (3, nth+6, nr+6, nx+6).

    Ghost rules per boundary kind: periodic -> wrapped interior point plus the
    period translation; axis -> the point across the axis (i, m, k+nth/2);
    entrance/exit/far field -> linear extrapolation in index space,
    r_{-m} = r_0 + m (r_0 - r_1)."""
    g = NGC
    _, nth, nr, nx = xyz.shape
    n = (nx, nr, nth)
    P = np.full((3, nth + 2 * g, nr + 2 * g, nx + 2 * g), np.nan, dtype=xyz.dtype)
    P[:, g:g + nth, g:g + nr, g:g + nx] = xyz
    period = np.asarray(prm["period"], dtype=float)
    for d in range(3):
        lo_kind, hi_kind = prm["bc"][2 * d], prm["bc"][2 * d + 1]
        L = _fill_region(P, d, g)                   # (3, a, b, n_d + 2g)
        nd = n[d]
        shift = period[d].reshape(3, 1, 1)
        for m in range(1, g + 1):
            lo, hi = g - m, g + nd - 1 + m
            if lo_kind == "periodic":
                L[..., lo] = L[..., g + nd - m] - shift
            elif lo_kind == "axis":
                # eta direction: the other (zeta) axis of L is axis 1
                L[..., lo] = np.roll(L[..., g + m - 1], -(n[2] // 2), axis=1)
            elif lo_kind == "axis_node":               # mirror through the axis node (C2)
                L[..., lo] = np.roll(L[..., g + m], -(n[2] // 2), axis=1)
            else:
                L[..., lo] = L[..., g] + m * (L[..., g] - L[..., g + 1])
            if hi_kind == "periodic":
                L[..., hi] = L[..., g + m - 1] + shift
            else:
                L[..., hi] = L[..., g + nd - 1] + m * (L[..., g + nd - 1] - L[..., g + nd - 2])
    return P


def metrics(P):
    """Metric terms on the state's padded box (two ghost layers).

    Derivatives of the coordinates are second-order central differences in
    index space (unit spacing).  Returns
      S : (3, 3, nth+4, nr+4, nx+4), S[d] = J^-1 grad(xi_d) (area vectors)
      V : (nth+4, nr+4, nx+4), V = J^-1 (the Jacobian determinant).
    The rows are the paper's metric-term formulas multiplied by J^-1; the eta
    row is the cofactor r_zeta x r_xi (reading R5)."""
    def central(ax):
        hi = [slice(None), slice(1, -1), slice(1, -1), slice(1, -1)]
        lo = list(hi)
        hi[ax] = slice(2, None)
        lo[ax] = slice(None, -2)
        return (P[tuple(hi)] - P[tuple(lo)]) / 2.0

    x_xi, y_xi, z_xi = central(3)
    x_eta, y_eta, z_eta = central(2)
    x_zeta, y_zeta, z_zeta = central(1)

    S = np.empty((3, 3) + x_xi.shape, dtype=P.dtype)
    # J^-1 (xi_x, xi_y, xi_z)
    S[0, 0] = y_eta * z_zeta - y_zeta * z_eta
    S[0, 1] = z_eta * x_zeta - z_zeta * x_eta
    S[0, 2] = x_eta * y_zeta - x_zeta * y_eta
    # J^-1 (eta_x, eta_y, eta_z)
    S[1, 0] = y_zeta * z_xi - y_xi * z_zeta
    S[1, 1] = z_zeta * x_xi - z_xi * x_zeta
    S[1, 2] = x_zeta * y_xi - x_xi * y_zeta
    # J^-1 (zeta_x, zeta_y, zeta_z)
    S[2, 0] = y_xi * z_eta - y_eta * z_xi
    S[2, 1] = z_xi * x_eta - z_eta * x_xi
    S[2, 2] = x_xi * y_eta - x_eta * y_xi
    # J^-1 = x_xi y_eta z_zeta + x_eta y_zeta z_xi + x_zeta y_xi z_eta
    #        - x_xi y_zeta z_eta - x_eta y_xi z_zeta - x_zeta y_eta z_xi
    V = (x_xi * y_eta * z_zeta + x_eta * y_zeta * z_xi + x_zeta * y_xi * z_eta
         - x_xi * y_zeta * z_eta - x_eta * y_xi * z_zeta - x_zeta * y_eta * z_xi)
    return dict(S=S, V=V)


def geometry(xyz, prm):
    """pad_coords + metrics."""
    return metrics(pad_coords(np.asarray(xyz), prm))


# ---------------------------------------------------------------------------
# state conversions
# ---------------------------------------------------------------------------
def primitives(Q, gamma):
    """(rho, u, v, w, p) from Q = (rho, rho u, rho v, rho w, E), with
    E = p/(gamma-1) + rho |u|^2/2 (System-I energy)."""
    rho = Q[0]
    u = Q[1] / rho
    v = Q[2] / rho
    w = Q[3] / rho
    p = (gamma - 1.0) * (Q[4] - 0.5 * rho * (u * u + v * v + w * w))
    return rho, u, v, w, p


def conserved(rho, u, v, w, p, gamma):
    return np.stack([rho, rho * u, rho * v, rho * w,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])


def pad_state(Q):
    """Interior (5, nth, nr, nx) -> padded (5, nth+4, nr+4, nx+4); ghosts NaN
    until fill_ghosts runs."""
    g = NG
    _, nth, nr, nx = Q.shape
    Qp = np.full((5, nth + 2 * g, nr + 2 * g, nx + 2 * g), np.nan, dtype=Q.dtype)
    Qp[:, g:-g, g:-g, g:-g] = Q
    return Qp


def interior(A):
    g = NG
    return A[..., g:-g, g:-g, g:-g]


# ---------------------------------------------------------------------------
# boundary conditions (section "Boundary Conditions")
# ---------------------------------------------------------------------------
def riemann_state(e, r, n, gamma):
    """Boundary state from Riemann invariants (far-field subsection).

    e, r: primitives (rho, u, v, w, p) inside / outside; n: outward unit
    normal (3, ...).  R+ = q_e + 2 a_e/(gamma-1), R- = q_r - 2 a_r/(gamma-1),
    q_f = (R+ + R-)/2, a_f = (gamma-1)(R+ - R-)/4.  Branches on M = q_e/a_e:
    M >= 1 interior state; M <= -1 outside state; q_e >= 0 subsonic exit
    (velocity corrected along n, entropy of e); else subsonic entrance
    (velocity corrected along n, entropy of r).  Returns primitives and the
    branch masks (sup_out, sup_in, sub_out)."""
    re, ue, ve, we, pe = e
    rr, ur, vr, wr, pr = r
    ae = np.sqrt(gamma * pe / re)
    ar = np.sqrt(gamma * pr / rr)
    qe = ue * n[0] + ve * n[1] + we * n[2]
    qr = ur * n[0] + vr * n[1] + wr * n[2]
    Rp = qe + 2.0 * ae / (gamma - 1.0)
    Rm = qr - 2.0 * ar / (gamma - 1.0)
    qf = 0.5 * (Rp + Rm)
    af = 0.25 * (gamma - 1.0) * (Rp - Rm)
    # subsonic exit: from the interior
    rho_o = (re ** gamma * af * af / (gamma * pe)) ** (1.0 / (gamma - 1.0))
    out = (rho_o,
           ue + (qf - qe) * n[0], ve + (qf - qe) * n[1], we + (qf - qe) * n[2],
           rho_o * af * af / gamma)
    # subsonic entrance: from the outside state
    rho_i = (rr ** gamma * af * af / (gamma * pr)) ** (1.0 / (gamma - 1.0))
    inn = (rho_i,
           ur + (qf - qr) * n[0], vr + (qf - qr) * n[1], wr + (qf - qr) * n[2],
           rho_i * af * af / gamma)
    M = np.real(qe / ae)
    sup_out = M >= 1.0
    sup_in = M <= -1.0
    sub_out = np.real(qe) >= 0.0
    f = []
    for c in range(5):
        rc = np.broadcast_to(r[c], np.shape(e[c]))
        f.append(np.where(sup_out, e[c], np.where(sup_in, rc,
                                                  np.where(sub_out, out[c], inn[c]))))
    return f, (sup_out, sup_in & ~sup_out, sub_out & ~sup_out & ~sup_in)


def _unit(Svec):
    mag = np.sqrt(Svec[0] * Svec[0] + Svec[1] * Svec[1] + Svec[2] * Svec[2])
    return Svec / mag


def fill_ghosts(Qp, geo, prm, inflow=None, held=None):
    """Fill the two ghost layers of the padded state in place.

    held: a padded state filled earlier (Q^n of schedule "step", L2) whose
    physical-face ghosts and centerline row are taken instead of evaluated.

    Order xi, eta, zeta (so that edge ghosts read already-filled values):
      xi-  periodic | entrance (data `inflow` = target primitives (5, nth, nr))
      xi+  periodic | exit (back pressure p_exit)
      eta- periodic | centerline: copy of (i, m, k + nth/2), m = 0, 1
      eta+ periodic | far field: Riemann invariants with the reference state
      zeta periodic (all i, j).
    Both ghost layers of a non-periodic face receive the same face state."""
    g = NG
    gamma = prm["gamma"]
    bc = prm["bc"]
    S, V = geo["S"], geo["V"]
    _, nthp, nrp, nxp = Qp.shape
    nth, nr, nx = nthp - 2 * g, nrp - 2 * g, nxp - 2 * g
    n = (nx, nr, nth)

    axis_node = bc[2] == "axis_node"
    if axis_node and held is not None:              # (L2) held centerline row
        Qp[:, g:g + nth, g, g:g + nx] = held[:, g:g + nth, g, g:g + nx]
    elif axis_node:                                 # (C1) axis row = mean of row j = 1
        ring = Qp[:, g:g + nth, g + 1, g:g + nx]
        Qp[:, g:g + nth, g, g:g + nx] = np.mean(ring, axis=1, keepdims=True)
    for d in range(3):
        lo_kind, hi_kind = bc[2 * d], bc[2 * d + 1]
        L = _fill_region(Qp, d, g)                  # (5, a, b, n_d + 2g)
        if held is not None:                        # (L2) held physical-face ghosts
            Lh = _fill_region(held, d, g)
            nd = n[d]
            if lo_kind in PHYSICAL_FACE_KINDS:
                L[..., :g] = Lh[..., :g]
            if hi_kind in PHYSICAL_FACE_KINDS:
                L[..., g + nd:] = Lh[..., g + nd:]
        Sd = _fill_region(S[d], d, g)               # (3, a, b, n_d + 2g)
        if axis_node and d == 0:                    # (C5) normals of the row j = 1
            Sd = Sd.copy()
            Sd[:, :, 0, :] = Sd[:, :, 1, :]
        nd = n[d]
        # periodic wraps
        if lo_kind == "periodic":
            for m in range(1, g + 1):
                L[..., g - m] = L[..., g + nd - m]
        if hi_kind == "periodic":
            for m in range(1, g + 1):
                L[..., g + nd - 1 + m] = L[..., g + m - 1]

        if lo_kind == "axis":
            for m in range(1, g + 1):
                L[..., g - m] = np.roll(L[..., g + m - 1], -(n[2] // 2), axis=1)
        if lo_kind == "axis_node":                  # (C2)
            for m in range(1, g + 1):
                L[..., g - m] = np.roll(L[..., g + m], -(n[2] // 2), axis=1)

        if held is not None:
            continue
        if lo_kind == "inflow":
            Qe = L[..., g]
            e = primitives(Qe, gamma)
            nrm = -_unit(Sd[..., g])                # outward normal at the entrance
            tgt = [np.asarray(inflow[c]) for c in range(5)]   # (nth, nr), like L[..., g]
            at = np.sqrt(gamma * tgt[4] / tgt[0])
            mn = -(tgt[1] * nrm[0] + tgt[2] * nrm[1] + tgt[3] * nrm[2]) / at
            f, (sup_out, _, _) = riemann_state(e, tgt, nrm, gamma)
            sup = np.real(mn) >= 1.0
            Qf = np.where(sup, conserved(*tgt, gamma),
                          np.where(sup_out, Qe, conserved(*f, gamma)))
            for m in range(1, g + 1):
                L[..., g - m] = Qf

        if hi_kind == "outflow":
            Qe = L[..., g + nd - 1]
            e = primitives(Qe, gamma)
            nrm = _unit(Sd[..., g + nd - 1])
            ae = np.sqrt(gamma * e[4] / e[0])
            qe = e[1] * nrm[0] + e[2] * nrm[1] + e[3] * nrm[2]
            sup = np.real(qe / ae) >= 1.0
            Qsub = conserved(e[0], e[1], e[2], e[3],
                             np.full_like(e[4], prm["p_exit"]), gamma)
            Qf = np.where(sup, Qe, Qsub)
            for m in range(1, g + 1):
                L[..., g + nd - 1 + m] = Qf

        if hi_kind == "farfield":
            Qe = L[..., g + nd - 1]
            e = primitives(Qe, gamma)
            nrm = _unit(Sd[..., g + nd - 1])
            ref = [np.asarray(c, dtype=float) for c in prm["ref_prim"]]
            f, (sup_out, _, _) = riemann_state(e, ref, nrm, gamma)
            Qf = np.where(sup_out, Qe, conserved(*f, gamma))
            for m in range(1, g + 1):
                L[..., g + nd - 1 + m] = Qf
    return Qp


# ---------------------------------------------------------------------------
# residual (section "Spatial Discretization")
# ---------------------------------------------------------------------------
def _lines(A, d, ng):
    """Direction-d lines of A at the interior of the two other directions
    (ng = ghost count of A along those directions); direction d last."""
    sl = [slice(None)] * A.ndim
    for dd in range(3):
        if dd != d:
            sl[_axis(A, dd)] = slice(ng, -ng)
    return np.moveaxis(A[tuple(sl)], _axis(A, d), -1)


def point_terms(Qp, geo, prm, visc=None, dyn=None):
    """Point quantities on the region where every index is in [-1, n].

    visc: held (mu, mu_t) over that region (schedule "step", L1), used in
    place of the values of this state; dyn: held coefficients of the
    dynamic model (D8), else computed from this state.

    Returns dict with (arrays over that region, shape (.., nth+2, nr+2, nx+2)):
      G[d]    = Fe^d - Fv^d, the inviscid minus viscous point flux (5 comps)
      lam[d]  = spectral radius lambda_d, lam_bar[d] its anisotropic scaling
      nu[d]   = pressure sensor along d
      mu, mu_t = molecular and SGS eddy viscosity (jet-viscosity units)
    and W over the whole padded box."""
    gamma = prm["gamma"]
    Cv = prm["visc_coef"]
    S_all, V_all = geo["S"], geo["V"]
    rho, u, v, w, p = primitives(Qp, gamma)
    E = Qp[4]
    T = gamma * p / rho                 # p = rho T / gamma (equation of state)
    a = np.sqrt(gamma * p / rho)

    c = (slice(1, -1),) * 3             # region one
    S = S_all[(slice(None), slice(None)) + c]
    V = V_all[c]
    r1 = lambda A: A[c]  # noqa: E731

    def delta(phi, d):
        """(phi_{+1} - phi_{-1})/2 along direction d, on region one."""
        ax = 2 - d
        hi = [slice(1, -1)] * 3
        lo = [slice(1, -1)] * 3
        hi[ax] = slice(2, None)
        lo[ax] = slice(None, -2)
        return (phi[tuple(hi)] - phi[tuple(lo)]) / 2.0

    def grad(phi):
        """Cartesian gradient by the chain rule: d phi/d x_m =
        sum_d (J^-1 grad xi_d)_m delta_d phi / J^-1."""
        dd = [delta(phi, d) for d in range(3)]
        return [(S[0, m] * dd[0] + S[1, m] * dd[1] + S[2, m] * dd[2]) / V
                for m in range(3)]

    out = {}
    # inviscid point fluxes (eq. hat-flux-G, contravariant velocity times J^-1)
    ru, rv, rw = r1(Qp[1]), r1(Qp[2]), r1(Qp[3])
    rho1, u1, v1, w1, p1, E1 = r1(rho), r1(u), r1(v), r1(w), r1(p), r1(E)
    Uc = [S[d, 0] * u1 + S[d, 1] * v1 + S[d, 2] * w1 for d in range(3)]
    Fe = [np.stack([rho1 * Uc[d],
                    ru * Uc[d] + p1 * S[d, 0],
                    rv * Uc[d] + p1 * S[d, 1],
                    rw * Uc[d] + p1 * S[d, 2],
                    (E1 + p1) * Uc[d]]) for d in range(3)]

    # viscous and SGS point fluxes (eqs. tau_mod, q_mod, hat-flux-Ev/Fv/Gv)
    if Cv != 0.0:
        Ssuth = prm["suth_S"]
        T1 = r1(T)
        mu = T1 ** 1.5 * (1.0 + Ssuth) / (T1 + Ssuth)      # Sutherland (R10)
        gu = [grad(u), grad(v), grad(w)]                    # gu[i][m] = d u_i / d x_m
        gT = grad(T)
        div = gu[0][0] + gu[1][1] + gu[2][2]
        if prm["sgs_model"] == 1 and prm["Cs"] != 0.0:
            Sij2 = 0.0
            for i in range(3):
                for j in range(3):
                    sij = 0.5 * (gu[i][j] + gu[j][i])
                    Sij2 = Sij2 + sij * sij
            Smag = np.sqrt(2.0 * Sij2)
            delta_f = rabs(V) ** (1.0 / 3.0)                # filter width (R9)
            mu_t = rho1 * (prm["Cs"] * delta_f) ** 2 * Smag / Cv   # (R7)
        elif prm["sgs_model"] == 2 and prm["Cs"] != 0.0:
            # Vreman model (subsection "Vreman Model"): alpha_ij = d u_j/d x_i,
            # beta_ij = Delta^2 alpha_mi alpha_mj, c = 2.5 Cs^2, mu_t = 0 where
            # alpha_ij alpha_ij = 0 (and where rounding makes B_beta <= 0)
            delta_f = rabs(V) ** (1.0 / 3.0)
            beta = [[delta_f ** 2 * (gu[i][0] * gu[j][0] + gu[i][1] * gu[j][1] + gu[i][2] * gu[j][2])
                     for j in range(3)] for i in range(3)]
            B = (beta[0][0] * beta[1][1] - beta[0][1] ** 2 + beta[0][0] * beta[2][2]
                 - beta[0][2] ** 2 + beta[1][1] * beta[2][2] - beta[1][2] ** 2)
            aa = sum(gu[i][j] ** 2 for i in range(3) for j in range(3))
            ok = (np.real(aa) > 0.0) & (np.real(B) > 0.0)
            ratio = np.sqrt(np.where(ok, B, 1.0) / np.where(ok, aa, 1.0))
            mu_t = np.where(ok, rho1 * (2.5 * prm["Cs"] ** 2) * ratio / Cv, 0.0 * rho1)
        elif prm["sgs_model"] == 3:
            # dynamic model (D1-D8): global coefficients, then the static forms
            if dyn is None:
                dyn = dynamic_coefficients(Qp, geo, prm)
            S2 = 0.0
            for i in range(3):
                for j in range(3):
                    S2 = S2 + (0.5 * (gu[i][j] + gu[j][i])) ** 2
            Smag2 = 2.0 * S2                                # |S|^2
            delta2 = rabs(V) ** (2.0 / 3.0)
            mu_t = rho1 * dyn["C_ds_eff"] * delta2 * np.sqrt(Smag2) / Cv      # (D5)
            p_sgs = (2.0 / 3.0) * dyn["C_I_eff"] * rho1 * delta2 * Smag2      # (D7)
            for d in range(3):
                Fe[d] = Fe[d] + np.stack([0.0 * p_sgs, p_sgs * S[d, 0], p_sgs * S[d, 1],
                                          p_sgs * S[d, 2], p_sgs * Uc[d]])
        else:
            mu_t = np.zeros_like(mu)
        if visc is not None:                                # (L1) held viscosities
            mu, mu_t = visc
        out["mu"], out["mu_t"] = mu, mu_t
        out["dyn"] = dyn
        Pr_sgs = dyn["Pr_eff"] if prm["sgs_model"] == 3 else prm["Pr_sgs"]
        tau = [[(mu + mu_t) * (gu[i][j] + gu[j][i] - (2.0 / 3.0 if i == j else 0.0) * div)
                for j in range(3)] for i in range(3)]
        kap = (mu / prm["Pr"] + mu_t / Pr_sgs) / (gamma - 1.0)
        q = [-kap * gT[j] for j in range(3)]                # (R6)
        vel = (u1, v1, w1)
        beta = [tau[0][j] * vel[0] + tau[1][j] * vel[1] + tau[2][j] * vel[2] - q[j]
                for j in range(3)]
        Fv = []
        for d in range(3):
            Fv.append(Cv * np.stack([
                np.zeros_like(u1),
                S[d, 0] * tau[0][0] + S[d, 1] * tau[0][1] + S[d, 2] * tau[0][2],
                S[d, 0] * tau[1][0] + S[d, 1] * tau[1][1] + S[d, 2] * tau[1][2],
                S[d, 0] * tau[2][0] + S[d, 1] * tau[2][1] + S[d, 2] * tau[2][2],
                S[d, 0] * beta[0] + S[d, 1] * beta[1] + S[d, 2] * beta[2]]))
        out["G"] = [Fe[d] - Fv[d] for d in range(3)]
    else:
        out["G"] = Fe

    # dissipation ingredients (spectral radii R4, sensor R3, W R1)
    a1 = r1(a)
    Smag_d = [np.sqrt(S[d, 0] ** 2 + S[d, 1] ** 2 + S[d, 2] ** 2) for d in range(3)]
    lam = [(rabs(Uc[d]) + a1 * Smag_d[d]) / rabs(V) for d in range(3)]
    lam_bar = []
    for d in range(3):
        o1, o2 = lam[(d + 1) % 3], lam[(d + 2) % 3]
        lam_bar.append(lam[d] * (1.0 + np.sqrt(o1 / lam[d]) + np.sqrt(o2 / lam[d])))
    nu = []
    for d in range(3):
        ax = 2 - d
        hi = [slice(1, -1)] * 3
        lo = [slice(1, -1)] * 3
        hi[ax] = slice(2, None)
        lo[ax] = slice(None, -2)
        pp, pm = p[tuple(hi)], p[tuple(lo)]
        nu.append(rabs(pp - 2.0 * p1 + pm) / (pp + 2.0 * p1 + pm))
    out.update(lam=lam, lam_bar=lam_bar, nu=nu, V=V,
               W=np.stack([Qp[0], Qp[1], Qp[2], Qp[3], Qp[4] + p]))
    if prm["bc"][2] == "axis_node":
        # (C3) region one starts at j = -1, so the axis row is index 1
        out["G"][1][..., 1, :] = 0.0
    return out


def test_filter(A):
    """Separable three-point test filter (1/4, 1/2, 1/4) along the last three
    axes (D1); the result is one point shorter at each end of each axis."""
    for ax in (-1, -2, -3):
        n = A.shape[ax]
        lo = np.take(A, range(0, n - 2), axis=ax)
        mid = np.take(A, range(1, n - 1), axis=ax)
        hi = np.take(A, range(2, n), axis=ax)
        A = 0.25 * lo + 0.5 * mid + 0.25 * hi
    return A


def dynamic_coefficients(Qp, geo, prm):
    """Coefficients C_I, C_ds and Pr_sgs of the dynamic model (subsection
    "Dynamic Smagorinsky Model"; readings D1-D6) from a padded state whose
    ghosts are filled.  Returns the raw ratios, the volume-weighted sums
    they come from, and the values used (C_I_eff, C_ds_eff, Pr_eff)."""
    if prm["bc"][2] == "axis_node":
        raise NotImplementedError("the dynamic model's test filter would average the axis "
                                  "row, where J^-1 = 0 leaves the strain undefined")
    gamma = prm["gamma"]
    rho, u, v, w, p = primitives(Qp, gamma)
    T = gamma * p / rho
    vel = (u, v, w)
    S_all, V_all = geo["S"], geo["V"]

    def grad_on(phi, S, V):
        """chain-rule gradient of phi (one point wider than S, V) on the
        region of S, V."""
        dd = []
        for d in range(3):
            ax = 2 - d
            hi = [slice(1, -1)] * 3
            lo = [slice(1, -1)] * 3
            hi[ax] = slice(2, None)
            lo[ax] = slice(None, -2)
            dd.append((phi[tuple(hi)] - phi[tuple(lo)]) / 2.0)
        return [(S[0, m] * dd[0] + S[1, m] * dd[1] + S[2, m] * dd[2]) / V for m in range(3)]

    r1 = (slice(1, -1),) * 3              # region one of the padded box
    it = (slice(2, -2),) * 3              # interior of the padded box
    S1, V1 = S_all[(slice(None), slice(None)) + r1], V_all[r1]
    Si, Vi = S_all[(slice(None), slice(None)) + it], V_all[it]
    # resolved strain, |S| and temperature gradient on region one
    gu = [grad_on(vel[i], S1, V1) for i in range(3)]
    gT = grad_on(T, S1, V1)
    Sij = [[0.5 * (gu[i][j] + gu[j][i]) for j in range(3)] for i in range(3)]
    Smag = np.sqrt(2.0 * sum(Sij[i][j] ** 2 for i in range(3) for j in range(3)))
    rho1 = rho[r1]
    # fields filtered from region one to the interior
    h_rSS = [[test_filter(rho1 * Smag * Sij[i][j]) for j in range(3)] for i in range(3)]
    h_rS2 = test_filter(rho1 * Smag ** 2)
    h_rST = [test_filter(rho1 * Smag * gT[j]) for j in range(3)]
    # state products filtered from the padded box to region one
    f_r = test_filter(rho)
    f_ru = [test_filter(rho * vel[i]) for i in range(3)]
    f_rT = test_filter(rho * T)
    # ... and their interior part
    c = (slice(1, -1),) * 3
    h_r = f_r[c]
    h_ru = [f_ru[i][c] for i in range(3)]
    h_rT = f_rT[c]
    h_ruu = [[test_filter(rho * vel[i] * vel[j])[c] for j in range(3)] for i in range(3)]
    h_ruT = [test_filter(rho * vel[j] * T)[c] for j in range(3)]
    # strain of u_hat and gradient of T_hat on the interior (D4, D6)
    uh = [f_ru[i] / f_r for i in range(3)]
    guh = [grad_on(uh[i], Si, Vi) for i in range(3)]
    gTh = grad_on(f_rT / f_r, Si, Vi)
    Shij = [[0.5 * (guh[i][j] + guh[j][i]) for j in range(3)] for i in range(3)]
    Shmag = np.sqrt(2.0 * sum(Shij[i][j] ** 2 for i in range(3) for j in range(3)))
    # resolved quantities at the interior
    Sc = [[Sij[i][j][c] for j in range(3)] for i in range(3)]
    Smc = Smag[c]
    gTc = [gT[j][c] for j in range(3)]
    D2 = rabs(Vi) ** (2.0 / 3.0)          # Delta^2 (R9)
    Dh2 = 4.0 * D2                        # Delta_hat = 2 Delta (D1)
    trS = Sc[0][0] + Sc[1][1] + Sc[2][2]
    L = [[h_ruu[i][j] - h_ru[i] * h_ru[j] / h_r for j in range(3)] for i in range(3)]
    Lll = L[0][0] + L[1][1] + L[2][2]
    LS = sum(L[i][j] * Sc[i][j] for i in range(3) for j in range(3))
    # C_I (eq. av_ci)
    N_I = Lll
    D_I = 2.0 * Dh2 * h_r * Shmag ** 2 - 2.0 * D2 * h_rS2
    # C_ds (eq. av_cd): numerator = A + C_I B (D3)
    A = LS - trS * Lll / 3.0
    B = trS * 2.0 * D2 * h_rS2 / 3.0
    h_rSS_S = sum(h_rSS[i][j] * Sc[i][j] for i in range(3) for j in range(3))
    h_rSmm = h_rSS[0][0] + h_rSS[1][1] + h_rSS[2][2]
    Sh_S = sum(Shij[i][j] * Sc[i][j] for i in range(3) for j in range(3))
    trSh = Shij[0][0] + Shij[1][1] + Shij[2][2]
    D_d = (2.0 * D2 * (h_rSS_S - h_rSmm * trS / 3.0)
           - 2.0 * Dh2 * (h_r * Shmag * Sh_S - h_r * Shmag * trSh * trS / 3.0))
    # Pr_sgs (eq. av_Pr_sgs, D6)
    N_P = sum(D2 * h_rST[j] * gTc[j] - Dh2 * h_r * Shmag * gTh[j] * gTc[j] for j in range(3))
    D_P = sum((h_ruT[j] - h_ru[j] * h_rT / h_r) * gTc[j] for j in range(3))
    sums = {k: float(np.sum(np.real(Vi * a))) for k, a in
            dict(N_I=N_I, D_I=D_I, A=A, B=B, D_d=D_d, N_P=N_P, D_P=D_P).items()}
    C_I = sums["N_I"] / sums["D_I"] if sums["D_I"] != 0.0 else 0.0
    C_I_eff = max(C_I, 0.0)
    # C_ds uses the C_I of the isotropic term actually modelled (D3, D5)
    C_ds = (sums["A"] + C_I_eff * sums["B"]) / sums["D_d"] if sums["D_d"] != 0.0 else 0.0
    C_ds_eff = max(C_ds, 0.0)
    Pr = C_ds_eff * sums["N_P"] / sums["D_P"] if sums["D_P"] != 0.0 else float("nan")
    Pr_eff = Pr if np.isfinite(Pr) and Pr > 0.0 else prm["Pr_sgs"]
    return dict(C_I=C_I, C_ds=C_ds, Pr_sgs=Pr, C_I_eff=C_I_eff, C_ds_eff=C_ds_eff,
                Pr_eff=Pr_eff, sums=sums)


def face_fluxes(pt, d, prm):
    """Numerical fluxes at the faces -1/2 .. n_d - 1/2 along direction d
    (eq. inv_flux_vec with the dissipation of eq. dissip_term), on the
    interior of the two other directions.  Shape (5, ..., n_d + 1)."""
    G = _lines(pt["G"][d], d, 1)           # (5, a, b, n_d + 2): points -1 .. n_d
    lb = _lines(pt["lam_bar"][d], d, 1)
    nu = _lines(pt["nu"][d], d, 1)
    V = _lines(pt["V"], d, 1)
    W = _lines(pt["W"], d, 2)              # (5, a, b, n_d + 4): points -2 .. n_d + 1
    GL, GR = G[..., :-1], G[..., 1:]       # L = -1 .. n_d - 1
    eps2 = prm["k2"] * rmax(nu[..., :-1], nu[..., 1:])
    eps4 = rmax(0.0 * eps2, prm["k4"] - eps2)
    lam_f = 0.5 * (lb[..., :-1] + lb[..., 1:])
    V_f = 0.5 * (V[..., :-1] + V[..., 1:])
    Wm, WL, WR, Wp = W[..., :-3], W[..., 1:-2], W[..., 2:-1], W[..., 3:]
    d4 = Wp - 3.0 * WR + 3.0 * WL - Wm
    if d == 1 and prm["bc"][2] == "axis_node":
        # (C4) the axis face is face index 1 (L = 0, R = 1)
        lam_f = lam_f.copy()
        lam_f[..., 1] = lb[..., 2]
        d4 = d4.copy()
        d4[..., 1] = Wp[..., 1] - 4.0 * WR[..., 1] + 3.0 * WL[..., 1]
    dis = lam_f * (eps2 * (WR - WL) - eps4 * d4)
    lo_kind, hi_kind = prm["bc"][2 * d], prm["bc"][2 * d + 1]
    if lo_kind in PHYSICAL_FACE_KINDS:     # R15
        dis[..., 0] = 0.0
    if hi_kind in PHYSICAL_FACE_KINDS:
        dis[..., -1] = 0.0
    return 0.5 * (GL + GR) - V_f * dis


def residual(Qp, geo, prm, visc=None, dyn=None):
    """R = RHS / V on the interior, for a padded state whose ghosts are
    filled; dQ/dt = -R (eq. spatial_discret with unit index spacing).
    visc, dyn: held viscosities and dynamic coefficients (see point_terms)."""
    axis_node = prm["bc"][2] == "axis_node"
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        pt = point_terms(Qp, geo, prm, visc, dyn)
        rhs = 0.0
        for d in range(3):
            F = face_fluxes(pt, d, prm)
            diff = F[..., 1:] - F[..., :-1]
            rhs = rhs + np.moveaxis(diff, -1, diff.ndim - 1 - d)
        R = rhs / interior(geo["V"])
    if axis_node:
        R[:, :, 0, :] = 0.0                          # (C1) the axis row is not advanced
    return R


def lambda_sum(Qp, geo, prm):
    """lambda_xi + lambda_eta + lambda_zeta on the interior."""
    gamma = prm["gamma"]
    Q = interior(Qp)
    S = interior(geo["S"])
    V = interior(geo["V"])
    rho, u, v, w, p = primitives(Q, gamma)
    a = np.sqrt(gamma * p / rho)
    tot = 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        for d in range(3):
            Uc = S[d, 0] * u + S[d, 1] * v + S[d, 2] * w
            tot = tot + (rabs(Uc) + a * np.sqrt(S[d, 0] ** 2 + S[d, 1] ** 2 + S[d, 2] ** 2)) / rabs(V)
    if prm["bc"][2] == "axis_node":
        tot = tot.copy()
        tot[:, 0, :] = 0.0                           # (C6) the axis row has V = 0
    return tot


def time_step(Q, geo, prm):
    """Global dt = CFL / max_interior(lambda sum) (reading R18)."""
    Qp = pad_state(Q)
    return prm["cfl"] / np.max(np.real(lambda_sum(Qp, geo, prm)))


def evaluate(Q, geo, prm, inflow=None):
    """Residual of an interior state: pad, fill ghosts, residual."""
    Qp = pad_state(np.asarray(Q))
    fill_ghosts(Qp, geo, prm, inflow)
    return residual(Qp, geo, prm)


# ---------------------------------------------------------------------------
# time marching (section "Time Marching Method")
# ---------------------------------------------------------------------------
def jameson_rk(Q0, resid, dt, alpha):
    """Q^(l) = Q^(0) - alpha_l dt R(Q^(l-1)), l = 1..len(alpha); returns the
    last stage.  `resid` maps a state to R."""
    Q = Q0
    for a in alpha:
        Q = Q0 - a * dt * resid(Q)
    return Q


def held_state(Q, geo, prm, inflow=None):
    """Schedule "step" (L1, L2, D8): the padded Q^n with its ghosts filled,
    its viscosities (mu, mu_t) on region one and its dynamic-model
    coefficients (None when inviscid / not dynamic)."""
    Hp = pad_state(np.asarray(Q))
    fill_ghosts(Hp, geo, prm, inflow)
    if prm["visc_coef"] == 0.0:
        return Hp, None, None
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        pt = point_terms(Hp, geo, prm)
    return Hp, (pt["mu"], pt["mu_t"]), pt["dyn"]


def rk5_step(Q, geo, prm, inflow=None, dt=None):
    """One RK5 time step of the interior state Q; dt from CFL when None.
    Returns (Q^{n+1}, dt)."""
    if dt is None:
        dt = time_step(Q, geo, prm)
    if prm.get("schedule", "stage") == "step":
        Hp, visc, dyn = held_state(Q, geo, prm, inflow)

        def resid(q):
            Qp = pad_state(q)
            fill_ghosts(Qp, geo, prm, inflow, held=Hp)
            return residual(Qp, geo, prm, visc, dyn)
    else:
        def resid(q):
            return evaluate(q, geo, prm, inflow)
    Qn = jameson_rk(np.asarray(Q), resid, dt, prm["rk_alpha"])
    return Qn, dt


def run(Q, geo, prm, inflow=None, steps=1, dt=None):
    """`steps` RK5 steps; returns (Q, list of dt)."""
    dts = []
    for _ in range(steps):
        Q, h = rk5_step(Q, geo, prm, inflow, dt)
        dts.append(h)
    return Q, dts
