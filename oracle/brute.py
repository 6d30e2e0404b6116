"""Scalar brute-force version of the oracle for tiny grids.

TEST INFRASTRUCTURE ONLY (see oracle/les.py for the readings of the paper).

Every quantity is computed point by point and face by face with plain Python
floats and dictionaries keyed by (i, j, k), written independently of the
vectorised oracle, so that slicing or axis mistakes in one show up as a
mismatch against the other.  Cost grows like n^3 with large constants: use
only on grids of a few hundred points.
"""
import math

NG = 2
NGC = 3


def _add(a, b):
    return [x + y for x, y in zip(a, b)]


def _sub(a, b):
    return [x - y for x, y in zip(a, b)]


def _scale(s, a):
    return [s * x for x in a]


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


class Brute:
    """Residual of the LES discretisation on a tiny grid, point by point."""

    def __init__(self, xyz, prm, inflow=None):
        self.prm = prm
        _, nth, nr, nx = xyz.shape
        self.n = (nx, nr, nth)
        self.inflow = inflow
        self.X = {}
        for k in range(nth):
            for j in range(nr):
                for i in range(nx):
                    self.X[(i, j, k)] = [float(xyz[c, k, j, i]) for c in range(3)]
        self._coord_ghosts()
        self._met = {}

    # -- index helpers -------------------------------------------------------
    @staticmethod
    def _shift(p, d, s):
        q = list(p)
        q[d] += s
        return tuple(q)

    def _ranges(self, d, g):
        """Index ranges of the other two directions when direction d is
        filled (order xi, eta, zeta)."""
        nx, nr, nth = self.n
        full = [range(-g, nx + g), range(-g, nr + g), range(-g, nth + g)]
        inner = [range(nx), range(nr), range(nth)]
        if d == 0:
            return [None, inner[1], inner[2]]
        if d == 1:
            return [full[0], None, inner[2]]
        return [full[0], full[1], None]

    def _points_on_plane(self, d, g, idx):
        rg = self._ranges(d, g)
        others = [e for e in range(3) if e != d]
        for a in rg[others[0]]:
            for b in rg[others[1]]:
                p = [0, 0, 0]
                p[d] = idx
                p[others[0]] = a
                p[others[1]] = b
                yield tuple(p)

    # -- coordinates ---------------------------------------------------------
    def _coord_ghosts(self):
        g = NGC
        bc = self.prm["bc"]
        per = self.prm["period"]
        for d in range(3):
            nd = self.n[d]
            for m in range(1, g + 1):
                for p in self._points_on_plane(d, g, -m):
                    kind = bc[2 * d]
                    if kind == "periodic":
                        self.X[p] = _sub(self.X[self._shift(p, d, nd)], list(per[d]))
                    elif kind == "axis":
                        i, j, k = p
                        src = (i, m - 1, (k + self.n[2] // 2) % self.n[2])
                        self.X[p] = list(self.X[src])
                    elif kind == "axis_node":          # mirror through the axis node
                        i, j, k = p
                        src = (i, m, (k + self.n[2] // 2) % self.n[2])
                        self.X[p] = list(self.X[src])
                    else:
                        b0 = self.X[self._shift(p, d, m)]
                        b1 = self.X[self._shift(p, d, m + 1)]
                        self.X[p] = _add(b0, _scale(m, _sub(b0, b1)))
                for p in self._points_on_plane(d, g, nd - 1 + m):
                    kind = bc[2 * d + 1]
                    if kind == "periodic":
                        self.X[p] = _add(self.X[self._shift(p, d, -nd)], list(per[d]))
                    else:
                        b0 = self.X[self._shift(p, d, -m)]
                        b1 = self.X[self._shift(p, d, -m - 1)]
                        self.X[p] = _add(b0, _scale(m, _sub(b0, b1)))

    def metric(self, p):
        """(S^xi, S^eta, S^zeta, V) at point p from central differences."""
        if p not in self._met:
            r = []
            for d in range(3):
                r.append(_scale(0.5, _sub(self.X[self._shift(p, d, 1)],
                                          self.X[self._shift(p, d, -1)])))
            Sx = _cross(r[1], r[2])
            Se = _cross(r[2], r[0])
            Sz = _cross(r[0], r[1])
            V = _dot(r[0], _cross(r[1], r[2]))
            self._met[p] = ([Sx, Se, Sz], V)
        return self._met[p]

    # -- state ---------------------------------------------------------------
    def prim(self, q):
        g = self.prm["gamma"]
        rho = q[0]
        u, v, w = q[1] / rho, q[2] / rho, q[3] / rho
        p = (g - 1.0) * (q[4] - 0.5 * rho * (u * u + v * v + w * w))
        return rho, u, v, w, p

    def cons(self, rho, u, v, w, p):
        g = self.prm["gamma"]
        return [rho, rho * u, rho * v, rho * w, p / (g - 1.0) + 0.5 * rho * (u * u + v * v + w * w)]

    def riemann(self, e, r, n):
        g = self.prm["gamma"]
        ae = math.sqrt(g * e[4] / e[0])
        ar = math.sqrt(g * r[4] / r[0])
        qe = e[1] * n[0] + e[2] * n[1] + e[3] * n[2]
        qr = r[1] * n[0] + r[2] * n[1] + r[3] * n[2]
        Rp = qe + 2.0 * ae / (g - 1.0)
        Rm = qr - 2.0 * ar / (g - 1.0)
        qf = 0.5 * (Rp + Rm)
        af = 0.25 * (g - 1.0) * (Rp - Rm)
        if qe / ae >= 1.0:
            return "copy", None
        if qe / ae <= -1.0:
            return "outside", list(r)
        src, qs = (e, qe) if qe >= 0.0 else (r, qr)
        rho = (src[0] ** g * af * af / (g * src[4])) ** (1.0 / (g - 1.0))
        return "sub", [rho, src[1] + (qf - qs) * n[0], src[2] + (qf - qs) * n[1],
                       src[3] + (qf - qs) * n[2], rho * af * af / g]

    def fill(self, Q, held=None):
        """Padded state dict from the interior array Q (5, nth, nr, nx).
        held: padded state dict of Q^n (schedule "step"): its centerline row
        and physical-face ghosts are taken, not evaluated."""
        nx, nr, nth = self.n
        g = NG
        prm = self.prm
        bc = prm["bc"]
        gam = prm["gamma"]
        S = {}
        for k in range(nth):
            for j in range(nr):
                for i in range(nx):
                    S[(i, j, k)] = [float(Q[c, k, j, i]) for c in range(5)]
        axis_node = bc[2] == "axis_node"
        if axis_node and held is not None:
            for i in range(nx):
                for k in range(nth):
                    S[(i, 0, k)] = list(held[(i, 0, k)])
        elif axis_node:
            # centerline: mean over the azimuth of the row j = 1, for every k
            for i in range(nx):
                mean = [sum(S[(i, 1, k)][c] for k in range(nth)) / nth for c in range(5)]
                for k in range(nth):
                    S[(i, 0, k)] = list(mean)
        for d in range(3):
            nd = self.n[d]
            # low side
            for m in range(1, g + 1):
                for p in self._points_on_plane(d, g, -m):
                    kind = bc[2 * d]
                    if held is not None and kind in ("inflow", "outflow", "farfield"):
                        S[p] = list(held[p])
                    elif kind == "periodic":
                        S[p] = list(S[self._shift(p, d, nd)])
                    elif kind == "axis":
                        i, j, k = p
                        S[p] = list(S[(i, m - 1, (k + nth // 2) % nth)])
                    elif kind == "axis_node":
                        i, j, k = p
                        S[p] = list(S[(i, m, (k + nth // 2) % nth)])
                    elif kind == "inflow":
                        e_pt = self._shift(p, d, m)
                        i, j, k = e_pt
                        n_pt = (i, 1, k) if axis_node and j == 0 else e_pt
                        Sx = self.metric(n_pt)[0][0]
                        mag = math.sqrt(_dot(Sx, Sx))
                        n = [-c / mag for c in Sx]
                        t = [float(self.inflow[c][k][j]) for c in range(5)]
                        at = math.sqrt(gam * t[4] / t[0])
                        mn = -(t[1] * n[0] + t[2] * n[1] + t[3] * n[2]) / at
                        if mn >= 1.0:
                            S[p] = self.cons(*t)
                        else:
                            br, f = self.riemann(self.prim(S[e_pt]), t, n)
                            S[p] = list(S[e_pt]) if br == "copy" else self.cons(*f)
            # high side
            for m in range(1, g + 1):
                for p in self._points_on_plane(d, g, nd - 1 + m):
                    kind = bc[2 * d + 1]
                    e_pt = self._shift(p, d, -m)
                    if held is not None and kind in ("inflow", "outflow", "farfield"):
                        S[p] = list(held[p])
                    elif kind == "periodic":
                        S[p] = list(S[self._shift(p, d, -nd)])
                    elif kind == "outflow":
                        e = self.prim(S[e_pt])
                        n_pt = (e_pt[0], 1, e_pt[2]) if axis_node and e_pt[1] == 0 else e_pt
                        Sx = self.metric(n_pt)[0][0]
                        mag = math.sqrt(_dot(Sx, Sx))
                        n = [c / mag for c in Sx]
                        ae = math.sqrt(gam * e[4] / e[0])
                        if (e[1] * n[0] + e[2] * n[1] + e[3] * n[2]) / ae >= 1.0:
                            S[p] = list(S[e_pt])
                        else:
                            S[p] = self.cons(e[0], e[1], e[2], e[3], prm["p_exit"])
                    elif kind == "farfield":
                        Sd = self.metric(e_pt)[0][d]
                        mag = math.sqrt(_dot(Sd, Sd))
                        n = [c / mag for c in Sd]
                        br, f = self.riemann(self.prim(S[e_pt]), list(prm["ref_prim"]), n)
                        S[p] = list(S[e_pt]) if br == "copy" else self.cons(*f)
        return S

    # -- point terms ---------------------------------------------------------
    def point(self, S, p):
        """Primitive and derived quantities needed at point p."""
        prm = self.prm
        gam = prm["gamma"]
        rho, u, v, w, pr = self.prim(S[p])
        T = gam * pr / rho
        return dict(rho=rho, u=u, v=v, w=w, p=pr, T=T, a=math.sqrt(gam * pr / rho), q=S[p])

    def gradients(self, S, p):
        """d(u,v,w,T)/dx_m at p, chain rule over central differences."""
        Sm, V = self.metric(p)
        dl = []
        for d in range(3):
            a = self.point(S, self._shift(p, d, 1))
            b = self.point(S, self._shift(p, d, -1))
            dl.append({f: 0.5 * (a[f] - b[f]) for f in ("u", "v", "w", "T")})
        out = {}
        for f in ("u", "v", "w", "T"):
            out[f] = [(Sm[0][m] * dl[0][f] + Sm[1][m] * dl[1][f] + Sm[2][m] * dl[2][f]) / V
                      for m in range(3)]
        return out

    def viscosity(self, S, p):
        """(mu, mu_sgs) at p in jet-viscosity units: Sutherland and the SGS
        model of the parameters."""
        prm = self.prm
        Cv = prm["visc_coef"]
        _, V = self.metric(p)
        P = self.point(S, p)
        gr = self.gradients(S, p)
        g = [gr["u"], gr["v"], gr["w"]]
        T = P["T"]
        Ss = prm["suth_S"]
        mu = T ** 1.5 * (1.0 + Ss) / (T + Ss)
        mut = 0.0
        if prm["sgs_model"] == 1 and prm["Cs"] != 0.0:
            s2 = 0.0
            for i in range(3):
                for j in range(3):
                    s2 += (0.5 * (g[i][j] + g[j][i])) ** 2
            delta = abs(V) ** (1.0 / 3.0)
            mut = P["rho"] * (prm["Cs"] * delta) ** 2 * math.sqrt(2.0 * s2) / Cv
        elif prm["sgs_model"] == 2 and prm["Cs"] != 0.0:
            # Vreman: alpha_ij = d u_j / d x_i, beta_ij = Delta^2 alpha_mi alpha_mj
            alpha = [[g[j][i] for j in range(3)] for i in range(3)]
            delta = abs(V) ** (1.0 / 3.0)
            beta = [[delta ** 2 * sum(alpha[m][i] * alpha[m][j] for m in range(3))
                     for j in range(3)] for i in range(3)]
            B = (beta[0][0] * beta[1][1] - beta[0][1] ** 2 + beta[0][0] * beta[2][2]
                 - beta[0][2] ** 2 + beta[1][1] * beta[2][2] - beta[1][2] ** 2)
            aa = sum(alpha[i][j] ** 2 for i in range(3) for j in range(3))
            c = 2.5 * prm["Cs"] ** 2
            mut = P["rho"] * c * math.sqrt(B / aa) / Cv if aa > 0.0 and B > 0.0 else 0.0
        return mu, mut

    def point_flux(self, S, p, d, visc=None):
        """Inviscid minus viscous point flux along d at p (5 components);
        visc: held {point: (mu, mu_sgs)} (schedule "step")."""
        prm = self.prm
        gam = prm["gamma"]
        Cv = prm["visc_coef"]
        Sm, V = self.metric(p)
        Sd = Sm[d]
        P = self.point(S, p)
        q = P["q"]
        Uc = Sd[0] * P["u"] + Sd[1] * P["v"] + Sd[2] * P["w"]
        F = [P["rho"] * Uc,
             q[1] * Uc + P["p"] * Sd[0],
             q[2] * Uc + P["p"] * Sd[1],
             q[3] * Uc + P["p"] * Sd[2],
             (q[4] + P["p"]) * Uc]
        if Cv == 0.0:
            return F
        gr = self.gradients(S, p)
        g = [gr["u"], gr["v"], gr["w"]]
        mu, mut = visc[p] if visc is not None else self.viscosity(S, p)
        div = g[0][0] + g[1][1] + g[2][2]
        tau = [[(mu + mut) * (g[i][j] + g[j][i] - (2.0 / 3.0 if i == j else 0.0) * div)
                for j in range(3)] for i in range(3)]
        kap = (mu / prm["Pr"] + mut / prm["Pr_sgs"]) / (gam - 1.0)
        vel = [P["u"], P["v"], P["w"]]
        beta = [sum(tau[i][j] * vel[i] for i in range(3)) + kap * gr["T"][j] for j in range(3)]
        Fv = [0.0] + [Cv * _dot(Sd, tau[i]) for i in range(3)] + [Cv * _dot(Sd, beta)]
        return [F[c] - Fv[c] for c in range(5)]

    def lambdas(self, S, p):
        Sm, V = self.metric(p)
        P = self.point(S, p)
        lam = []
        for d in range(3):
            Uc = _dot(Sm[d], [P["u"], P["v"], P["w"]])
            lam.append((abs(Uc) + P["a"] * math.sqrt(_dot(Sm[d], Sm[d]))) / abs(V))
        return lam

    def lam_bar(self, S, p, d):
        lam = self.lambdas(S, p)
        o1, o2 = lam[(d + 1) % 3], lam[(d + 2) % 3]
        return lam[d] * (1.0 + math.sqrt(o1 / lam[d]) + math.sqrt(o2 / lam[d]))

    def sensor(self, S, p, d):
        pp = self.point(S, self._shift(p, d, 1))["p"]
        pc = self.point(S, p)["p"]
        pm = self.point(S, self._shift(p, d, -1))["p"]
        return abs(pp - 2.0 * pc + pm) / (pp + 2.0 * pc + pm)

    def W(self, S, p):
        q = S[p]
        return [q[0], q[1], q[2], q[3], q[4] + self.point(S, p)["p"]]

    def face(self, S, L, d, visc=None):
        """Numerical flux at the face between L and L + e_d."""
        prm = self.prm
        R = self._shift(L, d, 1)
        axis_face = prm["bc"][2] == "axis_node" and d == 1 and L[1] == 0
        GL = [0.0] * 5 if axis_face else self.point_flux(S, L, d, visc)
        GR = self.point_flux(S, R, d, visc)
        e2 = prm["k2"] * max(self.sensor(S, L, d), self.sensor(S, R, d))
        e4 = max(0.0, prm["k4"] - e2)
        if axis_face:     # the axis point has V = 0: lambda_bar of the j = 1 point
            lam = self.lam_bar(S, R, d)
        else:
            lam = 0.5 * (self.lam_bar(S, L, d) + self.lam_bar(S, R, d))
        Vf = 0.5 * (self.metric(L)[1] + self.metric(R)[1])
        Wm = self.W(S, self._shift(L, d, -1))
        WL, WR = self.W(S, L), self.W(S, R)
        Wp = self.W(S, self._shift(R, d, 1))
        physical = (L[d] == -1 and prm["bc"][2 * d] in ("inflow", "outflow", "farfield")) or \
                   (L[d] == self.n[d] - 1 and prm["bc"][2 * d + 1] in ("inflow", "outflow", "farfield"))
        out = []
        for c in range(5):
            if axis_face:   # (Delta w)_{-1/2} = -(Delta w)_{1/2} at the centerline
                d4 = Wp[c] - 4.0 * WR[c] + 3.0 * WL[c]
            else:
                d4 = Wp[c] - 3.0 * WR[c] + 3.0 * WL[c] - Wm[c]
            dis = 0.0 if physical else lam * (e2 * (WR[c] - WL[c]) - e4 * d4)
            out.append(0.5 * (GL[c] + GR[c]) - Vf * dis)
        return out

    def residual(self, Q, held=None, visc=None):
        """R (5, nth, nr, nx) as nested lists -> returned as a dict of points.
        held, visc: schedule "step" (see fill and point_flux)."""
        S = self.fill(Q, held)
        nx, nr, nth = self.n
        R = {}
        for k in range(nth):
            for j in range(nr):
                for i in range(nx):
                    p = (i, j, k)
                    if j == 0 and self.prm["bc"][2] == "axis_node":
                        R[p] = [0.0] * 5          # the axis row is not advanced
                        continue
                    acc = [0.0] * 5
                    for d in range(3):
                        Fp = self.face(S, p, d, visc)
                        Fm = self.face(S, self._shift(p, d, -1), d, visc)
                        acc = [a + fp - fm for a, fp, fm in zip(acc, Fp, Fm)]
                    V = self.metric(p)[1]
                    R[p] = [a / V for a in acc]
        return R, S

    def step(self, Q, dt, schedule="stage"):
        """One five-stage step Q^(l) = Q^n - alpha_l dt R(Q^(l-1)) of the
        interior array Q (indexable as Q[c, k, j, i]); schedule "step"
        evaluates the ghosts of physical faces, the centerline row and
        (mu, mu_sgs) from Q^n only and holds them through the stages.
        Returns {point: 5 values}."""
        nx, nr, nth = self.n
        held = visc = None
        if schedule == "step":
            held = self.fill(Q)
            if self.prm["visc_coef"] != 0.0:
                visc = {}
                for p in held:
                    i, j, k = p
                    # region one; axis points (V = 0) carry no viscous flux
                    if -1 <= i <= nx and -1 <= j <= nr and -1 <= k <= nth and \
                            self.metric(p)[1] != 0.0:
                        visc[p] = self.viscosity(held, p)
        pts = [(i, j, k) for k in range(nth) for j in range(nr) for i in range(nx)]
        Q0 = {p: [float(Q[c, p[2], p[1], p[0]]) for c in range(5)] for p in pts}
        cur = Q0
        for a in self.prm["rk_alpha"]:
            R, _ = self.residual(_PointArray(cur), held, visc)
            cur = {p: [Q0[p][c] - a * dt * R[p][c] for c in range(5)] for p in pts}
        return cur


    def dynamic_sums(self, Q):
        """The seven J^-1-weighted interior sums of the dynamic model
        (subsection "Dynamic Smagorinsky Model", readings D1-D6): N_I, D_I
        (C_I = N_I / D_I), A, B, D_d (C_ds = (A + C_I+ B) / D_d), N_P, D_P
        (Pr_sgs = C_ds+ N_P / D_P), and for each the sum of the absolute
        values of its terms.  The test filter is the explicit 27-point
        product of (1/4, 1/2, 1/4) weights."""
        S = self.fill(Q)
        nx, nr, nth = self.n
        wt = (0.25, 0.5, 0.25)
        offs = [(a, b, c) for c in (-1, 0, 1) for b in (-1, 0, 1) for a in (-1, 0, 1)]

        def hat(fn, p, nf):
            tot = [0.0] * nf
            for a, b, c in offs:
                w = wt[a + 1] * wt[b + 1] * wt[c + 1]
                v = fn((p[0] + a, p[1] + b, p[2] + c))
                tot = [t + w * x for t, x in zip(tot, v)]
            return tot

        res = {}

        def resolved(p):
            """strain S_ij, |S|, grad T and the point values at p."""
            if p not in res:
                gr = self.gradients(S, p)
                g = [gr["u"], gr["v"], gr["w"]]
                Sij = [[0.5 * (g[i][j] + g[j][i]) for j in range(3)] for i in range(3)]
                Smag = math.sqrt(2.0 * sum(Sij[i][j] ** 2 for i in range(3) for j in range(3)))
                res[p] = (Sij, Smag, gr["T"], self.point(S, p))
            return res[p]

        def model_fields(p):
            """rho |S| S_ij (9), rho |S|^2, rho |S| dT/dx_j (3) at p."""
            Sij, Smag, gT, P = resolved(p)
            r = P["rho"]
            return ([r * Smag * Sij[i][j] for i in range(3) for j in range(3)]
                    + [r * Smag * Smag] + [r * Smag * gT[j] for j in range(3)])

        def state_fields(p):
            """rho, rho u_i, rho T, rho u_i u_j (9), rho u_j T (3) at p."""
            P = self.point(S, p)
            r, U = P["rho"], (P["u"], P["v"], P["w"])
            return ([r] + [r * U[i] for i in range(3)] + [r * P["T"]]
                    + [r * U[i] * U[j] for i in range(3) for j in range(3)]
                    + [r * U[j] * P["T"] for j in range(3)])

        hs = {}

        def hat_state(p):
            if p not in hs:
                hs[p] = hat(state_fields, p, 17)
            return hs[p]

        keys = ("N_I", "D_I", "A", "B", "D_d", "N_P", "D_P")
        sums = {k: 0.0 for k in keys}
        mags = {k: 0.0 for k in keys}
        for k in range(nth):
            for j in range(nr):
                for i in range(nx):
                    p = (i, j, k)
                    Sm, V = self.metric(p)
                    Sij, Smag, gT, _ = resolved(p)
                    trS = Sij[0][0] + Sij[1][1] + Sij[2][2]
                    hm = hat(model_fields, p, 13)
                    hSS = [[hm[3 * i2 + j2] for j2 in range(3)] for i2 in range(3)]
                    hS2, hST = hm[9], hm[10:13]
                    h = hat_state(p)
                    hr, hru, hrT = h[0], h[1:4], h[4]
                    hruu = [[h[5 + 3 * i2 + j2] for j2 in range(3)] for i2 in range(3)]
                    hruT = h[14:17]
                    # gradients of u_hat = hat(rho u)/hat(rho), T_hat = hat(rho T)/hat(rho)
                    dl = []
                    for d in range(3):
                        a, b = hat_state(self._shift(p, d, 1)), hat_state(self._shift(p, d, -1))
                        dl.append([0.5 * (a[1 + f] / a[0] - b[1 + f] / b[0]) for f in range(3)]
                                  + [0.5 * (a[4] / a[0] - b[4] / b[0])])
                    gh = [[(Sm[0][m] * dl[0][f] + Sm[1][m] * dl[1][f] + Sm[2][m] * dl[2][f]) / V
                           for m in range(3)] for f in range(4)]
                    Sh = [[0.5 * (gh[i2][j2] + gh[j2][i2]) for j2 in range(3)] for i2 in range(3)]
                    Shmag = math.sqrt(2.0 * sum(Sh[i2][j2] ** 2 for i2 in range(3) for j2 in range(3)))
                    trSh = Sh[0][0] + Sh[1][1] + Sh[2][2]
                    D2 = abs(V) ** (2.0 / 3.0)
                    Dh2 = 4.0 * D2
                    L = [[hruu[i2][j2] - hru[i2] * hru[j2] / hr for j2 in range(3)] for i2 in range(3)]
                    Lkk = L[0][0] + L[1][1] + L[2][2]
                    LS = sum(L[i2][j2] * Sij[i2][j2] for i2 in range(3) for j2 in range(3))
                    hSS_S = sum(hSS[i2][j2] * Sij[i2][j2] for i2 in range(3) for j2 in range(3))
                    hSkk = hSS[0][0] + hSS[1][1] + hSS[2][2]
                    ShS = sum(Sh[i2][j2] * Sij[i2][j2] for i2 in range(3) for j2 in range(3))
                    term = {
                        "N_I": Lkk,
                        "D_I": 2.0 * Dh2 * hr * Shmag ** 2 - 2.0 * D2 * hS2,
                        "A": LS - trS * Lkk / 3.0,
                        "B": trS * 2.0 * D2 * hS2 / 3.0,
                        "D_d": 2.0 * D2 * (hSS_S - hSkk * trS / 3.0)
                               - 2.0 * Dh2 * hr * Shmag * (ShS - trSh * trS / 3.0),
                        "N_P": sum(D2 * hST[m] * gT[m] - Dh2 * hr * Shmag * gh[3][m] * gT[m]
                                   for m in range(3)),
                        "D_P": sum((hruT[m] - hru[m] * hrT / hr) * gT[m] for m in range(3)),
                    }
                    for kk in keys:
                        sums[kk] += V * term[kk]
                        mags[kk] += abs(V * term[kk])
        return sums, mags


class _PointArray:
    """Q[c, k, j, i] view of a {(i, j, k): 5 values} dict."""

    def __init__(self, D):
        self.D = D

    def __getitem__(self, idx):
        c, k, j, i = idx
        return self.D[(i, j, k)][c]
