"""Differentiable lesjet operations for torch.autograd, a checkpointed RK5
rollout, and the far-field pressure functional.

Every derivative is one of the library's hand-written adjoints
(les_residual_vjp, les_rk5_step_vjp); torch only chains them with the
differentiable parameterisation of the inputs written by the caller.  The
time step is a constant of each operation (a CFL step is frozen at its value
before the rollout), and the boundary data other than the entrance target
(far-field state, back pressure) are constants.

States are padded FP64 tensors in the library layout (5, nth+4, nr+4, pitch);
only the interior enters R, so the cotangents of ghost entries are zero.
`pad_state` embeds an interior state differentiably.
"""
import math

import torch
import torch.nn.functional as F


def pad_state(solver, Q):
    """Padded copy of the interior state Q (5, nth, nr, nx); ghost entries and
    pitch padding are zero (the library fills ghosts itself)."""
    nx = solver.shape[0]
    return F.pad(Q, (2, solver.pitch - nx - 2, 2, 2, 2, 2))


def _inflow_in(solver, inflow):
    if inflow is not None:
        solver.set_inflow(inflow.detach())


class LesResidual(torch.autograd.Function):
    """R(Q; inflow data) with R on the interior and 0 elsewhere."""

    @staticmethod
    def forward(ctx, Qp, inflow, solver):
        _inflow_in(solver, inflow)
        R = solver.field(5, dtype=torch.float64, fill=0.0)
        solver.residual(Qp.detach().clone(), R)
        ctx.solver = solver
        ctx.save_for_backward(Qp, inflow)
        return R

    @staticmethod
    def backward(ctx, Rbar):
        Qp, inflow = ctx.saved_tensors
        s = ctx.solver
        _inflow_in(s, inflow)
        ib = s.new_inflow_bar() if inflow is not None and ctx.needs_input_grad[1] else None
        Qb = s.residual_vjp(Qp.detach().clone(), Rbar.contiguous(), inflow_bar=ib)
        return Qb, ib, None


class LesRK5Step(torch.autograd.Function):
    """One RK5 step with a fixed dt: Q^n -> Q^(n+1)."""

    @staticmethod
    def forward(ctx, Qp, inflow, solver, dt):
        _inflow_in(solver, inflow)
        Qn1 = Qp.detach().clone()
        solver.rk5_step(Qn1, 1, dt)
        ctx.solver, ctx.dt = solver, float(dt)
        ctx.save_for_backward(Qp, inflow)
        return Qn1

    @staticmethod
    def backward(ctx, Qbar):
        Qp, inflow = ctx.saved_tensors
        s = ctx.solver
        _inflow_in(s, inflow)
        ib = s.new_inflow_bar() if inflow is not None and ctx.needs_input_grad[1] else None
        Qb = s.rk5_step_vjp(Qp.detach().clone(), ctx.dt, Qbar.contiguous(), inflow_bar=ib)
        return Qb, ib, None, None


class SurfacePressure:
    """Acoustic-energy functional on the surface r ~ r_target of a cylindrical
    mesh: S(Q) = sum_{i,k} w_i r_s dtheta (p_{i,j_s,k} - p_inf)^2, with w the
    trapezoid weights of the axial node positions, r_s the radius of the
    chosen radial line and dtheta = 2 pi / nth.  Computed from the mesh
    coordinates xyz (3, nth, nr, nx) of the azimuthal plane k = 0."""

    def __init__(self, xyz, r_target, p_inf, gamma, device="cuda"):
        x = xyz[0, 0, 0, :].to(torch.float64)
        r = torch.sqrt(xyz[1, 0, :, 0].to(torch.float64) ** 2 + xyz[2, 0, :, 0].to(torch.float64) ** 2)
        self.js = int(torch.argmin((r - r_target).abs()))
        self.rs = float(r[self.js])
        nth = xyz.shape[1]
        h = x[1:] - x[:-1]
        w = torch.zeros_like(x)
        w[:-1] += 0.5 * h
        w[1:] += 0.5 * h
        self.w = (w * self.rs * (2.0 * math.pi / nth)).to(device)
        self.p_inf = float(p_inf)
        self.gm1 = float(gamma) - 1.0

    def __call__(self, solver, Qp):
        nx, nr, nth = solver.shape
        q = Qp[:, 2:2 + nth, 2 + self.js, 2:2 + nx]              # (5, nth, nx)
        ke = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]
        d = self.gm1 * (q[4] - ke) - self.p_inf
        return torch.sum(self.w.view(1, -1) * d * d)

    def grad(self, solver, Qp):
        """dS/dQ as a padded tensor (torch autograd over this formula)."""
        with torch.enable_grad():
            x = Qp.detach().requires_grad_(True)
            (g,) = torch.autograd.grad(self(solver, x), x)
        return g


class _Segment(torch.autograd.Function):
    """k RK5 steps from a checkpoint: (Q^m, inflow) -> (Q^(m+k), sum of
    dt S(Q^n) over n = m+1..m+k).  Only Q^m is kept; the backward recomputes
    the k states and runs the k step adjoints in reverse, adding
    dt dS/dQ^n at each step."""

    @staticmethod
    def forward(ctx, Qp, inflow, solver, dt, k, functional):
        _inflow_in(solver, inflow)
        Q = Qp.detach().clone()
        J = torch.zeros((), dtype=torch.float64, device=Qp.device)
        for _ in range(k):
            solver.rk5_step(Q, 1, dt)
            if functional is not None:
                J = J + dt * functional(solver, Q)
        ctx.solver, ctx.dt, ctx.k, ctx.functional = solver, float(dt), int(k), functional
        ctx.save_for_backward(Qp, inflow)
        return Q, J

    @staticmethod
    def backward(ctx, Qbar_end, Jbar):
        Qp, inflow = ctx.saved_tensors
        s, dt, k, fn = ctx.solver, ctx.dt, ctx.k, ctx.functional
        _inflow_in(s, inflow)
        states = [Qp.detach().clone()]
        for _ in range(k):
            q = states[-1].clone()
            s.rk5_step(q, 1, dt)
            states.append(q)
        b = Qbar_end.detach().clone() if Qbar_end is not None else torch.zeros_like(Qp)
        ib = s.new_inflow_bar() if inflow is not None and ctx.needs_input_grad[1] else None
        use_j = fn is not None and Jbar is not None
        if use_j:
            b = b + (float(Jbar) * dt) * fn.grad(s, states[k])
        for n in range(k, 0, -1):
            s.rk5_step_vjp(states[n - 1], dt, b, b, inflow_bar=ib)
            if use_j and n - 1 >= 1:
                b = b + (float(Jbar) * dt) * fn.grad(s, states[n - 1])
        return b, ib, None, None, None, None


def rollout(solver, Q0p, inflow, dt, nsteps, every=5, functional=None):
    """nsteps RK5 steps of fixed dt from the padded state Q0p, checkpointed
    every `every` steps; returns (Q^N, J) with J = sum_{n=1}^{N} dt S(Q^n)
    (zero without a functional).  Differentiable in Q0p and inflow."""
    Q = Q0p
    J = torch.zeros((), dtype=torch.float64, device=Q0p.device)
    done = 0
    while done < nsteps:
        k = min(every, nsteps - done)
        Q, Jseg = _Segment.apply(Q, inflow, solver, dt, k, functional)
        J = J + Jseg
        done += k
    return Q, J


def cfl_dt(solver, Qp):
    """The CFL time step of the padded FP64 state (one throw-away step)."""
    q = Qp.detach().clone()
    return float(solver.rk5_step(q, 1, 0.0)[0])
