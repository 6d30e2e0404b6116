"""Torch-facing wrapper of one lesjet context.

PyTorch provides device memory and the current HIP stream; every step of the
method runs in the library's kernels.  Fields live in the library's padded
layout (nvar, nth+4, nr+4, pitch) with two ghost layers; `interior` returns
the (nvar, nth, nr, nx) view.
"""
import torch

from . import binding as B


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


class Solver:
    """Mesh, metrics and boundary data of one LES problem on one GPU.

    params: dict of constants and boundary kinds (gamma, Pr, Pr_sgs,
    visc_coef, suth_S, Cs, k2, k4, cfl, rk_alpha, ref_prim, p_exit,
    sgs_model, bc, period); xyz: (3, nth, nr, nx) float64 coordinates (any
    device; copied); inflow: (5, nth, nr) entrance target primitives.
    precision: "fp64" or "fp32" (FP32 storage of stage states and metrics,
    FP64 Q^n and stage accumulation).
    """

    def __init__(self, params, xyz, inflow=None, precision="fp64", device="cuda",
                 keep_metrics=False):
        if not torch.cuda.is_available():
            raise RuntimeError("lesjet needs a HIP device; none is visible")
        self.device = torch.device(device)
        _, nth, nr, nx = xyz.shape
        self.shape = (nx, nr, nth)
        self.precision = precision
        self.prec = B.LES_FP32_STORAGE if precision == "fp32" else B.LES_FP64
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.params = dict(params)
        self.p = B.make_params(params, self.shape, self.prec)
        self.pitch, self.dims, self.vs = B.les_layout(self.p)
        xyz_d = xyz.to(self.device, torch.float64).contiguous()
        self.ctx = B.les_init_grid(self.p, xyz_d.data_ptr(), _stream(self.device))
        del xyz_d
        self.metrics64 = None
        out = None
        if keep_metrics:
            out = torch.zeros((10,) + self.dims, dtype=torch.float64, device=self.device)
        B.les_metrics(self.ctx, out.data_ptr() if out is not None else None, _stream(self.device))
        self.metrics64 = out
        if inflow is not None:
            self.set_inflow(inflow)

    # -- layout ---------------------------------------------------------------
    def field(self, nvar=5, dtype=None, fill=None):
        t = torch.empty((nvar,) + self.dims, dtype=dtype or self.dtype, device=self.device)
        if fill is not None:
            t.fill_(fill)
        return t

    def interior(self, F):
        nx, nr, nth = self.shape
        return F[:, 2:2 + nth, 2:2 + nr, 2:2 + nx]

    def pad(self, Q, dtype=None, fill=float("nan")):
        """Padded copy of an interior state (ghosts set to `fill`)."""
        F = self.field(Q.shape[0], dtype or self.dtype, fill)
        self.interior(F).copy_(Q)
        return F

    # -- entry points -----------------------------------------------------------
    def set_inflow(self, prim):
        self._inflow = prim.to(self.device, torch.float64).contiguous()
        B.les_set_inflow(self.ctx, self._inflow.data_ptr(), _stream(self.device))

    def fill_ghosts(self, Qp):
        assert Qp.dtype == self.dtype and tuple(Qp.shape[1:]) == self.dims and Qp.is_contiguous()
        B.les_fill_ghosts(self.ctx, Qp.data_ptr(), _stream(self.device))
        return Qp

    def residual(self, Qp, R=None):
        assert Qp.dtype == self.dtype and tuple(Qp.shape) == (5,) + self.dims and Qp.is_contiguous()
        if R is None:
            R = self.field(5, fill=float("nan"))
        B.les_residual(self.ctx, Qp.data_ptr(), R.data_ptr(), _stream(self.device))
        return R

    def residual_reference(self, Qp, R=None):
        """R(Q) by the two-pass reference kernels (validation)."""
        assert Qp.dtype == self.dtype and tuple(Qp.shape) == (5,) + self.dims and Qp.is_contiguous()
        if R is None:
            R = self.field(5, fill=float("nan"))
        B.les_residual_reference(self.ctx, Qp.data_ptr(), R.data_ptr(), _stream(self.device))
        return R

    def dynamic_coefficients(self, Qp):
        """Dynamic SGS model coefficients of the padded state Qp (storage
        type; ghosts filled in place): (C_I, C_ds, Pr_sgs) as computed, then
        as used."""
        assert Qp.dtype == self.dtype and tuple(Qp.shape) == (5,) + self.dims and Qp.is_contiguous()
        return B.les_dynamic_coefficients(self.ctx, Qp.data_ptr(), _stream(self.device))

    def rk5_step(self, Qn, nsteps=1, dt=0.0, dt_out=None):
        """Advance the padded FP64 state Qn in place; returns the per-step dt
        (device tensor of nsteps doubles)."""
        assert Qn.dtype == torch.float64 and tuple(Qn.shape) == (5,) + self.dims and Qn.is_contiguous()
        if dt_out is None:
            dt_out = torch.empty(max(int(nsteps), 1), dtype=torch.float64, device=self.device)
        B.les_rk5_step(self.ctx, Qn.data_ptr(), int(nsteps), float(dt), dt_out.data_ptr(),
                       _stream(self.device))
        return dt_out

    def _check_fp64_state(self, Q):
        assert Q.dtype == torch.float64 and tuple(Q.shape) == (5,) + self.dims and Q.is_contiguous()

    def new_inflow_bar(self):
        nx, nr, nth = self.shape
        return torch.zeros((5, nth, nr), dtype=torch.float64, device=self.device)

    def residual_vjp(self, Qp, Rbar, Qbar=None, inflow_bar=None):
        """(dR/dQ)^T Rbar at the padded FP64 state Qp (ghost fill included);
        the entrance-target cotangent is added to `inflow_bar` if given."""
        self._check_fp64_state(Qp)
        self._check_fp64_state(Rbar)
        if Qbar is None:
            Qbar = self.field(5, dtype=torch.float64)
        self._check_fp64_state(Qbar)
        B.les_residual_vjp(self.ctx, Qp.data_ptr(), Rbar.data_ptr(), Qbar.data_ptr(),
                           inflow_bar.data_ptr() if inflow_bar is not None else None,
                           _stream(self.device))
        return Qbar

    def rk5_step_vjp(self, Qn, dt, Qbar_np1, Qbar_n=None, inflow_bar=None):
        """Cotangent of Q^n from that of Q^(n+1) for one RK5 step of fixed dt."""
        self._check_fp64_state(Qn)
        self._check_fp64_state(Qbar_np1)
        if Qbar_n is None:
            Qbar_n = self.field(5, dtype=torch.float64)
        self._check_fp64_state(Qbar_n)
        B.les_rk5_step_vjp(self.ctx, Qn.data_ptr(), float(dt), Qbar_np1.data_ptr(),
                           Qbar_n.data_ptr(),
                           inflow_bar.data_ptr() if inflow_bar is not None else None,
                           _stream(self.device))
        return Qbar_n

    def diagnostics(self, Qn, stats=None):
        """Conservation totals (5 doubles, device) of the padded FP64 state;
        if `stats` = (sum1, sum2) of shape (5, nr, nx) is given, adds the
        azimuthal sums of (rho, u, v, w, p) and their squares."""
        assert Qn.dtype == torch.float64 and tuple(Qn.shape) == (5,) + self.dims and Qn.is_contiguous()
        totals = torch.empty(5, dtype=torch.float64, device=self.device)
        s1 = s2 = None
        if stats is not None:
            s1, s2 = stats
        B.les_diagnostics(self.ctx, Qn.data_ptr(), totals.data_ptr(),
                          s1.data_ptr() if s1 is not None else None,
                          s2.data_ptr() if s2 is not None else None, _stream(self.device))
        return totals

    def new_stats(self):
        nx, nr, _ = self.shape
        z = lambda: torch.zeros((5, nr, nx), dtype=torch.float64, device=self.device)  # noqa: E731
        return z(), z()

    def profile(self, enable=True):
        B.les_profile(self.ctx, enable)

    def profile_read(self):
        """(launches, total ms) of the residual stage kernel since the last
        read, timed with HIP events on the launch stream."""
        return B.les_profile_read(self.ctx)

    def query(self):
        return B.les_query(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            B.les_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
