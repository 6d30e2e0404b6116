"""Torch-facing wrapper of one lesjet context.

PyTorch provides device memory and the current HIP stream; every step of the
method runs in the library's kernels.  Fields live in the library's padded
layout (nvar, nth+4, nr+4, pitch) with two ghost layers; `interior` returns
the (nvar, nth, nr, nx) view.

Every tensor whose pointer crosses the C-ABI is checked first (type, dtype,
exact shape, device, contiguity) and a mismatch raises ValueError before
any library call: the kernels take raw pointers and sizes from the context,
so an undersized or mistyped buffer would otherwise be read or written out
of bounds.
"""
import torch

from . import binding as B


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


def _check_tensor(t, name, shape, dtype, device):
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch.Tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.device != device:
        raise ValueError(f"{name} is on device {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Solver:
    """Mesh, metrics and boundary data of one LES problem on one GPU.

    params: dict of constants and boundary kinds (gamma, Pr, Pr_sgs,
    visc_coef, suth_S, Cs, k2, k4, cfl, rk_alpha, ref_prim, p_exit,
    sgs_model, bc, period).  The mesh is either xyz, (3, nth, nr, nx) float64
    coordinates (host or device; copied), or grid = (X, R, TH), the 1-D maps
    of a cylindrical product mesh (x = X_i, y = R_j cos TH_k,
    z = R_j sin TH_k).  inflow: (5, nth, nr) entrance target primitives.
    precision: "fp64" or "fp32" (FP32 storage of stage states and metrics,
    FP64 Q^n and stage accumulation).
    """

    def __init__(self, params, xyz=None, inflow=None, precision="fp64", device="cuda",
                 keep_metrics=False, grid=None):
        if not torch.cuda.is_available():
            raise RuntimeError("lesjet needs a HIP device; none is visible")
        if (xyz is None) == (grid is None):
            raise ValueError("give exactly one of xyz and grid = (X, R, TH)")
        if precision not in ("fp64", "fp32"):
            raise ValueError(f"precision must be 'fp64' or 'fp32', got {precision!r}")
        dev = torch.device(device)
        if dev.type != "cuda":
            raise ValueError(f"device must be a HIP device, got {dev}")
        self.device = torch.device("cuda", dev.index if dev.index is not None
                                   else torch.cuda.current_device())
        if xyz is not None:
            if not isinstance(xyz, torch.Tensor) or xyz.dim() != 4 or xyz.shape[0] != 3:
                raise ValueError("xyz must be a (3, nth, nr, nx) tensor")
            _, nth, nr, nx = xyz.shape
            maps = None
        else:
            if len(grid) != 3:
                raise ValueError("grid must be (X, R, TH)")
            maps = [torch.as_tensor(a).to(torch.float64).contiguous() for a in grid]
            if any(m.dim() != 1 for m in maps):
                raise ValueError("X, R and TH must be 1-D")
            nx, nr, nth = (m.numel() for m in maps)
        self.shape = (int(nx), int(nr), int(nth))
        self.precision = precision
        self.prec = B.LES_FP32_STORAGE if precision == "fp32" else B.LES_FP64
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.params = dict(params)
        self.p = B.make_params(params, self.shape, self.prec)
        self.pitch, dims3, self.vs = B.les_layout(self.p)
        self.dims = tuple(dims3)
        st = _stream(self.device)
        if maps is not None:
            # host arrays: the library reads them during the call
            maps = [m.cpu() for m in maps]
            self.ctx = B.les_init_grid(self.p, None, maps[0].data_ptr(), maps[1].data_ptr(),
                                       maps[2].data_ptr(), st)
        else:
            # host or this device's memory; the library copies it
            src = xyz.to(torch.float64).contiguous()
            if src.device.type == "cuda" and src.device != self.device:
                src = src.to(self.device)
            self.ctx = B.les_init_grid(self.p, src.data_ptr(), None, None, None, st)
            del src
        self.metrics64 = None
        out = None
        if keep_metrics:
            out = torch.zeros((10,) + self.dims, dtype=torch.float64, device=self.device)
        B.les_metrics(self.ctx, out.data_ptr() if out is not None else None, st)
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

    # -- argument checks --------------------------------------------------------
    def _state(self, t, name, dtype=None):
        """A padded 5-variable field of the storage type (or `dtype`)."""
        return _check_tensor(t, name, (5,) + self.dims, dtype or self.dtype, self.device)

    def _inflow_bar(self, t):
        if t is None:
            return None
        nx, nr, nth = self.shape
        return _check_tensor(t, "inflow_bar", (5, nth, nr), torch.float64, self.device)

    # -- entry points -----------------------------------------------------------
    def set_inflow(self, prim):
        nx, nr, nth = self.shape
        if not isinstance(prim, torch.Tensor) or tuple(prim.shape) != (5, nth, nr):
            raise ValueError(f"inflow must be a (5, {nth}, {nr}) tensor")
        self._inflow = prim.to(self.device, torch.float64).contiguous()
        B.les_set_inflow(self.ctx, self._inflow.data_ptr(), _stream(self.device))

    def fill_ghosts(self, Qp):
        self._state(Qp, "Q")
        B.les_fill_ghosts(self.ctx, Qp.data_ptr(), _stream(self.device))
        return Qp

    def residual(self, Qp, R=None):
        self._state(Qp, "Q")
        if R is None:
            R = self.field(5, fill=float("nan"))
        self._state(R, "R")
        B.les_residual(self.ctx, Qp.data_ptr(), R.data_ptr(), _stream(self.device))
        return R

    def residual_reference(self, Qp, R=None):
        """R(Q) by the two-pass reference kernels (validation)."""
        self._state(Qp, "Q")
        if R is None:
            R = self.field(5, fill=float("nan"))
        self._state(R, "R")
        B.les_residual_reference(self.ctx, Qp.data_ptr(), R.data_ptr(), _stream(self.device))
        return R

    def dynamic_coefficients(self, Qp):
        """Dynamic SGS model coefficients of the padded state Qp (storage
        type; ghosts filled in place): (C_I, C_ds, Pr_sgs) as computed, then
        as used."""
        self._state(Qp, "Q")
        return B.les_dynamic_coefficients(self.ctx, Qp.data_ptr(), _stream(self.device))

    def rk5_step(self, Qn, nsteps=1, dt=0.0, dt_out=None):
        """Advance the padded FP64 state Qn in place; returns the per-step dt
        (device tensor of nsteps doubles)."""
        self._state(Qn, "Qn", torch.float64)
        nsteps = int(nsteps)
        if nsteps < 0:
            raise ValueError("nsteps must be >= 0")
        if dt_out is None:
            dt_out = torch.empty(max(nsteps, 1), dtype=torch.float64, device=self.device)
        if not isinstance(dt_out, torch.Tensor) or dt_out.dtype != torch.float64 \
                or dt_out.device != self.device or not dt_out.is_contiguous() \
                or dt_out.dim() != 1 or dt_out.numel() < nsteps:
            raise ValueError(f"dt_out must be a contiguous float64 vector of at least {nsteps} "
                             f"elements on {self.device}")
        B.les_rk5_step(self.ctx, Qn.data_ptr(), nsteps, float(dt), dt_out.data_ptr(),
                       _stream(self.device))
        return dt_out

    def new_inflow_bar(self):
        nx, nr, nth = self.shape
        return torch.zeros((5, nth, nr), dtype=torch.float64, device=self.device)

    def residual_vjp(self, Qp, Rbar, Qbar=None, inflow_bar=None):
        """(dR/dQ)^T Rbar at the padded FP64 state Qp (ghost fill included);
        the entrance-target cotangent is added to `inflow_bar` if given."""
        self._state(Qp, "Q", torch.float64)
        self._state(Rbar, "Rbar", torch.float64)
        if Qbar is None:
            Qbar = self.field(5, dtype=torch.float64)
        self._state(Qbar, "Qbar", torch.float64)
        ib = self._inflow_bar(inflow_bar)
        B.les_residual_vjp(self.ctx, Qp.data_ptr(), Rbar.data_ptr(), Qbar.data_ptr(),
                           ib.data_ptr() if ib is not None else None, _stream(self.device))
        return Qbar

    def rk5_step_vjp(self, Qn, dt, Qbar_np1, Qbar_n=None, inflow_bar=None):
        """Cotangent of Q^n from that of Q^(n+1) for one RK5 step of fixed dt."""
        self._state(Qn, "Qn", torch.float64)
        self._state(Qbar_np1, "Qbar_np1", torch.float64)
        if Qbar_n is None:
            Qbar_n = self.field(5, dtype=torch.float64)
        self._state(Qbar_n, "Qbar_n", torch.float64)
        ib = self._inflow_bar(inflow_bar)
        B.les_rk5_step_vjp(self.ctx, Qn.data_ptr(), float(dt), Qbar_np1.data_ptr(),
                           Qbar_n.data_ptr(), ib.data_ptr() if ib is not None else None,
                           _stream(self.device))
        return Qbar_n

    def diagnostics(self, Qn, stats=None):
        """Conservation totals (5 doubles, device) of the padded FP64 state;
        if `stats` = (sum1, sum2) of shape (5, nr, nx) is given, adds the
        azimuthal sums of (rho, u, v, w, p) and their squares."""
        self._state(Qn, "Qn", torch.float64)
        totals = torch.empty(5, dtype=torch.float64, device=self.device)
        s1 = s2 = None
        if stats is not None:
            nx, nr, _ = self.shape
            s1, s2 = stats
            for t, name in ((s1, "sum1"), (s2, "sum2")):
                if t is not None:
                    _check_tensor(t, name, (5, nr, nx), torch.float64, self.device)
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
        """(dims_padded (5, nth+4, nr+4, pitch), pitch, device bytes held)."""
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
