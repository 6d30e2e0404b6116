"""ctypes binding of liblesjet.so (include/lesjet.h).

Argument marshalling only: every function has the name and argument order of
its C counterpart, takes raw device pointers as Python ints, and raises
LesError on a negative status.  The library must have been built
(`python -m paper_2301_00817_amd.build`); importing this module without it
raises immediately — there is no fallback implementation.
"""
import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "liblesjet.so")

LES_OK, LES_EINVAL, LES_ENOMEM, LES_EHIP, LES_ENONFINITE, LES_ESTATE, LES_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
LES_FP64, LES_FP32_STORAGE = 0, 1
LES_SCHEDULE_STAGE, LES_SCHEDULE_STEP = 0, 1
SCHEDULE = {"stage": 0, "step": 1}
BC = {"periodic": 0, "axis": 1, "inflow": 2, "outflow": 3, "farfield": 4, "axis_node": 5}
SGS = {0: 0, 1: 1, 2: 2, 3: 3, "none": 0, "smagorinsky": 1, "vreman": 2, "dynamic": 3}
STATUS = {0: "LES_OK", -1: "LES_EINVAL", -2: "LES_ENOMEM", -3: "LES_EHIP",
          -4: "LES_ENONFINITE", -5: "LES_ESTATE", -6: "LES_EUNSUPPORTED"}


class LesError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class les_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("nr", ctypes.c_int32), ("nth", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 6),
        ("period", (ctypes.c_double * 3) * 3),
        ("gamma", ctypes.c_double), ("Pr", ctypes.c_double), ("Pr_sgs", ctypes.c_double),
        ("visc_coef", ctypes.c_double), ("suth_S", ctypes.c_double), ("Cs", ctypes.c_double),
        ("k2", ctypes.c_double), ("k4", ctypes.c_double), ("cfl", ctypes.c_double),
        ("rk_alpha", ctypes.c_double * 5), ("ref_prim", ctypes.c_double * 5),
        ("p_exit", ctypes.c_double),
        ("sgs_model", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
    ]


def make_params(prm, shape, precision=LES_FP64):
    """les_params from a parameter dict and the interior shape (nx, nr, nth)."""
    p = les_params()
    p.nx, p.nr, p.nth = (int(s) for s in shape)
    for f, kind in enumerate(prm["bc"]):
        p.bc[f] = BC[kind] if isinstance(kind, str) else int(kind)
    for d in range(3):
        for c in range(3):
            p.period[d][c] = float(prm["period"][d][c])
    for key in ("gamma", "Pr", "Pr_sgs", "visc_coef", "suth_S", "Cs", "k2", "k4", "cfl", "p_exit"):
        setattr(p, key, float(prm[key]))
    for l in range(5):
        p.rk_alpha[l] = float(prm["rk_alpha"][l])
    for c in range(5):
        p.ref_prim[c] = float(prm["ref_prim"][c])
    sgs = prm.get("sgs_model", 1)
    p.sgs_model = SGS[sgs] if isinstance(sgs, str) else int(sgs)
    p.precision = int(precision)
    sch = prm.get("schedule", "stage")
    p.schedule = SCHEDULE[sch] if isinstance(sch, str) else int(sch)
    return p


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2301_00817_amd.build` (there is no fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "les_validate": ([P(les_params)], ctypes.c_int),
        "les_layout": ([P(les_params), P(i64), P(i64 * 3), P(i64)], ctypes.c_int),
        "les_device_bytes": ([P(les_params), P(sz)], ctypes.c_int),
        "les_init_grid": ([P(vp), P(les_params), vp, vp, vp, vp, vp], ctypes.c_int),
        "les_metrics": ([vp, vp, vp], ctypes.c_int),
        "les_set_inflow": ([vp, vp, vp], ctypes.c_int),
        "les_fill_ghosts": ([vp, vp, vp], ctypes.c_int),
        "les_residual": ([vp, vp, vp, vp], ctypes.c_int),
        "les_residual_reference": ([vp, vp, vp, vp], ctypes.c_int),
        "les_dynamic_coefficients": ([vp, vp, P(dbl * 6), vp], ctypes.c_int),
        "les_rk5_step": ([vp, vp, i32, dbl, vp, vp], ctypes.c_int),
        "les_residual_vjp": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "les_rk5_step_vjp": ([vp, vp, dbl, vp, vp, vp, vp], ctypes.c_int),
        "les_diagnostics": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "les_diagnostics_noalloc": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "les_profile": ([vp, i32], ctypes.c_int),
        "les_profile_read": ([vp, P(i64), P(dbl)], ctypes.c_int),
        "les_query": ([vp, P(i64 * 4), P(i64), P(sz)], ctypes.c_int),
        "les_last_error": ([vp], ctypes.c_char_p),
        "les_free": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()
EXPORTS = ("les_validate", "les_layout", "les_device_bytes", "les_init_grid", "les_metrics",
           "les_set_inflow", "les_fill_ghosts", "les_residual", "les_residual_reference",
           "les_dynamic_coefficients",
           "les_rk5_step", "les_residual_vjp", "les_rk5_step_vjp", "les_diagnostics",
           "les_diagnostics_noalloc", "les_profile",
           "les_profile_read", "les_query",
           "les_last_error", "les_free")


def _check(code, ctx=None):
    if code != LES_OK:
        raise LesError(code, les_last_error(ctx))
    return code


def les_last_error(ctx=None):
    return _lib.les_last_error(ctx).decode()


def les_validate(params):
    return _check(_lib.les_validate(ctypes.byref(params)))


def les_layout(params):
    pitch, dims, vs = ctypes.c_int64(), (ctypes.c_int64 * 3)(), ctypes.c_int64()
    _check(_lib.les_layout(ctypes.byref(params), ctypes.byref(pitch), ctypes.byref(dims),
                           ctypes.byref(vs)))
    return pitch.value, tuple(dims), vs.value


def les_device_bytes(params):
    b = ctypes.c_size_t()
    _check(_lib.les_device_bytes(ctypes.byref(params), ctypes.byref(b)))
    return b.value


def les_init_grid(params, xyz_ptr=None, x_ptr=None, r_ptr=None, th_ptr=None, stream=0):
    """Context for a mesh given as xyz (3, nth, nr, nx) or as the 1-D maps X,
    R, TH of a cylindrical product mesh (pointers to host or device FP64)."""
    ctx = ctypes.c_void_p()
    _check(_lib.les_init_grid(ctypes.byref(ctx), ctypes.byref(params), xyz_ptr, x_ptr, r_ptr,
                              th_ptr, stream))
    return ctx.value


def les_metrics(ctx, metrics_out_ptr=None, stream=0):
    return _check(_lib.les_metrics(ctx, metrics_out_ptr, stream), ctx)


def les_set_inflow(ctx, prim_ptr, stream=0):
    return _check(_lib.les_set_inflow(ctx, prim_ptr, stream), ctx)


def les_fill_ghosts(ctx, q_ptr, stream=0):
    return _check(_lib.les_fill_ghosts(ctx, q_ptr, stream), ctx)


def les_residual(ctx, q_ptr, r_ptr, stream=0):
    return _check(_lib.les_residual(ctx, q_ptr, r_ptr, stream), ctx)


def les_residual_reference(ctx, q_ptr, r_ptr, stream=0):
    return _check(_lib.les_residual_reference(ctx, q_ptr, r_ptr, stream), ctx)


def les_dynamic_coefficients(ctx, q_ptr, stream=0):
    """(C_I, C_ds, Pr_sgs) as computed and as used, a 6-tuple of floats."""
    out = (ctypes.c_double * 6)()
    _check(_lib.les_dynamic_coefficients(ctx, q_ptr, ctypes.byref(out), stream), ctx)
    return tuple(out)


def les_rk5_step(ctx, qn_ptr, nsteps, dt_fixed=0.0, dt_out_ptr=None, stream=0):
    return _check(_lib.les_rk5_step(ctx, qn_ptr, int(nsteps), float(dt_fixed), dt_out_ptr, stream), ctx)


def les_residual_vjp(ctx, q_ptr, rbar_ptr, qbar_ptr, inflow_bar_ptr=None, stream=0):
    return _check(_lib.les_residual_vjp(ctx, q_ptr, rbar_ptr, qbar_ptr, inflow_bar_ptr, stream), ctx)


def les_rk5_step_vjp(ctx, qn_ptr, dt, qbar_np1_ptr, qbar_n_ptr, inflow_bar_ptr=None, stream=0):
    return _check(_lib.les_rk5_step_vjp(ctx, qn_ptr, float(dt), qbar_np1_ptr, qbar_n_ptr,
                                        inflow_bar_ptr, stream), ctx)


def les_diagnostics(ctx, qn_ptr, totals_ptr=None, sum1_ptr=None, sum2_ptr=None, stream=0):
    return _check(_lib.les_diagnostics(ctx, qn_ptr, totals_ptr, sum1_ptr, sum2_ptr, stream), ctx)


def les_diagnostics_noalloc(ctx, qn_ptr, totals_ptr=None, sum1_ptr=None, sum2_ptr=None, stream=0):
    return _check(_lib.les_diagnostics_noalloc(ctx, qn_ptr, totals_ptr, sum1_ptr, sum2_ptr, stream),
                  ctx)


def les_profile(ctx, enable):
    return _check(_lib.les_profile(ctx, int(bool(enable))), ctx)


def les_profile_read(ctx):
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(_lib.les_profile_read(ctx, ctypes.byref(n), ctypes.byref(ms)), ctx)
    return n.value, ms.value


def les_query(ctx):
    """(dims_padded (5, nth+4, nr+4, pitch), pitch, device bytes held)."""
    dims, pitch, b = (ctypes.c_int64 * 4)(), ctypes.c_int64(), ctypes.c_size_t()
    _check(_lib.les_query(ctx, ctypes.byref(dims), ctypes.byref(pitch), ctypes.byref(b)), ctx)
    return tuple(dims), pitch.value, b.value


def les_free(ctx):
    _lib.les_free(ctx)
