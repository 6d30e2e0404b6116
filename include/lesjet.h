/*
 * lesjet — explicit LES residual and five-stage Runge-Kutta step of the
 * filtered compressible Navier-Stokes equations (System-I energy form) on a
 * structured curvilinear mesh, for one AMD Instinct MI355X (gfx950).
 *
 * Method: Junqueira-Junior, Azevedo, Yamouni, Wolf, arXiv 2301.00817,
 * sections "Large Eddy Simulation Filtering", "Subgrid Scale Modeling"
 * (static Smagorinsky and Vreman models), "Transformation of Coordinates", "Numerical
 * Formulation" (centred fluxes, Turkel-Vatsa artificial dissipation, Jameson
 * 5-stage RK) and "Boundary Conditions".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Index directions: xi (i, axial, fastest in memory), eta (j, radial),
 * zeta (k, azimuthal).  Interior sizes nx, nr, nth.
 *
 * Padded field layout: a field of `nvar` variables is stored as
 *     F[v][k + 2][j + 2][i + 2],  i in [-2, nx+1], j in [-2, nr+1], k in [-2, nth+1]
 * with row pitch `pitch` elements (>= nx + 4, from les_layout), plane stride
 * (nr + 4) * pitch and variable stride (nth + 4) * (nr + 4) * pitch.
 * Two ghost layers on every face hold boundary / periodic values; the
 * library writes them (they are scratch from the caller's point of view).
 *
 * State Q: unhatted nondimensional conserved variables
 *     (rho, rho u, rho v, rho w, E),  E = p/(gamma-1) + rho |u|^2 / 2,
 * scaled by the jet density, jet sound speed and diameter
 * ("Dimensionless Formulation").  Residual R: dQ/dt = -R, R = RHS / J^-1
 * (eq. spatial_discret with unit index spacing).
 *
 * Pointers: arguments documented "device" are HIP device pointers owned by
 * the caller (e.g. torch tensor storage); "host" pointers are read during
 * the call only.  The library owns its context, metrics, stage buffers and
 * scratch, released by les_free.
 *
 * Streams: `stream` is a hipStream_t (NULL = default stream).  Work is
 * enqueued asynchronously unless stated otherwise.  A context must not be
 * used from two host threads at once, nor on two streams concurrently.
 *
 * Errors: every function returns LES_OK (0) or a negative code; nothing
 * aborts and no C++ exception crosses the ABI.  Arguments are validated
 * before any device work.  les_last_error gives a message.
 */
#ifndef LESJET_H
#define LESJET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct les_ctx les_ctx;

enum les_status {
  LES_OK = 0,
  LES_EINVAL = -1,        /* bad argument (sizes, pointers, boundary kinds) */
  LES_ENOMEM = -2,        /* device allocation failed */
  LES_EHIP = -3,          /* a HIP runtime call failed (message has details) */
  LES_ENONFINITE = -4,    /* time-step reduction met a NaN/Inf (diverged state) */
  LES_ESTATE = -5,        /* call order violated (e.g. residual before metrics) */
  LES_EUNSUPPORTED = -6   /* valid request this build does not provide */
};

enum les_precision {
  LES_FP64 = 0,           /* state, metrics and fluxes in FP64 */
  LES_FP32_STORAGE = 1    /* stage states, metrics, fluxes in FP32; Q^n and the
                             RK accumulation Q^n - alpha dt R in FP64 */
};

/* When the viscosities and boundary values are updated during an RK5 step
 * (section "The JAZzY code": the paper's iteration loop updates the
 * viscosity, the SGS viscosity and the boundary conditions once per
 * iteration, after the time marching). */
enum les_schedule {
  LES_SCHEDULE_STAGE = 0, /* everything recomputed from the state of every stage */
  LES_SCHEDULE_STEP = 1   /* mu + mu_sgs (and the conductivity) evaluated at
                             stage 1 from Q^n and held through the five stages;
                             ghosts of the entrance, exit and far-field faces
                             and the centerline row (LES_BC_AXIS_NODE) held
                             from Q^n; periodic and cross-axis ghosts copied
                             from each stage state.  Affects les_rk5_step only
                             (a single residual is the same in both). */
};

enum les_bc {
  LES_BC_PERIODIC = 0,    /* both faces of a direction; translation `period` */
  LES_BC_AXIS = 1,        /* eta-: ghosts are the points across the axis
                             (i, m, k + nth/2); needs even nth, zeta periodic */
  LES_BC_INFLOW = 2,      /* xi-: entrance; target primitives from les_set_inflow */
  LES_BC_OUTFLOW = 3,     /* xi+: exit with back pressure p_exit */
  LES_BC_FARFIELD = 4,    /* eta+: Riemann invariants with ref_prim */
  LES_BC_AXIS_NODE = 5    /* eta-: the row j = 0 lies on the axis (subsection
                             "Centerline Boundary Condition"): before every
                             residual it takes the azimuthal mean of the
                             conserved variables of row j = 1 and R = 0 there;
                             ghosts are the mirror points (i, m, k + nth/2);
                             the eta point flux vanishes on the axis; the axis
                             face uses lambda_bar of row 1 and the three-point
                             fourth difference W2 - 4 W1 + 3 W0; entrance and
                             exit normals of axis points are those of row 1;
                             the CFL maximum skips the axis.  The axis row of
                             the caller's state is derived data: the ghost fill
                             of les_residual / les_rk5_step writes the mean into
                             it, and les_rk5_step returns it as the mean of the
                             returned state's row 1.  Needs even nth.  The
                             adjoints follow: the axis row's cotangent is zero
                             (R does not depend on it), and les_rk5_step_vjp
                             first moves the cotangent of the returned axis
                             row to row 1 (the transpose of that mean). */
};

/* Subgrid-scale eddy viscosity (subsection "Subgrid Scale Modeling"), in
 * jet-viscosity units (divided by visc_coef), filter width |J^-1|^(1/3):
 *   SMAGORINSKY  mu_sgs = rho (Cs Delta)^2 sqrt(2 S_ij S_ij);
 *   VREMAN       mu_sgs = rho c sqrt(B_beta / (alpha_ij alpha_ij)), c = 2.5 Cs^2,
 *                alpha_ij = d u_j / d x_i, beta_ij = Delta^2 alpha_mi alpha_mj,
 *                B_beta = b11 b22 - b12^2 + b11 b33 - b13^2 + b22 b33 - b23^2,
 *                zero where alpha_ij alpha_ij = 0 (or B_beta <= 0 by rounding);
 *   DYNAMIC      (subsection "Dynamic Smagorinsky Model") mu_sgs = rho C_ds Delta^2 |S|
 *                plus the isotropic stress sigma_kk = 2 C_I rho Delta^2 |S|^2
 *                (sigma_kk / 3 added to the pressure of the momentum and energy
 *                fluxes) and Pr_sgs from the model; C_I, C_ds, Pr_sgs are global
 *                volume averages over the interior computed with the separable
 *                (1/4, 1/2, 1/4) test filter and Delta_hat = 2 Delta before
 *                every residual (LES_SCHEDULE_STEP: once per step); C_I, C_ds
 *                below zero are taken as zero, Pr_sgs falls back to the static
 *                value when not a positive number.  Cs is not used.  Holds 29
 *                FP64 scratch variables of the padded layout.  Not available
 *                with LES_BC_AXIS_NODE (les_validate: LES_EUNSUPPORTED). */
enum les_sgs {
  LES_SGS_NONE = 0,
  LES_SGS_SMAGORINSKY = 1,
  LES_SGS_VREMAN = 2,
  LES_SGS_DYNAMIC = 3
};

typedef struct les_params {
  int32_t nx, nr, nth;        /* interior points along xi, eta, zeta (each >= 5) */
  int32_t bc[6];              /* xi-, xi+, eta-, eta+, zeta-, zeta+ (enum les_bc) */
  double period[3][3];        /* translation vector added across the periodic
                                 faces of xi, eta, zeta (coordinates only) */
  double gamma;               /* ratio of specific heats */
  double Pr, Pr_sgs;          /* molecular and SGS Prandtl numbers */
  double visc_coef;           /* M/Re factor of the viscous fluxes (0: inviscid) */
  double suth_S;              /* Sutherland constant over the reference temperature */
  double Cs;                  /* Smagorinsky constant (Vreman: c = 2.5 Cs^2) */
  double k2, k4;              /* dissipation constants */
  double cfl;                 /* CFL number for the global time step */
  double rk_alpha[5];         /* stage coefficients alpha_1..alpha_5 */
  double ref_prim[5];         /* far-field state (rho, u, v, w, p) */
  double p_exit;              /* exit back pressure */
  int32_t sgs_model;          /* enum les_sgs */
  int32_t precision;          /* enum les_precision */
  int32_t schedule;           /* enum les_schedule */
} les_params;

/* ---- host-only helpers (no device work; callable without a GPU) -------- */

/* Validate `p` (sizes >= 5, consistent boundary kinds, finite positive
 * constants).  Returns LES_OK, LES_EINVAL, or LES_EUNSUPPORTED for a valid
 * combination this library does not provide. */
int les_validate(const les_params* p);

/* Padded layout for `p`: *pitch = row pitch in elements, dims[0..2] =
 * (nth+4, nr+4, pitch), *var_stride = elements per variable.  Returns
 * LES_EINVAL for invalid params, LES_EUNSUPPORTED if one variable exceeds
 * 2^31 - 1 elements. */
int les_layout(const les_params* p, int64_t* pitch, int64_t dims[3], int64_t* var_stride);

/* Device bytes the context will hold (metrics + stage buffers + scratch). */
int les_device_bytes(const les_params* p, size_t* bytes);

/* ---- context ------------------------------------------------------------ */

/* Create a context for a mesh given in one of two forms (exactly one):
 *   xyz         FP64, shape (3, nth, nr, nx), coordinates x, y, z of the
 *               interior points, i fastest; host or device memory (the
 *               runtime tells them apart); or
 *   X, R, TH    the 1-D maps of a cylindrical product mesh (section "Mesh
 *               Generation", tab:mesh-gen: the 3-D jet mesh is a 2-D axial-
 *               radial mesh rotated about the axis; here the 2-D mesh is the
 *               product of an axial and a radial distribution), X[nx],
 *               R[nr], TH[nth] FP64, host or device:
 *                 x = X[i],  y = R[j] cos(TH[k]),  z = R[j] sin(TH[k]),
 *               cos and sin evaluated on the host by the C library (a caller
 *               forming xyz with the same functions gets the same mesh
 *               bitwise); no 3-D coordinate array crosses the boundary.
 * The other form's pointers are NULL; both or neither given, or only some
 * of X, R, TH, is LES_EINVAL, as are non-finite maps.  Ghost coordinates
 * (three layers) are built on the device from the boundary kinds:
 * periodic -> wrapped point plus `period`; axis -> point (i, m, k + nth/2);
 * inflow/outflow/far field -> linear extrapolation in index space.
 * The inputs are copied; they may be freed after the call returns
 * (the call synchronises `stream`).  The environment variable LESJET_KCHUNK,
 * if set to a positive integer, overrides the number of azimuthal planes
 * one block of the fused kernel marches over (tuning and tests); with
 * LESJET_POISON=1 every device buffer the library allocates is filled with
 * NaN bit patterns (a test hook that exposes reads of unwritten memory).
 * Section "Transformation of
 * Coordinates"; the centerline and periodic subsections of "Boundary
 * Conditions". */
int les_init_grid(les_ctx** out, const les_params* p, const double* xyz, const double* X,
                  const double* R, const double* TH, void* stream);

/* Compute the metric terms J^-1 grad(xi), J^-1 grad(eta), J^-1 grad(zeta)
 * and J^-1 on the padded box by central differences of the coordinates
 * (metric-term and Jacobian equations of "Transformation of Coordinates";
 * the eta row taken as the cofactor r_zeta x r_xi).  Frees the coordinates.
 * If `metrics_out` (device, FP64, 10 padded variables in the order
 * Sxi_x, Sxi_y, Sxi_z, Seta_x .. Szeta_z, V) is not NULL the FP64 metrics
 * are copied there.  Must be called once before any residual. */
int les_metrics(les_ctx* c, double* metrics_out, void* stream);

/* Set the entrance target state: `prim_in` (device, FP64, shape (5, nth, nr),
 * primitives rho, u, v, w, p per entrance point).  Copied.  Section
 * "Entrance Boundary": a target with normal Mach >= 1 is imposed, otherwise
 * Riemann invariants with the target as outside state.  Required when
 * bc[0] == LES_BC_INFLOW. */
int les_set_inflow(les_ctx* c, const double* prim_in, void* stream);

/* Fill the ghost layers of Q (device, padded, 5 variables; FP64, or FP32 for
 * LES_FP32_STORAGE) in place: xi faces on the interior of eta/zeta, then eta
 * faces for all xi, then zeta faces everywhere (section "Boundary
 * Conditions").  Used internally before every residual; exported for tests. */
int les_fill_ghosts(les_ctx* c, void* Q, void* stream);

/* Residual R(Q) (section "Spatial Discretization"): fills the ghosts of Q in
 * place, then writes the interior of R (device, padded, 5 variables; FP64,
 * or FP32 for LES_FP32_STORAGE).  Ghost entries of R are not written. */
int les_residual(les_ctx* c, void* Q, void* R, void* stream);

/* The same residual computed by the two-pass reference kernels (a point
 * pass storing the point quantities of every point in library scratch, then
 * a face pass): simple indexing, several times the memory traffic.  For
 * validating the fused kernel on meshes the CPU oracle cannot handle. */
int les_residual_reference(les_ctx* c, void* Q, void* R, void* stream);

/* Coefficients of the dynamic SGS model (LES_SGS_DYNAMIC; subsection
 * "Dynamic Smagorinsky Model") for the state Q (device, padded, storage
 * type; its ghosts are filled in place): coef (host, 6 doubles) receives
 * C_I, C_ds and Pr_sgs as computed (Pr_sgs NaN when its denominator is 0),
 * then the values the residual uses (C_I and C_ds clipped at 0, Pr_sgs or
 * its static fallback).  Synchronises `stream`.  LES_EINVAL when the
 * context uses another SGS model. */
int les_dynamic_coefficients(les_ctx* c, void* Q, double* coef, void* stream);

/* Advance Qn (device, FP64, padded, 5 variables) by `nsteps` Jameson RK5
 * steps (section "Time Marching Method"):
 *   Q^(0) = Q^n,  Q^(l) = Q^(0) - alpha_l dt R(Q^(l-1)),  Q^(n+1) = Q^(5),
 * ghosts refilled before every residual (LES_SCHEDULE_STEP: see
 * les_schedule for what is held from Q^n).  dt_fixed > 0 uses that step;
 * dt_fixed <= 0 takes dt = cfl / max over the interior of
 * (lambda_xi + lambda_eta + lambda_zeta) of Q^n each step.  If `dt_out`
 * (device, nsteps doubles) is not NULL the steps used are stored there.
 * Synchronises `stream` once at the end to check the reductions; returns
 * LES_ENONFINITE if one was not finite (Qn is then undefined). */
int les_rk5_step(les_ctx* c, double* Qn, int32_t nsteps, double dt_fixed,
                 double* dt_out, void* stream);

/* Adjoint of the residual (FP64 precision and static or no SGS model only;
 * LES_EUNSUPPORTED otherwise):
 *   Qbar = (dR/dQ)^T Rbar,
 * the vector-Jacobian product of R (section "Spatial Discretization") as a
 * function of the interior of Q, the ghost fill of section "Boundary
 * Conditions" included, with the boundary data (entrance target, far-field
 * state, back pressure) held fixed.
 *   Q          device, FP64, padded, 5 variables; its ghost entries are
 *              overwritten by the ghost fill, the interior is read only.
 *   Rbar       device, same layout; only interior entries are read.
 *   Qbar       device, same layout, overwritten: interior = the cotangent,
 *              ghost entries and pitch padding = 0.  May alias Rbar.
 *   inflow_bar device, (5, nth, nr) doubles, or NULL: the cotangent of the
 *              entrance target (rho, u, v, w, p) is ADDED to it (only when
 *              xi- is an entrance).
 * Gather form without floating-point atomics: results are bitwise
 * reproducible.  Holds 28 scratch variables of the padded layout after the
 * first call.  Asynchronous on `stream`. */
int les_residual_vjp(les_ctx* c, double* Q, const double* Rbar, double* Qbar, double* inflow_bar,
                     void* stream);

/* Adjoint of one RK5 step with a fixed dt > 0 (section "Time Marching
 * Method"; a CFL step is frozen at its value): given the cotangent
 * Qbar_np1 of Q^(n+1), writes that of Q^n,
 *   b5 = Qbar_np1,  b(l-1) = -alpha_l dt (dR/dQ)^T(Q^(l-1)) b(l),
 *   Qbar_n = b5 + b4 + b3 + b2 + b1 + b0,
 * recomputing the stage states Q^(1..4) from Qn with the les_rk5_step
 * kernels.  Qn as in les_rk5_step (ghosts overwritten, interior unchanged);
 * ghost entries of Qbar_np1 are ignored, those of Qbar_n are zero;
 * Qbar_n may alias Qbar_np1; inflow_bar as in les_residual_vjp (added to).
 * FP64, LES_SCHEDULE_STAGE and static or no SGS model only
 * (LES_EUNSUPPORTED otherwise).  Holds 25
 * more padded variables after the first call.  Asynchronous on `stream`. */
int les_rk5_step_vjp(les_ctx* c, double* Qn, double dt, const double* Qbar_np1, double* Qbar_n,
                     double* inflow_bar, void* stream);

/* Diagnostics of the FP64 state Qn (device, padded), in a fixed summation
 * order (bitwise reproducible):
 *   totals (device, 5 doubles, or NULL): sum over the interior of J^-1 Q_c,
 *     the discrete conserved totals (constant on a periodic mesh);
 *   sum1, sum2 (device, (5, nr, nx) doubles each, or NULL): incremented by
 *     sum over k of phi and phi^2, phi = (rho, u, v, w, p), the accumulators
 *     of azimuthal and temporal mean and rms fields (the caller zeroes them).
 * Asynchronous on `stream`. */
int les_diagnostics(les_ctx* c, const double* Qn, double* totals, double* sum1, double* sum2,
                    void* stream);

/* The same diagnostics as les_diagnostics, allocating nothing: for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving or time-stepping loops, harnesses that forbid allocation).  The
 * per-block partial sums of the totals go to a static device array of the
 * library (80 KiB, at most 2048 blocks x 5 sums; every GPU the library runs
 * on holds one until the process ends) instead of a buffer allocated on
 * first use.  Sizes: any mesh the context accepts (the totals use at most
 * 2048 partial sums); LES_EUNSUPPORTED if a mesh needed more.  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other host threads, other contexts) race and must be serialised
 * by the caller.  Each call writes every partial sum before reading it, so
 * the array's previous contents never matter.  Asynchronous on `stream`. */
int les_diagnostics_noalloc(les_ctx* c, const double* Qn, double* totals, double* sum1,
                            double* sum2, void* stream);

/* Measurement support.  While enabled, every launch of the residual stage
 * kernel issued by les_residual and les_rk5_step is bracketed by a pair of
 * HIP events recorded on the call's stream, so the durations are those of
 * that kernel alone.  les_profile_read synchronises the recorded events,
 * returns the number of launches and their summed duration in milliseconds,
 * and clears the record.  Off by default (no events are recorded). */
int les_profile(les_ctx* c, int32_t enable);
int les_profile_read(les_ctx* c, int64_t* launches, double* total_ms);

/* Query the context: dims_padded = shape of a padded state (5, nth+4, nr+4,
 * pitch) (variable stride = dims_padded[1] * dims_padded[2] * pitch
 * elements), pitch = row pitch in elements, device_bytes = device memory the
 * library holds for the context.  Any output may be NULL. */
int les_query(const les_ctx* c, int64_t dims_padded[4], int64_t* pitch, size_t* device_bytes);

/* Message of the last failure on `c`, or of the calling thread when c is NULL
 * (e.g. after les_init_grid failed).  Never NULL. */
const char* les_last_error(const les_ctx* c);

/* Release the context and its device memory (synchronises the device). */
void les_free(les_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* LESJET_H */
