// Host-side launchers of the lesjet kernels (one translation unit per
// subsystem; the C-ABI in api.cpp calls these).
#pragma once

#include "common.hpp"

namespace lesjet {

// Padded coordinates with three ghost layers: from xyz (3, nth, nr, nx), host
// or device, or (xyz NULL) from the device table of a cylindrical product
// mesh X[nx], R[nr], cos(theta)[nth], sin(theta)[nth].
hipError_t launch_coords(const double* xyz, const double* tab, double* C, const CGrid& cg,
                         const int bc[6], const double period[3][3], hipStream_t s);

template <typename T>
hipError_t launch_metrics(const double* C, const CGrid& cg, T* M, const Grid& g, double* M64,
                          hipStream_t s);

// Axis row j = 0 := azimuthal mean of row j = 1 (centerline through the nodes).
template <typename T>
hipError_t launch_centerline(T* Q, const Grid& g, hipStream_t s);

// held != NULL: ghosts of physical faces (and the centerline row) are
// copied from `held` (a state filled earlier), the others traced as usual.
template <typename T>
hipError_t launch_ghosts(T* Q, const Grid& g, const T* M, const double* inflow, const Phys<T>& ph,
                         const int bc[6], const double ref_prim[5], double p_exit, const T* held,
                         hipStream_t s);

template <typename T>
hipError_t launch_residual_ref(const T* Q, const T* M, const Grid& g, const Phys<T>& ph, T* PT,
                               T* R, hipStream_t s);

template <typename T>
int fused_chunk(const Grid& g, int num_cu);

// dyn: coefficients of the dynamic SGS model (device, see launch_dynamic),
// read when ph.sgs == 3; may be NULL otherwise.
template <typename T>
hipError_t launch_fused(const T* Q, const T* M, const Grid& g, const Phys<T>& ph, int kc, int epi,
                        T* out, const double* Q0, double* Q64, double alpha, const double* dt,
                        const Phys<double>& ph64, unsigned long long* maxbits, int lag, T* visc,
                        const double* dyn, hipStream_t s);

// Dynamic Smagorinsky coefficients of the ghost-filled state Q: scratch SC
// (DYN_SCRATCH_VARS padded FP64 variables), part (7 doubles per block of
// dyn_blocks(g)), dyn (DYN_COEF_DOUBLES): [0] C_ds+ / Cv, [1] 1 / Pr_sgs,
// [2] (2/3) C_I+, [3..5] C_I, C_ds, Pr_sgs as computed, [6..12] the sums.
constexpr int DYN_SCRATCH_VARS = 29;
constexpr int DYN_COEF_DOUBLES = 16;
int dyn_blocks(const Grid& g);
template <typename T>
hipError_t launch_dynamic(const T* Q, const T* M, const Grid& g, double gamma, double Cv,
                          double Pr_static, double* SC, double* part, double* dyn,
                          hipStream_t s);

enum { FUSED_EPI_R = 0, FUSED_EPI_RK = 1, FUSED_EPI_RK_LAST = 2 };
// viscosity schedule of the stage kernel (same values as LAG_* of the
// point formulas): none, write the held values, read them
enum { FUSED_LAG_NONE = 0, FUSED_LAG_WRITE = 1, FUSED_LAG_READ = 2 };

template <typename TQ, typename TM>
hipError_t launch_lambda_max(const TQ* Q, const TM* M, const Grid& g, const Phys<double>& ph,
                             unsigned long long* maxbits, hipStream_t s);

hipError_t launch_dt_finalize(unsigned long long* maxbits, double cfl, double dt_fixed,
                              double* dt, double* dt_out, int* flag, hipStream_t s);

hipError_t launch_reset(unsigned long long* maxbits, int* flag, hipStream_t s);

template <typename T, typename TS>
hipError_t launch_rk_update(const double* Q0, const T* R, TS* Qout, double* Q64out, const Grid& g,
                            double alpha, const double* dt, hipStream_t s);

// Per-block partial sums of the diagnostics' totals: at most
// DIAG_MAX_PARTIALS blocks, 5 sums each.
constexpr int DIAG_MAX_PARTIALS = 2048;
int diag_partials(const Grid& g);

template <typename TM>
hipError_t launch_diagnostics(const double* Q, const TM* M, const Grid& g, const Phys<double>& ph,
                              double* part, double* totals, double* s1, double* s2, hipStream_t s);

// Residual adjoint (FP64): Qb = (dR/dQ)^T Rb on the padded layout (ghost
// entries zero); inflow_bar (5, nth, nr) accumulated when non-null.  Scratch
// SC of VJP_SCRATCH_VARS padded variables; Q's ghosts must be filled.
constexpr int VJP_SCRATCH_VARS = 28;
// Transpose of the axis-row mean (centerline through the nodes) on a
// cotangent field: the axis row's cotangent is spread over row 1, then zeroed.
hipError_t launch_centerline_transpose(double* Qb, const Grid& g, hipStream_t s);

hipError_t launch_residual_vjp(const double* Q, const double* M, const Grid& g,
                               const Phys<double>& ph, const int bc[6], const double ref_prim[5],
                               double p_exit, const double* inflow, const double* Rb, double* SC,
                               double* Qb, double* inflow_bar, hipStream_t s);
hipError_t launch_scale(const double* x, double a, double* y, long long n, hipStream_t s);
hipError_t launch_interior_copy(const double* x, double* y, const Grid& g, hipStream_t s);
hipError_t launch_accumulate(const double* x, double* y, long long n, hipStream_t s);

hipError_t launch_to_float(const double* a, float* b, long long n, hipStream_t s);

}  // namespace lesjet
