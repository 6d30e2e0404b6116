// Pointwise physics of the LES discretisation, written once for the compute
// type T (double or float) and used by every residual kernel.
//
// Point quantities (section "Transformation of Coordinates", eqs.
// hat-flux-G and hat-flux-Ev/Fv/Gv; section "Large Eddy Simulation
// Filtering"; Smagorinsky model):
//   G^d = Fe^d - Fv^d    inviscid minus viscous point flux along d,
//   lambda_bar^d         anisotropic spectral-radius scaling of the
//                        Turkel-Vatsa dissipation,
//   nu^d                 pressure sensor along d.
// Face flux (eqs. inv_flux_vec, dissip_term, eps_2_dissip, eps_4_dissip):
//   F = (G_L + G_R)/2 - V_f d,
//   d = lambda_f [eps2 (W_R - W_L) - eps4 (W_{R+1} - 3 W_R + 3 W_L - W_{L-1})].
//
// Readings of passages the paper leaves ambiguous: unhatted state with
// W = (rho, rho u, rho v, rho w, E + p) and V_f the face average of J^-1;
// minus sign between the two dissipation terms; sensor denominator
// p+ + 2p + p-; lambda_d = |U_d| + a |grad xi_d|; heat flux down the
// temperature gradient; mu_sgs = rho (Cs Delta)^2 |S| with Delta = |J^-1|^(1/3)
// in jet-viscosity units (divided by M/Re); viscous face flux as the mean of
// the two point fluxes from central-difference gradients.
#pragma once

#include "common.hpp"

namespace lesjet {

#if defined(__HIP_DEVICE_COMPILE__) && !defined(LESJET_IEEE_F64)
// FP64 square root and reciprocal from the hardware estimates refined by
// Newton-Raphson (Goldschmidt for the root): within an ulp of the correctly
// rounded results over the arguments the kernels meet (reciprocals of
// |x| in [1e-13, 1e6], either sign; roots of [1e-20, 1e12]; sqrt(0) = 0),
// at about half the instructions of the IEEE sequences (-DLESJET_IEEE_F64
// restores those).
__device__ __forceinline__ double nr_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double nr_sqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  g = fma(d, h, g);
  return x > 0.0 ? g : 0.0 * x;
}
#endif

template <typename T> __host__ __device__ __forceinline__ T tsqrt(T x);
#if defined(__HIP_DEVICE_COMPILE__) && !defined(LESJET_IEEE_F64)
template <> __host__ __device__ __forceinline__ double tsqrt<double>(double x) { return nr_sqrt(x); }
#else
template <> __host__ __device__ __forceinline__ double tsqrt<double>(double x) { return sqrt(x); }
#endif
// FP32 (the storage form only): the hardware square root (within an ulp)
// and a cube root from the hardware base-2 logarithm and exponential (within
// 4e-6 relative over the filter widths of the meshes), far inside that
// form's tolerances.
#if defined(__HIP_DEVICE_COMPILE__) && !defined(LESJET_IEEE_F32)
template <> __host__ __device__ __forceinline__ float tsqrt<float>(float x) {
  return __builtin_amdgcn_sqrtf(x);
}
#else
template <> __host__ __device__ __forceinline__ float tsqrt<float>(float x) { return sqrtf(x); }
#endif
template <typename T> __host__ __device__ __forceinline__ T tcbrt(T x);
template <> __host__ __device__ __forceinline__ double tcbrt<double>(double x) { return cbrt(x); }
#if defined(__HIP_DEVICE_COMPILE__) && !defined(LESJET_IEEE_F32)
template <> __host__ __device__ __forceinline__ float tcbrt<float>(float x) {
  // x > 0 here (|J^-1|); exp2(log2(x) / 3)
  return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 3.0f));
}
#else
template <> __host__ __device__ __forceinline__ float tcbrt<float>(float x) { return cbrtf(x); }
#endif
template <typename T> __host__ __device__ __forceinline__ T tpow(T x, T y);
template <> __host__ __device__ __forceinline__ double tpow<double>(double x, double y) { return pow(x, y); }
template <> __host__ __device__ __forceinline__ float tpow<float>(float x, float y) { return powf(x, y); }
template <typename T> __host__ __device__ __forceinline__ T tabs(T x);
template <> __host__ __device__ __forceinline__ double tabs<double>(double x) { return fabs(x); }
template <> __host__ __device__ __forceinline__ float tabs<float>(float x) { return fabsf(x); }
template <typename T> __host__ __device__ __forceinline__ T tmax(T a, T b);
template <> __host__ __device__ __forceinline__ double tmax<double>(double a, double b) { return fmax(a, b); }
template <> __host__ __device__ __forceinline__ float tmax<float>(float a, float b) { return fmaxf(a, b); }

// Reciprocal: Newton-refined in FP64 (above); the hardware approximation
// (1 ulp) in FP32, which serves only the FP32-storage form.
template <typename T> __host__ __device__ __forceinline__ T trcp(T x);
#if defined(__HIP_DEVICE_COMPILE__) && !defined(LESJET_IEEE_F64)
template <> __host__ __device__ __forceinline__ double trcp<double>(double x) { return nr_rcp(x); }
#else
template <> __host__ __device__ __forceinline__ double trcp<double>(double x) { return 1.0 / x; }
#endif
template <> __host__ __device__ __forceinline__ float trcp<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

// Primitive variables from Q = (rho, rho u, rho v, rho w, E); System-I energy
// E = p/(gamma-1) + rho |u|^2/2.
template <typename T>
struct Prim { T rho, u, v, w, p; };

template <typename T>
__host__ __device__ __forceinline__ Prim<T> primitives(const T q[5], const Phys<T>& ph) {
  Prim<T> s;
  s.rho = q[0];
  const T ir = trcp(q[0]);
  s.u = q[1] * ir;
  s.v = q[2] * ir;
  s.w = q[3] * ir;
  s.p = ph.gm1 * (q[4] - T(0.5) * q[0] * (s.u * s.u + s.v * s.v + s.w * s.w));
  return s;
}

// Temperature in jet units: p = rho T / gamma.
template <typename T>
__host__ __device__ __forceinline__ T temperature(const Prim<T>& s, const Phys<T>& ph) {
  return ph.gamma * s.p * trcp(s.rho);
}

// (u, v, w, T, p) of a state, the form the point computation consumes.
template <typename T>
__host__ __device__ __forceinline__ void prim5(const T q[5], const Phys<T>& ph, T pr[5]) {
  const T ir = trcp(q[0]);
  pr[0] = q[1] * ir;
  pr[1] = q[2] * ir;
  pr[2] = q[3] * ir;
  pr[4] = ph.gm1 * (q[4] - T(0.5) * q[0] * (pr[0] * pr[0] + pr[1] * pr[1] + pr[2] * pr[2]));
  pr[3] = ph.gamma * pr[4] * ir;
}

// Data a point needs: its state and primitives, the central differences of
// (u, v, w, T) and the pressure sensors along the three index directions
// (formed by the caller from the six neighbours, see `neighbour_terms`), its
// metrics.
template <typename T>
struct PointIn {
  T q[5];
  T pr[5];           // (u, v, w, T, p) of the point, from prim5
  T dl[3][4];        // (phi_{+1} - phi_{-1}) / 2 along d, phi = (u, v, w, T)
  T nu[3];           // pressure sensor along d
  T S[3][3];         // S[d] = J^-1 grad(xi_d)
  T V;               // J^-1
  T mt, kap;         // held mu + mu_sgs and conductivity (LAG_READ)
};

// Central differences and pressure sensor along one direction from the
// (u, v, w, T, p) of the -1 and +1 neighbours; p is the point's pressure.
template <typename T>
__host__ __device__ __forceinline__ void neighbour_terms(const T m[5], const T pl[5], T p, T dl[4],
                                                         T& nu) {
#pragma unroll
  for (int f = 0; f < 4; ++f) dl[f] = T(0.5) * (pl[f] - m[f]);
  const T num = pl[4] - T(2) * p + m[4];
  const T den = pl[4] + T(2) * p + m[4];
  nu = tabs(num) * trcp(den);
}

// Vreman's sqrt(B_beta / (alpha_ij alpha_ij)) divided by Delta^2, from the
// velocity gradient g[i][m] = d u_i / d x_m (alpha_mi = g[i][m]); zero where
// alpha_ij alpha_ij = 0 or B_beta <= 0 (rounding of a positive
// semi-definite minor sum).
template <typename T>
__host__ __device__ __forceinline__ T vreman_ratio(const T g[4][3]) {
  T b[3][3], aa = T(0);
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j)
      b[i][j] = g[i][0] * g[j][0] + g[i][1] * g[j][1] + g[i][2] * g[j][2];
  for (int i = 0; i < 3; ++i) aa += b[i][i];
  const T B = b[0][0] * b[1][1] - b[0][1] * b[0][1] + b[0][0] * b[2][2] - b[0][2] * b[0][2] +
              b[1][1] * b[2][2] - b[1][2] * b[1][2];
  return (aa > T(0) && B > T(0)) ? tsqrt(B * trcp(aa)) : T(0);
}

// 2 S_ij S_ij / 2 = S_ij S_ij with S_ij = (g_ij + g_ji) / 2 (each
// off-diagonal pair formed once), from g[i][m] = d u_i / d x_m.
template <typename T>
__host__ __device__ __forceinline__ T strain_sq(const T g[4][3]) {
  const T a01 = g[0][1] + g[1][0], a02 = g[0][2] + g[2][0], a12 = g[1][2] + g[2][1];
  return g[0][0] * g[0][0] + g[1][1] * g[1][1] + g[2][2] * g[2][2] +
         T(0.5) * (a01 * a01 + a02 * a02 + a12 * a12);
}

template <typename T>
struct PointOut {
  T G[3][5];
  T lb[3];
  T nu[3];
  T mt, kap;         // mu + mu_sgs and conductivity of the point (LAG_WRITE)
};

// Viscosity update schedule: computed from the point's own state (LAG_NONE),
// also returned for holding (LAG_WRITE), or taken from held values (LAG_READ).
enum { LAG_NONE = 0, LAG_WRITE = 1, LAG_READ = 2 };

// DYN: the dynamic SGS model's terms are compiled in (used when ph.sgs == 3);
// a separate instance so that the other models carry none of them.
template <typename T, int LAG = LAG_NONE, bool DYN = false>
__host__ __device__ inline void point_quantities(const PointIn<T>& in, const Phys<T>& ph,
                                                 PointOut<T>& out) {
  Prim<T> s;
  s.rho = in.q[0]; s.u = in.pr[0]; s.v = in.pr[1]; s.w = in.pr[2]; s.p = in.pr[4];
  const T Tt = in.pr[3];
  const T a = tsqrt(Tt);                       // a^2 = gamma p / rho = T
  const T iV = trcp(in.V);
  const T aiV = tabs(iV);

  T Uc[3];
  for (int d = 0; d < 3; ++d)
    Uc[d] = in.S[d][0] * s.u + in.S[d][1] * s.v + in.S[d][2] * s.w;

  // inviscid point fluxes
  for (int d = 0; d < 3; ++d) {
    out.G[d][0] = s.rho * Uc[d];
    out.G[d][1] = in.q[1] * Uc[d] + s.p * in.S[d][0];
    out.G[d][2] = in.q[2] * Uc[d] + s.p * in.S[d][1];
    out.G[d][3] = in.q[3] * Uc[d] + s.p * in.S[d][2];
    out.G[d][4] = (in.q[4] + s.p) * Uc[d];
  }

  if (ph.viscous) {
    // chain rule on the central differences
    const T (&dl)[3][4] = in.dl;
    T g[4][3];   // g[f][m] = d phi_f / d x_m, phi = (u, v, w, T)
    for (int f = 0; f < 4; ++f)
      for (int m = 0; m < 3; ++m)
        g[f][m] = (in.S[0][m] * dl[0][f] + in.S[1][m] * dl[1][f] + in.S[2][m] * dl[2][f]) * iV;

    T mt, kap;
    if (LAG == LAG_READ) {
      mt = in.mt;
      kap = in.kap;
    } else {
      const T mu = Tt * a * ph.suth1 * trcp(Tt + ph.suth);    // Sutherland
      T mut = T(0);
      if (ph.sgs == 1) {                                      // Smagorinsky
        const T s2 = strain_sq(g);
        const T delta = tcbrt(tabs(in.V));
        mut = s.rho * ph.sgs_coef * delta * delta * tsqrt(T(2) * s2);
      } else if (ph.sgs == 2) {                               // Vreman
        const T delta = tcbrt(tabs(in.V));
        mut = s.rho * ph.sgs_coef * delta * delta * vreman_ratio(g);
      } else if (DYN && ph.sgs == 3) {                        // dynamic: C_ds Delta^2 |S|
        const T s2 = strain_sq(g);
        const T delta = tcbrt(tabs(in.V));
        mut = s.rho * ph.sgs_coef * delta * delta * tsqrt(T(2) * s2);
      }
      mt = mu + mut;
      kap = (mu * ph.Pr_inv + mut * ph.Prs_inv) * ph.igm1;
      if (LAG == LAG_WRITE) {
        out.mt = mt;
        out.kap = kap;
      }
    }
    if (DYN && ph.sgs == 3) {
      // isotropic SGS stress of the dynamic model: sigma_kk / 3 =
      // (2/3) C_I rho Delta^2 |S|^2 acts as a pressure in the momentum and
      // energy point fluxes (stage |S|, coefficient of the launch)
      const T s2 = strain_sq(g);
      const T delta = tcbrt(tabs(in.V));
      const T psgs = ph.iso_coef * s.rho * delta * delta * (T(2) * s2);
      for (int d = 0; d < 3; ++d) {
        out.G[d][1] += psgs * in.S[d][0];
        out.G[d][2] += psgs * in.S[d][1];
        out.G[d][3] += psgs * in.S[d][2];
        out.G[d][4] += psgs * Uc[d];
      }
    }
    // the viscous coefficient M/Re folded into mu and kappa once: tau and
    // beta below are C_v tau_ij and C_v beta_j
    const T mtc = ph.Cv * mt, kapc = ph.Cv * kap;
    const T div = g[0][0] + g[1][1] + g[2][2];
    T tau[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = i; j < 3; ++j) {
        tau[i][j] = mtc * (g[i][j] + g[j][i] - (i == j ? T(2.0 / 3.0) * div : T(0)));
        tau[j][i] = tau[i][j];
      }
    T beta[3];
    for (int j = 0; j < 3; ++j)
      beta[j] = tau[0][j] * s.u + tau[1][j] * s.v + tau[2][j] * s.w + kapc * g[3][j];
    for (int d = 0; d < 3; ++d) {
      const T* Sd = in.S[d];
      out.G[d][1] -= Sd[0] * tau[0][0] + Sd[1] * tau[0][1] + Sd[2] * tau[0][2];
      out.G[d][2] -= Sd[0] * tau[1][0] + Sd[1] * tau[1][1] + Sd[2] * tau[1][2];
      out.G[d][3] -= Sd[0] * tau[2][0] + Sd[1] * tau[2][1] + Sd[2] * tau[2][2];
      out.G[d][4] -= Sd[0] * beta[0] + Sd[1] * beta[1] + Sd[2] * beta[2];
    }
  }

  // spectral radii and their anisotropic scaling
  T lam[3];
  for (int d = 0; d < 3; ++d) {
    const T* Sd = in.S[d];
    lam[d] = (tabs(Uc[d]) + a * tsqrt(Sd[0] * Sd[0] + Sd[1] * Sd[1] + Sd[2] * Sd[2])) * aiV;
  }
  // lambda_d + sqrt(lambda_d lambda_e) + sqrt(lambda_d lambda_f)
  //   = sqrt(lambda_d) (sqrt(lambda_d) + sqrt(lambda_e) + sqrt(lambda_f))
  const T r0 = tsqrt(lam[0]), r1 = tsqrt(lam[1]), r2 = tsqrt(lam[2]);
  const T rs = r0 + r1 + r2;
  out.lb[0] = r0 * rs;
  out.lb[1] = r1 * rs;
  out.lb[2] = r2 * rs;

  for (int d = 0; d < 3; ++d) out.nu[d] = in.nu[d];
}

// Dissipation vector W = (rho, rho u, rho v, rho w, E + p).
template <typename T>
__host__ __device__ __forceinline__ void wvec(const T q[5], const Phys<T>& ph, T W[5]) {
  const Prim<T> s = primitives(q, ph);
  W[0] = q[0]; W[1] = q[1]; W[2] = q[2]; W[3] = q[3]; W[4] = q[4] + s.p;
}

// Numerical flux at the face between L and R = L + 1 along one direction.
template <typename T>
__host__ __device__ __forceinline__ void face_flux(const T GL[5], const T GR[5], T lbL, T lbR,
                                                   T nuL, T nuR, T VL, T VR, const T Wm[5],
                                                   const T WL[5], const T WR[5], const T Wp[5],
                                                   bool physical, const Phys<T>& ph, T F[5]) {
  const T e2 = ph.k2 * tmax(nuL, nuR);
  const T e4 = tmax(T(0), ph.k4 - e2);
  const T lf = T(0.5) * (lbL + lbR);
  const T Vf = physical ? T(0) : T(0.5) * (VL + VR);
  // V_f d = a2 (W_R - W_L) - a4 ((W_{R+1} - W_{L-1}) - 3 (W_R - W_L))
  const T vl = Vf * lf, a2 = vl * e2, a4 = vl * e4;
  for (int c = 0; c < 5; ++c) {
    const T A = WR[c] - WL[c];
    const T B = (Wp[c] - Wm[c]) - T(3) * A;
    F[c] = T(0.5) * (GL[c] + GR[c]) - a2 * A + a4 * B;
  }
}

// Sum of the spectral radii lambda_xi + lambda_eta + lambda_zeta at a point
// (time-step restriction).
template <typename T>
__host__ __device__ __forceinline__ T lambda_sum(const T q[5], const T S[3][3], T V,
                                                 const Phys<T>& ph) {
  const Prim<T> s = primitives(q, ph);
  const T a = tsqrt(ph.gamma * s.p / s.rho);
  T tot = T(0);
  for (int d = 0; d < 3; ++d) {
    const T Uc = S[d][0] * s.u + S[d][1] * s.v + S[d][2] * s.w;
    tot += tabs(Uc) + a * tsqrt(S[d][0] * S[d][0] + S[d][1] * S[d][1] + S[d][2] * S[d][2]);
  }
  return tot / tabs(V);
}

// Riemann-invariant boundary state (far-field subsection of "Boundary
// Conditions"); e inside, r outside, n outward unit normal.  Returns the
// branch: 0 copy of e (supersonic exit), 1 outside state (supersonic
// entrance), 2 subsonic (f written).
template <typename T>
__host__ __device__ __forceinline__ int riemann(const Prim<T>& e, const Prim<T>& r, const T n[3],
                                                const Phys<T>& ph, Prim<T>& f) {
  const T ae = tsqrt(ph.gamma * e.p / e.rho);
  const T ar = tsqrt(ph.gamma * r.p / r.rho);
  const T qe = e.u * n[0] + e.v * n[1] + e.w * n[2];
  const T qr = r.u * n[0] + r.v * n[1] + r.w * n[2];
  if (qe / ae >= T(1)) return 0;
  if (qe / ae <= T(-1)) return 1;
  const T Rp = qe + T(2) * ae * ph.igm1;
  const T Rm = qr - T(2) * ar * ph.igm1;
  const T qf = T(0.5) * (Rp + Rm);
  const T af = T(0.25) * ph.gm1 * (Rp - Rm);
  const Prim<T>& src = qe >= T(0) ? e : r;
  const T qs = qe >= T(0) ? qe : qr;
  // entropy of the upwind side: rho_f = (rho^gamma a_f^2 / (gamma p))^(1/(gamma-1))
  const T base = tpow(src.rho, ph.gamma) * af * af / (ph.gamma * src.p);
  f.rho = tpow(base, ph.igm1);
  f.u = src.u + (qf - qs) * n[0];
  f.v = src.v + (qf - qs) * n[1];
  f.w = src.w + (qf - qs) * n[2];
  f.p = f.rho * af * af / ph.gamma;
  return 2;
}

template <typename T>
__host__ __device__ __forceinline__ void conserved(const Prim<T>& s, const Phys<T>& ph, T q[5]) {
  q[0] = s.rho;
  q[1] = s.rho * s.u;
  q[2] = s.rho * s.v;
  q[3] = s.rho * s.w;
  q[4] = s.p * ph.igm1 + T(0.5) * s.rho * (s.u * s.u + s.v * s.v + s.w * s.w);
}

}  // namespace lesjet
