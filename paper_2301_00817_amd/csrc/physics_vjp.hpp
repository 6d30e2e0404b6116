// Reverse mode (vector-Jacobian products) of the point and face functions
// of physics.hpp, written by hand: given the cotangents of the outputs,
// accumulate those of the inputs.  Used by the residual adjoint; FP64.
#pragma once

#include "physics.hpp"

namespace lesjet {

// Reverse of vreman_ratio: adds d(ratio)/d g[i][m] * rb to gb (zero where
// the forward clipped to zero).
template <typename T>
__host__ __device__ inline void vreman_ratio_vjp(const T g[4][3], T rb, T gb[4][3]) {
  T b[3][3], aa = T(0);
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j)
      b[i][j] = g[i][0] * g[j][0] + g[i][1] * g[j][1] + g[i][2] * g[j][2];
  for (int i = 0; i < 3; ++i) aa += b[i][i];
  const T B = b[0][0] * b[1][1] - b[0][1] * b[0][1] + b[0][0] * b[2][2] - b[0][2] * b[0][2] +
              b[1][1] * b[2][2] - b[1][2] * b[1][2];
  if (!(aa > T(0) && B > T(0))) return;
  const T iaa = trcp(aa);
  const T x = B * iaa;
  const T r = tsqrt(x);
  const T x_b = T(0.5) * rb * trcp(r);
  const T B_b = x_b * iaa;
  const T aa_b = -x_b * x * iaa;
  T bb[3][3];
  bb[0][0] = B_b * (b[1][1] + b[2][2]) + aa_b;
  bb[1][1] = B_b * (b[0][0] + b[2][2]) + aa_b;
  bb[2][2] = B_b * (b[0][0] + b[1][1]) + aa_b;
  bb[0][1] = T(-2) * b[0][1] * B_b;
  bb[0][2] = T(-2) * b[0][2] * B_b;
  bb[1][2] = T(-2) * b[1][2] * B_b;
  for (int m = 0; m < 3; ++m) {
    for (int i = 0; i < 3; ++i) gb[i][m] += T(2) * bb[i][i] * g[i][m];
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 3; ++j) {
        gb[i][m] += bb[i][j] * g[j][m];
        gb[j][m] += bb[i][j] * g[i][m];
      }
  }
}

// Cotangents of the inputs of point_quantities.
template <typename T>
struct PointBar {
  T q[5];            // direct dependence on the state of the point
  T pr[5];           // (u, v, w, T, p) of the point
  T dl[3][4];        // central differences
};

// Given Gb[d][c] = dL/dG^d_c and lbb[d] = dL/dlambda_bar^d, accumulate into
// `bar` (which the caller zeroes).  The sensors pass through the point
// function unchanged; their cotangents are handled by sensor_vjp.
template <typename T>
__host__ __device__ inline void point_quantities_vjp(const PointIn<T>& in, const Phys<T>& ph,
                                                     const T Gb[3][5], const T lbb[3],
                                                     PointBar<T>& bar) {
  const T rho = in.q[0], u = in.pr[0], v = in.pr[1], w = in.pr[2], Tt = in.pr[3], p = in.pr[4];
  const T vel[3] = {u, v, w};
  const T a = tsqrt(Tt);
  const T ia = trcp(a);                       // 1/T = ia^2
  const T iV = trcp(in.V);
  const T aiV = tabs(iV);
  T Uc[3], Uc_b[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d) Uc[d] = in.S[d][0] * u + in.S[d][1] * v + in.S[d][2] * w;
  T a_b = 0, Tt_b = 0, p_b = 0, rho_b = 0;
  T vel_b[3] = {0, 0, 0};

  // spectral radii and their anisotropic scaling
  {
    T lam[3], Sn[3];
    for (int d = 0; d < 3; ++d) {
      Sn[d] = tsqrt(in.S[d][0] * in.S[d][0] + in.S[d][1] * in.S[d][1] + in.S[d][2] * in.S[d][2]);
      lam[d] = (tabs(Uc[d]) + a * Sn[d]) * aiV;
    }
    const T s01 = tsqrt(lam[0] * lam[1]);
    const T s02 = tsqrt(lam[0] * lam[2]);
    const T s12 = tsqrt(lam[1] * lam[2]);
    // lb0 = l0 + s01 + s02, lb1 = l1 + s01 + s12, lb2 = l2 + s02 + s12
    const T s01_b = lbb[0] + lbb[1], s02_b = lbb[0] + lbb[2], s12_b = lbb[1] + lbb[2];
    T lam_b[3] = {lbb[0], lbb[1], lbb[2]};
    // d sqrt(x y)/dx = y / (2 sqrt(x y))
    if (s01 > T(0)) { const T h = T(0.5) * s01_b * trcp(s01); lam_b[0] += h * lam[1]; lam_b[1] += h * lam[0]; }
    if (s02 > T(0)) { const T h = T(0.5) * s02_b * trcp(s02); lam_b[0] += h * lam[2]; lam_b[2] += h * lam[0]; }
    if (s12 > T(0)) { const T h = T(0.5) * s12_b * trcp(s12); lam_b[1] += h * lam[2]; lam_b[2] += h * lam[1]; }
    for (int d = 0; d < 3; ++d) {
      Uc_b[d] += lam_b[d] * aiV * (Uc[d] < T(0) ? T(-1) : T(1));
      a_b += lam_b[d] * Sn[d] * aiV;
    }
  }

  if (ph.viscous) {
    const T (&dl)[3][4] = in.dl;
    T g[4][3];
    for (int f = 0; f < 4; ++f)
      for (int m = 0; m < 3; ++m)
        g[f][m] = (in.S[0][m] * dl[0][f] + in.S[1][m] * dl[1][f] + in.S[2][m] * dl[2][f]) * iV;
    const T iTS = trcp(Tt + ph.suth);
    const T mu = Tt * a * ph.suth1 * iTS;
    T mut = 0, Smag = 0, Csd2 = 0, sij[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) sij[i][j] = T(0.5) * (g[i][j] + g[j][i]);
    // mut = rho coef Delta^2 Smag with the model's shape factor Smag:
    // sqrt(2 S_ij S_ij) (Smagorinsky) or sqrt(B_beta / alpha.alpha) / Delta^2
    // (Vreman)
    if (ph.sgs) {
      const T delta = tcbrt(tabs(in.V));
      Csd2 = ph.sgs_coef * delta * delta;
      if (ph.sgs == 1) {
        T s2 = 0;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) s2 += sij[i][j] * sij[i][j];
        Smag = tsqrt(T(2) * s2);
      } else {
        Smag = vreman_ratio(g);
      }
      mut = rho * Csd2 * Smag;
    }
    const T mt = mu + mut;
    const T div = g[0][0] + g[1][1] + g[2][2];
    T tau[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        tau[i][j] = mt * (g[i][j] + g[j][i] - (i == j ? T(2.0 / 3.0) * div : T(0)));
    const T kap = (mu * ph.Pr_inv + mut * ph.Prs_inv) * ph.igm1;
    // G[d][1+i] -= Cv S[d].tau[i];  G[d][4] -= Cv S[d].beta
    T tau_b[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, beta_b[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d)
      for (int j = 0; j < 3; ++j) {
        for (int i = 0; i < 3; ++i) tau_b[i][j] -= ph.Cv * Gb[d][1 + i] * in.S[d][j];
        beta_b[j] -= ph.Cv * Gb[d][4] * in.S[d][j];
      }
    // beta[j] = sum_i tau[i][j] vel[i] + kap g[3][j]
    T kap_b = 0;
    T g_b[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int j = 0; j < 3; ++j) {
      for (int i = 0; i < 3; ++i) {
        tau_b[i][j] += beta_b[j] * vel[i];
        vel_b[i] += beta_b[j] * tau[i][j];
      }
      kap_b += beta_b[j] * g[3][j];
      g_b[3][j] += beta_b[j] * kap;
    }
    T mu_b = kap_b * ph.Pr_inv * ph.igm1;
    T mut_b = kap_b * ph.Prs_inv * ph.igm1;
    // tau[i][j] = mt (g[i][j] + g[j][i] - 2/3 delta_ij div)
    T mt_b = 0, trace_b = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        mt_b += tau_b[i][j] * (g[i][j] + g[j][i] - (i == j ? T(2.0 / 3.0) * div : T(0)));
        g_b[i][j] += mt * tau_b[i][j];
        g_b[j][i] += mt * tau_b[i][j];
      }
    for (int i = 0; i < 3; ++i) trace_b += tau_b[i][i];
    for (int i = 0; i < 3; ++i) g_b[i][i] -= T(2.0 / 3.0) * mt * trace_b;
    mu_b += mt_b;
    mut_b += mt_b;
    if (ph.sgs) {
      rho_b += mut_b * Csd2 * Smag;
      const T Smag_b = mut_b * rho * Csd2;
      if (ph.sgs == 1 && Smag > T(0)) {
        // Smag = sqrt(2 sum sij^2): dSmag/dg_ij = 2 sij / Smag
        const T h = T(2) * Smag_b * trcp(Smag);
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) g_b[i][j] += h * sij[i][j];
      } else if (ph.sgs == 2) {
        vreman_ratio_vjp(g, Smag_b, g_b);
      }
    }
    // Sutherland: dmu/dT = mu (3/(2T) - 1/(T + S))
    Tt_b += mu_b * mu * (T(1.5) * ia * ia - iTS);
    // g[f][m] = iV sum_d S[d][m] dl[d][f]
    for (int d = 0; d < 3; ++d)
      for (int f = 0; f < 4; ++f) {
        T acc = 0;
        for (int m = 0; m < 3; ++m) acc += in.S[d][m] * g_b[f][m];
        bar.dl[d][f] += acc * iV;
      }
  }

  // inviscid point fluxes
  for (int d = 0; d < 3; ++d) {
    rho_b += Gb[d][0] * Uc[d];
    Uc_b[d] += Gb[d][0] * rho;
    for (int i = 0; i < 3; ++i) {
      Uc_b[d] += Gb[d][1 + i] * in.q[1 + i];
      bar.q[1 + i] += Gb[d][1 + i] * Uc[d];
      p_b += Gb[d][1 + i] * in.S[d][i];
    }
    Uc_b[d] += Gb[d][4] * (in.q[4] + p);
    bar.q[4] += Gb[d][4] * Uc[d];
    p_b += Gb[d][4] * Uc[d];
  }
  for (int d = 0; d < 3; ++d)
    for (int i = 0; i < 3; ++i) vel_b[i] += Uc_b[d] * in.S[d][i];
  Tt_b += T(0.5) * a_b * ia;
  bar.q[0] += rho_b;
  bar.pr[0] += vel_b[0];
  bar.pr[1] += vel_b[1];
  bar.pr[2] += vel_b[2];
  bar.pr[3] += Tt_b;
  bar.pr[4] += p_b;
}

// Cotangent of the state from cotangents of (u, v, w, T, p) (reverse of prim5).
template <typename T>
__host__ __device__ inline void prim5_vjp(const T q[5], const Phys<T>& ph, const T prb[5],
                                          T qb[5]) {
  const T ir = trcp(q[0]);
  const T u = q[1] * ir, v = q[2] * ir, w = q[3] * ir;
  const T p = ph.gm1 * (q[4] - T(0.5) * q[0] * (u * u + v * v + w * w));
  // T = gamma p ir
  T p_b = prb[4] + prb[3] * ph.gamma * ir;
  T ir_b = prb[3] * ph.gamma * p;
  // p = gm1 (q4 - q0 |u|^2 / 2)
  T u_b[3] = {prb[0], prb[1], prb[2]};
  qb[4] += ph.gm1 * p_b;
  qb[0] -= ph.gm1 * T(0.5) * (u * u + v * v + w * w) * p_b;
  const T vel[3] = {u, v, w};
  for (int i = 0; i < 3; ++i) u_b[i] -= ph.gm1 * q[0] * vel[i] * p_b;
  // u_i = q_{1+i} ir
  for (int i = 0; i < 3; ++i) {
    qb[1 + i] += u_b[i] * ir;
    ir_b += u_b[i] * q[1 + i];
  }
  qb[0] -= ir_b * ir * ir;
}

// Sensor nu = |p+ - 2p + p-| / (p+ + 2p + p-): given its cotangent nb,
// the cotangent of each neighbour pressure (`side`) and of the centre
// pressure (`centre`).
template <typename T>
__host__ __device__ inline void sensor_vjp(T pm, T p0, T pp, T nb, T& side, T& centre) {
  const T num = pp - T(2) * p0 + pm;
  const T iden = trcp(pp + T(2) * p0 + pm);
  const T nu = tabs(num) * iden;
  const T sg = num < T(0) ? T(-1) : T(1);
  side = nb * (sg - nu) * iden;
  centre = nb * T(-2) * (sg + nu) * iden;
}

// Reverse of face_flux: accumulate the cotangents of G_L, G_R, lambda_bar_L/R,
// nu_L/R and W_{L-1}, W_L, W_R, W_{R+1} from Fb = dL/dF.
template <typename T>
__host__ __device__ inline void face_flux_vjp(const T lbL, const T lbR, const T nuL, const T nuR,
                                              const T VL, const T VR, const T Wm[5],
                                              const T WL[5], const T WR[5], const T Wp[5],
                                              bool physical, const Phys<T>& ph, const T Fb[5],
                                              T GbL[5], T GbR[5], T& lbbL, T& lbbR, T& nubL,
                                              T& nubR, T Wbm[5], T WbL[5], T WbR[5], T Wbp[5]) {
  for (int c = 0; c < 5; ++c) {
    GbL[c] += T(0.5) * Fb[c];
    GbR[c] += T(0.5) * Fb[c];
  }
  if (physical) return;
  const T e2 = ph.k2 * tmax(nuL, nuR);
  const T k4m = ph.k4 - e2;
  const T e4 = tmax(T(0), k4m);
  const T lf = T(0.5) * (lbL + lbR);
  const T Vf = T(0.5) * (VL + VR);
  T lf_b = 0, e2_b = 0, e4_b = 0;
  for (int c = 0; c < 5; ++c) {
    const T Db = -Vf * Fb[c];
    const T A = WR[c] - WL[c];
    const T B = Wp[c] - T(3) * WR[c] + T(3) * WL[c] - Wm[c];
    lf_b += Db * (e2 * A - e4 * B);
    e2_b += Db * lf * A;
    e4_b -= Db * lf * B;
    WbR[c] += lf * (e2 + T(3) * e4) * Db;
    WbL[c] -= lf * (e2 + T(3) * e4) * Db;
    Wbp[c] -= lf * e4 * Db;
    Wbm[c] += lf * e4 * Db;
  }
  if (k4m > T(0)) e2_b -= e4_b;
  lbbL += T(0.5) * lf_b;
  lbbR += T(0.5) * lf_b;
  if (nuL >= nuR) nubL += ph.k2 * e2_b;
  else nubR += ph.k2 * e2_b;
}

}  // namespace lesjet
