// Coefficients of the dynamic Smagorinsky model (subsection "Dynamic
// Smagorinsky Model"): C_I of the isotropic SGS stress, C_ds of the eddy
// viscosity and the SGS Prandtl number, each a ratio of two volume averages
// over the interior.  Test filter: the separable three-point filter
// (1/4, 1/2, 1/4) along each index direction, test width 2 Delta; Delta =
// |J^-1|^(1/3) stays outside the hats (the local width at the averaging
// point).  Computed in FP64 from the state of the storage type; the sums are
// fixed-order trees (reproducible).
//
//   k_dyn_fields  points of [-1, n]^3: rho |S| S_ij, rho |S|^2, rho |S| dT/dx_j
//                 (central differences, chain rule) and the filtered rho,
//                 rho u_i, rho T (27 points of the padded box);
//   k_dyn_sums    interior points: the remaining filtered quantities, the
//                 strain of u_hat = hat(rho u)/hat(rho) and the gradient of
//                 T_hat = hat(rho T)/hat(rho); per block, the J^-1-weighted
//                 sums of the seven numerator and denominator terms;
//   k_dyn_final   one block: the sums, the coefficients, clipping.
#include "launch.hpp"

namespace lesjet {

enum {
  DY_FS = 0,     // rho |S| S_ij, ij = 00 11 22 01 02 12
  DY_FS2 = 6,    // rho |S|^2
  DY_FT = 7,     // rho |S| dT/dx_j
  DY_HR = 10,    // hat(rho)
  DY_HRU = 11,   // hat(rho u_i)
  DY_HRT = 14,   // hat(rho T)
  DY_N = 15
};
static_assert(DY_N == DYN_SCRATCH_VARS, "dynamic-model scratch size");

constexpr int DY_BS = 256;
constexpr int DY_NSUM = 7;   // N_I, D_I, A, B, D_d, N_P, D_P
static_assert(DY_NSUM + 6 + 3 <= DYN_COEF_DOUBLES, "coefficient buffer size");

constexpr double FW[3] = {0.25, 0.5, 0.25};   // test-filter weights

struct PrimD {
  double rho, u, v, w, T, p;
};

template <typename T>
__device__ __forceinline__ PrimD prim_at(const T* __restrict__ Q, const Grid& g, int o,
                                         double gamma) {
  PrimD s;
  const double q0 = (double)Q[o], q1 = (double)Q[(long long)g.vs + o],
               q2 = (double)Q[2LL * g.vs + o], q3 = (double)Q[3LL * g.vs + o],
               q4 = (double)Q[4LL * g.vs + o];
  const double ir = 1.0 / q0;          // one division per point
  s.rho = q0;
  s.u = q1 * ir;
  s.v = q2 * ir;
  s.w = q3 * ir;
  s.p = (gamma - 1.0) * (q4 - 0.5 * q0 * (s.u * s.u + s.v * s.v + s.w * s.w));
  s.T = gamma * s.p * ir;
  return s;
}

// Resolved velocity and temperature gradients at o: central differences
// along the three index directions and the chain rule with the metrics.
template <typename T>
__device__ __forceinline__ void gradients(const T* __restrict__ Q, const T* __restrict__ M,
                                          const Grid& g, int o, double gamma, double gu[3][3],
                                          double gT[3]) {
  const int step[3] = {1, g.pitch, g.plane};
  double dl[3][4];
  for (int d = 0; d < 3; ++d) {
    const PrimD a = prim_at(Q, g, o + step[d], gamma), b = prim_at(Q, g, o - step[d], gamma);
    dl[d][0] = 0.5 * (a.u - b.u);
    dl[d][1] = 0.5 * (a.v - b.v);
    dl[d][2] = 0.5 * (a.w - b.w);
    dl[d][3] = 0.5 * (a.T - b.T);
  }
  const double iV = 1.0 / (double)M[9LL * g.vs + o];
  for (int m = 0; m < 3; ++m) {
    const double S0 = (double)M[(long long)m * g.vs + o];
    const double S1 = (double)M[(long long)(3 + m) * g.vs + o];
    const double S2 = (double)M[(long long)(6 + m) * g.vs + o];
    for (int f = 0; f < 3; ++f) gu[f][m] = (S0 * dl[0][f] + S1 * dl[1][f] + S2 * dl[2][f]) * iV;
    gT[m] = (S0 * dl[0][3] + S1 * dl[1][3] + S2 * dl[2][3]) * iV;
  }
}

__device__ __forceinline__ void strain(const double gu[3][3], double S[3][3], double& Smag) {
  double s2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S[i][j] = 0.5 * (gu[i][j] + gu[j][i]);
      s2 += S[i][j] * S[i][j];
    }
  Smag = sqrt(2.0 * s2);
}

// The 27-point product filter (weights FW[a] FW[b] FW[c], the separable
// three-point filter along i, j and k) of NF fields at o, accumulated point
// by point (few live registers); `val(o, v)` gives the fields at o.
template <int NF, typename F>
__device__ __forceinline__ void filter27(const Grid& g, int o, F val, double out[NF]) {
  for (int f = 0; f < NF; ++f) out[f] = 0.0;
  // few fields: unrolled (loads in flight together); many: rolled (registers)
  constexpr int U = NF <= 5 ? 3 : 1;
#pragma unroll U
  for (int dk = 0; dk < 3; ++dk)
#pragma unroll U
    for (int dj = 0; dj < 3; ++dj) {
      const double wjk = FW[dk] * FW[dj];
      const int ob = o + (dk - 1) * g.plane + (dj - 1) * g.pitch;
#pragma unroll
      for (int di = 0; di < 3; ++di) {
        double v[NF];
        val(ob + di - 1, v);
        const double w = wjk * FW[di];
        for (int f = 0; f < NF; ++f) out[f] += w * v[f];
      }
    }
}

template <typename T>
__global__ __launch_bounds__(DY_BS) void k_dyn_fields(const T* __restrict__ Q,
                                                      const T* __restrict__ M, Grid g,
                                                      double gamma, double* __restrict__ SC) {
  const int NX1 = g.nx + 2, NR1 = g.nr + 2, NT1 = g.nth + 2;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)NX1 * NR1 * NT1) return;
  const int i = (int)(t % NX1) - 1;
  const int j = (int)((t / NX1) % NR1) - 1;
  const int k = (int)(t / ((long long)NX1 * NR1)) - 1;
  const int o = g.at(i, j, k);
  double gu[3][3], gT[3], S[3][3], Smag;
  gradients(Q, M, g, o, gamma, gu, gT);
  strain(gu, S, Smag);
  const double rho = (double)Q[o];
  const double rS = rho * Smag;
  const int IJ[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  for (int q = 0; q < 6; ++q) SC[(long long)(DY_FS + q) * g.vs + o] = rS * S[IJ[q][0]][IJ[q][1]];
  SC[(long long)DY_FS2 * g.vs + o] = rho * Smag * Smag;
  for (int m = 0; m < 3; ++m) SC[(long long)(DY_FT + m) * g.vs + o] = rS * gT[m];
  // hat(rho), hat(rho u_i), hat(rho T) over the padded box
  double h[5];
  filter27<5>(g, o, [&](int oo, double v[5]) {
    const PrimD s = prim_at(Q, g, oo, gamma);
    v[0] = s.rho; v[1] = s.rho * s.u; v[2] = s.rho * s.v; v[3] = s.rho * s.w; v[4] = s.rho * s.T;
  }, h);
  SC[(long long)DY_HR * g.vs + o] = h[0];
  for (int c = 0; c < 3; ++c) SC[(long long)(DY_HRU + c) * g.vs + o] = h[1 + c];
  SC[(long long)DY_HRT * g.vs + o] = h[4];
}

template <typename T>
__global__ __launch_bounds__(DY_BS) void k_dyn_sums(const T* __restrict__ Q,
                                                    const T* __restrict__ M, Grid g,
                                                    double gamma, const double* __restrict__ SC,
                                                    double* __restrict__ part) {
  __shared__ double red[DY_NSUM][DY_BS];
  const long long tot = (long long)g.nx * g.nr * g.nth;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  double term[DY_NSUM] = {0, 0, 0, 0, 0, 0, 0};
  if (t < tot) {
    const int i = (int)(t % g.nx);
    const int j = (int)((t / g.nx) % g.nr);
    const int k = (int)(t / ((long long)g.nx * g.nr));
    const int o = g.at(i, j, k);
    // resolved strain and temperature gradient at the point
    double gu[3][3], gT[3], S[3][3], Smag;
    gradients(Q, M, g, o, gamma, gu, gT);
    strain(gu, S, Smag);
    const double trS = S[0][0] + S[1][1] + S[2][2];
    // filtered fields from [-1, n]^3
    double hF[10];
    filter27<10>(g, o, [&](int oo, double v[10]) {
      for (int q = 0; q < 10; ++q) v[q] = SC[(long long)q * g.vs + oo];
    }, hF);
    // filtered products of the padded state
    double hP[9];
    filter27<9>(g, o, [&](int oo, double v[9]) {
      const PrimD s = prim_at(Q, g, oo, gamma);
      const double uu[3] = {s.u, s.v, s.w};
      v[0] = s.rho * uu[0] * uu[0]; v[1] = s.rho * uu[1] * uu[1]; v[2] = s.rho * uu[2] * uu[2];
      v[3] = s.rho * uu[0] * uu[1]; v[4] = s.rho * uu[0] * uu[2]; v[5] = s.rho * uu[1] * uu[2];
      for (int c = 0; c < 3; ++c) v[6 + c] = s.rho * uu[c] * s.T;
    }, hP);
    const double hr = SC[(long long)DY_HR * g.vs + o];
    const double ihr = 1.0 / hr;
    double hru[3];
    for (int c = 0; c < 3; ++c) hru[c] = SC[(long long)(DY_HRU + c) * g.vs + o];
    const double hrT = SC[(long long)DY_HRT * g.vs + o];
    // strain of u_hat and gradient of T_hat (central differences of the
    // filtered fields at the neighbours, metrics of the point)
    const int step[3] = {1, g.pitch, g.plane};
    double dl[3][4];
    for (int d = 0; d < 3; ++d) {
      const int op = o + step[d], om = o - step[d];
      const double irp = 1.0 / SC[(long long)DY_HR * g.vs + op];
      const double irm = 1.0 / SC[(long long)DY_HR * g.vs + om];
      for (int c = 0; c < 3; ++c)
        dl[d][c] = 0.5 * (SC[(long long)(DY_HRU + c) * g.vs + op] * irp -
                          SC[(long long)(DY_HRU + c) * g.vs + om] * irm);
      dl[d][3] = 0.5 * (SC[(long long)DY_HRT * g.vs + op] * irp - SC[(long long)DY_HRT * g.vs + om] * irm);
    }
    const double V = (double)M[9LL * g.vs + o];
    const double iV = 1.0 / V;
    double guh[3][3], gTh[3];
    for (int m = 0; m < 3; ++m) {
      const double S0 = (double)M[(long long)m * g.vs + o];
      const double S1 = (double)M[(long long)(3 + m) * g.vs + o];
      const double S2 = (double)M[(long long)(6 + m) * g.vs + o];
      for (int f = 0; f < 3; ++f) guh[f][m] = (S0 * dl[0][f] + S1 * dl[1][f] + S2 * dl[2][f]) * iV;
      gTh[m] = (S0 * dl[0][3] + S1 * dl[1][3] + S2 * dl[2][3]) * iV;
    }
    double Sh[3][3], Shmag;
    strain(guh, Sh, Shmag);
    const double trSh = Sh[0][0] + Sh[1][1] + Sh[2][2];
    const double D2 = pow(fabs(V), 2.0 / 3.0);
    const double Dh2 = 4.0 * D2;
    // L_ij and the contractions
    const int IJ[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    double Lll = 0.0, LS = 0.0, hSS = 0.0, ShS = 0.0;
    for (int q = 0; q < 6; ++q) {
      const int a = IJ[q][0], b = IJ[q][1];
      const double w = a == b ? 1.0 : 2.0;            // symmetric: off-diagonals twice
      const double L = hP[q] - hru[a] * hru[b] * ihr;
      if (a == b) Lll += L;
      LS += w * L * S[a][b];
      hSS += w * hF[DY_FS + q] * S[a][b];
      ShS += w * Sh[a][b] * S[a][b];
    }
    const double hSmm = hF[DY_FS + 0] + hF[DY_FS + 1] + hF[DY_FS + 2];
    const double hS2 = hF[DY_FS2];
    double NP = 0.0, DP = 0.0;
    for (int m = 0; m < 3; ++m) {
      NP += D2 * hF[DY_FT + m] * gT[m] - Dh2 * hr * Shmag * gTh[m] * gT[m];
      DP += (hP[6 + m] - hru[m] * hrT * ihr) * gT[m];
    }
    term[0] = Lll;                                                     // N_I
    term[1] = 2.0 * Dh2 * hr * Shmag * Shmag - 2.0 * D2 * hS2;         // D_I
    term[2] = LS - trS * Lll / 3.0;                                    // A
    term[3] = trS * 2.0 * D2 * hS2 / 3.0;                              // B
    term[4] = 2.0 * D2 * (hSS - hSmm * trS / 3.0) -
              2.0 * Dh2 * (hr * Shmag * ShS - hr * Shmag * trSh * trS / 3.0);   // D_d
    term[5] = NP;
    term[6] = DP;
    for (int q = 0; q < DY_NSUM; ++q) term[q] *= V;
  }
  for (int q = 0; q < DY_NSUM; ++q) red[q][threadIdx.x] = term[q];
  __syncthreads();
  for (int w = DY_BS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < DY_NSUM; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < DY_NSUM) part[(long long)blockIdx.x * DY_NSUM + threadIdx.x] = red[threadIdx.x][0];
}

// dyn[0] = C_ds+ / Cv (eddy-viscosity coefficient in jet-viscosity units),
// dyn[1] = 1 / Pr_sgs used, dyn[2] = (2/3) C_I+, dyn[3..5] = C_I, C_ds,
// Pr_sgs as computed, dyn[6..12] = the seven sums.
__global__ __launch_bounds__(DY_BS) void k_dyn_final(const double* __restrict__ part, int nblk,
                                                     double Cv, double Pr_static,
                                                     double* __restrict__ dyn) {
  __shared__ double red[DY_NSUM][DY_BS];
  double acc[DY_NSUM] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblk; b += DY_BS)
    for (int q = 0; q < DY_NSUM; ++q) acc[q] += part[(long long)b * DY_NSUM + q];
  for (int q = 0; q < DY_NSUM; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = DY_BS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < DY_NSUM; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double N_I = red[0][0], D_I = red[1][0], A = red[2][0], B = red[3][0],
               D_d = red[4][0], N_P = red[5][0], D_P = red[6][0];
  const double C_I = D_I != 0.0 ? N_I / D_I : 0.0;
  const double C_Ip = fmax(C_I, 0.0);
  const double C_ds = D_d != 0.0 ? (A + C_Ip * B) / D_d : 0.0;
  const double C_dsp = fmax(C_ds, 0.0);
  const double Pr = D_P != 0.0 ? C_dsp * N_P / D_P : NAN;
  const double Pr_used = isfinite(Pr) && Pr > 0.0 ? Pr : Pr_static;
  dyn[0] = C_dsp / Cv;
  dyn[1] = 1.0 / Pr_used;
  dyn[2] = (2.0 / 3.0) * C_Ip;
  dyn[3] = C_I;
  dyn[4] = C_ds;
  dyn[5] = Pr;
  for (int q = 0; q < DY_NSUM; ++q) dyn[6 + q] = red[q][0];
}

int dyn_blocks(const Grid& g) {
  return (int)blocks_for((long long)g.nx * g.nr * g.nth, DY_BS);
}

template <typename T>
hipError_t launch_dynamic(const T* Q, const T* M, const Grid& g, double gamma, double Cv,
                          double Pr_static, double* SC, double* part, double* dyn,
                          hipStream_t s) {
  const long long n1 = (long long)(g.nx + 2) * (g.nr + 2) * (g.nth + 2);
  hipLaunchKernelGGL(k_dyn_fields<T>, dim3(blocks_for(n1, DY_BS)), dim3(DY_BS), 0, s, Q, M, g,
                     gamma, SC);
  const int nb = dyn_blocks(g);
  hipLaunchKernelGGL(k_dyn_sums<T>, dim3(nb), dim3(DY_BS), 0, s, Q, M, g, gamma,
                     (const double*)SC, part);
  hipLaunchKernelGGL(k_dyn_final, dim3(1), dim3(DY_BS), 0, s, (const double*)part, nb, Cv,
                     Pr_static, dyn);
  return hipGetLastError();
}

template hipError_t launch_dynamic<double>(const double*, const double*, const Grid&, double,
                                           double, double, double*, double*, double*,
                                           hipStream_t);
template hipError_t launch_dynamic<float>(const float*, const float*, const Grid&, double, double,
                                          double, double*, double*, double*, hipStream_t);

}  // namespace lesjet
