// Coefficients of the dynamic Smagorinsky model (subsection "Dynamic
// Smagorinsky Model"): C_I of the isotropic SGS stress, C_ds of the eddy
// viscosity and the SGS Prandtl number, each a ratio of two volume averages
// over the interior.  Test filter: the separable three-point filter
// (1/4, 1/2, 1/4) along each index direction, test width 2 Delta; Delta =
// |J^-1|^(1/3) stays outside the hats (the local width at the averaging
// point).  Computed in FP64 from the state of the storage type; the sums are
// fixed-order trees (reproducible).
//
// The separable filter is applied one direction at a time:
//   k_dyn_plane   per 32 x 8 tile of a plane, the primitives of the tile
//                 and two rings staged once in LDS: rho |S| S_ij,
//                 rho |S|^2, rho |S| dT/dx_j (central differences and the
//                 chain rule) formed once per point of the tile and its ring
//                 into LDS; rho, rho u_i, rho T, rho u_i u_j, rho u_i T
//                 formed from the staged primitives where read; all filtered
//                 along i and j and stored;
//   k_dyn_hat     points of [-1, n]^3: the filter along k of rho, rho u_i,
//                 rho T -> hat(rho), hat(rho u_i), hat(rho T);
//   k_dyn_sums    interior points: the filter along k of the other fields,
//                 the strain of u_hat = hat(rho u)/hat(rho) and the gradient
//                 of T_hat = hat(rho T)/hat(rho); per block, the
//                 J^-1-weighted sums of the seven numerator and denominator
//                 terms;
//   k_dyn_final   one block: the sums, the coefficients, clipping.
#include "launch.hpp"
#include "physics.hpp"

namespace lesjet {

// Fields filtered along i and j (index within the 24 filtered fields and
// scratch variable), then the fully filtered state.
enum {
  DY_FS = 0,     // rho |S| S_ij, ij = 00 11 22 01 02 12    (i, j in [0, n), k in [-1, n])
  DY_FS2 = 6,    // rho |S|^2
  DY_FT = 7,     // rho |S| dT/dx_j
  DY_PUU = 10,   // rho u_i u_j, ij = 00 11 22 01 02 12
  DY_PUT = 16,   // rho u_i T
  DY_NG = 19,    // fields used at interior points only
  DY_R = 19,     // rho, rho u_i, rho T                      (i, j in [-1, n], every plane)
  DY_NF = 24,
  DY_HR = 24,    // hat(rho)                                 ([-1, n]^3)
  DY_HRU = 25,   // hat(rho u_i)
  DY_HRT = 28,   // hat(rho T)
  DY_N = 29
};
static_assert(DY_N == DYN_SCRATCH_VARS, "dynamic-model scratch size");

constexpr int DY_BS = 256;
constexpr int DY_NXCD = 8;   // XCDs of the device (workgroups are dealt to them in turn)
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
  const double ir = trcp(q0);          // one reciprocal per point
  s.rho = q0;
  s.u = q1 * ir;
  s.v = q2 * ir;
  s.w = q3 * ir;
  s.p = (gamma - 1.0) * (q4 - 0.5 * q0 * (s.u * s.u + s.v * s.v + s.w * s.w));
  s.T = gamma * s.p * ir;
  return s;
}

// Velocity and temperature gradients at o from the central differences
// dl[d] of (u, v, w, T) along the three index directions (chain rule with
// the metrics of o).
template <typename T>
__device__ __forceinline__ void chain_rule(const double dl[3][4], const T* __restrict__ M,
                                           const Grid& g, int o, double gu[3][3], double gT[3]) {
  const double iV = trcp((double)M[9LL * g.vs + o]);
  for (int m = 0; m < 3; ++m) {
    const double S0 = (double)M[(long long)m * g.vs + o];
    const double S1 = (double)M[(long long)(3 + m) * g.vs + o];
    const double S2 = (double)M[(long long)(6 + m) * g.vs + o];
    for (int f = 0; f < 3; ++f) gu[f][m] = (S0 * dl[0][f] + S1 * dl[1][f] + S2 * dl[2][f]) * iV;
    gT[m] = (S0 * dl[0][3] + S1 * dl[1][3] + S2 * dl[2][3]) * iV;
  }
}

// Resolved gradients at o, the neighbours' primitives from global memory.
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
  chain_rule(dl, M, g, o, gu, gT);
}

__device__ __forceinline__ void strain(const double gu[3][3], double S[3][3], double& Smag) {
  double s2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S[i][j] = 0.5 * (gu[i][j] + gu[j][i]);
      s2 += S[i][j] * S[i][j];
    }
  Smag = tsqrt(2.0 * s2);
}

// Tiles of the columns [-2, n] x [-1, n] of a plane; every padded plane.
// Gradient fields on the tile and a one-point ring (DP_*), primitives on the
// tile and a two-point ring (DQ_*).
constexpr int DP_X = 32, DP_Y = 8, DP_HX = DP_X + 2, DP_HY = DP_Y + 2, DP_HP = DP_HX * DP_HY;
constexpr int DQ_HX = DP_X + 4, DQ_HY = DP_Y + 4, DQ_HP = DQ_HX * DQ_HY;

template <typename T>
__global__ __launch_bounds__(DP_X * DP_Y) void k_dyn_plane(const T* __restrict__ Q,
                                                           const T* __restrict__ M, Grid g,
                                                           double gamma, int tiles_x,
                                                           double* __restrict__ SC) {
  __shared__ double sP[5][DQ_HP];          // rho, u, v, w, T
  __shared__ double sG[DY_PUU][DP_HP];     // rho |S| S_ij, rho |S|^2, rho |S| dT/dx_j
  // tile columns start at padded index 0 (i = -2) so that each tile row is
  // whole 128-byte lines of the scratch arrays
  const int i0 = (blockIdx.x % tiles_x) * DP_X - NG, j0 = (blockIdx.x / tiles_x) * DP_Y - 1;
  const int k = (int)blockIdx.y - NG;
  // the gradient fields are needed on the planes [-1, n] (uniform per block)
  const bool kgrad = k >= -1 && k <= g.nth;
  const int tid = threadIdx.x;
  // primitives of the tile and two rings, clamped to the padded box (a
  // clamped slot feeds no stored value)
  for (int e = tid; e < DQ_HP; e += DP_X * DP_Y) {
    const int i = min(i0 - 2 + e % DQ_HX, g.nx + 1), j = min(j0 - 2 + e / DQ_HX, g.nr + 1);
    const PrimD s = prim_at(Q, g, g.at(max(i, -NG), max(j, -NG), k), gamma);
    sP[0][e] = s.rho;
    sP[1][e] = s.u;
    sP[2][e] = s.v;
    sP[3][e] = s.w;
    sP[4][e] = s.T;
  }
  __syncthreads();
  const int IJ[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  if (kgrad) {
    for (int e = tid; e < DP_HP; e += DP_X * DP_Y) {
      const int hx = e % DP_HX, hy = e / DP_HX;
      const int i = i0 - 1 + hx, j = j0 - 1 + hy;
      double F[DY_PUU];
      // only where an interior column's filter reads them
      if (i >= -1 && i <= g.nx && j >= -1 && j <= g.nr) {
        const int ep = (hy + 1) * DQ_HX + hx + 1;       // the same point among the primitives
        const int o = g.at(i, j, k);
        double dl[3][4];
        const int sd[2] = {1, DQ_HX};
        for (int d = 0; d < 2; ++d)
          for (int f = 0; f < 4; ++f) dl[d][f] = 0.5 * (sP[1 + f][ep + sd[d]] - sP[1 + f][ep - sd[d]]);
        const PrimD a = prim_at(Q, g, o + g.plane, gamma), b = prim_at(Q, g, o - g.plane, gamma);
        dl[2][0] = 0.5 * (a.u - b.u);
        dl[2][1] = 0.5 * (a.v - b.v);
        dl[2][2] = 0.5 * (a.w - b.w);
        dl[2][3] = 0.5 * (a.T - b.T);
        double gu[3][3], gT[3], S[3][3], Smag;
        chain_rule(dl, M, g, o, gu, gT);
        strain(gu, S, Smag);
        const double rho = sP[0][ep], rS = rho * Smag;
        for (int q = 0; q < 6; ++q) F[DY_FS + q] = rS * S[IJ[q][0]][IJ[q][1]];
        F[DY_FS2] = rho * Smag * Smag;
        for (int m = 0; m < 3; ++m) F[DY_FT + m] = rS * gT[m];
      } else {
        for (int f = 0; f < DY_PUU; ++f) F[f] = 0.0;
      }
      for (int f = 0; f < DY_PUU; ++f) sG[f][e] = F[f];
    }
    __syncthreads();
  }
  const int tx = tid % DP_X, ty = tid / DP_X;
  const int i = i0 + tx, j = j0 + ty;
  if (i > g.nx || j > g.nr) return;
  const int o = g.at(i, j, k);
  const bool inner_col = i >= 0 && i < g.nx && j >= 0 && j < g.nr && kgrad;
  // the state fields and the products, formed from the staged primitives
  // where the filter reads them
  double acc[DY_NF - DY_PUU];
  for (int f = 0; f < DY_NF - DY_PUU; ++f) acc[f] = 0.0;
  for (int b = 0; b < 3; ++b) {
    double row[DY_NF - DY_PUU];
    for (int f = 0; f < DY_NF - DY_PUU; ++f) row[f] = 0.0;
    for (int a = 0; a < 3; ++a) {
      const int e = (ty + 1 + b) * DQ_HX + tx + 1 + a;
      const double rho = sP[0][e], uu[3] = {sP[1][e], sP[2][e], sP[3][e]}, Tt = sP[4][e];
      row[DY_R - DY_PUU] += FW[a] * rho;
      for (int c = 0; c < 3; ++c) row[DY_R - DY_PUU + 1 + c] += FW[a] * (rho * uu[c]);
      row[DY_R - DY_PUU + 4] += FW[a] * (rho * Tt);
      if (inner_col) {
        for (int q = 0; q < 6; ++q) row[q] += FW[a] * (rho * uu[IJ[q][0]] * uu[IJ[q][1]]);
        for (int c = 0; c < 3; ++c) row[DY_PUT - DY_PUU + c] += FW[a] * (rho * uu[c] * Tt);
      }
    }
    for (int f = 0; f < DY_NF - DY_PUU; ++f) acc[f] += FW[b] * row[f];
  }
  for (int f = inner_col ? DY_PUU : DY_R; f < DY_NF; ++f) SC[(long long)f * g.vs + o] = acc[f - DY_PUU];
  if (!inner_col) return;
  for (int f = 0; f < DY_PUU; ++f) {
    double sum = 0.0;
    for (int b = 0; b < 3; ++b) {
      const int e = (ty + b) * DP_HX + tx;
      sum += FW[b] * (FW[0] * sG[f][e] + FW[1] * sG[f][e + 1] + FW[2] * sG[f][e + 2]);
    }
    SC[(long long)f * g.vs + o] = sum;
  }
}

// hat(rho), hat(rho u_i), hat(rho T) at the points of [-1, n]^3: the
// i-j-filtered fields filtered along k.  One thread per element of the rows
// j in [-1, n] of the planes [-1, n] (whole rows, so stores fill lines).
__global__ __launch_bounds__(DY_BS) void k_dyn_hat(Grid g, double* __restrict__ SC) {
  const long long rows = (long long)(g.nr + 2) * (g.nth + 2);
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= rows * g.pitch) return;
  const int i = (int)(t % g.pitch) - NG;
  const long long r = t / g.pitch;
  const int j = (int)(r % (g.nr + 2)) - 1, k = (int)(r / (g.nr + 2)) - 1;
  if (i < -1 || i > g.nx) return;
  const int o = g.at(i, j, k);
  for (int f = 0; f < 5; ++f) {
    const double* F = SC + (long long)(DY_R + f) * g.vs;
    SC[(long long)(DY_HR + f) * g.vs + o] =
        FW[0] * F[o - g.plane] + FW[1] * F[o] + FW[2] * F[o + g.plane];
  }
}

template <typename T>
__global__ __launch_bounds__(DY_BS) void k_dyn_sums(const T* __restrict__ Q,
                                                    const T* __restrict__ M, Grid g,
                                                    double gamma, const double* __restrict__ SC,
                                                    double* __restrict__ part) {
  __shared__ double red[DY_NSUM][DY_BS];
  // blocks of an interior plane dealt to the eight XCDs so that each XCD
  // walks its share of every plane in order (the k-neighbour planes are then
  // in its own L2)
  const int P = (g.nx * g.nr + DY_BS - 1) / DY_BS, Pmax = (P + DY_NXCD - 1) / DY_NXCD;
  const int hw = blockIdx.x, x = hw % DY_NXCD, r = hw / DY_NXCD;
  const int k = r / Pmax, pb = x * Pmax + r % Pmax;
  const int q0 = pb * DY_BS + (int)threadIdx.x;
  double term[DY_NSUM] = {0, 0, 0, 0, 0, 0, 0};
  if (k < g.nth && pb < P && q0 < g.nx * g.nr) {
    const int i = q0 % g.nx, j = q0 / g.nx;
    const int o = g.at(i, j, k);
    // resolved strain and temperature gradient at the point
    double gu[3][3], gT[3], S[3][3], Smag;
    gradients(Q, M, g, o, gamma, gu, gT);
    strain(gu, S, Smag);
    const double trS = S[0][0] + S[1][1] + S[2][2];
    // the other filtered fields: the i-j-filtered ones filtered along k
    double hF[DY_PUU], hP[DY_NG - DY_PUU];
    for (int f = 0; f < DY_NG; ++f) {
      const double* F = SC + (long long)f * g.vs;
      const double v = FW[0] * F[o - g.plane] + FW[1] * F[o] + FW[2] * F[o + g.plane];
      if (f < DY_PUU) hF[f] = v; else hP[f - DY_PUU] = v;
    }
    const double hr = SC[(long long)DY_HR * g.vs + o];
    const double ihr = trcp(hr);
    double hru[3];
    for (int c = 0; c < 3; ++c) hru[c] = SC[(long long)(DY_HRU + c) * g.vs + o];
    const double hrT = SC[(long long)DY_HRT * g.vs + o];
    // strain of u_hat and gradient of T_hat (central differences of the
    // filtered fields at the neighbours, metrics of the point)
    const int step[3] = {1, g.pitch, g.plane};
    double dl[3][4];
    for (int d = 0; d < 3; ++d) {
      const int op = o + step[d], om = o - step[d];
      const double irp = trcp(SC[(long long)DY_HR * g.vs + op]);
      const double irm = trcp(SC[(long long)DY_HR * g.vs + om]);
      for (int c = 0; c < 3; ++c)
        dl[d][c] = 0.5 * (SC[(long long)(DY_HRU + c) * g.vs + op] * irp -
                          SC[(long long)(DY_HRU + c) * g.vs + om] * irm);
      dl[d][3] = 0.5 * (SC[(long long)DY_HRT * g.vs + op] * irp - SC[(long long)DY_HRT * g.vs + om] * irm);
    }
    const double V = (double)M[9LL * g.vs + o];
    const double iV = trcp(V);
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
    const double cV = cbrt(fabs(V));
    const double D2 = cV * cV;                       // Delta^2 = |J^-1|^(2/3)
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
  const int P = (g.nx * g.nr + DY_BS - 1) / DY_BS;
  return DY_NXCD * ((P + DY_NXCD - 1) / DY_NXCD) * g.nth;
}

template <typename T>
hipError_t launch_dynamic(const T* Q, const T* M, const Grid& g, double gamma, double Cv,
                          double Pr_static, double* SC, double* part, double* dyn,
                          hipStream_t s) {
  const int tiles_x = (g.nx + 3 + DP_X - 1) / DP_X, tiles_y = (g.nr + 2 + DP_Y - 1) / DP_Y;
  hipLaunchKernelGGL(k_dyn_plane<T>, dim3(tiles_x * tiles_y, g.nth + 2 * NG), dim3(DP_X * DP_Y), 0, s,
                     Q, M, g, gamma, tiles_x, SC);
  const long long nrow = (long long)(g.nr + 2) * (g.nth + 2) * g.pitch;
  hipLaunchKernelGGL(k_dyn_hat, dim3(blocks_for(nrow, DY_BS)), dim3(DY_BS), 0, s, g, SC);
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
