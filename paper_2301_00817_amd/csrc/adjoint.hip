// Adjoint of the residual: Qbar = (dR/dQ)^T Rbar, where R is the residual of
// section "Spatial Discretization" evaluated after the ghost fill of section
// "Boundary Conditions", so the derivative includes the boundary maps (with
// the boundary data held fixed; the entrance-data cotangent is returned
// separately).  FP64, gather form: every output is accumulated by one
// thread, with no floating-point atomics, so results are deterministic.
//
// Passes (28 scratch variables in the padded layout):
//   1. pressure of every padded point; 1 / J^-1, lambda_bar^d and nu^d of
//      every point of [-1, n]^3 (zero at the other padded points);
//   2. per padded point: cotangents of its G^d, lambda_bar^d, nu^d and W
//      from the (up to) four faces per direction whose stencil contains it,
//      then (points of [-1, n]^3) the reverse of the point function; the
//      part of the state cotangent that depends on the point alone is
//      finished here, the cotangents of its central differences and sensor
//      neighbour pressures are stored.  The xi and eta lines of a 32 x 8
//      tile are staged in LDS, the zeta line of each point is held in
//      registers;
//   3. per padded point: the neighbours' contributions through its
//      primitives are added -> cotangent of the padded state;
//   4. transposes of the ghost fill in reverse order (zeta, eta, xi): ghost
//      cotangents go to the points they were computed from, through the
//      exact Jacobians of the boundary states (dual numbers);
//   5. centerline through the nodes (axis_node): the transpose of the
//      azimuthal mean that sets the axis row from row 1.
// With axis_node the axis row has R = 0 and J^-1 = 0: its Rbar is ignored,
// its eta point flux is the constant 0 and its point function is not
// reversed (only its pressure sensors, which the axis face uses); the axis
// face takes lambda_bar of row 1 and the fourth difference W2 - 4 W1 + 3 W0.
#include "bc.hpp"
#include "launch.hpp"
#include "physics_vjp.hpp"

namespace lesjet {

namespace {

__device__ __forceinline__ bool in_r1(const Grid& g, int i, int j, int k) {
  return i >= -1 && i <= g.nx && j >= -1 && j <= g.nr && k >= -1 && k <= g.nth;
}
__device__ __forceinline__ bool interior(const Grid& g, int i, int j, int k) {
  return i >= 0 && i < g.nx && j >= 0 && j < g.nr && k >= 0 && k < g.nth;
}

__device__ __forceinline__ void load5d(const double* A, const Grid& g, int o, double q[5]) {
#pragma unroll
  for (int c = 0; c < 5; ++c) q[c] = A[(long long)c * g.vs + o];
}

__device__ __forceinline__ double pressure(const double q[5], const Phys<double>& ph) {
  const double ir = trcp(q[0]);
  const double u = q[1] * ir, v = q[2] * ir, w = q[3] * ir;
  return ph.gm1 * (q[4] - 0.5 * q[0] * (u * u + v * v + w * w));
}

}  // namespace

// scratch layout (variables of the padded layout)
enum {
  S_LB = 0,    // lambda_bar^d, points of [-1, n]^3
  S_NU = 3,    // nu^d, points of [-1, n]^3
  S_IV = 6,    // 1 / J^-1, points of [-1, n]^3
  S_P = 7,     // pressure of every padded point
  S_PQ = 8,    // state cotangent of the point's own terms
  S_DL = 13,   // cotangents of the central differences (d, u v w T), [-1, n]^3
  S_NC = 25,   // cotangent of each sensor neighbour pressure (d), [-1, n]^3
  S_N = 28
};
static_assert(S_N == VJP_SCRATCH_VARS, "scratch size");

// Points of a padded plane by plane and XCD: workgroups are dealt to the
// eight XCDs (each with its own L2) in turn; the block id is remapped so
// that each XCD takes one eighth of every plane's blocks (256 points, or
// one tile, each) and walks the planes in order, so the k-neighbour planes
// a block reads were brought into the same L2 shortly before (with a plain
// linear order a block's k-neighbours were fetched by blocks on other XCDs).
constexpr int ADJ_NXCD = 8;
struct PlaneMap {
  int P;      // blocks per plane
  int Pmax;   // of them per XCD
};

static PlaneMap plane_map(int blocks_per_plane) {
  PlaneMap pm;
  pm.P = blocks_per_plane;
  pm.Pmax = (pm.P + ADJ_NXCD - 1) / ADJ_NXCD;
  return pm;
}

static unsigned plane_map_grid(const PlaneMap& pm, const Grid& g) {
  return (unsigned)(ADJ_NXCD * pm.Pmax * (g.nth + 2 * NG));
}

// Plane index (0 .. nth + 3) and block within the plane, or false for the
// blocks that fill up the last XCD's share.
__device__ __forceinline__ bool plane_block(const Grid& g, PlaneMap pm, int& kk, int& p) {
  const int hw = blockIdx.x, x = hw % ADJ_NXCD, r = hw / ADJ_NXCD;
  kk = r / pm.Pmax;
  p = x * pm.Pmax + r % pm.Pmax;
  return kk < g.nth + 2 * NG && p < pm.P;
}

// Pass 1, one thread per padded point: its pressure; for points of
// [-1, n]^3 also 1 / J^-1, lambda_bar^d and nu^d (the face dissipation
// coefficients, as in the point function), zero at the others.  One block
// per 32 x 8 tile of a padded plane (tile columns from padded index 0, so
// that stores fill lines); the pressures of the tile and a one-point ring
// are formed once into LDS for the sensors' xi and eta neighbours.
constexpr int PT_X = 32, PT_Y = 8, PT_HX = PT_X + 2, PT_HP = PT_HX * (PT_Y + 2);

__global__ __launch_bounds__(PT_X * PT_Y) void k_adj_prep(const double* __restrict__ Q,
                                                          const double* __restrict__ M, Grid g,
                                                          Phys<double> ph, PlaneMap pm,
                                                          int tiles_x, double* __restrict__ SC) {
  __shared__ double sp[PT_HP];
  int kk, pb;
  if (!plane_block(g, pm, kk, pb)) return;   // uniform over the block
  const int i0 = (pb % tiles_x) * PT_X - NG, j0 = (pb / tiles_x) * PT_Y - NG, k = kk - NG;
  const int tx = threadIdx.x % PT_X, ty = threadIdx.x / PT_X;
  const int i = i0 + tx, j = j0 + ty;
  const bool live = i < g.nx + NG && j < g.nr + NG;
  const bool r1 = live && in_r1(g, i, j, k);
  const int o = live ? g.at(i, j, k) : 0;
  // the point's own loads go out with the staging loads (one round trip
  // instead of two)
  double q[5], qm[5], qp[5];
  if (live) load5d(Q, g, o, q);
  if (r1) {
    load5d(Q, g, o - g.plane, qm);
    load5d(Q, g, o + g.plane, qp);
  }
  for (int e = threadIdx.x; e < PT_HP; e += PT_X * PT_Y) {
    // clamped to the padded box: a clamped slot feeds no stored value
    const int ie = min(max(i0 - 1 + e % PT_HX, -NG), g.nx + NG - 1);
    const int je = min(max(j0 - 1 + e / PT_HX, -NG), g.nr + NG - 1);
    double qe[5];
    load5d(Q, g, g.at(ie, je, k), qe);
    sp[e] = pressure(qe, ph);
  }
  __syncthreads();
  if (!live) return;
  const int slot = (ty + 1) * PT_HX + tx + 1;
  double pr[5];
  prim5(q, ph, pr);
  SC[(long long)S_P * g.vs + o] = pr[4];
  if (!r1) {
    // no face uses these; written so that no pass reads unset memory
    for (int d = 0; d < 3; ++d) {
      SC[(long long)(S_LB + d) * g.vs + o] = 0.0;
      SC[(long long)(S_NU + d) * g.vs + o] = 0.0;
    }
    SC[(long long)S_IV * g.vs + o] = 0.0;
    return;
  }
  // J^-1 = 0 on the axis row of a centerline-through-the-nodes mesh: no face
  // uses its lambda_bar and its Rbar is ignored, so 0 is stored there
  const bool axis_row = ph.axis_node && j == 0;
  const double iV = axis_row ? 0.0 : trcp(M[9LL * g.vs + o]);
  SC[(long long)S_IV * g.vs + o] = iV;
  const double a = tsqrt(pr[3]);
  const double aiV = fabs(iV);
  double lam[3];
  for (int d = 0; d < 3; ++d) {
    const double S0 = M[(long long)(3 * d) * g.vs + o], S1 = M[(long long)(3 * d + 1) * g.vs + o],
                 S2 = M[(long long)(3 * d + 2) * g.vs + o];
    const double Uc = S0 * pr[0] + S1 * pr[1] + S2 * pr[2];
    lam[d] = (fabs(Uc) + a * tsqrt(S0 * S0 + S1 * S1 + S2 * S2)) * aiV;
    double pl, pu;
    if (d < 2) {                       // in the plane: from LDS
      const int sd = d == 0 ? 1 : PT_HX;
      pl = sp[slot - sd];
      pu = sp[slot + sd];
    } else {
      pl = pressure(qm, ph);
      pu = pressure(qp, ph);
    }
    const double num = pu - 2.0 * pr[4] + pl, den = pu + 2.0 * pr[4] + pl;
    SC[(long long)(S_NU + d) * g.vs + o] = fabs(num) * trcp(den);
  }
  const double s01 = tsqrt(lam[0] * lam[1]), s02 = tsqrt(lam[0] * lam[2]),
               s12 = tsqrt(lam[1] * lam[2]);
  SC[(long long)(S_LB + 0) * g.vs + o] = lam[0] + s01 + s02;
  SC[(long long)(S_LB + 1) * g.vs + o] = lam[1] + s01 + s12;
  SC[(long long)(S_LB + 2) * g.vs + o] = lam[2] + s02 + s12;
}

// Coefficients of one face L | L+1 along d: the flux cotangent
// Fb = Rbar/J^-1 (L) - Rbar/J^-1 (L+1) (interior terms only) and, for a
// face with dissipation, lambda_f, eps2, eps4, V_f.
struct FaceCoef {
  double Fb[5];
  double lf, e2, e4, k4m, Vf;
  bool nu_left;   // the eps2 max takes the left sensor
  bool dis;       // the face carries dissipation
};

// Face L | L+1 from the line arrays (line points f and f+1).  Only the
// coefficients of existing faces (L in [-1, n-1]) are used by the caller.
__device__ __forceinline__ void line_face(const double rt[5][5], const double lbl[5],
                                          const double nul[5], const double vl[5], int f, int d,
                                          int L, int n, const Phys<double>& ph, FaceCoef& fc) {
  for (int c = 0; c < 5; ++c) fc.Fb[c] = rt[f][c] - rt[f + 1][c];   // rt is zero off the interior
  fc.dis = !((L == -1 && ph.phys_face[d][0]) || (L == n - 1 && ph.phys_face[d][1]));
  const double nuL = nul[f], nuR = nul[f + 1];
  // the axis face (centerline through the nodes) takes lambda_bar of row 1
  const bool axis = ph.axis_node && d == 1 && L == 0;
  fc.lf = axis ? lbl[f + 1] : 0.5 * (lbl[f] + lbl[f + 1]);
  fc.Vf = 0.5 * (vl[f] + vl[f + 1]);
  fc.nu_left = nuL >= nuR;
  fc.e2 = ph.k2 * fmax(nuL, nuR);
  fc.k4m = ph.k4 - fc.e2;
  fc.e4 = fmax(0.0, fc.k4m);
}

// Reverse of the dissipation of a face at one of its two inner points:
// adds the cotangent of that point's W (sign +1 for the right point, -1 for
// the left), of its lambda_bar and (when the eps2 max took its sensor) of
// its nu.  D = lf (e2 (W_R - W_L) - e4 (W_{R+1} - 3 W_R + 3 W_L - W_{L-1}))
// enters the flux as -V_f D.
__device__ __forceinline__ void face_self(const FaceCoef& f, const double* Wm, const double* WL,
                                          const double* WR, const double* Wp, double sign,
                                          bool takes_nu, const Phys<double>& ph, double wb[5],
                                          double& lbb, double& nub) {
  double lf_b = 0.0, e2_b = 0.0, e4_b = 0.0;
  for (int c = 0; c < 5; ++c) {
    const double Db = -f.Vf * f.Fb[c];
    const double A = WR[c] - WL[c];
    const double B = Wp[c] - 3.0 * WR[c] + 3.0 * WL[c] - Wm[c];
    lf_b += Db * (f.e2 * A - f.e4 * B);
    e2_b += Db * f.lf * A;
    e4_b -= Db * f.lf * B;
    wb[c] += sign * f.lf * (f.e2 + 3.0 * f.e4) * Db;
  }
  if (f.k4m > 0.0) e2_b -= e4_b;
  lbb += 0.5 * lf_b;
  if (takes_nu) nub += ph.k2 * e2_b;
}

// The same at an inner point of the axis face, where
// D = lf (e2 (W1 - W0) - e4 (W2 - 4 W1 + 3 W0)) and lf = lambda_bar(1):
// W1 (the right point) takes lf (e2 + 4 e4), W0 lf (-e2 - 3 e4), and the
// whole lf cotangent goes to the right point's lambda_bar.
__device__ __forceinline__ void face_self_axis(const FaceCoef& f, const double* W0, const double* W1,
                                               const double* W2, bool right, bool takes_nu,
                                               const Phys<double>& ph, double wb[5], double& lbb,
                                               double& nub) {
  double lf_b = 0.0, e2_b = 0.0, e4_b = 0.0;
  for (int c = 0; c < 5; ++c) {
    const double Db = -f.Vf * f.Fb[c];
    const double A = W1[c] - W0[c];
    const double B = W2[c] - 4.0 * W1[c] + 3.0 * W0[c];
    lf_b += Db * (f.e2 * A - f.e4 * B);
    e2_b += Db * f.lf * A;
    e4_b -= Db * f.lf * B;
    wb[c] += (right ? f.lf * (f.e2 + 4.0 * f.e4) : -f.lf * (f.e2 + 3.0 * f.e4)) * Db;
  }
  if (f.k4m > 0.0) e2_b -= e4_b;
  if (right) lbb += lf_b;
  if (takes_nu) nub += ph.k2 * e2_b;
}

// Line p-2 .. p+2 along zeta, its values loaded into registers by the
// caller: per point V, 1/J^-1, Rbar (5), lambda_bar^zeta, nu^zeta, and the
// state (5) and pressure.  Points outside the padded box, reached only when
// p is a ghost, are clamped to its edge (no existing face uses them).
// Rbar / J^-1 is zero off the interior (and on the axis row of a
// centerline-through-the-nodes mesh, where R = 0); W = (rho, rho u, rho v,
// rho w, E + p).
struct ZetaLine {
  const double (*zc)[9];
  const double (*zw)[6];
  bool row_inner;
  int s, n;
  __device__ __forceinline__ void coef(int m, double rt[5], double& lb, double& nu, double& v) const {
    const int k = min(max(s + m - 2, -NG), n - 1 + NG);
    const bool inner = row_inner && k >= 0 && k < n;
    v = zc[m][0];
    for (int q = 0; q < 5; ++q) rt[q] = inner ? zc[m][2 + q] * zc[m][1] : 0.0;
    lb = zc[m][7];
    nu = zc[m][8];
  }
  __device__ __forceinline__ void w(int m, double W[5]) const {
    for (int q = 0; q < 5; ++q) W[q] = zw[m][q];
    W[4] += zw[m][5];
  }
};

// Contributions of the four faces along d whose stencil holds p (line
// position s of n interior points): p's W (wb), its G^d (gbd), lambda_bar^d
// (lbb) and nu^d (nub).
template <class Line>
__device__ __forceinline__ void dir_part(const Line& ln, int s, int d, int n, const Phys<double>& ph,
                                         double wb[5], double gbd[5], double& lbb, double& nub) {
  // face L = s-2+f joins line points f and f+1
  double rt[5][5], lbl[5], nul[5], vl[5];
  for (int m = 0; m < 5; ++m) ln.coef(m, rt[m], lbl[m], nul[m], vl[m]);
  FaceCoef fo[2], fb, fc;
  // faces exist for L in [-1, n-1]
  const bool ha = s - 2 >= -1, hd = s + 1 <= n - 1;
  const bool hb = s - 1 >= -1 && s - 1 <= n - 1, hc = s >= -1 && s <= n - 1;
  line_face(rt, lbl, nul, vl, 0, d, s - 2, n, ph, fo[0]);
  line_face(rt, lbl, nul, vl, 3, d, s + 1, n, ph, fo[1]);
  line_face(rt, lbl, nul, vl, 1, d, s - 1, n, ph, fb);
  line_face(rt, lbl, nul, vl, 2, d, s, n, ph, fc);
  // axis face (centerline through the nodes): face L = 0 along eta
  const bool axd = ph.axis_node && d == 1;
  // faces L = s-2 and s+1: p is the outer point of their 4-point stencil
  // (the axis face has no point -1 in its stencil)
  if (ha && fo[0].dis)
    for (int c = 0; c < 5; ++c) wb[c] += fo[0].lf * fo[0].e4 * fo[0].Vf * fo[0].Fb[c];
  if (hd && fo[1].dis && !(axd && s + 1 == 0))
    for (int c = 0; c < 5; ++c) wb[c] -= fo[1].lf * fo[1].e4 * fo[1].Vf * fo[1].Fb[c];
  // faces L = s-1 (p is its right point) and L = s (p is its left point)
  for (int c = 0; c < 5; ++c) gbd[c] = 0.5 * ((hb ? fb.Fb[c] : 0.0) + (hc ? fc.Fb[c] : 0.0));
  const bool db = hb && fb.dis, dc = hc && fc.dis;
  if (db || dc) {
    double W[5][5];
    for (int m = 0; m < 5; ++m) ln.w(m, W[m]);
    if (db && axd && s - 1 == 0)
      face_self_axis(fb, W[1], W[2], W[3], true, !fb.nu_left, ph, wb, lbb, nub);
    else if (db)
      face_self(fb, W[0], W[1], W[2], W[3], 1.0, !fb.nu_left, ph, wb, lbb, nub);
    if (dc && axd && s == 0)
      face_self_axis(fc, W[2], W[3], W[4], false, fc.nu_left, ph, wb, lbb, nub);
    else if (dc)
      face_self(fc, W[1], W[2], W[3], W[4], -1.0, fc.nu_left, ph, wb, lbb, nub);
  }
}

// Second half of pass 2 at p, once the face contributions are summed: for
// p in [-1, n]^3 the reverse of the point function (skipped on the axis row
// of a centerline-through-the-nodes mesh, whose eta flux is the constant 0
// and whose other outputs are unused since J^-1 = 0 there), the sensor
// reverse and the writes of S_NC, S_DL; for every p the reverse of the
// primitives -> S_PQ.
template <class Prim>
__device__ __forceinline__ void point_part(const double* __restrict__ M, double* __restrict__ SC,
                                           const Grid& g, int o, bool r1,
                                           bool axis_row, const Phys<double>& ph, const Prim& pv,
                                           const double gb[3][5], double lbb[3], const double nub[3],
                                           const double wb[5]) {
  double q[5];
  pv.state(q);
  double qb[5], prb[5] = {0, 0, 0, 0, 0};
  for (int c = 0; c < 5; ++c) qb[c] = wb[c];
  prb[4] = wb[4];                                  // W5 = E + p
  if (r1) {
    PointIn<double> in;
    for (int c = 0; c < 5; ++c) {
      in.q[c] = q[c];
      in.pr[c] = pv.own(c);
    }
    double pm[3], pp[3];
    for (int d = 0; d < 3; ++d) {
      double m[5], pl[5];
      pv.nb(d, -1, m);
      pv.nb(d, 1, pl);
      for (int f = 0; f < 4; ++f) in.dl[d][f] = 0.5 * (pl[f] - m[f]);
      in.nu[d] = 0.0;                        // not used by the reverse
      pm[d] = m[4];
      pp[d] = pl[4];
      for (int c = 0; c < 3; ++c) in.S[d][c] = M[(long long)(3 * d + c) * g.vs + o];
    }
    in.V = pv.vol();
    PointBar<double> bar = {};
    if (!axis_row) point_quantities_vjp(in, ph, gb, lbb, bar);
    for (int d = 0; d < 3; ++d) {
      double side, centre;
      sensor_vjp(pm[d], in.pr[4], pp[d], nub[d], side, centre);
      bar.pr[4] += centre;
      SC[(long long)(S_NC + d) * g.vs + o] = side;
      for (int f = 0; f < 4; ++f) SC[(long long)(S_DL + 4 * d + f) * g.vs + o] = bar.dl[d][f];
    }
    for (int c = 0; c < 5; ++c) {
      qb[c] += bar.q[c];
      prb[c] += bar.pr[c];
    }
  }
  prim5_vjp(q, ph, prb, qb);
  for (int c = 0; c < 5; ++c) SC[(long long)(S_PQ + c) * g.vs + o] = qb[c];
}

// Pass 2, one thread per padded point p: the cotangents that the faces
// whose stencils contain p send to its point quantities (G^d, lambda_bar^d,
// nu^d) and to its W; then, for p in [-1, n]^3, the reverse of the point
// function.  Writes the state cotangent of everything that depends on p
// alone (S_PQ) and the cotangents of p's central differences and sensor
// neighbour pressures (S_DL, S_NC), which pass 3 hands to the neighbours.
//
// One block per 32 x 8 tile of a padded plane.  The block stages once, in
// LDS, what the xi and eta lines of its points read (the tile and two points
// on each side, clamped to the padded box): Rbar / J^-1, lambda_bar and nu
// along xi and eta, J^-1, the state and the primitives.  Each thread loads
// its zeta line from global memory into registers before the staging (the
// two sets of loads overlap); the metrics come from global memory.
constexpr int AT_X = 32, AT_Y = 8, AT_HX = AT_X + 4, AT_HY = AT_Y + 4, AT_HP = AT_HX * AT_HY;
enum { L_RT = 0, L_LB = 5, L_NU = 7, L_V = 9, L_Q = 10, L_PR = 15, L_N = 20 };

struct LdsLine {
  const double* sh;   // [L_N][AT_HP]
  int slot;           // slot of line point 0
  int stride;         // 1 along xi, AT_HX along eta
  int d;
  __device__ __forceinline__ void coef(int m, double rt[5], double& lb, double& nu, double& v) const {
    const int e = slot + m * stride;
    for (int c = 0; c < 5; ++c) rt[c] = sh[(L_RT + c) * AT_HP + e];
    lb = sh[(L_LB + d) * AT_HP + e];
    nu = sh[(L_NU + d) * AT_HP + e];
    v = sh[L_V * AT_HP + e];
  }
  __device__ __forceinline__ void w(int m, double W[5]) const {
    const int e = slot + m * stride;
    for (int c = 0; c < 5; ++c) W[c] = sh[(L_Q + c) * AT_HP + e];
    W[4] += sh[(L_PR + 4) * AT_HP + e];
  }
};

// State and primitives of p, primitives of its neighbours p -+ 1 along d
// (LDS in the plane, global state along zeta), J^-1 of p.
struct LdsPoint {
  const double* sh;
  const double* Q;
  const Phys<double>* ph;
  int slot, vs, o, plane;
  __device__ __forceinline__ void state(double q[5]) const {
    for (int c = 0; c < 5; ++c) q[c] = sh[(L_Q + c) * AT_HP + slot];
  }
  __device__ __forceinline__ double own(int c) const { return sh[(L_PR + c) * AT_HP + slot]; }
  __device__ __forceinline__ void nb(int d, int sg, double pr[5]) const {
    if (d < 2) {
      const int e = slot + sg * (d == 0 ? 1 : AT_HX);
      for (int c = 0; c < 5; ++c) pr[c] = sh[(L_PR + c) * AT_HP + e];
    } else {
      double qn[5];
      for (int c = 0; c < 5; ++c) qn[c] = Q[(long long)c * vs + o + sg * plane];
      prim5(qn, *ph, pr);
    }
  }
  __device__ __forceinline__ double vol() const { return sh[L_V * AT_HP + slot]; }
};

__global__ __launch_bounds__(256) void k_adj_main(const double* __restrict__ Q,
                                                  const double* __restrict__ M, Grid g,
                                                  Phys<double> ph, PlaneMap pm, int tiles_x,
                                                  const double* __restrict__ Rb,
                                                  double* __restrict__ SC) {
  __shared__ double sh[L_N * AT_HP];
  int kk, pb;
  if (!plane_block(g, pm, kk, pb)) return;   // uniform over the block
  const int i0 = (pb % tiles_x) * AT_X - NG, j0 = (pb / tiles_x) * AT_Y - NG, k = kk - NG;
  const int tx = threadIdx.x % AT_X, ty = threadIdx.x / AT_X;
  const int pos[3] = {i0 + tx, j0 + ty, k};
  const bool live = pos[0] < g.nx + NG && pos[1] < g.nr + NG;
  // zeta faces exist where (i, j) is interior
  const bool zeta = live && pos[0] >= 0 && pos[0] < g.nx && pos[1] >= 0 && pos[1] < g.nr;
  // the zeta line's values, loaded ahead of the staging so that both sets
  // of loads are in flight together (0.72 -> 0.655 ms per VJP on 2.05 M
  // points against loading them after the staging)
  double zc[5][9], zw[5][6];
  if (zeta) {
    const int o = g.at(pos[0], pos[1], pos[2]);
    for (int m = 0; m < 5; ++m) {
      const int om = o + (min(max(k + m - 2, -NG), g.nth - 1 + NG) - k) * g.plane;
      zc[m][0] = M[9LL * g.vs + om];
      zc[m][1] = SC[(long long)S_IV * g.vs + om];
      for (int c = 0; c < 5; ++c) zc[m][2 + c] = Rb[(long long)c * g.vs + om];
      zc[m][7] = SC[(long long)(S_LB + 2) * g.vs + om];
      zc[m][8] = SC[(long long)(S_NU + 2) * g.vs + om];
      for (int c = 0; c < 5; ++c) zw[m][c] = Q[(long long)c * g.vs + om];
      zw[m][5] = SC[(long long)S_P * g.vs + om];
    }
  }
  for (int e = threadIdx.x; e < AT_HP; e += 256) {
    const int i = min(max(i0 + e % AT_HX - 2, -NG), g.nx - 1 + NG);
    const int j = min(max(j0 + e / AT_HX - 2, -NG), g.nr - 1 + NG);
    const int oe = g.at(i, j, k);
    double q[5], pr[5];
    load5d(Q, g, oe, q);
    prim5(q, ph, pr);
    const double V = M[9LL * g.vs + oe], iV = SC[(long long)S_IV * g.vs + oe];
    // R has no entries off the interior nor on a centerline row
    const bool inner = interior(g, i, j, k) && !(ph.axis_node && j == 0);
    for (int c = 0; c < 5; ++c) {
      sh[(L_RT + c) * AT_HP + e] = inner ? Rb[(long long)c * g.vs + oe] * iV : 0.0;
      sh[(L_Q + c) * AT_HP + e] = q[c];
      sh[(L_PR + c) * AT_HP + e] = pr[c];
    }
    for (int d = 0; d < 2; ++d) {
      sh[(L_LB + d) * AT_HP + e] = SC[(long long)(S_LB + d) * g.vs + oe];
      sh[(L_NU + d) * AT_HP + e] = SC[(long long)(S_NU + d) * g.vs + oe];
    }
    sh[L_V * AT_HP + e] = V;
  }
  __syncthreads();
  if (!live) return;
  const int slot = (ty + 2) * AT_HX + tx + 2;
  const int nn[3] = {g.nx, g.nr, g.nth};
  const int o = g.at(pos[0], pos[1], pos[2]);
  const bool r1 = in_r1(g, pos[0], pos[1], pos[2]);
  double gb[3][5], lbb[3] = {0, 0, 0}, nub[3] = {0, 0, 0}, wb[5] = {0, 0, 0, 0, 0};
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 5; ++c) gb[d][c] = 0.0;
  if (zeta) {
    const ZetaLine ln = {zc, zw, !(ph.axis_node && pos[1] == 0), pos[2], g.nth};
    dir_part(ln, pos[2], 2, g.nth, ph, wb, gb[2], lbb[2], nub[2]);
  }
  for (int d = 0; d < 2; ++d) {
    // faces along d exist only where p is interior in the other directions
    const int d1 = d + 1, d2 = d == 0 ? 2 : d - 1;
    if (pos[d1] < 0 || pos[d1] >= nn[d1] || pos[d2] < 0 || pos[d2] >= nn[d2]) continue;
    const int stride = d == 0 ? 1 : AT_HX;
    const LdsLine ln = {sh, slot - 2 * stride, stride, d};
    dir_part(ln, pos[d], d, nn[d], ph, wb, gb[d], lbb[d], nub[d]);
  }
  const LdsPoint pv = {sh, Q, &ph, slot, g.vs, o, g.plane};
  point_part(M, SC, g, o, r1, ph.axis_node && pos[1] == 0, ph, pv, gb, lbb, nub, wb);
}

// Pass 3: cotangent of the padded state = own part + the neighbours'
// central-difference and sensor contributions through this point's
// primitives.  One thread per element of a variable, so the pitch padding
// beyond the padded box is written (zero) too.
__global__ __launch_bounds__(256) void k_adj_gather(const double* __restrict__ Q, Grid g,
                                                    Phys<double> ph,
                                                    PlaneMap pm, const double* __restrict__ SC,
                                                    double* __restrict__ Qb) {
  // 256-element blocks of a padded plane (pitch included) by plane and XCD
  int kk, p;
  if (!plane_block(g, pm, kk, p)) return;
  const int q = p * 256 + threadIdx.x;
  if (q >= g.plane) return;
  const int o = kk * g.plane + q;
  const int pos[3] = {o % g.pitch - NG, (o % g.plane) / g.pitch - NG, o / g.plane - NG};
  if (pos[0] >= g.nx + NG) {
    for (int c = 0; c < 5; ++c) Qb[(long long)c * g.vs + o] = 0.0;
    return;
  }
  const int step[3] = {1, g.pitch, g.plane};
  double prb[5] = {0, 0, 0, 0, 0};
  bool any = false;
  for (int d = 0; d < 3; ++d) {
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      int p2[3] = {pos[0], pos[1], pos[2]};
      p2[d] += sgn;
      if (!in_r1(g, p2[0], p2[1], p2[2])) continue;
      any = true;
      const int om = o + sgn * step[d];
      // this point is the +1 neighbour of om when sgn = -1, the -1 when sgn = +1
      const double h = sgn < 0 ? 0.5 : -0.5;
      for (int f = 0; f < 4; ++f) prb[f] += h * SC[(long long)(S_DL + 4 * d + f) * g.vs + om];
      prb[4] += SC[(long long)(S_NC + d) * g.vs + om];
    }
  }
  double qb[5];
  for (int c = 0; c < 5; ++c) qb[c] = SC[(long long)(S_PQ + c) * g.vs + o];
  if (any) {
    double q[5];
    load5d(Q, g, o, q);
    prim5_vjp(q, ph, prb, qb);
  }
  for (int c = 0; c < 5; ++c) Qb[(long long)c * g.vs + o] = qb[c];
}

// ---- ghost-fill transposes ---------------------------------------------------
// Qb(src) += Qb(ghost), Qb(ghost) = 0 for the NG ghosts of one side, all five
// variables, every load issued before any store (the NG sources and NG
// ghosts must be 2 NG distinct points).
__device__ __forceinline__ void addT_side(double* Qb, const Grid& g, const int osrc[NG],
                                          const int oghost[NG]) {
  double vs[5][NG], vg[5][NG];
  for (int c = 0; c < 5; ++c)
    for (int m = 0; m < NG; ++m) {
      vs[c][m] = Qb[(long long)c * g.vs + osrc[m]];
      vg[c][m] = Qb[(long long)c * g.vs + oghost[m]];
    }
  for (int c = 0; c < 5; ++c)
    for (int m = 0; m < NG; ++m) {
      Qb[(long long)c * g.vs + osrc[m]] = vs[c][m] + vg[c][m];
      Qb[(long long)c * g.vs + oghost[m]] = 0.0;
    }
}

// One thread per padded (i, j) column and variable.  With nth >= 5 the 2 NG
// ghost planes and the 2 NG interior planes they were copied from are all
// distinct, so the thread issues its loads before its stores.
__global__ __launch_bounds__(256) void k_adjT_zeta(double* __restrict__ Qb, Grid g) {
  const int NX = g.nx + 2 * NG, NR = g.nr + 2 * NG;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 5 * NX * NR) return;
  const int c = t / (NX * NR), r = t - c * (NX * NR);
  const int i = r % NX - NG, j = r / NX - NG;
  double* F = Qb + (long long)c * g.vs;
  int og[2 * NG], os[2 * NG];
  for (int m = 1; m <= NG; ++m) {
    og[m - 1] = g.at(i, j, -m);
    os[m - 1] = g.at(i, j, g.nth - m);
    og[NG + m - 1] = g.at(i, j, g.nth - 1 + m);
    os[NG + m - 1] = g.at(i, j, m - 1);
  }
  double vg[2 * NG], vs[2 * NG];
  for (int m = 0; m < 2 * NG; ++m) { vg[m] = F[og[m]]; vs[m] = F[os[m]]; }
  for (int m = 0; m < 2 * NG; ++m) { F[os[m]] = vs[m] + vg[m]; F[og[m]] = 0.0; }
}

// sum of the two ghost cotangents of a face, pulled back through the exact
// Jacobian (dual numbers) of the face state with respect to the interior
// state qe (and, for the entrance, the target primitives).
__global__ __launch_bounds__(256) void k_adjT_eta(const double* __restrict__ Q, const double* __restrict__ M,
                           double* __restrict__ Qb, Grid g, double gamma, int lo_kind,
                           int hi_kind, BPrim<double> ref) {
  // one thread per (i, k) and face; with nr >= 5 the two faces touch
  // disjoint ghosts and disjoint interior points
  const int NX = g.nx + 2 * NG;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nf = NX * g.nth;
  if (t >= 2 * nf) return;
  const bool lo = t < nf;
  const int ik = lo ? t : t - nf;
  const int i = ik % NX - NG, k = ik / NX;
  if (!lo) { lo_kind = -1; } else { hi_kind = -1; }
  int os[NG], og[NG];
  if (lo_kind == BC_PERIODIC) {
    for (int m = 1; m <= NG; ++m) { os[m - 1] = g.at(i, g.nr - m, k); og[m - 1] = g.at(i, -m, k); }
    addT_side(Qb, g, os, og);
  } else if (lo_kind == BC_AXIS) {
    // gather form: the ghost (i, -m, k + nth/2) was copied from (i, m - 1, k)
    // (nth is even, so the map is an involution of k)
    const int kk = (k + g.nth / 2) % g.nth;
    for (int m = 1; m <= NG; ++m) { os[m - 1] = g.at(i, m - 1, k); og[m - 1] = g.at(i, -m, kk); }
    addT_side(Qb, g, os, og);
  } else if (lo_kind == BC_AXIS_NODE) {
    // mirror through the axis node: the ghost (i, -m, k + nth/2) was copied
    // from (i, m, k)
    const int kk = (k + g.nth / 2) % g.nth;
    for (int m = 1; m <= NG; ++m) { os[m - 1] = g.at(i, m, k); og[m - 1] = g.at(i, -m, kk); }
    addT_side(Qb, g, os, og);
  }
  if (hi_kind == BC_PERIODIC) {
    for (int m = 1; m <= NG; ++m) { os[m - 1] = g.at(i, m - 1, k); og[m - 1] = g.at(i, g.nr - 1 + m, k); }
    addT_side(Qb, g, os, og);
  } else if (hi_kind == BC_FARFIELD) {
    const int oe = g.at(i, g.nr - 1, k);
    double fb[5] = {0, 0, 0, 0, 0};
    for (int m = 1; m <= NG; ++m) {
      const int og = g.at(i, g.nr - 1 + m, k);
      for (int c = 0; c < 5; ++c) {
        fb[c] += Qb[(long long)c * g.vs + og];
        Qb[(long long)c * g.vs + og] = 0.0;
      }
    }
    double n[3];
    {
      const double a = M[3LL * g.vs + oe], b = M[4LL * g.vs + oe], c = M[5LL * g.vs + oe];
      const double inv = 1.0 / sqrt(a * a + b * b + c * c);
      n[0] = a * inv; n[1] = b * inv; n[2] = c * inv;
    }
    Dual<5> qd[5], fd[5];
    for (int c = 0; c < 5; ++c) { qd[c] = Dual<5>(Q[(long long)c * g.vs + oe]); qd[c].d[c] = 1.0; }
    BPrim<Dual<5>> rd = {Dual<5>(ref.rho), Dual<5>(ref.u), Dual<5>(ref.v), Dual<5>(ref.w),
                         Dual<5>(ref.p)};
    bc_farfield(qd, rd, n, gamma, fd);
    for (int jv = 0; jv < 5; ++jv) {
      double acc = 0.0;
      for (int c = 0; c < 5; ++c) acc += fb[c] * fd[c].d[jv];
      Qb[(long long)jv * g.vs + oe] += acc;
    }
  }
}

__global__ __launch_bounds__(64) void k_adjT_xi(const double* __restrict__ Q, const double* __restrict__ M,
                          double* __restrict__ Qb, Grid g, const double* __restrict__ inflow,
                          double* __restrict__ inflow_bar, double gamma, int lo_kind, int hi_kind,
                          double p_exit, int axis_node) {
  // one thread per (j, k) and face: the faces touch disjoint ghosts and
  // disjoint interior points
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nf = g.nr * g.nth;
  if (t >= 2 * nf) return;
  const bool lo = t < nf;
  const int jk = lo ? t : t - nf;
  const int j = jk % g.nr, k = jk / g.nr;
  if (!lo) { lo_kind = -1; } else { hi_kind = -1; }
  auto take = [&](int oe, int side, double fb[5]) {
    for (int c = 0; c < 5; ++c) fb[c] = 0.0;
    for (int m = 1; m <= NG; ++m) {
      const int og = side < 0 ? g.at(-m, j, k) : g.at(g.nx - 1 + m, j, k);
      for (int c = 0; c < 5; ++c) {
        fb[c] += Qb[(long long)c * g.vs + og];
        Qb[(long long)c * g.vs + og] = 0.0;
      }
    }
  };
  // boundary normals; on the axis row those of row 1 (S^xi vanishes there)
  const int jn = axis_node && j == 0 ? 1 : j;
  auto normal = [&](int oe, double sgn, double n[3]) {
    oe += (jn - j) * g.pitch;
    const double a = M[0LL * g.vs + oe], b = M[1LL * g.vs + oe], c = M[2LL * g.vs + oe];
    const double inv = sgn / sqrt(a * a + b * b + c * c);
    n[0] = a * inv; n[1] = b * inv; n[2] = c * inv;
  };
  if (lo_kind == BC_PERIODIC) {
    int os[NG], og[NG];
    for (int m = 1; m <= NG; ++m) { os[m - 1] = g.at(g.nx - m, j, k); og[m - 1] = g.at(-m, j, k); }
    addT_side(Qb, g, os, og);
  } else if (lo_kind == BC_INFLOW) {
    const int oe = g.at(0, j, k);
    double fb[5], n[3];
    take(oe, -1, fb);
    normal(oe, -1.0, n);
    const long long sp = (long long)g.nth * g.nr, it = (long long)k * g.nr + j;
    Dual<10> qd[5], fd[5];
    for (int c = 0; c < 5; ++c) { qd[c] = Dual<10>(Q[(long long)c * g.vs + oe]); qd[c].d[c] = 1.0; }
    BPrim<Dual<10>> tg;
    Dual<10>* tp[5] = {&tg.rho, &tg.u, &tg.v, &tg.w, &tg.p};
    for (int c = 0; c < 5; ++c) { *tp[c] = Dual<10>(inflow[c * sp + it]); tp[c]->d[5 + c] = 1.0; }
    bc_inflow(qd, tg, n, gamma, fd);
    for (int jv = 0; jv < 10; ++jv) {
      double acc = 0.0;
      for (int c = 0; c < 5; ++c) acc += fb[c] * fd[c].d[jv];
      if (jv < 5) Qb[(long long)jv * g.vs + oe] += acc;
      else if (inflow_bar) inflow_bar[(jv - 5) * sp + it] += acc;
    }
  }
  if (hi_kind == BC_PERIODIC) {
    int os[NG], og[NG];
    for (int m = 1; m <= NG; ++m) { os[m - 1] = g.at(m - 1, j, k); og[m - 1] = g.at(g.nx - 1 + m, j, k); }
    addT_side(Qb, g, os, og);
  } else if (hi_kind == BC_OUTFLOW) {
    const int oe = g.at(g.nx - 1, j, k);
    double fb[5], n[3];
    take(oe, 1, fb);
    normal(oe, 1.0, n);
    Dual<5> qd[5], fd[5];
    for (int c = 0; c < 5; ++c) { qd[c] = Dual<5>(Q[(long long)c * g.vs + oe]); qd[c].d[c] = 1.0; }
    bc_outflow(qd, n, gamma, p_exit, fd);
    for (int jv = 0; jv < 5; ++jv) {
      double acc = 0.0;
      for (int c = 0; c < 5; ++c) acc += fb[c] * fd[c].d[jv];
      Qb[(long long)jv * g.vs + oe] += acc;
    }
  }
}

// Transpose of the axis-row mean: Q(i, 0, k) = mean over k' of Q(i, 1, k'),
// so the axis row's cotangent, summed over k, is spread evenly over row 1
// and the axis row's own cotangent is zero.  One block per i, fixed-order
// FP64 tree over k.
constexpr int CLT_BS = 256;
__global__ __launch_bounds__(CLT_BS) void k_adjT_centerline(double* __restrict__ Qb, Grid g) {
  __shared__ double red[5][CLT_BS];
  const int i = blockIdx.x;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int k = threadIdx.x; k < g.nth; k += CLT_BS) {
    const int o = g.at(i, 0, k);
    for (int c = 0; c < 5; ++c) acc[c] += Qb[(long long)c * g.vs + o];
  }
  for (int c = 0; c < 5; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = CLT_BS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 5; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  for (int k = threadIdx.x; k < g.nth; k += CLT_BS) {
    const int o0 = g.at(i, 0, k), o1 = g.at(i, 1, k);
    for (int c = 0; c < 5; ++c) {
      Qb[(long long)c * g.vs + o1] += red[c][0] / g.nth;
      Qb[(long long)c * g.vs + o0] = 0.0;
    }
  }
}

hipError_t launch_centerline_transpose(double* Qb, const Grid& g, hipStream_t s) {
  hipLaunchKernelGGL(k_adjT_centerline, dim3(g.nx), dim3(CLT_BS), 0, s, Qb, g);
  return hipGetLastError();
}

// Element-wise kernels of the RK5-step adjoint.  x and y may be the same
// array (the step adjoint scales a cotangent in place, and Qbar_n may alias
// Qbar_np1): each thread reads its element before writing it and touches no
// other, so the pointers carry no __restrict__.
__global__ void k_scale(const double* x, double a, double* y, long long n) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t < n) y[t] = a * x[t];
}

__global__ void k_accumulate(const double* __restrict__ x, double* __restrict__ y, long long n) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t < n) y[t] += x[t];
}

// y = x on the interior, 0 on ghosts and pitch padding (5 variables); x and
// y may alias (see above).
__global__ void k_interior_copy(const double* x, double* y, Grid g) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= 5LL * g.vs) return;
  const int o = (int)(t % g.vs);
  const int i = o % g.pitch - NG, j = (o % g.plane) / g.pitch - NG, k = o / g.plane - NG;
  y[t] = interior(g, i, j, k) ? x[t] : 0.0;
}

hipError_t launch_interior_copy(const double* x, double* y, const Grid& g, hipStream_t s) {
  hipLaunchKernelGGL(k_interior_copy, dim3(blocks_for(5LL * g.vs, 256)), dim3(256), 0, s, x, y, g);
  return hipGetLastError();
}

hipError_t launch_scale(const double* x, double a, double* y, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, a, y, n);
  return hipGetLastError();
}

hipError_t launch_accumulate(const double* x, double* y, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_accumulate, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t launch_residual_vjp(const double* Q, const double* M, const Grid& g,
                               const Phys<double>& ph, const int bc[6], const double ref_prim[5],
                               double p_exit, const double* inflow, const double* Rb, double* SC,
                               double* Qb, double* inflow_bar, hipStream_t s) {
  const int ptiles_x = (g.nx + 2 * NG + PT_X - 1) / PT_X;
  const PlaneMap ppm = plane_map(ptiles_x * ((g.nr + 2 * NG + PT_Y - 1) / PT_Y));
  hipLaunchKernelGGL(k_adj_prep, dim3(plane_map_grid(ppm, g)), dim3(PT_X * PT_Y), 0, s, Q, M, g, ph,
                     ppm, ptiles_x, SC);
  const int tiles_x = (g.nx + 2 * NG + AT_X - 1) / AT_X;
  const PlaneMap tpm = plane_map(tiles_x * ((g.nr + 2 * NG + AT_Y - 1) / AT_Y));
  hipLaunchKernelGGL(k_adj_main, dim3(plane_map_grid(tpm, g)), dim3(256), 0, s, Q, M, g, ph, tpm,
                     tiles_x, Rb, SC);
  const PlaneMap gpm = plane_map((g.plane + 255) / 256);
  hipLaunchKernelGGL(k_adj_gather, dim3(plane_map_grid(gpm, g)), dim3(256), 0, s, Q, g, ph, gpm, SC,
                     Qb);
  const double gamma = ph.gamma;
  hipLaunchKernelGGL(k_adjT_zeta, dim3(blocks_for(5LL * (g.nx + 2 * NG) * (g.nr + 2 * NG), 256)),
                     dim3(256), 0, s, Qb, g);
  BPrim<double> ref = {ref_prim[0], ref_prim[1], ref_prim[2], ref_prim[3], ref_prim[4]};
  hipLaunchKernelGGL(k_adjT_eta, dim3(blocks_for(2LL * (g.nx + 2 * NG) * g.nth, 256)), dim3(256),
                     0, s, Q, M, Qb, g, gamma, bc[2], bc[3], ref);
  hipLaunchKernelGGL(k_adjT_xi, dim3(blocks_for(2LL * g.nr * g.nth, 64)), dim3(64), 0, s, Q, M, Qb,
                     g, inflow, inflow_bar, gamma, bc[0], bc[1], p_exit, ph.axis_node);
  if (bc[2] == BC_AXIS_NODE)
    hipLaunchKernelGGL(k_adjT_centerline, dim3(g.nx), dim3(CLT_BS), 0, s, Qb, g);
  return hipGetLastError();
}

}  // namespace lesjet
