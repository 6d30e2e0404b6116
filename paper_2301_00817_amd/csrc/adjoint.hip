// Adjoint of the residual: Qbar = (dR/dQ)^T Rbar, where R is the residual of
// section "Spatial Discretization" evaluated after the ghost fill of section
// "Boundary Conditions", so the derivative includes the boundary maps (with
// the boundary data held fixed; the entrance-data cotangent is returned
// separately).  FP64, gather form: every output is accumulated by one
// thread, with no floating-point atomics, so results are deterministic.
//
// Passes (scratch arrays in the padded layout):
//   1. point quantities G^d, lambda_bar^d, nu^d of every point of [-1, n]^3
//      (the two-pass reference point kernel);
//   2. per point: cotangents of its point quantities and of its W from the
//      (up to) four faces per direction whose stencil contains it;
//   3. per point of [-1, n]^3: reverse of the point function -> cotangents
//      of the state, of (u, v, w, T, p), of the central differences and of
//      the neighbours' pressures;
//   4. per padded point: gather the neighbours' contributions, reverse the
//      primitive map -> cotangent of the padded state;
//   5. transposes of the ghost fill in reverse order (zeta, eta, xi): ghost
//      cotangents go to the points they were computed from, through the
//      exact Jacobians of the boundary states (dual numbers).
#include "bc.hpp"
#include "launch.hpp"
#include "physics.hpp"

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
  const double ir = 1.0 / q[0];
  const double u = q[1] * ir, v = q[2] * ir, w = q[3] * ir;
  return ph.gm1 * (q[4] - 0.5 * q[0] * (u * u + v * v + w * w));
}

__device__ __forceinline__ void wvec_at(const double* Q, const Grid& g, int o,
                                        const Phys<double>& ph, double W[5]) {
  load5d(Q, g, o, W);
  W[4] += pressure(W, ph);
}

}  // namespace

// scratch layout (variables of the padded layout)
enum { A2_GB = 0, A2_LBB = 15, A2_NUB = 18, A2_WB = 21, A2_N = 26 };
enum { A3_QD = 0, A3_PRB = 5, A3_DLB = 10, A3_NC = 22, A3_N = 25 };
static_assert(21 + A2_N + A3_N == VJP_SCRATCH_VARS, "scratch size");

// Pass 2: face adjoints gathered at each padded point.
__global__ __launch_bounds__(256) void k_adj_face(const double* __restrict__ Q, const double* __restrict__ M, Grid g,
                           Phys<double> ph, const double* __restrict__ PT,
                           const double* __restrict__ Rb, double* __restrict__ A2) {
  const int NX = g.nx + 2 * NG, NR = g.nr + 2 * NG, NT = g.nth + 2 * NG;
  const long long tot = (long long)NX * NR * NT;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= tot) return;
  const int pos[3] = {(int)(t % NX) - NG, (int)((t / NX) % NR) - NG,
                      (int)(t / ((long long)NX * NR)) - NG};
  const int nn[3] = {g.nx, g.nr, g.nth};
  const int step[3] = {1, g.pitch, g.plane};
  const int o = g.at(pos[0], pos[1], pos[2]);
  double gb[3][5] = {}, lbb[3] = {}, nub[3] = {}, wb[5] = {};
  for (int d = 0; d < 3; ++d) {
    const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    if (pos[d1] < 0 || pos[d1] >= nn[d1] || pos[d2] < 0 || pos[d2] >= nn[d2]) continue;
    const int s = pos[d];
    for (int L = s - 2; L <= s + 1; ++L) {
      if (L < -1 || L > nn[d] - 1) continue;
      const int oL = o + (L - s) * step[d];
      const int oR = oL + step[d];
      double Fb[5];
      for (int c = 0; c < 5; ++c) {
        const double a = L >= 0 ? Rb[(long long)c * g.vs + oL] / M[9LL * g.vs + oL] : 0.0;
        const double b = L + 1 <= nn[d] - 1 ? Rb[(long long)c * g.vs + oR] / M[9LL * g.vs + oR] : 0.0;
        Fb[c] = a - b;
      }
      const int role = s - L;   // -1: L-1, 0: L, 1: R, 2: R+1
      if (role == 0 || role == 1)
        for (int c = 0; c < 5; ++c) gb[d][c] += 0.5 * Fb[c];
      const bool physical = (L == -1 && ph.phys_face[d][0]) || (L == nn[d] - 1 && ph.phys_face[d][1]);
      if (physical) continue;
      double Wm[5], WL[5], WR[5], Wp[5];
      wvec_at(Q, g, oL - step[d], ph, Wm);
      wvec_at(Q, g, oL, ph, WL);
      wvec_at(Q, g, oR, ph, WR);
      wvec_at(Q, g, oR + step[d], ph, Wp);
      double GbL[5] = {}, GbR[5] = {}, Wbm[5] = {}, WbL[5] = {}, WbR[5] = {}, Wbp[5] = {};
      double lbbL = 0, lbbR = 0, nubL = 0, nubR = 0;
      face_flux_vjp(PT[(long long)(15 + d) * g.vs + oL], PT[(long long)(15 + d) * g.vs + oR],
                    PT[(long long)(18 + d) * g.vs + oL], PT[(long long)(18 + d) * g.vs + oR],
                    M[9LL * g.vs + oL], M[9LL * g.vs + oR], Wm, WL, WR, Wp, false, ph, Fb, GbL,
                    GbR, lbbL, lbbR, nubL, nubR, Wbm, WbL, WbR, Wbp);
      const double* wsel = role == -1 ? Wbm : role == 0 ? WbL : role == 1 ? WbR : Wbp;
      for (int c = 0; c < 5; ++c) wb[c] += wsel[c];
      if (role == 0) { lbb[d] += lbbL; nub[d] += nubL; }
      if (role == 1) { lbb[d] += lbbR; nub[d] += nubR; }
    }
  }
  for (int d = 0; d < 3; ++d) {
    for (int c = 0; c < 5; ++c) A2[(long long)(A2_GB + 5 * d + c) * g.vs + o] = gb[d][c];
    A2[(long long)(A2_LBB + d) * g.vs + o] = lbb[d];
    A2[(long long)(A2_NUB + d) * g.vs + o] = nub[d];
  }
  for (int c = 0; c < 5; ++c) A2[(long long)(A2_WB + c) * g.vs + o] = wb[c];
}

// Pass 3: reverse of the point function at the points of [-1, n]^3.
__global__ __launch_bounds__(256) void k_adj_point(const double* __restrict__ Q, const double* __restrict__ M, Grid g,
                            Phys<double> ph, const double* __restrict__ A2,
                            double* __restrict__ A3) {
  const int NX1 = g.nx + 2, NR1 = g.nr + 2, NT1 = g.nth + 2;
  const long long tot = (long long)NX1 * NR1 * NT1;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= tot) return;
  const int i = (int)(t % NX1) - 1;
  const int j = (int)((t / NX1) % NR1) - 1;
  const int k = (int)(t / ((long long)NX1 * NR1)) - 1;
  const int o = g.at(i, j, k);
  const int step[3] = {1, g.pitch, g.plane};
  PointIn<double> in;
  load5d(Q, g, o, in.q);
  prim5(in.q, ph, in.pr);
  double pm[3], pp[3];
  for (int d = 0; d < 3; ++d) {
    double q[5], m[5], pl[5];
    load5d(Q, g, o - step[d], q);
    prim5(q, ph, m);
    load5d(Q, g, o + step[d], q);
    prim5(q, ph, pl);
    neighbour_terms(m, pl, in.pr[4], in.dl[d], in.nu[d]);
    pm[d] = m[4];
    pp[d] = pl[4];
    for (int c = 0; c < 3; ++c) in.S[d][c] = M[(long long)(3 * d + c) * g.vs + o];
  }
  in.V = M[9LL * g.vs + o];
  double Gb[3][5], lbb[3];
  for (int d = 0; d < 3; ++d) {
    for (int c = 0; c < 5; ++c) Gb[d][c] = A2[(long long)(A2_GB + 5 * d + c) * g.vs + o];
    lbb[d] = A2[(long long)(A2_LBB + d) * g.vs + o];
  }
  PointBar<double> bar = {};
  point_quantities_vjp(in, ph, Gb, lbb, bar);
  double nc[3];
  for (int d = 0; d < 3; ++d) {
    double side, centre;
    sensor_vjp(pm[d], in.pr[4], pp[d], A2[(long long)(A2_NUB + d) * g.vs + o], side, centre);
    bar.pr[4] += centre;
    nc[d] = side;
  }
  for (int c = 0; c < 5; ++c) {
    A3[(long long)(A3_QD + c) * g.vs + o] = bar.q[c];
    A3[(long long)(A3_PRB + c) * g.vs + o] = bar.pr[c];
  }
  for (int d = 0; d < 3; ++d) {
    for (int f = 0; f < 4; ++f) A3[(long long)(A3_DLB + 4 * d + f) * g.vs + o] = bar.dl[d][f];
    A3[(long long)(A3_NC + d) * g.vs + o] = nc[d];
  }
}

// Pass 4: cotangent of the padded state; one thread per element of a
// variable, so the pitch padding beyond the padded box is written (zero) too.
__global__ __launch_bounds__(256) void k_adj_gather(const double* __restrict__ Q, Grid g, Phys<double> ph,
                             const double* __restrict__ A2, const double* __restrict__ A3,
                             double* __restrict__ Qb) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= g.vs) return;
  const int pos[3] = {o % g.pitch - NG, (o % g.plane) / g.pitch - NG, o / g.plane - NG};
  if (pos[0] >= g.nx + NG) {
    for (int c = 0; c < 5; ++c) Qb[(long long)c * g.vs + o] = 0.0;
    return;
  }
  const int step[3] = {1, g.pitch, g.plane};
  double qb[5], prb[5] = {0, 0, 0, 0, 0};
  for (int c = 0; c < 5; ++c) qb[c] = A2[(long long)(A2_WB + c) * g.vs + o];
  prb[4] += qb[4];                               // W5 = E + p
  if (in_r1(g, pos[0], pos[1], pos[2]))
    for (int c = 0; c < 5; ++c) {
      qb[c] += A3[(long long)(A3_QD + c) * g.vs + o];
      prb[c] += A3[(long long)(A3_PRB + c) * g.vs + o];
    }
  for (int d = 0; d < 3; ++d) {
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      int p2[3] = {pos[0], pos[1], pos[2]};
      p2[d] += sgn;
      if (!in_r1(g, p2[0], p2[1], p2[2])) continue;
      const int om = o + sgn * step[d];
      // this point is the +1 neighbour of om when sgn = -1, the -1 when sgn = +1
      const double h = sgn < 0 ? 0.5 : -0.5;
      for (int f = 0; f < 4; ++f) prb[f] += h * A3[(long long)(A3_DLB + 4 * d + f) * g.vs + om];
      prb[4] += A3[(long long)(A3_NC + d) * g.vs + om];
    }
  }
  double q[5];
  load5d(Q, g, o, q);
  prim5_vjp(q, ph, prb, qb);
  for (int c = 0; c < 5; ++c) Qb[(long long)c * g.vs + o] = qb[c];
}

// ---- ghost-fill transposes ---------------------------------------------------
__device__ __forceinline__ void addT(double* Qb, const Grid& g, int osrc, int oghost) {
  for (int c = 0; c < 5; ++c) {
    Qb[(long long)c * g.vs + osrc] += Qb[(long long)c * g.vs + oghost];
    Qb[(long long)c * g.vs + oghost] = 0.0;
  }
}

__global__ void k_adjT_zeta(double* __restrict__ Qb, Grid g) {
  const int NX = g.nx + 2 * NG, NR = g.nr + 2 * NG;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NX * NR) return;
  const int i = t % NX - NG, j = t / NX - NG;
  for (int m = 1; m <= NG; ++m) {
    addT(Qb, g, g.at(i, j, g.nth - m), g.at(i, j, -m));
    addT(Qb, g, g.at(i, j, m - 1), g.at(i, j, g.nth - 1 + m));
  }
}

// sum of the two ghost cotangents of a face, pulled back through the exact
// Jacobian (dual numbers) of the face state with respect to the interior
// state qe (and, for the entrance, the target primitives).
__global__ __launch_bounds__(256) void k_adjT_eta(const double* __restrict__ Q, const double* __restrict__ M,
                           double* __restrict__ Qb, Grid g, double gamma, int lo_kind,
                           int hi_kind, BPrim<double> ref) {
  const int NX = g.nx + 2 * NG;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NX * g.nth) return;
  const int i = t % NX - NG, k = t / NX;
  if (lo_kind == BC_PERIODIC) {
    for (int m = 1; m <= NG; ++m) addT(Qb, g, g.at(i, g.nr - m, k), g.at(i, -m, k));
  } else if (lo_kind == BC_AXIS) {
    // gather form: the ghost (i, -m, k + nth/2) was copied from (i, m - 1, k)
    // (nth is even, so the map is an involution of k)
    const int kk = (k + g.nth / 2) % g.nth;
    for (int m = 1; m <= NG; ++m) addT(Qb, g, g.at(i, m - 1, k), g.at(i, -m, kk));
  }
  if (hi_kind == BC_PERIODIC) {
    for (int m = 1; m <= NG; ++m) addT(Qb, g, g.at(i, m - 1, k), g.at(i, g.nr - 1 + m, k));
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

__global__ __launch_bounds__(256) void k_adjT_xi(const double* __restrict__ Q, const double* __restrict__ M,
                          double* __restrict__ Qb, Grid g, const double* __restrict__ inflow,
                          double* __restrict__ inflow_bar, double gamma, int lo_kind, int hi_kind,
                          double p_exit) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.nr * g.nth) return;
  const int j = t % g.nr, k = t / g.nr;
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
  auto normal = [&](int oe, double sgn, double n[3]) {
    const double a = M[0LL * g.vs + oe], b = M[1LL * g.vs + oe], c = M[2LL * g.vs + oe];
    const double inv = sgn / sqrt(a * a + b * b + c * c);
    n[0] = a * inv; n[1] = b * inv; n[2] = c * inv;
  };
  if (lo_kind == BC_PERIODIC) {
    for (int m = 1; m <= NG; ++m) addT(Qb, g, g.at(g.nx - m, j, k), g.at(-m, j, k));
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
    for (int m = 1; m <= NG; ++m) addT(Qb, g, g.at(m - 1, j, k), g.at(g.nx - 1 + m, j, k));
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

__global__ void k_scale(const double* __restrict__ x, double a, double* __restrict__ y,
                        long long n) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t < n) y[t] = a * x[t];
}

__global__ void k_accumulate(const double* __restrict__ x, double* __restrict__ y, long long n) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t < n) y[t] += x[t];
}

// y = x on the interior, 0 on ghosts and pitch padding (5 variables).
__global__ void k_interior_copy(const double* __restrict__ x, double* __restrict__ y, Grid g) {
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
                               double p_exit, const double* inflow, const double* Rb, double* PT,
                               double* A2, double* A3, double* Qb, double* inflow_bar,
                               hipStream_t s) {
  hipError_t e = launch_residual_ref<double>(Q, M, g, ph, PT, nullptr, s);   // pass 1
  if (e != hipSuccess) return e;
  const long long npad = (long long)(g.nx + 2 * NG) * (g.nr + 2 * NG) * (g.nth + 2 * NG);
  const long long nr1 = (long long)(g.nx + 2) * (g.nr + 2) * (g.nth + 2);
  hipLaunchKernelGGL(k_adj_face, dim3(blocks_for(npad, 256)), dim3(256), 0, s, Q, M, g, ph, PT, Rb,
                     A2);
  hipLaunchKernelGGL(k_adj_point, dim3(blocks_for(nr1, 256)), dim3(256), 0, s, Q, M, g, ph, A2, A3);
  hipLaunchKernelGGL(k_adj_gather, dim3(blocks_for(g.vs, 256)), dim3(256), 0, s, Q, g, ph, A2, A3,
                     Qb);
  const double gamma = ph.gamma;
  hipLaunchKernelGGL(k_adjT_zeta, dim3(blocks_for((long long)(g.nx + 2 * NG) * (g.nr + 2 * NG), 256)),
                     dim3(256), 0, s, Qb, g);
  BPrim<double> ref = {ref_prim[0], ref_prim[1], ref_prim[2], ref_prim[3], ref_prim[4]};
  hipLaunchKernelGGL(k_adjT_eta, dim3(blocks_for((long long)(g.nx + 2 * NG) * g.nth, 256)), dim3(256),
                     0, s, Q, M, Qb, g, gamma, bc[2], bc[3], ref);
  hipLaunchKernelGGL(k_adjT_xi, dim3(blocks_for((long long)g.nr * g.nth, 256)), dim3(256), 0, s, Q,
                     M, Qb, g, inflow, inflow_bar, gamma, bc[0], bc[1], p_exit);
  return hipGetLastError();
}

}  // namespace lesjet
