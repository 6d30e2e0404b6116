// Host-side checks of the library's device functions (compiled for the CPU):
// each hand-written reverse-mode function against central finite differences
// of its forward function, and the dual-number boundary Jacobians against
// finite differences.  Test infrastructure; not part of the library.
#include <math.h>
#include <stdint.h>

#include <random>

#include "bc.hpp"
#include "physics_vjp.hpp"

using namespace lesjet;

namespace {

Phys<double> make_phys(int sgs) {
  Phys<double> ph;
  ph.gamma = 1.4; ph.gm1 = 0.4; ph.igm1 = 1.0 / 0.4;
  ph.Pr_inv = 1.0 / 0.72; ph.Prs_inv = 1.0 / 0.9;
  ph.Cv = 0.02; ph.suth = 110.4 / 288.15; ph.suth1 = 1.0 + ph.suth;
  ph.sgs_coef = (sgs == 2 ? 2.5 : 1.0) * 0.148 * 0.148 / ph.Cv;
  ph.iso_coef = 0.0;
  ph.k2 = 0.25; ph.k4 = 0.016;
  ph.viscous = 1; ph.sgs = sgs; ph.axis_node = 0;
  for (int d = 0; d < 3; ++d) ph.phys_face[d][0] = ph.phys_face[d][1] = 0;
  return ph;
}

struct Rng {
  std::mt19937_64 g;
  explicit Rng(uint64_t s) : g(s) {}
  double u(double a, double b) { return std::uniform_real_distribution<double>(a, b)(g); }
};

void random_point(Rng& r, PointIn<double>& in) {
  const double rho = r.u(0.8, 1.2), u = r.u(-0.5, 0.5), v = r.u(-0.5, 0.5), w = r.u(-0.5, 0.5);
  const double p = r.u(0.6, 0.8);
  in.q[0] = rho; in.q[1] = rho * u; in.q[2] = rho * v; in.q[3] = rho * w;
  in.q[4] = p / 0.4 + 0.5 * rho * (u * u + v * v + w * w);
  in.pr[0] = u; in.pr[1] = v; in.pr[2] = w; in.pr[3] = 1.4 * p / rho; in.pr[4] = p;
  for (int d = 0; d < 3; ++d) {
    for (int f = 0; f < 4; ++f) in.dl[d][f] = r.u(-0.1, 0.1);
    in.nu[d] = r.u(0.0, 0.05);
    for (int c = 0; c < 3; ++c) in.S[d][c] = (d == c ? 1.0 : 0.0) * 0.04 + r.u(-0.01, 0.01);
  }
  in.V = r.u(0.006, 0.01);
}

double point_objective(const PointIn<double>& in, const Phys<double>& ph, const double Gb[3][5],
                       const double lbb[3]) {
  PointOut<double> o;
  point_quantities(in, ph, o);
  double L = 0;
  for (int d = 0; d < 3; ++d) {
    for (int c = 0; c < 5; ++c) L += Gb[d][c] * o.G[d][c];
    L += lbb[d] * o.lb[d];
  }
  return L;
}

}  // namespace

extern "C" {

// Relative error of <bar, dir> against the central difference of the
// objective sum Gb.G + lbb.lambda_bar along a random direction of (q, pr, dl).
double check_point_vjp(uint64_t seed, int sgs) {
  Rng r(seed);
  const Phys<double> ph = make_phys(sgs);
  PointIn<double> in;
  random_point(r, in);
  double Gb[3][5], lbb[3];
  for (int d = 0; d < 3; ++d) {
    for (int c = 0; c < 5; ++c) Gb[d][c] = r.u(-1, 1);
    lbb[d] = r.u(-1, 1);
  }
  PointBar<double> bar = {};
  point_quantities_vjp(in, ph, Gb, lbb, bar);
  double dq[5], dpr[5], ddl[3][4];
  double ana = 0;
  for (int c = 0; c < 5; ++c) { dq[c] = r.u(-1, 1); ana += bar.q[c] * dq[c]; }
  for (int c = 0; c < 5; ++c) { dpr[c] = r.u(-1, 1); ana += bar.pr[c] * dpr[c]; }
  for (int d = 0; d < 3; ++d)
    for (int f = 0; f < 4; ++f) { ddl[d][f] = r.u(-1, 1); ana += bar.dl[d][f] * ddl[d][f]; }
  const double h = 1e-6;
  PointIn<double> a = in, b = in;
  for (int c = 0; c < 5; ++c) {
    a.q[c] += h * dq[c] * 0.1; b.q[c] -= h * dq[c] * 0.1;
    a.pr[c] += h * dpr[c] * 0.1; b.pr[c] -= h * dpr[c] * 0.1;
  }
  for (int d = 0; d < 3; ++d)
    for (int f = 0; f < 4; ++f) { a.dl[d][f] += h * ddl[d][f] * 0.1; b.dl[d][f] -= h * ddl[d][f] * 0.1; }
  const double fd = (point_objective(a, ph, Gb, lbb) - point_objective(b, ph, Gb, lbb)) / (2 * h * 0.1);
  return fabs(fd - ana) / fmax(fabs(fd), 1e-30);
}

double check_face_vjp(uint64_t seed, int nu_regime) {
  Rng r(seed);
  const Phys<double> ph = make_phys(0);
  double GL[5], GR[5], Wm[5], WL[5], WR[5], Wp[5], Fb[5];
  for (int c = 0; c < 5; ++c) {
    GL[c] = r.u(-1, 1); GR[c] = r.u(-1, 1);
    Wm[c] = r.u(0.5, 1.5); WL[c] = r.u(0.5, 1.5); WR[c] = r.u(0.5, 1.5); Wp[c] = r.u(0.5, 1.5);
    Fb[c] = r.u(-1, 1);
  }
  double lbL = r.u(20, 40), lbR = r.u(20, 40);
  // regime 0: both dissipation terms active; 1: eps4 switched off
  double nuL = nu_regime ? r.u(0.07, 0.1) : r.u(0.0, 0.03), nuR = nu_regime ? r.u(0.07, 0.1) : r.u(0.0, 0.03);
  const double VL = r.u(0.5, 1.0), VR = r.u(0.5, 1.0);
  double gbL[5] = {0}, gbR[5] = {0}, wbm[5] = {0}, wbL[5] = {0}, wbR[5] = {0}, wbp[5] = {0};
  double lbbL = 0, lbbR = 0, nubL = 0, nubR = 0;
  face_flux_vjp(lbL, lbR, nuL, nuR, VL, VR, Wm, WL, WR, Wp, false, ph, Fb, gbL, gbR, lbbL, lbbR,
                nubL, nubR, wbm, wbL, wbR, wbp);
  // direction
  double dGL[5], dGR[5], dWm[5], dWL[5], dWR[5], dWp[5];
  double ana = 0;
  for (int c = 0; c < 5; ++c) {
    dGL[c] = r.u(-1, 1); dGR[c] = r.u(-1, 1); dWm[c] = r.u(-1, 1); dWL[c] = r.u(-1, 1);
    dWR[c] = r.u(-1, 1); dWp[c] = r.u(-1, 1);
    ana += gbL[c] * dGL[c] + gbR[c] * dGR[c] + wbm[c] * dWm[c] + wbL[c] * dWL[c] + wbR[c] * dWR[c] +
           wbp[c] * dWp[c];
  }
  const double dlbL = r.u(-1, 1), dlbR = r.u(-1, 1), dnuL = r.u(-1, 1), dnuR = r.u(-1, 1);
  ana += lbbL * dlbL + lbbR * dlbR + nubL * dnuL + nubR * dnuR;
  auto obj = [&](double s) {
    double a[5], b[5], m[5], l[5], rr[5], pp[5], F[5];
    for (int c = 0; c < 5; ++c) {
      a[c] = GL[c] + s * dGL[c]; b[c] = GR[c] + s * dGR[c]; m[c] = Wm[c] + s * dWm[c];
      l[c] = WL[c] + s * dWL[c]; rr[c] = WR[c] + s * dWR[c]; pp[c] = Wp[c] + s * dWp[c];
    }
    face_flux(a, b, lbL + s * dlbL, lbR + s * dlbR, nuL + s * dnuL * 1e-3, nuR + s * dnuR * 1e-3,
              VL, VR, m, l, rr, pp, false, ph, F);
    double L = 0;
    for (int c = 0; c < 5; ++c) L += Fb[c] * F[c];
    return L;
  };
  // the sensors move by 1e-3 of the step (stay on one side of the max)
  ana -= nubL * dnuL + nubR * dnuR;
  ana += (nubL * dnuL + nubR * dnuR) * 1e-3;
  const double h = 1e-6;
  const double fd = (obj(h) - obj(-h)) / (2 * h);
  return fabs(fd - ana) / fmax(fabs(fd), 1e-30);
}

double check_prim_vjp(uint64_t seed) {
  Rng r(seed);
  const Phys<double> ph = make_phys(0);
  double q[5];
  q[0] = r.u(0.8, 1.2); q[1] = r.u(-0.5, 0.5); q[2] = r.u(-0.5, 0.5); q[3] = r.u(-0.5, 0.5);
  q[4] = r.u(1.8, 2.2);
  double prb[5], qb[5] = {0}, dq[5];
  for (int c = 0; c < 5; ++c) { prb[c] = r.u(-1, 1); dq[c] = r.u(-1, 1); }
  prim5_vjp(q, ph, prb, qb);
  double ana = 0;
  for (int c = 0; c < 5; ++c) ana += qb[c] * dq[c];
  auto obj = [&](double s) {
    double a[5], pr[5];
    for (int c = 0; c < 5; ++c) a[c] = q[c] + s * dq[c];
    prim5(a, ph, pr);
    double L = 0;
    for (int c = 0; c < 5; ++c) L += prb[c] * pr[c];
    return L;
  };
  const double h = 1e-6;
  const double fd = (obj(h) - obj(-h)) / (2 * h);
  return fabs(fd - ana) / fmax(fabs(fd), 1e-30);
}

double check_sensor_vjp(uint64_t seed) {
  Rng r(seed);
  const double pm = r.u(0.6, 0.8), p0 = r.u(0.6, 0.8), pp = r.u(0.6, 0.8), nb = r.u(-1, 1);
  double side, centre;
  sensor_vjp(pm, p0, pp, nb, side, centre);
  const double dm = r.u(-1, 1), d0 = r.u(-1, 1), dp = r.u(-1, 1);
  const double ana = side * (dm + dp) + centre * d0;
  auto nu = [&](double s) {
    const double a = pm + s * dm, b = p0 + s * d0, c = pp + s * dp;
    return nb * fabs(c - 2 * b + a) / (c + 2 * b + a);
  };
  const double h = 1e-7;
  const double fd = (nu(h) - nu(-h)) / (2 * h);
  return fabs(fd - ana) / fmax(fabs(fd), 1e-30);
}

// Dual-number Jacobian of a boundary state against central differences
// (kind 0 entrance, 1 exit, 2 far field); `mach` scales the normal velocity.
double check_bc_jacobian(uint64_t seed, int kind, double mach) {
  Rng r(seed);
  const double gamma = 1.4;
  double n[3] = {r.u(-1, 1), r.u(-1, 1), r.u(-1, 1)};
  const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int c = 0; c < 3; ++c) n[c] /= nn;
  const double rho = r.u(0.9, 1.1), p = r.u(0.65, 0.75);
  const double a = sqrt(gamma * p / rho);
  double vel[3];
  for (int c = 0; c < 3; ++c) vel[c] = mach * a * n[c] + r.u(-0.1, 0.1);
  double qe[5] = {rho, rho * vel[0], rho * vel[1], rho * vel[2],
                  p / (gamma - 1) + 0.5 * rho * (vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2])};
  BPrim<double> ref = {r.u(0.9, 1.1), r.u(-0.1, 0.1), r.u(-0.1, 0.1), r.u(-0.1, 0.1), r.u(0.65, 0.75)};
  auto state = [&](const double* q, double* f) {
    if (kind == 0) bc_inflow(q, ref, n, gamma, f);
    else if (kind == 1) bc_outflow(q, n, gamma, 0.7, f);
    else bc_farfield(q, ref, n, gamma, f);
  };
  Dual<5> qd[5], fd[5];
  for (int c = 0; c < 5; ++c) { qd[c] = Dual<5>(qe[c]); qd[c].d[c] = 1.0; }
  BPrim<Dual<5>> refd = {Dual<5>(ref.rho), Dual<5>(ref.u), Dual<5>(ref.v), Dual<5>(ref.w), Dual<5>(ref.p)};
  if (kind == 0) bc_inflow(qd, refd, n, gamma, fd);
  else if (kind == 1) bc_outflow(qd, n, gamma, 0.7, fd);
  else bc_farfield(qd, refd, n, gamma, fd);
  double worst = 0;
  const double h = 1e-7;
  for (int j = 0; j < 5; ++j) {
    double qa[5], qb[5], fa[5], fb[5];
    for (int c = 0; c < 5; ++c) { qa[c] = qe[c]; qb[c] = qe[c]; }
    qa[j] += h; qb[j] -= h;
    state(qa, fa);
    state(qb, fb);
    for (int c = 0; c < 5; ++c) {
      const double num = (fa[c] - fb[c]) / (2 * h);
      worst = fmax(worst, fabs(num - fd[c].d[j]) / fmax(1.0, fabs(num)));
    }
  }
  return worst;
}

}  // extern "C"
