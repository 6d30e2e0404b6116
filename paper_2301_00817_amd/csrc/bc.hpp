// Boundary face states of section "Boundary Conditions", written once for a
// generic scalar S: double or float in the ghost-fill kernels, and a
// forward-mode dual number in the adjoint, which needs their exact
// Jacobians.  Constants are doubles cast to S; branch tests act on values.
//
//   entrance: a target with normal Mach >= 1 is imposed; otherwise Riemann
//             invariants with the target as outside state (normal -xi);
//   exit:     copy when the normal Mach is >= 1, else interior rho, u, v, w
//             with the back pressure;
//   far field: Riemann invariants with the reference state (normal eta).
// Riemann invariants: R+ = q_e + 2 a_e/(gamma-1), R- = q_r - 2 a_r/(gamma-1),
// q_f = (R+ + R-)/2, a_f = (gamma-1)(R+ - R-)/4; M = q_e/a_e >= 1 copies the
// interior, <= -1 takes the outside state, otherwise the velocity is
// corrected along the unit normal and the entropy is taken from the upwind
// side (interior when q_e >= 0).
#pragma once

#include <math.h>

#include "common.hpp"

namespace lesjet {

// ---- forward-mode dual numbers ---------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
  __host__ __device__ Dual() : v(0.0) {
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
  __host__ __device__ Dual(double x) : v(x) {  // NOLINT: implicit constant
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
};

template <int N>
__host__ __device__ inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v;
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N>
__host__ __device__ inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <int N>
__host__ __device__ inline Dual<N> dsqrt(const Dual<N>& a) {
  Dual<N> r; r.v = ::sqrt(a.v);
  const double h = 0.5 / r.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * h;
  return r;
}
template <int N>
__host__ __device__ inline Dual<N> dpow(const Dual<N>& a, double y) {
  Dual<N> r; r.v = ::pow(a.v, y);
  const double g = y * r.v / a.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * g;
  return r;
}

__host__ __device__ inline double sval(double x) { return x; }
__host__ __device__ inline float sval(float x) { return x; }
template <int N>
__host__ __device__ inline double sval(const Dual<N>& x) { return x.v; }

__host__ __device__ inline double ssqrt(double x) { return ::sqrt(x); }
__host__ __device__ inline float ssqrt(float x) { return sqrtf(x); }
template <int N>
__host__ __device__ inline Dual<N> ssqrt(const Dual<N>& x) { return dsqrt(x); }
__host__ __device__ inline double spow(double x, double y) { return ::pow(x, y); }
__host__ __device__ inline float spow(float x, double y) { return powf(x, (float)y); }
template <int N>
__host__ __device__ inline Dual<N> spow(const Dual<N>& x, double y) { return dpow(x, y); }

// ---- boundary face states ------------------------------------------------------
template <typename S>
struct BPrim { S rho, u, v, w, p; };

template <typename S>
__host__ __device__ inline BPrim<S> bc_prim(const S q[5], double gamma) {
  BPrim<S> s;
  s.rho = q[0];
  s.u = q[1] / q[0];
  s.v = q[2] / q[0];
  s.w = q[3] / q[0];
  s.p = S(gamma - 1.0) * (q[4] - S(0.5) * q[0] * (s.u * s.u + s.v * s.v + s.w * s.w));
  return s;
}

template <typename S>
__host__ __device__ inline void bc_cons(const BPrim<S>& s, double gamma, S q[5]) {
  q[0] = s.rho;
  q[1] = s.rho * s.u;
  q[2] = s.rho * s.v;
  q[3] = s.rho * s.w;
  q[4] = s.p * S(1.0 / (gamma - 1.0)) + S(0.5) * s.rho * (s.u * s.u + s.v * s.v + s.w * s.w);
}

// Riemann-invariant state; returns 0 copy interior, 1 outside state,
// 2 subsonic state written to f.
template <typename S>
__host__ __device__ inline int bc_riemann(const BPrim<S>& e, const BPrim<S>& r, const double n[3],
                                          double gamma, BPrim<S>& f) {
  const double gm1 = gamma - 1.0;
  const S ae = ssqrt(S(gamma) * e.p / e.rho);
  const S ar = ssqrt(S(gamma) * r.p / r.rho);
  const S qe = e.u * S(n[0]) + e.v * S(n[1]) + e.w * S(n[2]);
  const S qr = r.u * S(n[0]) + r.v * S(n[1]) + r.w * S(n[2]);
  const double M = sval(qe) / sval(ae);
  if (M >= 1.0) return 0;
  if (M <= -1.0) return 1;
  const S Rp = qe + S(2.0 / gm1) * ae;
  const S Rm = qr - S(2.0 / gm1) * ar;
  const S qf = S(0.5) * (Rp + Rm);
  const S af = S(0.25 * gm1) * (Rp - Rm);
  const bool out = sval(qe) >= 0.0;
  const BPrim<S>& src = out ? e : r;
  const S qs = out ? qe : qr;
  const S base = spow(src.rho, gamma) * af * af / (S(gamma) * src.p);
  f.rho = spow(base, 1.0 / gm1);
  f.u = src.u + (qf - qs) * S(n[0]);
  f.v = src.v + (qf - qs) * S(n[1]);
  f.w = src.w + (qf - qs) * S(n[2]);
  f.p = f.rho * af * af / S(gamma);
  return 2;
}

// Entrance ghost state from the interior state qe and the target primitives;
// n is the outward unit normal.
template <typename S>
__host__ __device__ inline void bc_inflow(const S qe[5], const BPrim<S>& tgt, const double n[3],
                                          double gamma, S qf[5]) {
  const double at = ::sqrt(gamma * sval(tgt.p) / sval(tgt.rho));
  const double mn = -(sval(tgt.u) * n[0] + sval(tgt.v) * n[1] + sval(tgt.w) * n[2]) / at;
  if (mn >= 1.0) {
    bc_cons(tgt, gamma, qf);
    return;
  }
  BPrim<S> f;
  const int br = bc_riemann(bc_prim(qe, gamma), tgt, n, gamma, f);
  if (br == 0)
    for (int c = 0; c < 5; ++c) qf[c] = qe[c];
  else if (br == 1)
    bc_cons(tgt, gamma, qf);
  else
    bc_cons(f, gamma, qf);
}

template <typename S>
__host__ __device__ inline void bc_outflow(const S qe[5], const double n[3], double gamma,
                                           double p_exit, S qf[5]) {
  BPrim<S> e = bc_prim(qe, gamma);
  const double ae = ::sqrt(gamma * sval(e.p) / sval(e.rho));
  const double qn = sval(e.u) * n[0] + sval(e.v) * n[1] + sval(e.w) * n[2];
  if (qn / ae >= 1.0) {
    for (int c = 0; c < 5; ++c) qf[c] = qe[c];
    return;
  }
  e.p = S(p_exit);
  bc_cons(e, gamma, qf);
}

template <typename S>
__host__ __device__ inline void bc_farfield(const S qe[5], const BPrim<S>& ref, const double n[3],
                                            double gamma, S qf[5]) {
  BPrim<S> f;
  const int br = bc_riemann(bc_prim(qe, gamma), ref, n, gamma, f);
  if (br == 0)
    for (int c = 0; c < 5; ++c) qf[c] = qe[c];
  else if (br == 1)
    bc_cons(ref, gamma, qf);
  else
    bc_cons(f, gamma, qf);
}

}  // namespace lesjet
