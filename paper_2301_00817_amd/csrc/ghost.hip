// Ghost layers of the state from the boundary conditions (section "Boundary
// Conditions"), filled in the order xi, eta, zeta so that edge ghosts read
// values that are already set:
//   xi-  periodic | entrance: target imposed when its normal Mach >= 1, else
//        Riemann invariants with the target as outside state;
//   xi+  periodic | exit: copy when supersonic, else interior rho, u, v, w
//        with the back pressure;
//   eta- periodic | centerline: the points across the axis (i, m, k + nth/2);
//   eta+ periodic | far field: Riemann invariants with the reference state;
//   zeta periodic.
// Both ghost layers of a non-periodic face receive the same face state.
#include "bc.hpp"
#include "launch.hpp"

namespace lesjet {

template <typename T>
__device__ __forceinline__ void load5(const T* Q, int vs, int o, T q[5]) {
#pragma unroll
  for (int c = 0; c < 5; ++c) q[c] = Q[(long long)c * vs + o];
}
template <typename T>
__device__ __forceinline__ void store5(T* Q, int vs, int o, const T q[5]) {
#pragma unroll
  for (int c = 0; c < 5; ++c) Q[(long long)c * vs + o] = q[c];
}
// Unit normal S^d / |S^d| (times sgn) at offset o, in FP64 for the
// boundary formulas.
template <typename T>
__device__ __forceinline__ void unit_normal(const T* M, int vs, int o, int d, double sgn,
                                            double n[3]) {
  const double a = (double)M[(long long)(3 * d + 0) * vs + o];
  const double b = (double)M[(long long)(3 * d + 1) * vs + o];
  const double c = (double)M[(long long)(3 * d + 2) * vs + o];
  const double inv = sgn / sqrt(a * a + b * b + c * c);
  n[0] = a * inv; n[1] = b * inv; n[2] = c * inv;
}

// xi faces, one thread per (j, k) of the interior and face (the two faces
// read interior points only and write disjoint ghosts).
template <typename T>
__global__ void k_ghost_xi(T* __restrict__ Q, Grid g, const T* __restrict__ M,
                           const double* __restrict__ inflow, double gamma, int lo_kind,
                           int hi_kind, double p_exit) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nf = g.nr * g.nth;
  if (t >= 2 * nf) return;
  const bool lo = t < nf;
  const int jk = lo ? t : t - nf;
  const int j = jk % g.nr, k = jk / g.nr;
  if (!lo) { lo_kind = -1; } else { hi_kind = -1; }
  T q[5];
  if (lo_kind == BC_PERIODIC) {
    for (int m = 1; m <= NG; ++m) {
      load5(Q, g.vs, g.at(g.nx - m, j, k), q);
      store5(Q, g.vs, g.at(-m, j, k), q);
    }
  } else if (lo_kind == BC_INFLOW) {
    const int oe = g.at(0, j, k);
    T qe[5];
    load5(Q, g.vs, oe, qe);
    double n[3];
    unit_normal(M, g.vs, oe, 0, -1.0, n);
    BPrim<T> tg;
    const long long sp = (long long)g.nth * g.nr, it = (long long)k * g.nr + j;
    tg.rho = (T)inflow[0 * sp + it];
    tg.u = (T)inflow[1 * sp + it];
    tg.v = (T)inflow[2 * sp + it];
    tg.w = (T)inflow[3 * sp + it];
    tg.p = (T)inflow[4 * sp + it];
    bc_inflow(qe, tg, n, gamma, q);
    for (int m = 1; m <= NG; ++m) store5(Q, g.vs, g.at(-m, j, k), q);
  }
  if (hi_kind == BC_PERIODIC) {
    for (int m = 1; m <= NG; ++m) {
      load5(Q, g.vs, g.at(m - 1, j, k), q);
      store5(Q, g.vs, g.at(g.nx - 1 + m, j, k), q);
    }
  } else if (hi_kind == BC_OUTFLOW) {
    const int oe = g.at(g.nx - 1, j, k);
    T qe[5];
    load5(Q, g.vs, oe, qe);
    double n[3];
    unit_normal(M, g.vs, oe, 0, 1.0, n);
    bc_outflow(qe, n, gamma, p_exit, q);
    for (int m = 1; m <= NG; ++m) store5(Q, g.vs, g.at(g.nx - 1 + m, j, k), q);
  }
}

// eta faces, one thread per (i, k), i over the padded range, k interior.
template <typename T>
__global__ void k_ghost_eta(T* __restrict__ Q, Grid g, const T* __restrict__ M, double gamma,
                            int lo_kind, int hi_kind, BPrim<T> ref) {
  const int NX = g.nx + 2 * NG;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NX * g.nth) return;
  const int i = t % NX - NG, k = t / NX;
  T q[5];
  if (lo_kind == BC_PERIODIC) {
    for (int m = 1; m <= NG; ++m) {
      load5(Q, g.vs, g.at(i, g.nr - m, k), q);
      store5(Q, g.vs, g.at(i, -m, k), q);
    }
  } else if (lo_kind == BC_AXIS) {
    const int kk = (k + g.nth / 2) % g.nth;
    for (int m = 1; m <= NG; ++m) {
      load5(Q, g.vs, g.at(i, m - 1, kk), q);
      store5(Q, g.vs, g.at(i, -m, k), q);
    }
  }
  if (hi_kind == BC_PERIODIC) {
    for (int m = 1; m <= NG; ++m) {
      load5(Q, g.vs, g.at(i, m - 1, k), q);
      store5(Q, g.vs, g.at(i, g.nr - 1 + m, k), q);
    }
  } else if (hi_kind == BC_FARFIELD) {
    const int oe = g.at(i, g.nr - 1, k);
    T qe[5];
    load5(Q, g.vs, oe, qe);
    double n[3];
    unit_normal(M, g.vs, oe, 1, 1.0, n);
    bc_farfield(qe, ref, n, gamma, q);
    for (int m = 1; m <= NG; ++m) store5(Q, g.vs, g.at(i, g.nr - 1 + m, k), q);
  }
}

// zeta faces (periodic), one thread per (i, j) of the padded plane.
template <typename T>
__global__ void k_ghost_zeta(T* __restrict__ Q, Grid g) {
  const int NX = g.nx + 2 * NG, NR = g.nr + 2 * NG;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NX * NR) return;
  const int i = t % NX - NG, j = t / NX - NG;
  T q[5];
  for (int m = 1; m <= NG; ++m) {
    load5(Q, g.vs, g.at(i, j, g.nth - m), q);
    store5(Q, g.vs, g.at(i, j, -m), q);
    load5(Q, g.vs, g.at(i, j, m - 1), q);
    store5(Q, g.vs, g.at(i, j, g.nth - 1 + m), q);
  }
}

template <typename T>
hipError_t launch_ghosts(T* Q, const Grid& g, const T* M, const double* inflow,
                         const Phys<T>& ph, const int bc[6], const double ref_prim[5],
                         double p_exit, hipStream_t s) {
  const int bs = 256;
  const double gamma = (double)ph.gamma;
  hipLaunchKernelGGL(k_ghost_xi<T>, dim3(blocks_for(2LL * g.nr * g.nth, 64)), dim3(64), 0, s, Q,
                     g, M, inflow, gamma, bc[0], bc[1], p_exit);
  BPrim<T> ref;
  ref.rho = (T)ref_prim[0]; ref.u = (T)ref_prim[1]; ref.v = (T)ref_prim[2];
  ref.w = (T)ref_prim[3]; ref.p = (T)ref_prim[4];
  hipLaunchKernelGGL(k_ghost_eta<T>, dim3(blocks_for((long long)(g.nx + 2 * NG) * g.nth, bs)),
                     dim3(bs), 0, s, Q, g, M, gamma, bc[2], bc[3], ref);
  hipLaunchKernelGGL(k_ghost_zeta<T>,
                     dim3(blocks_for((long long)(g.nx + 2 * NG) * (g.nr + 2 * NG), bs)), dim3(bs),
                     0, s, Q, g);
  return hipGetLastError();
}

template hipError_t launch_ghosts<double>(double*, const Grid&, const double*, const double*,
                                          const Phys<double>&, const int*, const double*, double,
                                          hipStream_t);
template hipError_t launch_ghosts<float>(float*, const Grid&, const float*, const double*,
                                         const Phys<float>&, const int*, const double*, double,
                                         hipStream_t);

}  // namespace lesjet
