// Ghost layers of the state from the boundary conditions (section "Boundary
// Conditions"), defined as sweeps in the order xi, eta, zeta so that edge
// ghosts take values that are already set:
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

// The fill is defined as three sweeps in the order xi (j, k interior), eta
// (i padded, k interior), zeta (i, j padded), each reading what the earlier
// ones wrote.  One launch evaluates it directly: every ghost point traces
// its value back through the sweeps (zeta wrap, then the eta rule, then the
// xi rule) to interior points, so all ghost points are independent and
// filled in parallel.

// State of (i, j, k), i padded, j and k interior, after the xi sweep.
// With a centerline through the nodes j = 0 (axis_node), the boundary
// normals of axis points are those of row j = 1 (S^xi vanishes on the axis).
template <typename T>
__device__ __forceinline__ void xi_value(const T* __restrict__ Q, const Grid& g,
                                         const T* __restrict__ M,
                                         const double* __restrict__ inflow, double gamma,
                                         int lo_kind, int hi_kind, double p_exit, int axis_node,
                                         int i, int j, int k, T q[5]) {
  const int jn = axis_node && j == 0 ? 1 : j;
  if (i >= 0 && i < g.nx) {
    load5(Q, g.vs, g.at(i, j, k), q);
  } else if (i < 0) {
    if (lo_kind == BC_PERIODIC) {
      load5(Q, g.vs, g.at(i + g.nx, j, k), q);
    } else {                                   // entrance: both layers get the face state
      const int oe = g.at(0, j, k);
      T qe[5];
      load5(Q, g.vs, oe, qe);
      double n[3];
      unit_normal(M, g.vs, g.at(0, jn, k), 0, -1.0, n);
      BPrim<T> tg;
      const long long sp = (long long)g.nth * g.nr, it = (long long)k * g.nr + j;
      tg.rho = (T)inflow[0 * sp + it];
      tg.u = (T)inflow[1 * sp + it];
      tg.v = (T)inflow[2 * sp + it];
      tg.w = (T)inflow[3 * sp + it];
      tg.p = (T)inflow[4 * sp + it];
      bc_inflow(qe, tg, n, gamma, q);
    }
  } else {
    if (hi_kind == BC_PERIODIC) {
      load5(Q, g.vs, g.at(i - g.nx, j, k), q);
    } else {                                   // exit
      const int oe = g.at(g.nx - 1, j, k);
      T qe[5];
      load5(Q, g.vs, oe, qe);
      double n[3];
      unit_normal(M, g.vs, g.at(g.nx - 1, jn, k), 0, 1.0, n);
      bc_outflow(qe, n, gamma, p_exit, q);
    }
  }
}

// One thread per ghost point: the zeta layers of the whole padded plane, the
// eta layers (i padded, k interior), the xi layers (j, k interior).
// held != nullptr: a ghost point whose trace ends in a physical-face rule
// (entrance, exit, far field) takes the value of `held` at the same point,
// which is that rule evaluated on the held state.
// 64-thread blocks, at least six waves per SIMD: the FP64 instance fits 80
// VGPRs without spilling (81 unbounded, five waves); eight waves spill.
constexpr int GH_BS = 64;
template <typename T>
__global__ __launch_bounds__(GH_BS, 6) void k_ghost_all(T* __restrict__ Q, Grid g, const T* __restrict__ M,
                            const double* __restrict__ inflow, double gamma, int xlo, int xhi,
                            int elo, int ehi, double p_exit, BPrim<T> ref,
                            const T* __restrict__ held) {
  // 32-bit index arithmetic: the ghost points number 4 (NX NR + NX nth +
  // nr nth), far below 2^32 for every mesh the library accepts
  const unsigned NX = g.nx + 2 * NG, NR = g.nr + 2 * NG, nth = g.nth, nr = g.nr;
  const unsigned nz = 2u * NG * NX * NR, ne = 2u * NG * NX * nth, nxg = 2u * NG * nr * nth;
  unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (t < nz) {
    const unsigned r = t / NX;
    i = (int)(t - r * NX) - NG;
    const unsigned l = r / NR;                          // 0..3 -> -2, -1, nth, nth+1
    j = (int)(r - l * NR) - NG;
    k = l < NG ? (int)l - NG : g.nth + ((int)l - NG);
  } else if ((t -= nz) < ne) {
    const unsigned r = t / NX;
    i = (int)(t - r * NX) - NG;
    const unsigned l = r % (2 * NG);
    j = l < NG ? (int)l - NG : g.nr + ((int)l - NG);
    k = (int)(r / (2 * NG));
  } else if ((t -= ne) < nxg) {
    const unsigned l = t % (2 * NG);
    i = l < NG ? (int)l - NG : g.nx + ((int)l - NG);
    const unsigned r = t / (2 * NG);
    j = (int)(r % nr);
    k = (int)(r / nr);
  } else {
    return;
  }
  const int og = g.at(i, j, k);
  if (held && ((i < 0 && xlo != BC_PERIODIC) || (i >= g.nx && xhi != BC_PERIODIC) ||
               (j >= g.nr && ehi != BC_PERIODIC))) {
    T h[5];
    load5(held, g.vs, og, h);
    store5(Q, g.vs, og, h);
    return;
  }
  // zeta sweep (periodic): the wrapped point
  int kw = k < 0 ? k + g.nth : (k >= g.nth ? k - g.nth : k);
  const int an = elo == BC_AXIS_NODE;
  // eta sweep
  T q[5];
  if (j >= 0 && j < g.nr) {
    xi_value(Q, g, M, inflow, gamma, xlo, xhi, p_exit, an, i, j, kw, q);
  } else if (j < 0) {
    if (elo == BC_PERIODIC)
      xi_value(Q, g, M, inflow, gamma, xlo, xhi, p_exit, an, i, j + g.nr, kw, q);
    else if (elo == BC_AXIS)                     // across the axis
      xi_value(Q, g, M, inflow, gamma, xlo, xhi, p_exit, an, i, -1 - j, (kw + g.nth / 2) % g.nth, q);
    else                                         // mirror through the axis node
      xi_value(Q, g, M, inflow, gamma, xlo, xhi, p_exit, an, i, -j, (kw + g.nth / 2) % g.nth, q);
  } else {
    if (ehi == BC_PERIODIC) {
      xi_value(Q, g, M, inflow, gamma, xlo, xhi, p_exit, an, i, j - g.nr, kw, q);
    } else {                                     // far field from the state at (i, nr-1)
      T qe[5];
      xi_value(Q, g, M, inflow, gamma, xlo, xhi, p_exit, an, i, g.nr - 1, kw, qe);
      double n[3];
      unit_normal(M, g.vs, g.at(i, g.nr - 1, kw), 1, 1.0, n);
      bc_farfield(qe, ref, n, gamma, q);
    }
  }
  store5(Q, g.vs, og, q);
}

// Centerline through the nodes j = 0: the axis row takes the azimuthal mean
// of the conserved variables of row j = 1 (one block per i, a fixed-order
// FP64 tree over k, so the value is the same for every k and reproducible).
constexpr int CL_BS = 256;

// held row (schedule with held boundary values)
template <typename T>
__global__ void k_centerline_held(T* __restrict__ Q, Grid g, const T* __restrict__ held) {
  const int i = blockIdx.x;
  for (int k = threadIdx.x; k < g.nth; k += blockDim.x) {
    const int o = g.at(i, 0, k);
    for (int c = 0; c < 5; ++c) Q[(long long)c * g.vs + o] = held[(long long)c * g.vs + o];
  }
}

template <typename T>
__global__ void k_centerline(T* __restrict__ Q, Grid g) {
  __shared__ double red[5][CL_BS];
  const int i = blockIdx.x;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int k = threadIdx.x; k < g.nth; k += CL_BS) {
    const int o = g.at(i, 1, k);
    for (int c = 0; c < 5; ++c) acc[c] += (double)Q[(long long)c * g.vs + o];
  }
  for (int c = 0; c < 5; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = CL_BS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 5; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  for (int k = threadIdx.x; k < g.nth; k += CL_BS) {
    const int o = g.at(i, 0, k);
    for (int c = 0; c < 5; ++c) Q[(long long)c * g.vs + o] = (T)(red[c][0] / g.nth);
  }
}

template <typename T>
hipError_t launch_centerline(T* Q, const Grid& g, hipStream_t s) {
  hipLaunchKernelGGL(k_centerline<T>, dim3(g.nx), dim3(CL_BS), 0, s, Q, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ghosts(T* Q, const Grid& g, const T* M, const double* inflow,
                         const Phys<T>& ph, const int bc[6], const double ref_prim[5],
                         double p_exit, const T* held, hipStream_t s) {
  if (bc[2] == BC_AXIS_NODE) {
    if (held)
      hipLaunchKernelGGL(k_centerline_held<T>, dim3(g.nx), dim3(CL_BS), 0, s, Q, g, held);
    else
      hipLaunchKernelGGL(k_centerline<T>, dim3(g.nx), dim3(CL_BS), 0, s, Q, g);
  }
  const double gamma = (double)ph.gamma;
  BPrim<T> ref;
  ref.rho = (T)ref_prim[0]; ref.u = (T)ref_prim[1]; ref.v = (T)ref_prim[2];
  ref.w = (T)ref_prim[3]; ref.p = (T)ref_prim[4];
  const long long NX = g.nx + 2 * NG, NR = g.nr + 2 * NG;
  const long long n = 2LL * NG * (NX * NR + NX * g.nth + (long long)g.nr * g.nth);
  hipLaunchKernelGGL(k_ghost_all<T>, dim3(blocks_for(n, GH_BS)), dim3(GH_BS), 0, s, Q, g, M, inflow,
                     gamma, bc[0], bc[1], bc[2], bc[3], p_exit, ref, held);
  return hipGetLastError();
}

template hipError_t launch_centerline<double>(double*, const Grid&, hipStream_t);
template hipError_t launch_ghosts<double>(double*, const Grid&, const double*, const double*,
                                          const Phys<double>&, const int*, const double*, double,
                                          const double*, hipStream_t);
template hipError_t launch_ghosts<float>(float*, const Grid&, const float*, const double*,
                                         const Phys<float>&, const int*, const double*, double,
                                         const float*, hipStream_t);

}  // namespace lesjet
