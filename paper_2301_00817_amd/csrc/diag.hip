// Diagnostics of a state: conservation totals and azimuthal statistics.
//
//   totals[c] = sum over the interior of J^-1 Q_c   (c = rho, rho u, rho v,
//               rho w, E): the discrete conserved quantities, constant in
//               time on a periodic mesh because every face flux enters its
//               two cells with opposite signs;
//   sum1[c](i, j) += sum_k phi_c,  sum2[c](i, j) += sum_k phi_c^2  with
//               phi = (rho, u, v, w, p): accumulators of the azimuthal (and,
//               over calls, temporal) mean and rms fields.
//
// Both reductions run in a fixed order (per-block tree, then one block over
// the partials in block order; one thread per (i, j) over k), so repeated
// runs are bitwise identical.  FP64 throughout.
#include "launch.hpp"
#include "physics.hpp"

namespace lesjet {

constexpr int DIAG_BS = 256;

template <typename TM>
__global__ void k_totals_partial(const double* __restrict__ Q, const TM* __restrict__ M, Grid g,
                                 double* __restrict__ part) {
  __shared__ double red[5][DIAG_BS];
  const long long tot = (long long)g.nx * g.nr * g.nth;
  double acc[5] = {0, 0, 0, 0, 0};
  for (long long t = blockIdx.x * (long long)DIAG_BS + threadIdx.x; t < tot;
       t += (long long)gridDim.x * DIAG_BS) {
    const int i = (int)(t % g.nx);
    const int j = (int)((t / g.nx) % g.nr);
    const int k = (int)(t / ((long long)g.nx * g.nr));
    const int o = g.at(i, j, k);
    const double V = (double)M[9LL * g.vs + o];
    for (int c = 0; c < 5; ++c) acc[c] += V * Q[(long long)c * g.vs + o];
  }
  for (int c = 0; c < 5; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = DIAG_BS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 5; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 5) part[(long long)threadIdx.x * gridDim.x + blockIdx.x] = red[threadIdx.x][0];
}

__global__ void k_totals_final(const double* __restrict__ part, int nparts,
                               double* __restrict__ totals) {
  __shared__ double red[DIAG_BS];
  for (int c = 0; c < 5; ++c) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nparts; b += DIAG_BS) a += part[(long long)c * nparts + b];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = DIAG_BS / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) totals[c] = red[0];
    __syncthreads();
  }
}

__global__ void k_azimuthal_stats(const double* __restrict__ Q, Grid g, Phys<double> ph,
                                  double* __restrict__ s1, double* __restrict__ s2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.nx * g.nr) return;
  const int i = t % g.nx, j = t / g.nx;
  double a1[5] = {0, 0, 0, 0, 0}, a2[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < g.nth; ++k) {
    const int o = g.at(i, j, k);
    double q[5];
    for (int c = 0; c < 5; ++c) q[c] = Q[(long long)c * g.vs + o];
    const Prim<double> s = primitives(q, ph);
    const double f[5] = {s.rho, s.u, s.v, s.w, s.p};
    for (int c = 0; c < 5; ++c) { a1[c] += f[c]; a2[c] += f[c] * f[c]; }
  }
  const long long sp = (long long)g.nx * g.nr;
  for (int c = 0; c < 5; ++c) {
    if (s1) s1[c * sp + t] += a1[c];
    if (s2) s2[c * sp + t] += a2[c];
  }
}

int diag_partials(const Grid& g) {
  const long long n = (long long)g.nx * g.nr * g.nth;
  long long b = (n + DIAG_BS - 1) / DIAG_BS;
  return (int)(b > DIAG_MAX_PARTIALS ? DIAG_MAX_PARTIALS : (b < 1 ? 1 : b));
}

template <typename TM>
hipError_t launch_diagnostics(const double* Q, const TM* M, const Grid& g,
                              const Phys<double>& ph, double* part, double* totals, double* s1,
                              double* s2, hipStream_t s) {
  if (totals) {
    const int nb = diag_partials(g);
    hipLaunchKernelGGL((k_totals_partial<TM>), dim3(nb), dim3(DIAG_BS), 0, s, Q, M, g, part);
    hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(DIAG_BS), 0, s, part, nb, totals);
  }
  if (s1 || s2)
    hipLaunchKernelGGL(k_azimuthal_stats, dim3(blocks_for((long long)g.nx * g.nr, 256)), dim3(256),
                       0, s, Q, g, ph, s1, s2);
  return hipGetLastError();
}

template hipError_t launch_diagnostics<double>(const double*, const double*, const Grid&,
                                               const Phys<double>&, double*, double*, double*,
                                               double*, hipStream_t);
template hipError_t launch_diagnostics<float>(const double*, const float*, const Grid&,
                                              const Phys<double>&, double*, double*, double*,
                                              double*, hipStream_t);

}  // namespace lesjet
