// Time-step reduction and Runge-Kutta stage update (section "Time Marching
// Method", eq. localdt): Q^(l) = Q^(0) - alpha_l dt R(Q^(l-1)) with one
// global dt = CFL / max over the interior of (lambda_xi + lambda_eta +
// lambda_zeta).  The maximum is taken with an integer atomic on the bit
// pattern of non-negative doubles, which orders like the values and makes
// the result independent of scheduling; a NaN sorts above every number so a
// diverged state cannot hide.
#include "launch.hpp"
#include "physics.hpp"

namespace lesjet {

template <typename TQ, typename TM>
__global__ void k_lambda_max(const TQ* __restrict__ Q, const TM* __restrict__ M, Grid g,
                             Phys<double> ph, unsigned long long* __restrict__ maxbits) {
  __shared__ double red[256];
  const long long tot = (long long)g.nx * g.nr * g.nth;
  double local = 0.0;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < tot;
       t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t % g.nx);
    const int j = (int)((t / g.nx) % g.nr);
    const int k = (int)(t / ((long long)g.nx * g.nr));
    if (ph.axis_node && j == 0) continue;    // centerline row is not advanced
    const int o = g.at(i, j, k);
    double q[5], S[3][3];
    for (int c = 0; c < 5; ++c) q[c] = (double)Q[(long long)c * g.vs + o];
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) S[d][c] = (double)M[(long long)(3 * d + c) * g.vs + o];
    const double x = lambda_sum(q, S, (double)M[9LL * g.vs + o], ph);
    if (x != x || x > local) local = x;      // keeps a NaN once seen
  }
  red[threadIdx.x] = local;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double b = red[threadIdx.x + w];
      if (b != b || b > red[threadIdx.x]) red[threadIdx.x] = b;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    atomicMax(maxbits, (unsigned long long)__double_as_longlong(red[0]));
}

// dt for one step; resets the reduction slot for the next step.
__global__ void k_dt_finalize(unsigned long long* maxbits, double cfl, double dt_fixed,
                              double* dt, double* dt_out, int* flag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double h;
  if (dt_fixed > 0.0) {
    h = dt_fixed;
  } else {
    const double m = __longlong_as_double((long long)*maxbits);
    h = cfl / m;
    if (!(m > 0.0) || !isfinite(h)) *flag = 1;
  }
  *maxbits = 0ull;
  *dt = h;
  if (dt_out) *dt_out = h;
}

__global__ void k_reset(unsigned long long* maxbits, int* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) { *maxbits = 0ull; *flag = 0; }
}

// Q_out = Q0 - alpha dt R on the interior; accumulation in FP64.  Q0 and
// Q_out may be the same array (last stage), so they are not restrict.
template <typename T, typename TS>
__global__ void k_rk_update(const double* Q0, const T* __restrict__ R, TS* Qout,
                            double* Q64out, Grid g, double alpha, const double* __restrict__ dt) {
  const long long tot = (long long)g.nx * g.nr * g.nth;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= tot) return;
  const int i = (int)(t % g.nx);
  const int j = (int)((t / g.nx) % g.nr);
  const int k = (int)(t / ((long long)g.nx * g.nr));
  const int o = g.at(i, j, k);
  const double ad = alpha * (*dt);
  for (int c = 0; c < 5; ++c) {
    const long long oc = (long long)c * g.vs + o;
    const double v = Q0[oc] - ad * (double)R[oc];
    Qout[oc] = (TS)v;
    if (Q64out) Q64out[oc] = v;
  }
}

// FP64 -> FP32 copy of a whole padded field (start of an FP32-storage call).
__global__ void k_to_float(const double* __restrict__ a, float* __restrict__ b, long long n) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x)
    b[t] = (float)a[t];
}

template <typename TQ, typename TM>
hipError_t launch_lambda_max(const TQ* Q, const TM* M, const Grid& g, const Phys<double>& ph,
                             unsigned long long* maxbits, hipStream_t s) {
  const long long n = (long long)g.nx * g.nr * g.nth;
  long long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL((k_lambda_max<TQ, TM>), dim3((unsigned)b), dim3(256), 0, s, Q, M, g, ph,
                     maxbits);
  return hipGetLastError();
}

hipError_t launch_dt_finalize(unsigned long long* maxbits, double cfl, double dt_fixed,
                              double* dt, double* dt_out, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_dt_finalize, dim3(1), dim3(64), 0, s, maxbits, cfl, dt_fixed, dt, dt_out,
                     flag);
  return hipGetLastError();
}

hipError_t launch_reset(unsigned long long* maxbits, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, maxbits, flag);
  return hipGetLastError();
}

template <typename T, typename TS>
hipError_t launch_rk_update(const double* Q0, const T* R, TS* Qout, double* Q64out, const Grid& g,
                            double alpha, const double* dt, hipStream_t s) {
  const long long n = (long long)g.nx * g.nr * g.nth;
  hipLaunchKernelGGL((k_rk_update<T, TS>), dim3(blocks_for(n, 256)), dim3(256), 0, s, Q0, R, Qout,
                     Q64out, g, alpha, dt);
  return hipGetLastError();
}

hipError_t launch_to_float(const double* a, float* b, long long n, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_to_float, dim3((unsigned)blocks), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

template hipError_t launch_lambda_max<double, double>(const double*, const double*, const Grid&,
                                                      const Phys<double>&, unsigned long long*,
                                                      hipStream_t);
template hipError_t launch_lambda_max<double, float>(const double*, const float*, const Grid&,
                                                     const Phys<double>&, unsigned long long*,
                                                     hipStream_t);
template hipError_t launch_rk_update<double, double>(const double*, const double*, double*,
                                                     double*, const Grid&, double, const double*,
                                                     hipStream_t);
template hipError_t launch_rk_update<float, float>(const double*, const float*, float*, double*,
                                                   const Grid&, double, const double*,
                                                   hipStream_t);

}  // namespace lesjet
