// Two-pass residual (reference form of the fused kernel): a point pass that
// writes the point quantities G^d, lambda_bar^d, nu^d of every point whose
// indices lie in [-1, n] to scratch arrays, and a face pass that forms the
// six face fluxes of each interior point and R = RHS / J^-1 (section
// "Spatial Discretization").  Simple indexing, one thread per point, no
// shared memory; it moves several times the algorithmic bytes and serves as
// the on-device cross-check of the fused kernel.
#include "launch.hpp"
#include "physics.hpp"

namespace lesjet {

template <typename T>
__device__ __forceinline__ void uvwTp(const T* Q, int vs, int o, const Phys<T>& ph, T out[5]) {
  T q[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) q[c] = Q[(long long)c * vs + o];
  prim5(q, ph, out);
}

template <typename T>
__global__ void k_point_pass(const T* __restrict__ Q, const T* __restrict__ M, Grid g, Phys<T> ph,
                             T* __restrict__ PT) {
  const int NX1 = g.nx + 2, NR1 = g.nr + 2, NT1 = g.nth + 2;
  const long long tot = (long long)NX1 * NR1 * NT1;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= tot) return;
  const int i = (int)(t % NX1) - 1;
  const int j = (int)((t / NX1) % NR1) - 1;
  const int k = (int)(t / ((long long)NX1 * NR1)) - 1;
  const int o = g.at(i, j, k);
  const int step[3] = {1, g.pitch, g.plane};
  PointIn<T> in;
#pragma unroll
  for (int c = 0; c < 5; ++c) in.q[c] = Q[(long long)c * g.vs + o];
  prim5(in.q, ph, in.pr);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T m[5], pl[5];
    uvwTp(Q, g.vs, o - step[d], ph, m);
    uvwTp(Q, g.vs, o + step[d], ph, pl);
    neighbour_terms(m, pl, in.pr[4], in.dl[d], in.nu[d]);
#pragma unroll
    for (int c = 0; c < 3; ++c) in.S[d][c] = M[(long long)(3 * d + c) * g.vs + o];
  }
  in.V = M[9LL * g.vs + o];
  PointOut<T> out;
  point_quantities<T, LAG_NONE, true>(in, ph, out);
  if (ph.axis_node && j == 0)          // centerline through the nodes: no eta point flux
    for (int c = 0; c < 5; ++c) out.G[1][c] = T(0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int c = 0; c < 5; ++c) PT[(long long)(5 * d + c) * g.vs + o] = out.G[d][c];
    PT[(long long)(15 + d) * g.vs + o] = out.lb[d];
    PT[(long long)(18 + d) * g.vs + o] = out.nu[d];
  }
}

template <typename T>
__global__ void k_face_pass(const T* __restrict__ Q, const T* __restrict__ M, Grid g, Phys<T> ph,
                            const T* __restrict__ PT, T* __restrict__ R) {
  const long long tot = (long long)g.nx * g.nr * g.nth;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= tot) return;
  const int i = (int)(t % g.nx);
  const int j = (int)((t / g.nx) % g.nr);
  const int k = (int)(t / ((long long)g.nx * g.nr));
  const int o = g.at(i, j, k);
  const int step[3] = {1, g.pitch, g.plane};
  const int pos[3] = {i, j, k};
  const int nn[3] = {g.nx, g.nr, g.nth};
  T rhs[5] = {0, 0, 0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    const int s = step[d];
    T W[5][5];   // points o-2s .. o+2s
    for (int m = 0; m < 5; ++m) {
      T q[5];
      for (int c = 0; c < 5; ++c) q[c] = Q[(long long)c * g.vs + o + (m - 2) * s];
      wvec(q, ph, W[m]);
    }
    T G[3][5], lb[3], nu[3], V[3];
    for (int m = 0; m < 3; ++m) {
      const int op = o + (m - 1) * s;
      for (int c = 0; c < 5; ++c) G[m][c] = PT[(long long)(5 * d + c) * g.vs + op];
      lb[m] = PT[(long long)(15 + d) * g.vs + op];
      nu[m] = PT[(long long)(18 + d) * g.vs + op];
      V[m] = M[9LL * g.vs + op];
    }
    T Fm[5], Fp[5];
    const bool phys_m = pos[d] == 0 && ph.phys_face[d][0];
    const bool phys_p = pos[d] == nn[d] - 1 && ph.phys_face[d][1];
    // axis face (centerline through the nodes): lambda_bar of row 1 and the
    // three-point fourth difference (W(-1) replaced by W(1))
    const bool axis_face = ph.axis_node && d == 1 && j == 1;
    face_flux(G[0], G[1], axis_face ? lb[1] : lb[0], lb[1], nu[0], nu[1], V[0], V[1],
              axis_face ? W[2] : W[0], W[1], W[2], W[3], phys_m, ph, Fm);
    face_flux(G[1], G[2], lb[1], lb[2], nu[1], nu[2], V[1], V[2], W[1], W[2], W[3], W[4], phys_p,
              ph, Fp);
    for (int c = 0; c < 5; ++c) rhs[c] += Fp[c] - Fm[c];
  }
  const T iV = trcp(M[9LL * g.vs + o]);
  const bool axis_row = ph.axis_node && j == 0;   // not advanced
  for (int c = 0; c < 5; ++c) R[(long long)c * g.vs + o] = axis_row ? T(0) : rhs[c] * iV;
}

template <typename T>
hipError_t launch_residual_ref(const T* Q, const T* M, const Grid& g, const Phys<T>& ph, T* PT,
                               T* R, hipStream_t s) {
  const long long n1 = (long long)(g.nx + 2) * (g.nr + 2) * (g.nth + 2);
  hipLaunchKernelGGL(k_point_pass<T>, dim3(blocks_for(n1, 256)), dim3(256), 0, s, Q, M, g, ph, PT);
  if (!R) return hipGetLastError();   // point quantities only
  const long long n = (long long)g.nx * g.nr * g.nth;
  hipLaunchKernelGGL(k_face_pass<T>, dim3(blocks_for(n, 256)), dim3(256), 0, s, Q, M, g, ph, PT, R);
  return hipGetLastError();
}

template hipError_t launch_residual_ref<double>(const double*, const double*, const Grid&,
                                                const Phys<double>&, double*, double*, hipStream_t);
template hipError_t launch_residual_ref<float>(const float*, const float*, const Grid&,
                                               const Phys<float>&, float*, float*, hipStream_t);

}  // namespace lesjet
