// Mesh set-up: padded coordinates with three ghost layers, and the metric
// terms J^-1 grad(xi_d) and J^-1 on the padded state box (section
// "Transformation of Coordinates": metric-term and Jacobian equations, the
// eta row taken as the cofactor r_zeta x r_xi).
#include "launch.hpp"

namespace lesjet {

// Interior coordinates of a cylindrical product mesh into the padded
// coordinate array: x = X_i, y = R_j cos(theta_k), z = R_j sin(theta_k).
// tab = X[nx], R[nr], cos(theta)[nth], sin(theta)[nth] (the two tables of
// the angles are formed on the host).
__global__ void k_coord_product(const double* __restrict__ tab, double* __restrict__ C, CGrid g) {
  const double* X = tab;
  const double* R = X + g.nx;
  const double* ct = R + g.nr;
  const double* st = ct + g.nth;
  const long long n = (long long)g.nx * g.nr * g.nth;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t % g.nx);
    const int j = (int)((t / g.nx) % g.nr);
    const int k = (int)(t / ((long long)g.nx * g.nr));
    const int o = g.at(i, j, k);
    C[o] = X[i];
    C[(long long)g.vs + o] = R[j] * ct[k];
    C[2LL * g.vs + o] = R[j] * st[k];
  }
}

// Ghost coordinates along direction `dir` for one (a, b) line.  Fill order
// xi, eta, zeta: xi on the interior of eta/zeta, eta for all xi and the
// interior of zeta, zeta everywhere.
__global__ void k_coord_ghost(double* __restrict__ C, CGrid g, int dir, int lo_kind, int hi_kind,
                              double3 per) {
  const int n[3] = {g.nx, g.nr, g.nth};
  int na, nb, a0, b0;
  if (dir == 0) { na = g.nr; nb = g.nth; a0 = 0; b0 = 0; }
  else if (dir == 1) { na = g.nx + 2 * NGC; nb = g.nth; a0 = -NGC; b0 = 0; }
  else { na = g.nx + 2 * NGC; nb = g.nr + 2 * NGC; a0 = -NGC; b0 = -NGC; }
  const long long tot = (long long)na * nb;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= tot) return;
  const int a = a0 + (int)(t % na);
  const int b = b0 + (int)(t / na);
  const int nd = n[dir];
  auto idx = [&](int s) -> int {   // point with index s along dir
    if (dir == 0) return g.at(s, a, b);
    if (dir == 1) return g.at(a, s, b);
    return g.at(a, b, s);
  };
  const double pv[3] = {per.x, per.y, per.z};
  for (int m = 1; m <= NGC; ++m) {
    for (int c = 0; c < 3; ++c) {
      double* X = C + (long long)c * g.vs;
      // low side
      double lo;
      if (lo_kind == BC_PERIODIC) {
        lo = X[idx(nd - m)] - pv[c];
      } else if (lo_kind == BC_AXIS) {
        // dir == 1: the point across the axis, (i, m-1, k + nth/2)
        const int kk = (b + g.nth / 2) % g.nth;
        lo = X[g.at(a, m - 1, kk)];
      } else if (lo_kind == BC_AXIS_NODE) {
        // dir == 1: the mirror point through the axis node, (i, m, k + nth/2)
        const int kk = (b + g.nth / 2) % g.nth;
        lo = X[g.at(a, m, kk)];
      } else {
        lo = X[idx(0)] + m * (X[idx(0)] - X[idx(1)]);
      }
      X[idx(-m)] = lo;
      double hi;
      if (hi_kind == BC_PERIODIC) {
        hi = X[idx(m - 1)] + pv[c];
      } else {
        hi = X[idx(nd - 1)] + m * (X[idx(nd - 1)] - X[idx(nd - 2)]);
      }
      X[idx(nd - 1 + m)] = hi;
    }
  }
}

// Metrics at every point of the padded state box; T is the storage type.
template <typename T>
__global__ void k_metrics(const double* __restrict__ C, CGrid cg, T* __restrict__ M, Grid g,
                          double* __restrict__ M64) {
  const int NX = g.nx + 2 * NG, NR = g.nr + 2 * NG, NT = g.nth + 2 * NG;
  const long long tot = (long long)NX * NR * NT;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < tot;
       t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t % NX) - NG;
    const int j = (int)((t / NX) % NR) - NG;
    const int k = (int)(t / ((long long)NX * NR)) - NG;
    double r[3][3];   // r[d][c] = d x_c / d xi_d
    for (int c = 0; c < 3; ++c) {
      const double* X = C + (long long)c * cg.vs;
      r[0][c] = 0.5 * (X[cg.at(i + 1, j, k)] - X[cg.at(i - 1, j, k)]);
      r[1][c] = 0.5 * (X[cg.at(i, j + 1, k)] - X[cg.at(i, j - 1, k)]);
      r[2][c] = 0.5 * (X[cg.at(i, j, k + 1)] - X[cg.at(i, j, k - 1)]);
    }
    const double x_xi = r[0][0], y_xi = r[0][1], z_xi = r[0][2];
    const double x_et = r[1][0], y_et = r[1][1], z_et = r[1][2];
    const double x_ze = r[2][0], y_ze = r[2][1], z_ze = r[2][2];
    double m[10];
    m[0] = y_et * z_ze - y_ze * z_et;   // J^-1 xi_x
    m[1] = z_et * x_ze - z_ze * x_et;   // J^-1 xi_y
    m[2] = x_et * y_ze - x_ze * y_et;   // J^-1 xi_z
    m[3] = y_ze * z_xi - y_xi * z_ze;   // J^-1 eta_x
    m[4] = z_ze * x_xi - z_xi * x_ze;   // J^-1 eta_y
    m[5] = x_ze * y_xi - x_xi * y_ze;   // J^-1 eta_z
    m[6] = y_xi * z_et - y_et * z_xi;   // J^-1 zeta_x
    m[7] = z_xi * x_et - z_et * x_xi;   // J^-1 zeta_y
    m[8] = x_xi * y_et - x_et * y_xi;   // J^-1 zeta_z
    m[9] = x_xi * y_et * z_ze + x_et * y_ze * z_xi + x_ze * y_xi * z_et
         - x_xi * y_ze * z_et - x_et * y_xi * z_ze - x_ze * y_et * z_xi;   // J^-1
    const int o = g.at(i, j, k);
    for (int c = 0; c < 10; ++c) M[(long long)c * g.vs + o] = (T)m[c];
    if (M64)
      for (int c = 0; c < 10; ++c) M64[(long long)c * g.vs + o] = m[c];
  }
}

static unsigned grid_stride_blocks(long long n) {
  long long b = (n + 255) / 256;
  return (unsigned)(b > 65536 ? 65536 : (b < 1 ? 1 : b));
}

hipError_t launch_coords(const double* xyz, const double* tab, double* C, const CGrid& cg,
                         const int bc[6], const double period[3][3], hipStream_t s) {
  const long long n = (long long)cg.nx * cg.nr * cg.nth;
  if (xyz) {
    // (3, nth, nr, nx) dense, host or device: one pitched copy per variable
    // and plane (the runtime takes the direction from the addresses)
    for (int c = 0; c < 3; ++c)
      for (int k = 0; k < cg.nth; ++k) {
        const double* src = xyz + (long long)c * n + (long long)k * cg.nx * cg.nr;
        double* dst = C + (long long)c * cg.vs + cg.at(0, 0, k);
        const hipError_t e = hipMemcpy2DAsync(dst, (size_t)cg.pitch * sizeof(double), src,
                                              (size_t)cg.nx * sizeof(double),
                                              (size_t)cg.nx * sizeof(double), (size_t)cg.nr,
                                              hipMemcpyDefault, s);
        if (e != hipSuccess) return e;
      }
  } else {
    hipLaunchKernelGGL(k_coord_product, dim3(grid_stride_blocks(n)), dim3(256), 0, s, tab, C, cg);
  }
  for (int d = 0; d < 3; ++d) {
    long long lines;
    if (d == 0) lines = (long long)cg.nr * cg.nth;
    else if (d == 1) lines = (long long)(cg.nx + 2 * NGC) * cg.nth;
    else lines = (long long)(cg.nx + 2 * NGC) * (cg.nr + 2 * NGC);
    const double3 per = make_double3(period[d][0], period[d][1], period[d][2]);
    hipLaunchKernelGGL(k_coord_ghost, dim3(blocks_for(lines, 256)), dim3(256), 0, s, C, cg, d,
                       bc[2 * d], bc[2 * d + 1], per);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_metrics(const double* C, const CGrid& cg, T* M, const Grid& g, double* M64,
                          hipStream_t s) {
  const long long n = (long long)(g.nx + 2 * NG) * (g.nr + 2 * NG) * (g.nth + 2 * NG);
  hipLaunchKernelGGL(k_metrics<T>, dim3(grid_stride_blocks(n)), dim3(256), 0, s, C, cg, M, g, M64);
  return hipGetLastError();
}

template hipError_t launch_metrics<double>(const double*, const CGrid&, double*, const Grid&,
                                           double*, hipStream_t);
template hipError_t launch_metrics<float>(const double*, const CGrid&, float*, const Grid&,
                                          double*, hipStream_t);

}  // namespace lesjet
