// Internal definitions shared by the lesjet HIP sources: padded layouts,
// physical constants in the compute precision, launch helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lesjet {

constexpr int NG = 2;    // ghost layers of state, metrics and residual arrays
constexpr int NGC = 3;   // ghost layers of the coordinate array

// Padded layout of a field: F[v][k + NG][j + NG][i + NG].  Offsets inside
// one variable fit in 32 bits (checked at context creation); the variable
// stride is applied to 64-bit base pointers.
struct Grid {
  int nx, nr, nth;
  int pitch;        // row pitch in elements
  int plane;        // (nr + 2 NG) * pitch
  int vs;           // (nth + 2 NG) * plane
  __host__ __device__ __forceinline__ int at(int i, int j, int k) const {
    return (k + NG) * plane + (j + NG) * pitch + (i + NG);
  }
};

// Same for the coordinate array (three ghost layers).
struct CGrid {
  int nx, nr, nth;
  int pitch, plane, vs;
  __host__ __device__ __forceinline__ int at(int i, int j, int k) const {
    return (k + NGC) * plane + (j + NGC) * pitch + (i + NGC);
  }
};

// Boundary kinds (values of the public enum les_bc).
enum : int {
  BC_PERIODIC = 0, BC_AXIS = 1, BC_INFLOW = 2, BC_OUTFLOW = 3, BC_FARFIELD = 4, BC_AXIS_NODE = 5
};

// Constants of the discretisation in compute precision T.
template <typename T>
struct Phys {
  T gamma, gm1, igm1;     // gamma, gamma - 1, 1/(gamma - 1)
  T Pr_inv, Prs_inv;      // 1/Pr, 1/Pr_sgs
  T Cv;                   // visc_coef = M/Re
  T suth, suth1;          // S, 1 + S (Sutherland)
  T sgs_coef;             // Smagorinsky Cs^2 / Cv, Vreman 2.5 Cs^2 / Cv, dynamic
                          // C_ds / Cv (eddy viscosity in jet-viscosity units)
  T iso_coef;             // dynamic: (2/3) C_I (isotropic SGS stress), else 0
  T k2, k4;
  int viscous;            // Cv != 0
  int sgs;                // 0 none, 1 Smagorinsky, 2 Vreman, 3 dynamic (sgs_coef,
                          // Prs_inv and iso_coef set per launch from the device)
  int axis_node;          // eta- is a centerline through the mesh nodes j = 0
  int phys_face[3][2];    // face -1/2 / n-1/2 along d is a physical boundary
};

template <typename T>
struct Vec5 { T v[5]; };

// Sizes of the state arrays a kernel touches, per launch.
inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace lesjet
