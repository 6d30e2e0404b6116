// Fused residual / Runge-Kutta stage kernel (section "Spatial
// Discretization" with the stage update of eq. localdt as an epilogue).
//
// Work decomposition (2.5-D): a block of Tile<T>::X x Tile<T>::Y threads
// owns a ring-1 tile of (i, j) columns and marches along k over a chunk of
// planes.  For each plane kk it
//   (a) writes the state and primitives of the plane (ring-2 tile, two-point
//       halo for the fourth differences) to LDS,
//   (b) computes the point quantities G^d, lambda_bar^d, nu^d of every
//       ring-1 column, with in-plane neighbours from LDS and the kk-1, kk+1
//       neighbours from the thread's own registers, and publishes the xi and
//       eta ones in LDS,
//   (c) evaluates the in-plane faces i - 1/2 and j - 1/2 of each column from
//       LDS and publishes their fluxes; after a barrier each interior column
//       takes its flux differences from LDS and forms the zeta face kk-1/2
//       from registers (point quantities of plane kk-1 are kept from the
//       previous iteration), which completes R at plane kk-1.
// Every point quantity of a ring-1 column is computed once per plane, every
// face flux once.  HBM traffic per interior point and stage: Q (in), the 10
// metric arrays, Q^(0) and the output, the halos coming from L2.
//
// Epilogues: EPI_R writes R; EPI_RK writes Q^(l) = Q^(0) - alpha dt R
// (accumulated in FP64, stored in the stage type); EPI_RK_LAST also writes
// Q^(n+1) in FP64 and reduces max(lambda_xi + lambda_eta + lambda_zeta) of
// the new state for the next step's dt.
#pragma once

#include "launch.hpp"
#include "physics.hpp"
#include "plane_io.hpp"

namespace lesjet {

// Tile shape per precision (threads along i and j of a ring-1 tile):
// FP64 16 x 16 (LDS 79 KB, two blocks per CU), FP32 32 x 8 (LDS 40 KB, four
// blocks per CU); both measured fastest among 64x8, 32x8 and 16x16 on the
// jet meshes.
template <typename T> struct Tile;
template <> struct Tile<double> { static constexpr int X = 16, Y = 16, PER_CU = 2; };
template <> struct Tile<float> { static constexpr int X = 32, Y = 8, PER_CU = 4; };

constexpr int NPQ = 8;                // G(5), lambda_bar, nu, V per direction

enum { EPI_R = 0, EPI_RK = 1, EPI_RK_LAST = 2 };

// Global memory is addressed plane by plane (plane_io.hpp): one 32-bit
// offset register per column serves every variable and plane of the march.

// Byte offset of a column a thread reads: outside the padded box the nearest
// point of it (finite data that no output uses; clamping instead of a
// default value spares the moves that would set the default before every
// load).
template <typename T>
__device__ __forceinline__ unsigned q_col(const Grid& g, int i, int j) {
  return col_off<T>(g, min(max(i, -NG), g.nx + NG - 1), min(max(j, -NG), g.nr + NG - 1));
}

template <typename T>
__device__ __forceinline__ void load_q(const T* Q, const Grid& g, unsigned col, int k, T q[5]) {
#pragma unroll
  for (int c = 0; c < 5; ++c) q[c] = gld(Q, g, c, k, col);
}

template <typename T>
__device__ __forceinline__ void load_metrics(const T* M, const Grid& g, unsigned col, int k,
                                             T m[10]) {
#pragma unroll
  for (int c = 0; c < 10; ++c) m[c] = gld(M, g, c, k, col);
}

// Workgroups are dealt to the eight XCDs (each with its own L2) in turn.  The
// hardware id is remapped so that XCD x receives a contiguous run of tiles,
// i fastest, then j, then the k-chunk: tiles that share halos run at the
// same time on the same L2.
constexpr int NXCD = 8;

struct TileMap {
  int gx, gy, gz;       // tiles along i, j and k-chunks
  int per_xcd;          // ceil(gx gy gz / NXCD)
};

// The FP64 kernel has registers left at two waves per SIMD: it loads Q^(0)
// of the output point an iteration ahead (FP32 at 128 VGPRs does not, nor
// the FP64 last stage, whose registers carry metric terms instead).
template <typename T> struct PrefetchQ0 { static constexpr bool on = sizeof(T) == 8; };

// The last stage of a step evaluates the next step's CFL sum at its output
// point, which needs that point's metric terms, loaded two planes earlier
// and no longer in L2 (reloading them cost the FP64 kernel 10 ms, a sixth
// of the stage, on 1e9 points).  The stage carries them from the previous
// plane in registers instead: FP64 frees the registers by loading Q^(0) and
// the next plane's border where they are used rather than ahead; FP32 runs
// that stage at three waves per SIMD (at four it spills).

// Wave priority: the FP64 kernel (two waves per SIMD, bound by latency)
// raises its waves' issue priority from the face phase to the end of the
// epilogue, so that a wave that has its plane in LDS finishes the plane and
// reaches the next plane's loads ahead of the waves still in the point
// phase.  Measured on MI355X: 10 % less time per launch on the 5.9 M-point
// jet (one round of blocks, two per CU for the whole launch), about 2 % on
// meshes of 0.1 to 1 billion points; the FP32 kernel, bound by its ALUs,
// gains nothing from it.
template <typename T> struct WavePrio { static constexpr bool on = sizeof(T) == 8; };

// Register budget: FP64 two waves per SIMD (up to 256 VGPRs), FP32 four
// (128), three (168) in the last stage.
template <typename T> struct FusedOcc;
template <> struct FusedOcc<double> { static constexpr int waves = 2; };
template <> struct FusedOcc<float> { static constexpr int waves = 4; };
template <typename T, int EPI> struct FusedOccE { static constexpr int waves = FusedOcc<T>::waves; };
template <> struct FusedOccE<float, EPI_RK_LAST> { static constexpr int waves = 3; };

// AXIS: the eta- face is a centerline through mesh nodes (row j = 0 on the
// axis); a separate instance so that the common case carries none of it.
// LAG: viscosity schedule (LAG_NONE; LAG_WRITE also stores mu + mu_sgs and
// the conductivity of every point the block evaluates into `visc`, two
// padded variables; LAG_READ takes them from there).  The tiling is the same
// in every stage, so the points read are those written; points shared by
// two blocks are written twice with the same value.
template <typename T, int EPI, bool AXIS, int LAG, bool DYN>
__global__ void __launch_bounds__(Tile<T>::X * Tile<T>::Y, (FusedOccE<T, EPI>::waves))
k_fused(const T* __restrict__ Qin, const T* __restrict__ M, Grid g, Phys<T> ph_arg, int kc,
        TileMap tm, T* out, const double* Q0, double* Q64, double alpha,
        const double* __restrict__ dtp, Phys<double> ph64, unsigned long long* __restrict__ maxbits,
        T* __restrict__ visc, const double* __restrict__ dyn) {
  Phys<T> ph = ph_arg;
  if (DYN) {   // dynamic model: coefficients of this state, from the device
    ph.sgs_coef = (T)dyn[0];
    ph.Prs_inv = (T)dyn[1];
    ph.iso_coef = (T)dyn[2];
  }
  constexpr int FB_X = Tile<T>::X;              // threads along i (ring-1 columns)
  constexpr int FB_Y = Tile<T>::Y;              // threads along j
  constexpr int FT_X = FB_X - 2;                // interior outputs along i
  constexpr int FT_Y = FB_Y - 2;                // interior outputs along j
  constexpr int FR_X = FB_X + 2;                // ring-2 tile
  constexpr int FR_Y = FB_Y + 2;
  constexpr int NBORDER = FR_X * FR_Y - FB_X * FB_Y;   // ring-2 points without a thread
  // plane state and primitives (one buffer: a second would save a barrier
  // per plane but costs a resident block per CU in either precision)
  __shared__ T sQ[5][FR_Y][FR_X];
  __shared__ T sP[5][FR_Y][FR_X];
  __shared__ T sX[NPQ][FB_Y][FB_X];
  __shared__ T sE[NPQ][FB_Y][FB_X];
  // fluxes of the faces i - 1/2 (xi) and j - 1/2 (eta) of each column: each
  // in-plane face is evaluated once, by the column on its + side, and read
  // by both neighbours (evaluating it from both sides cost 11-14 % more time
  // in FP64 and the registers of a fourth FP32 block per CU)
  __shared__ T sFx[5][FB_Y][FB_X];
  __shared__ T sFe[5][FB_Y][FB_X];
  __shared__ double sRed[(FB_X * FB_Y + 63) / 64];

  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * FB_X + tx;
  const int hw = blockIdx.x;
  const int tile = (hw % NXCD) * tm.per_xcd + hw / NXCD;
  if (tile >= tm.gx * tm.gy * tm.gz) return;          // uniform for the block
  const int bx = tile % tm.gx;
  const int by = (tile / tm.gx) % tm.gy;
  const int bz = tile / (tm.gx * tm.gy);
  const int i0 = bx * FT_X, j0 = by * FT_Y;
  const int k0 = bz * kc;
  const int k1 = min(k0 + kc, g.nth);
  const int i = i0 - 1 + tx, j = j0 - 1 + ty;
  const bool col_ok = i >= -1 && i <= g.nx && j >= -1 && j <= g.nr;   // needed ring-1 column
  const bool interior = tx >= 1 && tx <= FT_X && ty >= 1 && ty <= FT_Y && i < g.nx && j < g.nr;
  // columns that evaluate their xi face i - 1/2 / eta face j - 1/2
  const bool xface = tx >= 1 && ty >= 1 && ty <= FT_Y && i <= g.nx && j < g.nr;
  const bool eface = ty >= 1 && tx >= 1 && tx <= FT_X && j <= g.nr && i < g.nx;

  // ring-2 border point handled by this thread (if tid < NBORDER)
  const bool has_b = tid < NBORDER;
  int brx = 0, bry = 0;
  if (tid < FR_X) { bry = 0; brx = tid; }
  else if (tid < 2 * FR_X) { bry = FR_Y - 1; brx = tid - FR_X; }
  else { const int r = tid - 2 * FR_X; bry = 1 + (r >> 1); brx = (r & 1) ? FR_X - 1 : 0; }
  const int bi = i0 - 2 + brx, bj = j0 - 2 + bry;
  // Byte offsets within a plane of the own column and of the border point.
  // Every column that produces or feeds an output lies in the padded box,
  // where the clamp is the identity, so oq is also the offset of the output
  // point; the columns beyond [-1, n] read metrics and held viscosities of
  // ghost columns, whose point quantities no face uses.  oq64: the same
  // column in the FP64 arrays (Q^(0), Q^(n+1)).
  const unsigned oq = q_col<T>(g, i, j), oob = q_col<T>(g, bi, bj);
  const unsigned oq64 = sizeof(T) == 8 ? oq : 2u * oq;

  const bool axis_row = AXIS && j == 0;      // centerline row (not advanced)
  const bool axis_face = AXIS && j == 1;     // face j - 1/2 is the axis face
  // physical-boundary faces i - 1/2 and j - 1/2 of this column (the face
  // i - 1/2 of column i = nx is the face nx - 1/2)
  const bool phys_xf = (i == 0 && ph.phys_face[0][0]) || (i == g.nx && ph.phys_face[0][1]);
  const bool phys_ef = (j == 0 && ph.phys_face[1][0]) || (j == g.nr && ph.phys_face[1][1]);

  // ---- rolling column state ------------------------------------------------
  // The state and primitives of the current plane kk live in LDS once phase
  // (a) has written them; registers carry only what the march needs next.
  T Wa[5], Wb[5];        // W at kk-2, kk-1 (zeta fourth difference)
  T Qd[5], Pd[5];        // Q and (u, v, w, T, p) at kk+1
  T Pb[5];               // (u, v, w, T, p) at kk-1
  T Qn[5];               // Q at kk+2, in flight
  T met[10], metn[10];   // metrics at (i, j, kk) and the prefetch for kk+1
  T lag[2], lagn[2];     // held (mu + mu_sgs, conductivity), same planes (LAG_READ)
  constexpr bool CS = EPI == EPI_RK_LAST;        // metric terms carried (above)
  constexpr bool DEFER = CS && sizeof(T) == 8;    // loads deferred to free registers
  constexpr bool PQ0 = EPI != EPI_R && !CS && PrefetchQ0<T>::on;
  // the own column two planes ahead is loaded at the top of the iteration
  // in FP64 stages 1-4, after the point phase elsewhere (measured: the FP64
  // last stage 2 % and FP32 stages 1 % faster, FP64 stages 1-4 4 % slower)
  constexpr bool LATE_QN = sizeof(T) == 4 || CS;
  double q0p[5];         // Q^(0) at (i, j, kk-1), loaded at the top of iteration kk
  const double ad_pre = PQ0 ? alpha * (*dtp) : 0.0;
  auto load_lag = [&](int kk, T v[2]) {
    // columns beyond [-1, n] read the nearest held column (all of [-1, n]^3
    // is written at stage 1); no output uses them
    v[0] = gld(visc, g, 0, kk, oq);
    v[1] = gld(visc, g, 1, kk, oq);
  };
  // zeta-face state of plane kk-1 (interior columns)
  T Gz[5], lbz = 0, nuz = 0, Vz = 0;
  T acc[5];              // RHS at kk-1 without its zeta face kk-1/2:
                         // in-plane faces minus the zeta face kk-3/2
  double lmax = 0.0;
  T Sp[9];               // last stage: metric terms of plane kk-1

  {
    T q[5], pc[5];
    load_q(Qin, g, oq, k0 - 2, q);
    prim5(q, ph, Pb);                    // primitives at kk-1 = k0-2
#pragma unroll
    for (int c = 0; c < 5; ++c) Wa[c] = q[c];
    Wa[4] += Pb[4];
    load_q(Qin, g, oq, k0 - 1, q);       // plane kk = k0-1 of the own column
    prim5(q, ph, pc);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      sQ[c][ty + 1][tx + 1] = q[c];
      sP[c][ty + 1][tx + 1] = pc[c];
    }
    load_q(Qin, g, oq, k0, Qd);
    prim5(Qd, ph, Pd);
    load_metrics(M, g, oq, k0 - 1, met);
    if (LAG == LAG_READ) load_lag(k0 - 1, lag);
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) { Wb[c] = Wa[c]; Gz[c] = 0; acc[c] = 0; }

  if (has_b) {                           // border of the first plane
    T bq[5], bp[5];
    load_q(Qin, g, oob, k0 - 1, bq);
    prim5(bq, ph, bp);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      sQ[c][bry][brx] = bq[c];
      sP[c][bry][brx] = bp[c];
    }
  }

  for (int kk = k0 - 1; kk <= k1; ++kk) {
    const bool more = kk < k1;
    // metric loads of the next plane (and, early, the own column two planes
    // ahead), in flight during (b)
    if (more) {
      if (!LATE_QN && kk + 2 <= k1 + 1) load_q(Qin, g, oq, kk + 2, Qn);
      load_metrics(M, g, oq, kk + 1, metn);
      if (LAG == LAG_READ) load_lag(kk + 1, lagn);
    }
    if (PQ0 && interior && kk - 1 >= k0) {
#pragma unroll
      for (int c = 0; c < 5; ++c) q0p[c] = gld(Q0, g, c, kk - 1, oq64);
    }
    // (a) plane kk is in LDS (written before the loop or at the end of the
    // previous iteration)
    __syncthreads();

    // (b) point quantities at (i, j, kk)
    PointIn<T> in;
    PointOut<T> po;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      in.q[c] = sQ[c][ty + 1][tx + 1];
      in.pr[c] = sP[c][ty + 1][tx + 1];
    }
    {
      T m[5], pl[5];
#pragma unroll
      for (int f = 0; f < 5; ++f) { m[f] = sP[f][ty + 1][tx]; pl[f] = sP[f][ty + 1][tx + 2]; }
      neighbour_terms(m, pl, in.pr[4], in.dl[0], in.nu[0]);
#pragma unroll
      for (int f = 0; f < 5; ++f) { m[f] = sP[f][ty][tx + 1]; pl[f] = sP[f][ty + 2][tx + 1]; }
      neighbour_terms(m, pl, in.pr[4], in.dl[1], in.nu[1]);
      neighbour_terms(Pb, Pd, in.pr[4], in.dl[2], in.nu[2]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int c = 0; c < 3; ++c) in.S[d][c] = met[3 * d + c];
    in.V = met[9];
    if (LAG == LAG_READ) { in.mt = lag[0]; in.kap = lag[1]; }
    point_quantities<T, LAG, DYN>(in, ph, po);
    if (LAG == LAG_WRITE && col_ok && ph.viscous) {
      gst(visc, g, 0, kk, oq, po.mt);
      gst(visc, g, 1, kk, oq, po.kap);
    }
    if (AXIS && axis_row) {
      // centerline through the nodes: S^eta = 0 on the axis, so the eta
      // point flux vanishes (its viscous part, singular at V = 0, is not used)
#pragma unroll
      for (int c = 0; c < 5; ++c) po.G[1][c] = T(0);
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      sX[c][ty][tx] = po.G[0][c];
      sE[c][ty][tx] = po.G[1][c];
    }
    sX[5][ty][tx] = po.lb[0];
    sX[6][ty][tx] = po.nu[0];
    sX[7][ty][tx] = in.V;
    sE[5][ty][tx] = po.lb[1];
    sE[6][ty][tx] = po.nu[1];
    sE[7][ty][tx] = in.V;
    // border of the next plane, in flight during the face phase
    T Bn[5];
    if (!DEFER && more && has_b) load_q(Qin, g, oob, kk + 1, Bn);
    if (LATE_QN && more && kk + 2 <= k1 + 1) load_q(Qin, g, oq, kk + 2, Qn);
    __syncthreads();

    // (c) faces
    if (WavePrio<T>::on) __builtin_amdgcn_s_setprio(1);
    auto wload = [&](int yy, int xx, T w[5]) {      // W = Q with E replaced by E + p
#pragma unroll
      for (int c = 0; c < 4; ++c) w[c] = sQ[c][yy][xx];
      w[4] = sQ[4][yy][xx] + sP[4][yy][xx];
    };
    if (kk >= k0 && kk < k1) {
      // in-plane faces of the output planes, one per column and direction
      T Wm[5], Wl[5], Wr[5], Wp[5], F[5], GA[5], GB[5];
      if (xface) {
        wload(ty + 1, tx - 1, Wm); wload(ty + 1, tx, Wl); wload(ty + 1, tx + 1, Wr);
        wload(ty + 1, tx + 2, Wp);
#pragma unroll
        for (int c = 0; c < 5; ++c) { GA[c] = sX[c][ty][tx - 1]; GB[c] = sX[c][ty][tx]; }
        face_flux(GA, GB, sX[5][ty][tx - 1], sX[5][ty][tx], sX[6][ty][tx - 1], sX[6][ty][tx],
                  sX[7][ty][tx - 1], sX[7][ty][tx], Wm, Wl, Wr, Wp, phys_xf, ph, F);
#pragma unroll
        for (int c = 0; c < 5; ++c) sFx[c][ty][tx] = F[c];
      }
      if (eface) {
        // axis face: lambda_bar of row 1 and the three-point fourth
        // difference W(2) - 4 W(1) + 3 W(0), i.e. the standard formula with
        // W(-1) replaced by W(1); done by choosing the rows read
        const int rm = AXIS && axis_face ? ty + 1 : ty - 1;
        const int rl = AXIS && axis_face ? ty : ty - 1;
        wload(rm, tx + 1, Wm); wload(ty, tx + 1, Wl); wload(ty + 1, tx + 1, Wr);
        wload(ty + 2, tx + 1, Wp);
#pragma unroll
        for (int c = 0; c < 5; ++c) { GA[c] = sE[c][ty - 1][tx]; GB[c] = sE[c][ty][tx]; }
        face_flux(GA, GB, sE[5][rl][tx], sE[5][ty][tx], sE[6][ty - 1][tx], sE[6][ty][tx],
                  sE[7][ty - 1][tx], sE[7][ty][tx], Wm, Wl, Wr, Wp, phys_ef, ph, F);
#pragma unroll
        for (int c = 0; c < 5; ++c) sFe[c][ty][tx] = F[c];
      }
    }
    __syncthreads();
    if (interior && kk >= k0) {
      const bool emit = kk - 1 >= k0;       // R at (i, j, kk-1) completes here
      // flux differences of the in-plane faces (output planes only)
      T rhs[5] = {0, 0, 0, 0, 0};
      if (kk < k1) {
#pragma unroll
        for (int c = 0; c < 5; ++c)
          rhs[c] = sFx[c][ty][tx + 1] - sFx[c][ty][tx] + sFe[c][ty + 1][tx] - sFe[c][ty][tx];
      }
      // zeta face kk-1/2: L = kk-1 (registers), R = kk
      T Wc[5], Wd[5], Fk[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) { Wc[c] = sQ[c][ty + 1][tx + 1]; Wd[c] = Qd[c]; }
      Wc[4] += sP[4][ty + 1][tx + 1];
      Wd[4] += Pd[4];
      face_flux(Gz, po.G[2], lbz, po.lb[2], nuz, po.nu[2], Vz, in.V, Wa, Wb, Wc, Wd, false, ph, Fk);
      if (emit) {
        // the epilogue's loads ahead of its stores (the compiler cannot order
        // buffer accesses of different arrays by itself): Q^(0) of the output
        // point (loaded an iteration ahead where registers allow) and, at the
        // last stage, its metric terms for the next step's dt (carried in
        // registers from the previous plane)
        double q0[5], S[3][3];
        if (EPI != EPI_R) {
#pragma unroll
          for (int c = 0; c < 5; ++c) q0[c] = PQ0 ? q0p[c] : gld(Q0, g, c, kk - 1, oq64);
        }
        if (EPI == EPI_RK_LAST) {
#pragma unroll
          for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int c = 0; c < 3; ++c) S[d][c] = (double)Sp[3 * d + c];
        }
        const T iV = trcp(Vz);
        T R[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) R[c] = AXIS && axis_row ? T(0) : (acc[c] + Fk[c]) * iV;
        if (EPI == EPI_R) {
#pragma unroll
          for (int c = 0; c < 5; ++c) gst(out, g, c, kk - 1, oq, R[c]);
        } else {
          const double ad = PQ0 ? ad_pre : alpha * (*dtp);
          double qn[5];
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            qn[c] = q0[c] - ad * (double)R[c];
            gst(out, g, c, kk - 1, oq, (T)qn[c]);
            if (EPI == EPI_RK_LAST && Q64) gst(Q64, g, c, kk - 1, oq64, qn[c]);
          }
          if (EPI == EPI_RK_LAST) {
            const double x = lambda_sum(qn, S, (double)Vz, ph64);
            if (!(AXIS && axis_row) && (x != x || x > lmax)) lmax = x;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 5; ++c) acc[c] = rhs[c] - Fk[c];
    }
    if (WavePrio<T>::on) __builtin_amdgcn_s_setprio(0);
    // keep the zeta-direction point quantities of plane kk, roll the window
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      Gz[c] = po.G[2][c];
      Wa[c] = Wb[c];
      Wb[c] = sQ[c][ty + 1][tx + 1];     // own state of plane kk, re-read from LDS
      Pb[c] = sP[c][ty + 1][tx + 1];
    }
    Wb[4] += Pb[4];
    lbz = po.lb[2];
    nuz = po.nu[2];
    Vz = in.V;
    // plane kk is read by other threads until the barrier after the face
    // fluxes; what follows reads only the thread's own column, which the
    // next plane's border writes never touch
    if (more) {
      // plane kk+1 goes to LDS: own column and ring-2 border
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        sQ[c][ty + 1][tx + 1] = Qd[c];
        sP[c][ty + 1][tx + 1] = Pd[c];
        Qd[c] = Qn[c];
      }
      if (has_b) {
        if (DEFER) load_q(Qin, g, oob, kk + 1, Bn);
        T bp[5];
        prim5(Bn, ph, bp);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          sQ[c][bry][brx] = Bn[c];
          sP[c][bry][brx] = bp[c];
        }
      }
      prim5(Qd, ph, Pd);
      if (CS) {
#pragma unroll
        for (int c = 0; c < 9; ++c) Sp[c] = met[c];
      }
#pragma unroll
      for (int c = 0; c < 10; ++c) met[c] = metn[c];
      if (LAG == LAG_READ) { lag[0] = lagn[0]; lag[1] = lagn[1]; }
    }
  }

  if (EPI == EPI_RK_LAST) {
    // block max of the lambda sums, then one integer atomic per block
    double v = lmax;
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(v, off, 64);
      if (o != o || o > v) v = o;
    }
    if ((tid & 63) == 0) sRed[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double b = sRed[0];
      for (int w = 1; w < (FB_X * FB_Y + 63) / 64; ++w)
        if (sRed[w] != sRed[w] || sRed[w] > b) b = sRed[w];
      atomicMax(maxbits, (unsigned long long)__double_as_longlong(b));
    }
  }
}

template <typename T>
int fused_chunk(const Grid& g, int num_cu) {
  constexpr int FT_X = Tile<T>::X - 2, FT_Y = Tile<T>::Y - 2;
  num_cu *= Tile<T>::PER_CU;          // resident blocks (the FP32 last stage, at
                                      // three per CU, takes the same length)
  const long long tiles = (long long)((g.nx + FT_X - 1) / FT_X) * ((g.nr + FT_Y - 1) / FT_Y);
  // pick the chunk length that minimises (rounds of resident blocks) x (planes per block),
  // over every length from 4 planes to the cap (lengths that divide the
  // azimuth leave no short last chunk: against powers of two only, 5.6 % on
  // the 128 x 128 x 360 mesh and 3.1 % on 1700 x 1700 x 360 in FP64, 1.4-1.6 %
  // in FP32, 0.5 % on 1250 x 640 x 1250).
  // FP32 (four blocks per CU) stops at 16 planes: longer chunks measured
  // slower on large meshes (4 % at 1e8 points, 8 % at 1e9), the resident
  // blocks of a round drifting apart in k and sharing fewer halo lines in
  // L2.  FP64 (two blocks per CU) takes 64 planes when that fits one round
  // (the 5.9 M-point mesh: 4 % faster than 32) and at most 32 otherwise:
  // the same time within 1 % on 1e8 and 1e9 points, with 12 % (32) to 21 %
  // (16) fewer bytes crossing the L2 boundary than with 64.
  const auto choose = [&](int kc_max, long long* rounds_out) {
    int best = g.nth;
    long long best_rounds = 0;
    double best_cost = 1e300;
    for (int kc = 4; kc <= kc_max; ++kc) {
      const long long nb = tiles * ((g.nth + kc - 1) / kc);
      const long long rounds = (nb + num_cu - 1) / num_cu;
      const double cost = (double)rounds * (kc + 2);
      if (cost < best_cost) { best_cost = cost; best = kc; best_rounds = rounds; }
    }
    *rounds_out = best_rounds;
    return best;
  };
  long long rounds = 0;
  if (sizeof(T) == 4) return choose(16, &rounds);
  const int kc64 = choose(64, &rounds);
  return rounds <= 1 ? kc64 : choose(32, &rounds);
}

template <typename T>
hipError_t launch_fused(const T* Q, const T* M, const Grid& g, const Phys<T>& ph, int kc, int epi,
                        T* out, const double* Q0, double* Q64, double alpha, const double* dt,
                        const Phys<double>& ph64, unsigned long long* maxbits, int lag, T* visc,
                        const double* dyn, hipStream_t s) {
  if (ph.sgs == 3 && !dyn) return hipErrorInvalidValue;
  // instances: LAG_NONE with every epilogue, LAG_WRITE with EPI_RK (stage 1),
  // LAG_READ with EPI_RK and EPI_RK_LAST (stages 2-5)
  if (lag != LAG_NONE && (!visc || epi == EPI_R || (lag == LAG_WRITE && epi != EPI_RK)))
    return hipErrorInvalidValue;
  constexpr int FT_X = Tile<T>::X - 2, FT_Y = Tile<T>::Y - 2;
  TileMap tm;
  tm.gx = (g.nx + FT_X - 1) / FT_X;
  tm.gy = (g.nr + FT_Y - 1) / FT_Y;
  tm.gz = (g.nth + kc - 1) / kc;
  const long long ntiles = (long long)tm.gx * tm.gy * tm.gz;
  tm.per_xcd = (int)((ntiles + NXCD - 1) / NXCD);
  const dim3 grid((unsigned)(tm.per_xcd * NXCD));
  const dim3 block(Tile<T>::X, Tile<T>::Y, 1);
#define LESJET_FUSED(E, A, L)                                                          \
  do {                                                                                 \
    if (ph.sgs == 3)                                                                   \
      hipLaunchKernelGGL((k_fused<T, E, A, L, true>), grid, block, 0, s, Q, M, g, ph, kc, tm, \
                         out, Q0, Q64, alpha, dt, ph64, maxbits, visc, dyn);           \
    else                                                                               \
      hipLaunchKernelGGL((k_fused<T, E, A, L, false>), grid, block, 0, s, Q, M, g, ph, kc, tm, \
                         out, Q0, Q64, alpha, dt, ph64, maxbits, visc, dyn);           \
  } while (0)
#define LESJET_FUSED_EPI(A)                                                        \
  if (lag == LAG_WRITE) LESJET_FUSED(EPI_RK, A, LAG_WRITE);                        \
  else if (lag == LAG_READ) {                                                      \
    if (epi == EPI_RK) LESJET_FUSED(EPI_RK, A, LAG_READ);                          \
    else LESJET_FUSED(EPI_RK_LAST, A, LAG_READ);                                   \
  } else if (epi == EPI_R) LESJET_FUSED(EPI_R, A, LAG_NONE);                       \
  else if (epi == EPI_RK) LESJET_FUSED(EPI_RK, A, LAG_NONE);                       \
  else LESJET_FUSED(EPI_RK_LAST, A, LAG_NONE);
  if (ph.axis_node) {
    LESJET_FUSED_EPI(true)
  } else {
    LESJET_FUSED_EPI(false)
  }
#undef LESJET_FUSED_EPI
#undef LESJET_FUSED
  return hipGetLastError();
}

}  // namespace lesjet
