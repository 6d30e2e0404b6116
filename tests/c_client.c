/* A plain C client of the library: the jet workload advanced through the
 * C-ABI alone (HIP runtime for device memory, no Python).  Test helper:
 * tests/test_gpu_c_client.py writes the inputs, runs this program, and
 * compares its output with the same steps taken through the Python binding.
 *
 *   c_client IN OUT
 * IN:  int32 nx, nr, nth, nsteps, precision; then FP64 X[nx], R[nr],
 *      TH[nth], the interior state (5, nth, nr, nx) and the entrance
 *      primitives (5, nth, nr).
 * OUT: FP64 dt[nsteps] and the interior state after the steps.
 * Exit status 0 on success, a small positive number naming the failed step
 * otherwise (the library's message on stderr). */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lesjet.h"

static int fail(int code, const char* what, les_ctx* c) {
  fprintf(stderr, "c_client: %s failed: %s\n", what, les_last_error(c));
  return code;
}

int main(int argc, char** argv) {
  FILE* f;
  int32_t hdr[5];
  int nx, nr, nth, nsteps;
  size_t nint, ninf, k, j, i, v;
  double *X, *R, *TH, *Qi, *inflow_h, *Qp_h, *dt_h;
  double *Q_d = NULL, *inflow_d = NULL, *dt_d = NULL;
  les_params p;
  les_ctx* c = NULL;
  int64_t pitch, dims[3], vs;
  if (argc != 3) return 2;
  f = fopen(argv[1], "rb");
  if (!f || fread(hdr, sizeof hdr, 1, f) != 1) return 3;
  nx = hdr[0]; nr = hdr[1]; nth = hdr[2]; nsteps = hdr[3];
  nint = (size_t)5 * nth * nr * nx;
  ninf = (size_t)5 * nth * nr;
  X = malloc(nx * sizeof(double)); R = malloc(nr * sizeof(double));
  TH = malloc(nth * sizeof(double)); Qi = malloc(nint * sizeof(double));
  inflow_h = malloc(ninf * sizeof(double)); dt_h = malloc(nsteps * sizeof(double));
  if (!X || !R || !TH || !Qi || !inflow_h || !dt_h) return 4;
  if (fread(X, sizeof(double), nx, f) != (size_t)nx || fread(R, sizeof(double), nr, f) != (size_t)nr ||
      fread(TH, sizeof(double), nth, f) != (size_t)nth || fread(Qi, sizeof(double), nint, f) != nint ||
      fread(inflow_h, sizeof(double), ninf, f) != ninf)
    return 5;
  fclose(f);

  /* the jet workload's constants */
  memset(&p, 0, sizeof p);
  p.nx = nx; p.nr = nr; p.nth = nth;
  p.bc[0] = LES_BC_INFLOW; p.bc[1] = LES_BC_OUTFLOW; p.bc[2] = LES_BC_AXIS;
  p.bc[3] = LES_BC_FARFIELD; p.bc[4] = LES_BC_PERIODIC; p.bc[5] = LES_BC_PERIODIC;
  p.gamma = 1.4; p.Pr = 0.72; p.Pr_sgs = 0.9; p.visc_coef = 1.4 / 1.5e6;
  p.suth_S = 110.4 / 288.15; p.Cs = 0.148; p.k2 = 0.25; p.k4 = 0.016; p.cfl = 0.5;
  p.rk_alpha[0] = 0.25; p.rk_alpha[1] = 1.0 / 6.0; p.rk_alpha[2] = 0.375;
  p.rk_alpha[3] = 0.5; p.rk_alpha[4] = 1.0;
  p.ref_prim[0] = 1.0; p.ref_prim[1] = 0.05; p.ref_prim[4] = 1.0 / 1.4;
  p.p_exit = 1.0 / 1.4;
  p.sgs_model = LES_SGS_SMAGORINSKY; p.precision = hdr[4]; p.schedule = LES_SCHEDULE_STAGE;

  if (les_layout(&p, &pitch, dims, &vs) != LES_OK) return fail(6, "les_layout", NULL);
  /* the 1-D maps are host memory; the library forms the mesh on the device */
  if (les_init_grid(&c, &p, NULL, X, R, TH, NULL) != LES_OK) return fail(7, "les_init_grid", NULL);
  if (les_metrics(c, NULL, NULL) != LES_OK) return fail(8, "les_metrics", c);

  /* padded state: interior from the input, ghosts filled by the library */
  Qp_h = calloc((size_t)5 * vs, sizeof(double));
  if (!Qp_h) return 4;
  for (v = 0; v < 5; ++v)
    for (k = 0; k < (size_t)nth; ++k)
      for (j = 0; j < (size_t)nr; ++j)
        for (i = 0; i < (size_t)nx; ++i)
          Qp_h[v * vs + ((k + 2) * dims[1] + (j + 2)) * pitch + (i + 2)] =
              Qi[((v * nth + k) * nr + j) * nx + i];
  if (hipMalloc((void**)&Q_d, (size_t)5 * vs * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&inflow_d, ninf * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&dt_d, nsteps * sizeof(double)) != hipSuccess)
    return 9;
  if (hipMemcpy(Q_d, Qp_h, (size_t)5 * vs * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(inflow_d, inflow_h, ninf * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return 10;
  if (les_set_inflow(c, inflow_d, NULL) != LES_OK) return fail(11, "les_set_inflow", c);
  if (les_rk5_step(c, Q_d, nsteps, 0.0, dt_d, NULL) != LES_OK) return fail(12, "les_rk5_step", c);
  if (hipMemcpy(Qp_h, Q_d, (size_t)5 * vs * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(dt_h, dt_d, nsteps * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return 13;
  for (v = 0; v < 5; ++v)
    for (k = 0; k < (size_t)nth; ++k)
      for (j = 0; j < (size_t)nr; ++j)
        for (i = 0; i < (size_t)nx; ++i)
          Qi[((v * nth + k) * nr + j) * nx + i] =
              Qp_h[v * vs + ((k + 2) * dims[1] + (j + 2)) * pitch + (i + 2)];
  f = fopen(argv[2], "wb");
  if (!f || fwrite(dt_h, sizeof(double), nsteps, f) != (size_t)nsteps ||
      fwrite(Qi, sizeof(double), nint, f) != nint)
    return 14;
  fclose(f);
  les_free(c);
  (void)hipFree(Q_d); (void)hipFree(inflow_d); (void)hipFree(dt_d);
  free(X); free(R); free(TH); free(Qi); free(inflow_h); free(Qp_h); free(dt_h);
  return 0;
}
