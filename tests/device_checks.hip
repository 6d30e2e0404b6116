// Device-side check library of the fast arithmetic of the kernels (built by
// build.py for gfx950 beside the product library; loaded only by the GPU
// tests).  Evaluates, for each argument x, the functions the kernels use in
// place of the IEEE operations:
//   FP64: nr_rcp (1/x) and nr_sqrt (Newton / Goldschmidt refinements of the
//         hardware estimates), through trcp<double> and tsqrt<double>;
//   FP32: trcp<float>, tsqrt<float>, tcbrt<float> (hardware reciprocal,
//         square root, and exp2(log2(x) / 3)), on (float)x.
// out[0..n) = rcp64, out[n..2n) = sqrt64, out[2n..3n) = rcp32,
// out[3n..4n) = sqrt32, out[4n..5n) = cbrt32 (FP32 results widened).
#include "physics.hpp"

using namespace lesjet;

__global__ void k_fastmath(const double* __restrict__ x, double* __restrict__ out, long long n) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double v = x[t];
  const float f = (float)v;
  out[t] = trcp<double>(v);
  out[n + t] = tsqrt<double>(v);
  out[2 * n + t] = (double)trcp<float>(f);
  out[3 * n + t] = (double)tsqrt<float>(f);
  out[4 * n + t] = (double)tcbrt<float>(f);
}

extern "C" int lesjet_check_fastmath(const double* x, double* out, long long n, void* stream) {
  if (!x || !out || n <= 0) return -1;
  hipLaunchKernelGGL(k_fastmath, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, x, out, n);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}
