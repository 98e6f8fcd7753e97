// Device twin of the synthetic line generator (see linegen_core.h): one thread per line.
#include <hip/hip_runtime.h>
#include "linegen_core.h"

__global__ void lg_kernel(lg_recipe r, uint64_t seed, int64_t i0, int64_t count,
                          double* __restrict__ nu, double* __restrict__ S, double* __restrict__ E,
                          double* __restrict__ g, double* __restrict__ n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  double a, b, c, d, e;
  lg_line(&r, seed, (uint64_t)(i0 + k), &a, &b, &c, &d, &e);
  nu[k] = a; S[k] = b; E[k] = c; g[k] = d; n[k] = e;
}

extern "C" int lg_generate_device(const lg_recipe* r, uint64_t seed, int64_t i0, int64_t count,
                                  double* nu, double* S, double* E, double* g, double* n,
                                  hipStream_t stream) {
  if (count <= 0) return 0;
  const int threads = 256;
  int64_t blocks = (count + threads - 1) / threads;
  hipLaunchKernelGGL(lg_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream,
                     *r, seed, i0, count, nu, S, E, g, n);
  return (int)hipGetLastError();
}
