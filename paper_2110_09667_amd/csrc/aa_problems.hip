// aa_problems.hip -- model fixed-point maps and seeded input generators.
//
// G(u) = u - omega (A u + c u^3 - f), A the (2 dim + 1)-point Dirichlet
// Laplacian on an s^dim grid (x fastest) scaled by 1/h^2: the 1D Poisson,
// 3D nonlinear and 2D batched workloads all use it (dim = 1, 3, 2).
#include <math.h>

#include "aa_passes.h"

namespace aa {

__global__ __launch_bounds__(256) void k_stencil(int dim, int64_t s, double ih2, double omega,
                                                 double c, const double* __restrict__ f,
                                                 const double* __restrict__ u,
                                                 double* __restrict__ out, int64_t n) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x)
    out[p] = stencil_point(u, f, dim, s, ih2, omega, c, p);
}

hipError_t launch_stencil(int dim, int64_t s, double h, double omega, double c,
                          const double* f, const double* u, double* out, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  int64_t n = s;
  if (dim >= 2) n *= s;
  if (dim >= 3) n *= s;
  int64_t blocks = (n + 255) / 256;
  int grid = (int)(blocks < 65536 ? blocks : 65536);
  hipLaunchKernelGGL(k_stencil, dim3(grid), dim3(256), 0, st, dim, s, 1.0 / (h * h), omega, c,
                     f, u, out, n);
  return hipGetLastError();
}

// counter origin of stream (seed, stream_id)
static uint64_t stream_base(uint64_t seed, uint64_t stream_id) {
  return sm64_mix_host(sm64_mix_host(seed) + stream_id);
}

__global__ void k_fill_uniform(double* out, int64_t n, uint64_t base, double lo, double hi) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = lo + (hi - lo) * u01(base + (uint64_t)i);
}

__global__ void k_fill_normal(double* out, int64_t n, uint64_t base, uint64_t offset) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = normal_at(base, offset + (uint64_t)i);
}

hipError_t launch_fill_uniform(double* out, int64_t n, uint64_t seed, uint64_t stream_id,
                               uint64_t offset, double lo, double hi, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  int64_t blocks = (n + 255) / 256;
  int grid = (int)(blocks < 65536 ? blocks : 65536);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_fill_uniform, dim3(grid), dim3(256), 0, st, out, n,
                     stream_base(seed, stream_id) + offset, lo, hi);
  return hipGetLastError();
}

hipError_t launch_fill_normal(double* out, int64_t n, uint64_t seed, uint64_t stream_id,
                              uint64_t offset, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  int64_t blocks = (n + 255) / 256;
  int grid = (int)(blocks < 65536 ? blocks : 65536);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_fill_normal, dim3(grid), dim3(256), 0, st, out, n,
                     stream_base(seed, stream_id), offset);
  return hipGetLastError();
}

}  // namespace aa
