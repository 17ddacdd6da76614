// aa_problems.hip -- model fixed-point maps and seeded input generators.
//
// G(u) = u - omega (A u + c u^3 - f), A the (2 dim + 1)-point Dirichlet
// Laplacian on an s^dim grid (x fastest) scaled by 1/h^2: the 1D Poisson,
// 3D nonlinear and 2D batched workloads all use it (dim = 1, 3, 2).
#include <math.h>

#include "aa_passes.h"

namespace aa {

// XCD-aware mapping: the hardware hands consecutive workgroups to the 8 XCDs
// in turn, so blockIdx.x % 8 names the XCD.  Each XCD is given one contiguous
// range of logical blocks (in order), so the y- and z-neighbours a workgroup
// reads were loaded by earlier workgroups of the same XCD and are still in
// that XCD's L2 (a z-plane of the 256^3 grid is 512 KiB; the L2 is 4 MiB).
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t q = nb / kXcds, r = nb % kXcds;
  const int64_t x = b % kXcds;
  return x * q + (x < r ? x : r) + b / kXcds;
}

__global__ __launch_bounds__(256) void k_stencil(int dim, int64_t s, double ih2, double omega,
                                                 double c, const double* __restrict__ f,
                                                 const double* __restrict__ u,
                                                 double* __restrict__ out, int64_t n,
                                                 int64_t chunk) {
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t p0 = lb * chunk;
  const int64_t p1 = p0 + chunk < n ? p0 + chunk : n;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x)
    out[p] = stencil_point(u, f, dim, s, ih2, omega, c, p);
}

hipError_t launch_stencil(int dim, int64_t s, double h, double omega, double c,
                          const double* f, const double* u, double* out, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  int64_t n = s;
  if (dim >= 2) n *= s;
  if (dim >= 3) n *= s;
  const int64_t blocks = (n + 255) / 256;
  const int grid = (int)(blocks < 65536 ? blocks : 65536);
  // points per logical block: a multiple of the workgroup size covering n
  const int64_t chunk = ((n + grid - 1) / grid + 255) / 256 * 256;
  hipLaunchKernelGGL(k_stencil, dim3(grid), dim3(256), 0, st, dim, s, 1.0 / (h * h), omega, c,
                     f, u, out, n, chunk);
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
