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

// dim >= 2: one workgroup per tile of TY consecutive grid rows (y0 .. y0+TY-1
// at one z), its threads along x: the tile's coordinates come from one scalar
// division per workgroup instead of three 64-bit divisions per point (256^3:
// 151 -> 142 us).  Same arithmetic, in the same order, as stencil_point.
// Tiles of 4, 8 or 16 rows (more y neighbours found in the workgroup's own
// reads) measured no faster in 3D and slower in 2D (fewer workgroups), so a
// tile is one row.  f and the output are streamed non-temporally
// (AA_STENCIL_NT, default on: 142 -> 136 us at 256^3, 112 -> 104 us in 2D).
#ifndef AA_STENCIL_TY
#define AA_STENCIL_TY 1
#endif
#ifndef AA_STENCIL_NT
#define AA_STENCIL_NT 1
#endif
constexpr int kStencilTY = AA_STENCIL_TY;

__global__ __launch_bounds__(256) void k_stencil_tile(int dim, int s, double ih2, double omega,
                                                      double c, const double* __restrict__ f,
                                                      const double* __restrict__ u,
                                                      double* __restrict__ out, int ntile_y) {
  const int b = blockIdx.x;
  const int z = b / ntile_y, y0 = (b % ntile_y) * kStencilTY;  // z = 0 in 2D
  const int64_t s2 = (int64_t)s * s;
  for (int ty = 0; ty < kStencilTY; ++ty) {
    const int y = y0 + ty;
    if (y >= s) break;
    const int64_t base = (int64_t)z * s2 + (int64_t)y * s;
    for (int x = threadIdx.x; x < s; x += blockDim.x) {
      const int64_t p = base + x;
      const double up = u[p];
      double nb = 0.0;
      if (x > 0) nb += u[p - 1];
      if (x < s - 1) nb += u[p + 1];
      if (y > 0) nb += u[p - s];
      if (y < s - 1) nb += u[p + s];
      if (dim >= 3) {
        if (z > 0) nb += u[p - s2];
        if (z < s - 1) nb += u[p + s2];
      }
      const double au = (2.0 * dim * up - nb) * ih2;
#if AA_STENCIL_NT
      __builtin_nontemporal_store(up - omega * (au + c * up * up * up - __builtin_nontemporal_load(f + p)), out + p);
#else
      out[p] = up - omega * (au + c * up * up * up - f[p]);
#endif
    }
  }
}

hipError_t launch_stencil(int dim, int64_t s, double h, double omega, double c,
                          const double* f, const double* u, double* out, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  int64_t n = s;
  if (dim >= 2) n *= s;
  if (dim >= 3) n *= s;
  if (dim >= 2 && s <= 65536) {
    const int64_t ntile_y = (s + kStencilTY - 1) / kStencilTY;
    const int64_t nwg = ntile_y * (dim >= 3 ? s : 1);
    hipLaunchKernelGGL(k_stencil_tile, dim3((unsigned)nwg), dim3(s < 256 ? (s + 63) / 64 * 64 : 256),
                       0, st, dim, (int)s, 1.0 / (h * h), omega, c, f, u, out, (int)ntile_y);
    return hipGetLastError();
  }
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
