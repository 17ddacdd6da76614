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

// The generators write far more than the caches hold and nothing reads it back
// at once: non-temporal stores.  (Ordinary stores leave the caches full of
// dirty lines, and the next kernel's reads then share HBM with their write-
// back: a 20-vector read pass ran 12 % slower right after a 512 MiB fill.)

// counter origin of stream (seed, stream_id)
static uint64_t stream_base(uint64_t seed, uint64_t stream_id) {
  return sm64_mix_host(sm64_mix_host(seed) + stream_id);
}

__global__ void k_fill_uniform(double* out, int64_t n, uint64_t base, double lo, double hi) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(lo + (hi - lo) * u01(base + (uint64_t)i), out + i);
}

__global__ void k_fill_normal(double* out, int64_t n, uint64_t base, uint64_t offset) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(normal_at(base, offset + (uint64_t)i), out + i);
}

// ---------------------------------------------------------------------------
// EM update of a three-component normal mixture's means (Sec. 5.3)
// ---------------------------------------------------------------------------

struct EmArgs {
  const double* x; int64_t N;      // samples
  const double* u;                 // current vector: the means are u[0..2]
  double coef[3];                  // alpha_i / (sqrt(2 pi) sigma_i)
  double inv2s2[3];                // 1 / (2 sigma_i^2)
  double* partials;                // [6][grid]: sum x w_i, then sum w_i
};

constexpr int kEmWG = 256;
constexpr int kEmMaxGrid = 1024;

// Per sample k: p_i = alpha_i / (sqrt(2 pi) sigma_i) exp(-(x_k - mu_i)^2 /
// (2 sigma_i^2)), w_i = p_i / sum_j p_j; each lane accumulates x_k w_i and
// w_i over its samples (grid stride), then one fixed-order reduction per
// workgroup writes the workgroup's six partial sums.
__global__ __launch_bounds__(kEmWG) void k_em_partials(EmArgs a) {
  const double m0 = a.u[0], m1 = a.u[1], m2 = a.u[2];
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t k = (int64_t)blockIdx.x * kEmWG + threadIdx.x; k < a.N;
       k += (int64_t)gridDim.x * kEmWG) {
    const double x = a.x[k];
    const double d0 = x - m0, d1 = x - m1, d2 = x - m2;
    const double p0 = a.coef[0] * exp(-(d0 * d0) * a.inv2s2[0]);
    const double p1 = a.coef[1] * exp(-(d1 * d1) * a.inv2s2[1]);
    const double p2 = a.coef[2] * exp(-(d2 * d2) * a.inv2s2[2]);
    const double tot = p0 + p1 + p2;
    const double w0 = p0 / tot, w1 = p1 / tot, w2 = p2 / tot;
    acc[0] += x * w0;
    acc[1] += x * w1;
    acc[2] += x * w2;
    acc[3] += w0;
    acc[4] += w1;
    acc[5] += w2;
  }
  const double r = multi_reduce<8>(acc);  // lane l < 8: value l over the wave
  __shared__ double s_w[kEmWG / 64][8];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane < 8) s_w[w][lane] = r;
  __syncthreads();
  if (threadIdx.x < 6) {
    double t = 0.0;
    for (int q = 0; q < kEmWG / 64; ++q) t += s_w[q][threadIdx.x];
    a.partials[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

// Every workgroup sums the G partials of the six values in the same fixed
// order (so all agree bit for bit), forms G(mu)_i = sum x w_i / sum w_i and
// writes its share of the replicas: out[3 r + i] = G(mu)_i.
__global__ __launch_bounds__(kEmWG) void k_em_broadcast(const double* __restrict__ partials,
                                                        int G, double* __restrict__ out,
                                                        int64_t nrep) {
  __shared__ double s_g[3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (w == 0) {
    double t[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      double v = 0.0;
      for (int g = lane; g < G; g += 64) v += partials[(size_t)c * G + g];
      t[c] = wave_sum(v);
    }
    if (lane < 3) s_g[lane] = t[lane] / t[lane + 3];
  }
  __syncthreads();
  const double g0 = s_g[0], g1 = s_g[1], g2 = s_g[2];
  for (int64_t r = (int64_t)blockIdx.x * kEmWG + threadIdx.x; r < nrep;
       r += (int64_t)gridDim.x * kEmWG) {
    out[3 * r] = g0;
    out[3 * r + 1] = g1;
    out[3 * r + 2] = g2;
  }
}

hipError_t launch_em(const double alpha[3], const double sigma[3], const double* x, int64_t N,
                     const double* u, double* out, int64_t n, double* work, hipStream_t st) {
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  EmArgs a{};
  a.x = x;
  a.N = N;
  a.u = u;
  for (int i = 0; i < 3; ++i) {
    a.coef[i] = alpha[i] * 0.39894228040143267793994605993438 / sigma[i];
    a.inv2s2[i] = 1.0 / (2.0 * sigma[i] * sigma[i]);
  }
  a.partials = work;
  int64_t g = (N + kEmWG - 1) / kEmWG;
  const int G = (int)(g > kEmMaxGrid ? kEmMaxGrid : g);
  hipLaunchKernelGGL(k_em_partials, dim3(G), dim3(kEmWG), 0, st, a);
  const int64_t nrep = n / 3;
  int64_t gb = (nrep + kEmWG - 1) / kEmWG;
  const int GB = (int)(gb > 2048 ? 2048 : (gb < 1 ? 1 : gb));
  hipLaunchKernelGGL(k_em_broadcast, dim3(GB), dim3(kEmWG), 0, st, work, G, out, nrep);
  return hipGetLastError();
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
