// aa_pde2d.hip -- fixed-point maps of the paper's 2D test problems: the
// steady heat equation with a nonlinear term (Sec. 5.1, both terms) and the
// Bratu problem (Sec. 5.2).  Each evaluation G(u) = A^{-1} rhs(u) solves a
// Poisson system, A = -L_h the 5-point Dirichlet Laplacian on an N x N
// interior grid (x fastest, h = 1 / (N + 1)), by the preconditioned conjugate
// gradient with one geometric-multigrid V(1,1) cycle as the preconditioner:
// red-black Gauss-Seidel (red then black before the coarse correction, black
// then red after it, so the cycle is symmetric), full weighting, bilinear
// interpolation, coarse point I at fine point 2 I + 1, and coarse operators
// whose last row and column keep the boundary at its true distance h (the
// 1D Galerkin products; diagonal 1 + 2^level in units of 1/H^2).
//
// Layout and launches.  Every level's vectors are N_l x N_l row-major
// arrays in the workspace.  Levels of more than 32 points per side run as
// grid-wide kernels with one thread per point (rows across blockIdx.y, x
// across threads: neighbour loads are coalesced, no divisions); the levels
// from 32 points down run in one kernel of one workgroup with every array in
// LDS.  A PCG iteration is 4 launches per grid-wide level, the coarse
// kernel and 2 vector kernels; the whole working set at N = 1024 (~60 MB)
// stays in the Infinity Cache, so the launches are latency bound.
//
// Reductions (r.z, p.q, r.r): each workgroup stores its partial sum, and
// every workgroup of the kernel that needs the value sums all partials itself
// in one fixed order (the same value everywhere, deterministic).  No device-
// scope fence (on gfx950 a release fence writes the whole L2 back: with one
// per workgroup the vector kernels took 28 us instead of ~10) and no
// finalize launch.  The stopping test runs on the device at the start of each
// iteration; once it holds, every later kernel returns at once, so the host
// may enqueue iterations ahead and read the state only now and then.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "aa_device.h"

namespace aa {
namespace pde {

constexpr int kBX = 256;           // threads per workgroup of the grid-wide kernels
constexpr int kMaxWG = 1024;       // workgroups of a grid-wide kernel (partials)
constexpr int kCoarseN = 32;       // levels of at most this many points per side in LDS
constexpr int kCoarseWG = 1024;    // threads of the coarse kernel
constexpr int kCoarseLds = 3 * (1024 + 256 + 64 + 16 + 4 + 1);
constexpr int kMaxLevels = 32;

// integer state words
enum : int { I_DONE = 0, I_ITERS = 1, I_CONV = 2, I_COUNT = 64 };
// scalar slots: r.r of the right-hand side, rho of the previous iteration
enum : int { S_RR0 = 0, S_RHO_PREV = 1, S_COUNT = 8 };

struct Lev {
  int N;
  double H2;     // spacing squared
  double dlast;  // last diagonal entry of the level's 1D operator, times H^2
  double* r;     // right-hand side (level 0: the PCG residual)
  double* e;     // pre-smoothed correction
  double* z;     // post-smoothed correction (the cycle's output on the level)
};

struct Pcg {
  double* sc;        // S_RR0, S_RHO_PREV
  int* ist;          // I_DONE, I_ITERS, I_CONV
  double* p_rr;      // partials of r.r (k_init, k_update), kMaxWG each
  double* p_rho;     // partials of r.z (the cycle's last kernel on the fine grid)
  double* p_pq;      // partials of p.q (k_dir)
  int np_fine;       // partials of the fine-grid vector kernels (their workgroups)
  int np_rho;        // partials of r.z: np_fine, or 1 from the coarse kernel
  double tol2;
  int max_iter;
  int fixed;         // >= 0: exactly this many iterations
};

// --------------------------------------------------------------------------
// point operations (shared by the grid-wide kernels and the LDS kernel)
// --------------------------------------------------------------------------

__device__ __forceinline__ double diag_at(int i, int j, int N, double dl) {
  return ((i == N - 1) ? dl : 2.0) + ((j == N - 1) ? dl : 2.0);
}

// sum of the four neighbours (zero outside), left, right, below, above
__device__ __forceinline__ double nb_sum(const double* u, int i, int j, int N) {
  const int64_t p = (int64_t)j * N + i;
  const double l = i > 0 ? u[p - 1] : 0.0;
  const double r = i < N - 1 ? u[p + 1] : 0.0;
  const double d = j > 0 ? u[p - N] : 0.0;
  const double a = j < N - 1 ? u[p + N] : 0.0;
  return ((l + r) + d) + a;
}

// red pre-smoothing from a zero start at red point (i, j)
__device__ __forceinline__ double red0(const double* r, int i, int j, int N, double H2,
                                       double dl) {
  return H2 * r[(int64_t)j * N + i] / diag_at(i, j, N, dl);
}

// pre-smoothing (red then black Gauss-Seidel from E = 0) at (i, j)
__device__ __forceinline__ double pre_point(const double* r, int i, int j, int N, double H2,
                                            double dl) {
  if (((i + j) & 1) == 0) return red0(r, i, j, N, H2, dl);
  const double l = i > 0 ? red0(r, i - 1, j, N, H2, dl) : 0.0;
  const double rt = i < N - 1 ? red0(r, i + 1, j, N, H2, dl) : 0.0;
  const double d = j > 0 ? red0(r, i, j - 1, N, H2, dl) : 0.0;
  const double a = j < N - 1 ? red0(r, i, j + 1, N, H2, dl) : 0.0;
  return (H2 * r[(int64_t)j * N + i] + (((l + rt) + d) + a)) / diag_at(i, j, N, dl);
}

// residual r - A e at (i, j); zero outside the grid
__device__ __forceinline__ double res_point(const double* r, const double* e, int i, int j,
                                            int N, double H2, double dl) {
  if (i < 0 || j < 0 || i >= N || j >= N) return 0.0;
  const int64_t p = (int64_t)j * N + i;
  return r[p] - (diag_at(i, j, N, dl) * e[p] - nb_sum(e, i, j, N)) / H2;
}

// full weighting of the residual at coarse point (I, J): along x, then y
__device__ __forceinline__ double restrict_point(const double* r, const double* e, int I, int J,
                                                 int N, double H2, double dl) {
  const int ic = 2 * I + 1, jc = 2 * J + 1;
  double row[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int j = jc - 1 + t;
    row[t] = 0.5 * res_point(r, e, ic - 1, j, N, H2, dl) + res_point(r, e, ic, j, N, H2, dl) +
             0.5 * res_point(r, e, ic + 1, j, N, H2, dl);
  }
  return (0.5 * row[0] + row[1] + 0.5 * row[2]) / 4.0;
}

// bilinear interpolation of the coarse correction (Nc per side) at fine (i, j):
// along x, then y; coarse index -1 is the boundary
__device__ __forceinline__ double interp_x(const double* ec, int i, int J, int Nc) {
  const double* row = ec + (int64_t)J * Nc;
  if (i & 1) return row[(i - 1) >> 1];
  const int I = i >> 1;
  return (I > 0 ? 0.5 * row[I - 1] : 0.0) + 0.5 * row[I];
}

__device__ __forceinline__ double interp_point(const double* ec, int i, int j, int Nc) {
  if (j & 1) return interp_x(ec, i, (j - 1) >> 1, Nc);
  const int J = j >> 1;
  return (J > 0 ? 0.5 * interp_x(ec, i, J - 1, Nc) : 0.0) + 0.5 * interp_x(ec, i, J, Nc);
}

// corrected pre-smoothed value e + P e_c at (i, j) (ec null: no correction)
__device__ __forceinline__ double corr_at(const double* e, const double* ec, int i, int j, int N,
                                          int Nc) {
  const double v = e[(int64_t)j * N + i];
  return ec ? v + interp_point(ec, i, j, Nc) : v;
}

// after the coarse correction: red points e + P e_c; black points their
// Gauss-Seidel value from the corrected red neighbours
__device__ __forceinline__ double post_black_point(const double* r, const double* e,
                                                   const double* ec, int i, int j, int N, int Nc,
                                                   double H2, double dl) {
  if (((i + j) & 1) == 0) return corr_at(e, ec, i, j, N, Nc);
  const double l = i > 0 ? corr_at(e, ec, i - 1, j, N, Nc) : 0.0;
  const double rt = i < N - 1 ? corr_at(e, ec, i + 1, j, N, Nc) : 0.0;
  const double d = j > 0 ? corr_at(e, ec, i, j - 1, N, Nc) : 0.0;
  const double a = j < N - 1 ? corr_at(e, ec, i, j + 1, N, Nc) : 0.0;
  return (H2 * r[(int64_t)j * N + i] + (((l + rt) + d) + a)) / diag_at(i, j, N, dl);
}

// the final red half-sweep at red point (i, j) from the black values in z
__device__ __forceinline__ double post_red_point(const double* r, const double* z, int i, int j,
                                                 int N, double H2, double dl) {
  return (H2 * r[(int64_t)j * N + i] + nb_sum(z, i, j, N)) / diag_at(i, j, N, dl);
}

// --------------------------------------------------------------------------
// reductions: each workgroup stores its sum; the consumers add the partials
// in index order (per thread, then the fixed tree of block_sum)
// --------------------------------------------------------------------------

__device__ double block_sum(double v, double* lds4) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds4[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) s += lds4[k];
  return s;
}

// this workgroup's sum of v, stored as its partial
__device__ void partial_store(double v, double* parts) {
  __shared__ double lds[16];
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) parts[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// the sum of np partials, in one fixed order (every workgroup gets the same)
__device__ double sum_parts(const double* parts, int np) {
  __shared__ double lds[16];
  double acc = 0.0;
  for (int k = threadIdx.x; k < np; k += blockDim.x) acc += parts[k];
  return block_sum(acc, lds);
}

// The stopping test before iteration k (every workgroup decides alike; the
// first records it, and at k = 0 keeps r.r of the right-hand side).  Returns
// true when the solve has ended.
__device__ __forceinline__ bool pcg_check(const Pcg& a, int k) {
  if (a.ist[I_DONE]) return true;
  const double rr = sum_parts(a.p_rr, a.np_fine);
  const double rr0 = k == 0 ? rr : a.sc[S_RR0];
  if (k == 0 && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) a.sc[S_RR0] = rr;
  bool stop;
  int conv;
  if (a.fixed >= 0) {
    stop = k >= a.fixed;
    conv = 1;
  } else {
    conv = rr <= a.tol2 * rr0;
    stop = conv || k >= a.max_iter;
  }
  if (stop && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    a.ist[I_DONE] = 1;
    a.ist[I_ITERS] = k;
    a.ist[I_CONV] = conv;
  }
  return stop;
}

// --------------------------------------------------------------------------
// grid-wide level kernels: thread (x, row) over points (i, j), rows strided
// --------------------------------------------------------------------------

#define PDE_ROWS(N) for (int j = blockIdx.y; j < (N); j += gridDim.y)
#define PDE_COLS(N) for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < (N); i += gridDim.x * blockDim.x)

__global__ __launch_bounds__(kBX) void k_pre(Lev L, Pcg a, int k, int check) {
  if (check ? pcg_check(a, k) : a.ist[I_DONE] != 0) return;
  PDE_ROWS(L.N) PDE_COLS(L.N) L.e[(int64_t)j * L.N + i] = pre_point(L.r, i, j, L.N, L.H2, L.dlast);
}

__global__ __launch_bounds__(kBX) void k_restrict(Lev L, Lev C, Pcg a) {
  if (a.ist[I_DONE]) return;
  PDE_ROWS(C.N) PDE_COLS(C.N)
    C.r[(int64_t)j * C.N + i] = restrict_point(L.r, L.e, i, j, L.N, L.H2, L.dlast);
}

__global__ __launch_bounds__(kBX) void k_post_black(Lev L, const double* ec, int Nc, Pcg a) {
  if (a.ist[I_DONE]) return;
  PDE_ROWS(L.N) PDE_COLS(L.N)
    L.z[(int64_t)j * L.N + i] = post_black_point(L.r, L.e, ec, i, j, L.N, Nc, L.H2, L.dlast);
}

// final red half-sweep; on level 0 also rho_k = r . z
__global__ __launch_bounds__(kBX) void k_post_red(Lev L, Pcg a, int k, int dot) {
  if (a.ist[I_DONE]) return;
  double acc = 0.0;
  PDE_ROWS(L.N) PDE_COLS(L.N) {
    const int64_t p = (int64_t)j * L.N + i;
    double zv;
    if (((i + j) & 1) == 0) {
      zv = post_red_point(L.r, L.z, i, j, L.N, L.H2, L.dlast);
      L.z[p] = zv;
    } else {
      zv = L.z[p];
    }
    if (dot) acc = fma(L.r[p], zv, acc);
  }
  if (dot) partial_store(acc, a.p_rho);
}

// --------------------------------------------------------------------------
// the levels from 32 points per side down: one workgroup, arrays in LDS
// --------------------------------------------------------------------------

struct CoarseArgs {
  const double* r_in;  // right-hand side of the first coarse level (global)
  double* z_out;       // its post-smoothed correction (global)
  int N[kMaxLevels];   // sizes of the coarse levels
  double H2[kMaxLevels];
  double dl[kMaxLevels];
  int nlev;
};

__global__ __launch_bounds__(kCoarseWG) void k_coarse(CoarseArgs c, Pcg a, int k, int check,
                                                      int dot) {
  if (check ? pcg_check(a, k) : a.ist[I_DONE] != 0) return;
  __shared__ double buf[kCoarseLds];
  __shared__ int sN[kMaxLevels], soff[kMaxLevels];
  __shared__ double sH2[kMaxLevels], sdl[kMaxLevels];
  const int t = threadIdx.x, nt = blockDim.x;
  if (t == 0) {
    int off = 0;
    for (int l = 0; l < c.nlev; ++l) {
      sN[l] = c.N[l];
      sH2[l] = c.H2[l];
      sdl[l] = c.dl[l];
      soff[l] = off;
      off += 3 * c.N[l] * c.N[l];
    }
  }
  __syncthreads();
  // level l: right-hand side R(l), pre-smoothed E(l), post-smoothed Z(l)
#define R_(l) (buf + soff[l])
#define E_(l) (buf + soff[l] + sN[l] * sN[l])
#define Z_(l) (buf + soff[l] + 2 * sN[l] * sN[l])
  for (int p = t; p < sN[0] * sN[0]; p += nt) R_(0)[p] = c.r_in[p];
  __syncthreads();
  for (int l = 0; l < c.nlev; ++l) {
    const int N = sN[l];
    for (int p = t; p < N * N; p += nt) E_(l)[p] = pre_point(R_(l), p % N, p / N, N, sH2[l], sdl[l]);
    __syncthreads();
    if (l + 1 < c.nlev) {
      const int Nc = sN[l + 1];
      for (int p = t; p < Nc * Nc; p += nt)
        R_(l + 1)[p] = restrict_point(R_(l), E_(l), p % Nc, p / Nc, N, sH2[l], sdl[l]);
      __syncthreads();
    }
  }
  for (int l = c.nlev - 1; l >= 0; --l) {
    const int N = sN[l];
    const double* ec = l + 1 < c.nlev ? Z_(l + 1) : nullptr;
    const int Nc = l + 1 < c.nlev ? sN[l + 1] : 0;
    for (int p = t; p < N * N; p += nt)
      Z_(l)[p] = post_black_point(R_(l), E_(l), ec, p % N, p / N, N, Nc, sH2[l], sdl[l]);
    __syncthreads();
    for (int p = t; p < N * N; p += nt) {
      const int i = p % N, j = p / N;
      if (((i + j) & 1) == 0) Z_(l)[p] = post_red_point(R_(l), Z_(l), i, j, N, sH2[l], sdl[l]);
    }
    __syncthreads();
  }
  double acc = 0.0;
  for (int p = t; p < sN[0] * sN[0]; p += nt) {
    c.z_out[p] = Z_(0)[p];
    if (dot) acc = fma(R_(0)[p], Z_(0)[p], acc);
  }
#undef R_
#undef E_
#undef Z_
  if (dot) partial_store(acc, a.p_rho);
}

// --------------------------------------------------------------------------
// PCG vector kernels (level 0)
// --------------------------------------------------------------------------

__device__ __forceinline__ double c_term(int problem, double u) {
  if (problem == AA_PDE_HEAT_NL1) {
    const double eu = exp(u);
    const double d = u - eu;
    return u + u * eu + u * exp(-u) + d * d;
  }
  return 100.0 * (u - u * u);  // AA_PDE_HEAT_NL2
}

// r = rhs(u) (heat: c(u) - b; Bratu: lambda e^u; plain solve: d_rhs), x = 0,
// r.r; resets the solve state
__global__ __launch_bounds__(kBX) void k_init(int problem, double lambda, const double* b,
                                              const double* u, double* x, double* r, int N,
                                              Pcg a) {
  double acc = 0.0;
  PDE_ROWS(N) PDE_COLS(N) {
    const int64_t p = (int64_t)j * N + i;
    double v;
    if (problem == AA_PDE_BRATU) v = lambda * exp(u[p]);
    else if (problem == 0) v = u[p];
    else v = c_term(problem, u[p]) - b[p];
    r[p] = v;
    x[p] = 0.0;
    acc = fma(v, v, acc);
  }
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    a.ist[I_DONE] = 0;
    a.ist[I_ITERS] = 0;
    a.ist[I_CONV] = 0;
  }
  partial_store(acc, a.p_rr);
}

// p = z + beta p_prev (beta = rho_k / rho_{k-1}; p = z at k = 0), q = A p, p.q
__global__ __launch_bounds__(kBX) void k_dir(const double* z, const double* p_prev,
                                             double* p_cur, double* q, int N, double ih2, Pcg a,
                                             int k) {
  if (a.ist[I_DONE]) return;
  const bool first = k == 0;
  const double rho = sum_parts(a.p_rho, a.np_rho);
  const double beta = first ? 0.0 : rho / a.sc[S_RHO_PREV];
  double acc = 0.0;
  PDE_ROWS(N) PDE_COLS(N) {
    const int64_t p = (int64_t)j * N + i;
#define PN(o) (first ? z[o] : z[o] + beta * p_prev[o])
    const double pc = PN(p);
    const double l = i > 0 ? PN(p - 1) : 0.0;
    const double rt = i < N - 1 ? PN(p + 1) : 0.0;
    const double d = j > 0 ? PN(p - N) : 0.0;
    const double up = j < N - 1 ? PN(p + N) : 0.0;
#undef PN
    const double qv = (4.0 * pc - (((l + rt) + d) + up)) * ih2;
    p_cur[p] = pc;
    q[p] = qv;
    acc = fma(pc, qv, acc);
  }
  partial_store(acc, a.p_pq);
}

// alpha = rho_k / (p.q); x += alpha p; r -= alpha q; r.r -> rr[k + 1]
__global__ __launch_bounds__(kBX) void k_update(const double* p_cur, const double* q, double* x,
                                                double* r, int N, Pcg a, int k) {
  if (a.ist[I_DONE]) return;
  const double rho = sum_parts(a.p_rho, a.np_rho);
  const double alpha = rho / sum_parts(a.p_pq, a.np_fine);
  // rho_k for the next iteration's beta (k_dir read the previous one already)
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) a.sc[S_RHO_PREV] = rho;
  double acc = 0.0;
  PDE_ROWS(N) PDE_COLS(N) {
    const int64_t p = (int64_t)j * N + i;
    x[p] = fma(alpha, p_cur[p], x[p]);
    const double rv = fma(-alpha, q[p], r[p]);
    r[p] = rv;
    acc = fma(rv, rv, acc);
  }
  partial_store(acc, a.p_rr);
}

__global__ void k_reset(int* ist) {
  if (threadIdx.x < I_COUNT) ist[threadIdx.x] = 0;
}

#undef PDE_ROWS
#undef PDE_COLS

}  // namespace pde
}  // namespace aa

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

using namespace aa::pde;

struct aa_pde2d {
  int N;
  int problem;
  double lambda, tol;
  int max_iter, fixed;
  hipStream_t st;
  int nlev, first_coarse;  // levels >= first_coarse run in k_coarse
  Lev lev[kMaxLevels];
  double *r, *z, *e0, *p[2], *q, *sc, *p_rr, *p_rho, *p_pq;
  int* ist;
  int last_iters, last_conv, predicted;
};

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// sizes of the hierarchy: halve while even; the coarse part must fit one
// workgroup's LDS (the first size of at most 32 points per side is reached)
int hierarchy(int64_t N, int* sizes) {
  int L = 0;
  int64_t n = N;
  while (true) {
    if (L >= kMaxLevels) return -1;
    sizes[L++] = (int)n;
    if (n % 2 != 0) break;
    n /= 2;
  }
  return L;
}

int first_coarse_level(const int* sizes, int L) {
  for (int l = 0; l < L; ++l)
    if (sizes[l] <= kCoarseN) return l;
  return -1;
}

size_t layout(int64_t N, int max_iter, const int* sizes, int L, aa_pde2d* c, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const size_t n = (size_t)N * (size_t)N;
  (void)max_iter;
  int* ist = (int*)take(I_COUNT * sizeof(int));
  double* sc = (double*)take(S_COUNT * sizeof(double));
  double* p_rr = (double*)take(kMaxWG * sizeof(double));
  double* p_rho = (double*)take(kMaxWG * sizeof(double));
  double* p_pq = (double*)take(kMaxWG * sizeof(double));
  double* r = (double*)take(n * 8);
  double* z = (double*)take(n * 8);
  double* e0 = (double*)take(n * 8);
  double* p0 = (double*)take(n * 8);
  double* p1 = (double*)take(n * 8);
  double* q = (double*)take(n * 8);
  if (c) {
    c->ist = ist;
    c->sc = sc;
    c->p_rr = p_rr;
    c->p_rho = p_rho;
    c->p_pq = p_pq;
    c->r = r;
    c->z = z;
    c->e0 = e0;
    c->p[0] = p0;
    c->p[1] = p1;
    c->q = q;
  }
  const double h = 1.0 / (double)(N + 1);
  for (int l = 0; l < L; ++l) {
    const size_t nl = (size_t)sizes[l] * (size_t)sizes[l];
    double *lr = r, *le = e0, *lz = z;
    if (l > 0) {
      lr = (double*)take(nl * 8);
      le = (double*)take(nl * 8);
      lz = (double*)take(nl * 8);
    }
    if (c) {
      const double H = h * (double)(1ll << l);
      c->lev[l] = Lev{sizes[l], H * H, 1.0 + (double)(1ll << l), lr, le, lz};
    }
  }
  return off;
}

dim3 grid_for(int N) {
  const int gx = (N + kBX - 1) / kBX;
  int gy = kMaxWG / gx;
  if (gy < 1) gy = 1;
  if (gy > N) gy = N;
  return dim3((unsigned)gx, (unsigned)gy);
}

dim3 block_for(int N) {
  const int bx = N >= kBX ? kBX : ((N + 63) / 64) * 64;
  return dim3((unsigned)bx);
}

Pcg pcg_args(const aa_pde2d* c) {
  Pcg a;
  a.sc = c->sc;
  a.ist = c->ist;
  a.p_rr = c->p_rr;
  a.p_rho = c->p_rho;
  a.p_pq = c->p_pq;
  const dim3 g = grid_for(c->N);
  a.np_fine = (int)(g.x * g.y);
  a.np_rho = c->first_coarse == 0 ? 1 : a.np_fine;  // r.z from the coarse kernel
  a.tol2 = c->tol * c->tol;
  a.max_iter = c->max_iter;
  a.fixed = c->fixed;
  return a;
}

// one V-cycle on r (level 0) into z; `check` runs the stopping test before
// iteration k in the first kernel, `dot` stores rho_k = r . z
hipError_t launch_vcycle(const aa_pde2d* c, const Pcg& a, int k, int check, int dot) {
  const int fc = c->first_coarse;
  for (int l = 0; l < fc; ++l) {
    const Lev& L = c->lev[l];
    hipLaunchKernelGGL(k_pre, grid_for(L.N), block_for(L.N), 0, c->st, L, a, k, check && l == 0);
    const Lev& Cl = c->lev[l + 1];
    hipLaunchKernelGGL(k_restrict, grid_for(Cl.N), block_for(Cl.N), 0, c->st, L, Cl, a);
  }
  CoarseArgs ca;
  memset(&ca, 0, sizeof(ca));
  ca.r_in = c->lev[fc].r;
  ca.z_out = c->lev[fc].z;
  ca.nlev = c->nlev - fc;
  for (int l = fc; l < c->nlev; ++l) {
    ca.N[l - fc] = c->lev[l].N;
    ca.H2[l - fc] = c->lev[l].H2;
    ca.dl[l - fc] = c->lev[l].dlast;
  }
  hipLaunchKernelGGL(k_coarse, dim3(1), dim3(kCoarseWG), 0, c->st, ca, a, k, check && fc == 0,
                     dot && fc == 0);
  for (int l = fc - 1; l >= 0; --l) {
    const Lev& L = c->lev[l];
    const Lev& Cl = c->lev[l + 1];
    hipLaunchKernelGGL(k_post_black, grid_for(L.N), block_for(L.N), 0, c->st, L,
                       (const double*)Cl.z, Cl.N, a);
    hipLaunchKernelGGL(k_post_red, grid_for(L.N), block_for(L.N), 0, c->st, L, a, k,
                       dot && l == 0);
  }
  return hipGetLastError();
}

hipError_t launch_iteration(const aa_pde2d* c, const Pcg& a, int k, double* x) {
  hipError_t e = launch_vcycle(c, a, k, 1, 1);
  if (e != hipSuccess) return e;
  const int N = c->N;
  const double h = 1.0 / (double)(N + 1);
  double* pc = c->p[k & 1];
  const double* pp = c->p[(k + 1) & 1];
  hipLaunchKernelGGL(k_dir, grid_for(N), block_for(N), 0, c->st, (const double*)c->z, pp, pc,
                     c->q, N, 1.0 / (h * h), a, k);
  hipLaunchKernelGGL(k_update, grid_for(N), block_for(N), 0, c->st, (const double*)pc,
                     (const double*)c->q, x, c->r, N, a, k);
  return hipGetLastError();
}

aa_status hipst(hipError_t e) { return e == hipSuccess ? AA_OK : AA_EHIP; }

// the PCG solve of A x = rhs(problem, u): enqueue iterations, read the state
// now and then (a first batch sized by the previous solve)
aa_status solve(aa_pde2d* c, int problem, const double* b, const double* u, double* x) {
  (void)hipGetLastError();
  const Pcg a = pcg_args(c);
  const int N = c->N;
  hipLaunchKernelGGL(k_init, grid_for(N), block_for(N), 0, c->st, problem, c->lambda, b, u, x,
                     c->r, N, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return AA_EHIP;
  const int last = c->fixed >= 0 ? c->fixed : c->max_iter;
  int k = 0;
  int batch = c->predicted + 1;
  int st[3] = {0, 0, 0};
  while (true) {
    for (int t = 0; t < batch && k <= last; ++t, ++k) {
      e = launch_iteration(c, a, k, x);
      if (e != hipSuccess) return AA_EHIP;
    }
    e = hipMemcpyAsync(st, c->ist, sizeof(st), hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) return AA_EHIP;
    if (st[I_DONE]) break;
    if (k > last) return AA_EHIP;  // not reached: the test before iteration `last` stops
    batch = 2;
  }
  c->last_iters = st[I_ITERS];
  c->last_conv = st[I_CONV];
  c->predicted = st[I_ITERS];
  return AA_OK;
}

}  // namespace

extern "C" {

aa_status aa_pde2d_workspace_size(int64_t N, int max_iter, size_t* bytes) {
  if (!bytes || N < 1 || N > 65536 || max_iter < 1 || max_iter > 100000) return AA_EINVAL;
  int sizes[kMaxLevels];
  const int L = hierarchy(N, sizes);
  if (L < 1 || first_coarse_level(sizes, L) < 0) return AA_EINVAL;
  *bytes = layout(N, max_iter, sizes, L, nullptr, nullptr);
  return AA_OK;
}

aa_status aa_pde2d_init(aa_pde2d** ctx, int64_t N, int problem, double lambda, double tol,
                        int max_iter, void* d_workspace, size_t bytes, void* stream) {
  if (!ctx) return AA_EINVAL;
  *ctx = nullptr;
  if (problem != AA_PDE_HEAT_NL1 && problem != AA_PDE_HEAT_NL2 && problem != AA_PDE_BRATU)
    return AA_EINVAL;
  if (!(tol >= 0.0) || !isfinite(lambda) || !d_workspace || ((uintptr_t)d_workspace & 255))
    return AA_EINVAL;
  size_t need = 0;
  aa_status s = aa_pde2d_workspace_size(N, max_iter, &need);
  if (s != AA_OK) return s;
  if (bytes < need) return AA_ENOSPACE;
  aa_pde2d* c = (aa_pde2d*)calloc(1, sizeof(aa_pde2d));
  if (!c) return AA_EINVAL;
  c->N = (int)N;
  c->problem = problem;
  c->lambda = lambda;
  c->tol = tol;
  c->max_iter = max_iter;
  c->fixed = -1;
  c->st = (hipStream_t)stream;
  int sizes[kMaxLevels];
  c->nlev = hierarchy(N, sizes);
  c->first_coarse = first_coarse_level(sizes, c->nlev);
  layout(N, max_iter, sizes, c->nlev, c, (char*)d_workspace);
  c->predicted = 8;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, c->st, c->ist);
  if (hipGetLastError() != hipSuccess) {
    free(c);
    return AA_EHIP;
  }
  *ctx = c;
  return AA_OK;
}

aa_status aa_pde2d_set_iters(aa_pde2d* c, int iters) {
  if (!c || iters < -1 || iters > c->max_iter) return AA_EINVAL;
  c->fixed = iters;
  return AA_OK;
}

aa_status aa_pde2d_apply(aa_pde2d* c, const double* d_b, const double* d_u, double* d_out) {
  if (!c || !d_u || !d_out) return AA_EINVAL;
  if (c->problem != AA_PDE_BRATU && !d_b) return AA_EINVAL;
  return solve(c, c->problem, d_b, d_u, d_out);
}

aa_status aa_pde2d_solve(aa_pde2d* c, const double* d_rhs, double* d_x) {
  if (!c || !d_rhs || !d_x) return AA_EINVAL;
  return solve(c, 0, nullptr, d_rhs, d_x);
}

aa_status aa_pde2d_vcycle(aa_pde2d* c, const double* d_r, double* d_z) {
  if (!c || !d_r || !d_z) return AA_EINVAL;
  (void)hipGetLastError();
  const size_t n = (size_t)c->N * (size_t)c->N;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, c->st, c->ist);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(c->r, d_r, n * 8, hipMemcpyDeviceToDevice, c->st);
  if (e == hipSuccess) e = launch_vcycle(c, pcg_args(c), 0, 0, 0);
  if (e == hipSuccess) e = hipMemcpyAsync(d_z, c->z, n * 8, hipMemcpyDeviceToDevice, c->st);
  return hipst(e);
}

aa_status aa_pde2d_last(const aa_pde2d* c, int* h_iters, int* h_converged) {
  if (!c) return AA_EINVAL;
  if (h_iters) *h_iters = c->last_iters;
  if (h_converged) *h_converged = c->last_conv;
  return AA_OK;
}

aa_status aa_pde2d_set_stream(aa_pde2d* c, void* stream) {
  if (!c) return AA_EINVAL;
  c->st = (hipStream_t)stream;
  return AA_OK;
}

aa_status aa_pde2d_destroy(aa_pde2d* c) {
  free(c);
  return AA_OK;
}

}  // extern "C"
