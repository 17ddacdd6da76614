// aa_mlp.hip -- the mixing-weight network of the learned-guarded AA step.
//
// 230 -> 256 -> 256 -> 256 -> 21 (padded to 256 in / 64 out), GELU (erf form),
// BF16 operands on the matrix cores with FP32 accumulation, FP32 master
// weights, Adam.  Everything is a dense contraction here, so every product is
// one LDS-tiled GEMM on gfx950's v_mfma_f32_16x16x32_bf16 (64 x 64 tile per
// workgroup, one 16-row strip per wave, K in steps of 32: half the MFMA
// issues and LDS passes of the 16-deep form); operand strides let the same kernel compute
// the forward products, the input gradients (times W^T) and the weight
// gradients (H^T times dZ).  The network is small and latency-bound.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <new>
#include <vector>

#include "aa_device.h"

namespace aa {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Operand and result layout of v_mfma_f32_16x16x32_bf16: lane l supplies
// A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16], e < 8, and
// register r of its result holds D[mfma_row(l, r)][l % 16].
__device__ __forceinline__ int mfma_row(int lane, int r) { return 4 * (lane >> 4) + r; }

struct GemmArgs {
  const uint16_t* a; int64_t sa0, sa1;  // A(m, k) = a[m sa0 + k sa1]
  const uint16_t* b; int64_t sb0, sb1;  // B(k, n) = b[k sb0 + n sb1]
  float* c; int64_t ldc;                // C(m, n) = c[m ldc + n]
  const float* bias;                    // added per column (may be null)
  int M, N, K;
  int accumulate;                       // C += A B instead of C = A B (+ bias)
};

constexpr int GT = 64;   // tile edge
constexpr int GK = 32;   // K step of one MFMA
constexpr int GKP = 40;  // LDS row stride (bf16 elements) of the K-major tiles: 80 bytes,
                         // 16-byte aligned rows for the 8-element operand reads

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[GT * GKP];  // [m][k]
  __shared__ __align__(16) uint16_t Bs[GT * GKP];  // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  v4f acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += GK) {
#pragma unroll
    for (int e = tid; e < GT * GK; e += 256) {
      const int r = e / GK, kk = e % GK;
      const int m = m0 + r, n = n0 + r, k = k0 + kk;
      As[r * GKP + kk] = (m < g.M && k < g.K) ? g.a[m * g.sa0 + k * g.sa1] : (uint16_t)0;
      Bs[r * GKP + kk] = (n < g.N && k < g.K) ? g.b[k * g.sb0 + n * g.sb1] : (uint16_t)0;
    }
    __syncthreads();
    const int ar = 16 * w + (lane & 15), ak = 8 * (lane >> 4);
    const v8bf af = *reinterpret_cast<const v8bf*>(&As[ar * GKP + ak]);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int bn = 16 * nb + (lane & 15);
      const v8bf bfr = *reinterpret_cast<const v8bf*>(&Bs[bn * GKP + ak]);
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr, acc[nb], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + 16 * w + mfma_row(lane, r), n = n0 + 16 * nb + (lane & 15);
      if (m < g.M && n < g.N) {
        float v = acc[nb][r];
        float* p = g.c + m * g.ldc + n;
        if (g.accumulate)
          *p += v;
        else
          *p = v + (g.bias ? g.bias[n] : 0.f);
      }
    }
}

// out[r][j] = bf16(in[r][j]) for j < ncols_in, 0 for ncols_in <= j < ncols_out.
__global__ void k_cast_pad(const float* in, int ld_in, int ncols_in, uint16_t* out, int ncols_out,
                           int rows) {
  const int64_t tot = (int64_t)rows * ncols_out;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / ncols_out), j = (int)(i % ncols_out);
    out[i] = j < ncols_in ? f2bf(in[(int64_t)r * ld_in + j]) : (uint16_t)0;
  }
}

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// h = bf16(gelu(z))
__global__ void k_gelu_bf16(const float* z, uint16_t* h, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    h[i] = f2bf(gelu_f(z[i]));
}

// dz = dh * gelu'(z); dzb = bf16(dz)
__global__ void k_gelu_back(const float* dh, const float* z, float* dz, uint16_t* dzb, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = dh[i] * gelu_grad_f(z[i]);
    dz[i] = v;
    dzb[i] = f2bf(v);
  }
}

// db[j] += sum_r dz[r][j] (fixed order over r; one thread per column)
// Bias gradient db[j] += sum_r dz[r][j] in two fixed-order stages: block
// (x, y) sums columns 64x..64x+63 over the y-th of kColSplit row slices (four
// row phases per thread, combined in LDS) into part[y][j]; k_colsum_fin adds
// the kColSplit partial sums in order.
constexpr int kColSplit = 32;

__global__ __launch_bounds__(256) void k_colsum_part(const float* dz, int rows, int cols,
                                                     float* part) {
  __shared__ float red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + tx;
  const int per = (rows + kColSplit - 1) / kColSplit;
  const int r0 = blockIdx.y * per, r1 = r0 + per < rows ? r0 + per : rows;
  float s = 0.f;
  if (j < cols)
    for (int r = r0 + ty; r < r1; r += 4) s += dz[(int64_t)r * cols + j];
  red[ty][tx] = s;
  __syncthreads();
  if (ty == 0 && j < cols)
    part[(size_t)blockIdx.y * cols + j] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

__global__ void k_colsum_fin(const float* part, int cols, float* db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int y = 0; y < kColSplit; ++y) s += part[(size_t)y * cols + j];
  db[j] += s;
}

// out[r][j] = z[r][j] for j < 21 (network output)
__global__ void k_take_out(const float* z, int ldz, float* out, int rows, int ncols) {
  const int64_t tot = (int64_t)rows * ncols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = z[(i / ncols) * ldz + (i % ncols)];
}

// Adam on FP32 master weights; clears the gradient; refreshes the BF16 copy.
__global__ void k_adam(float* p, float* g, float* m, float* v, uint16_t* pb, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float upd = lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    const float pi = p[i] - upd;
    p[i] = pi;
    pb[i] = f2bf(pi);
    g[i] = 0.f;
  }
}

__global__ void k_to_bf16(const float* p, uint16_t* pb, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    pb[i] = f2bf(p[i]);
}

__global__ void k_fillf(float* p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// W (din x dout, row-major): N(0,1) * scale on the live block (rows < fin,
// cols < fout), element (r, c) from counter r * dout + c of the stream.
__global__ void k_init_layer(float* W, int din, int dout, int fin, int fout, uint64_t base,
                             float scale) {
  const int64_t tot = (int64_t)din * dout;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / dout), c = (int)(i % dout);
    W[i] = (r < fin && c < fout) ? (float)normal_at(base, (uint64_t)i) * scale : 0.f;
  }
}

// dz = [dout | 0] padded to ncols_out columns; dzb = bf16(dz)
__global__ void k_pad_out(const float* dout, int ncols_in, float* dz, uint16_t* dzb, int ncols_out,
                          int rows) {
  const int64_t tot = (int64_t)rows * ncols_out;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / ncols_out), j = (int)(i % ncols_out);
    const float v = j < ncols_in ? dout[(int64_t)r * ncols_in + j] : 0.f;
    dz[i] = v;
    dzb[i] = f2bf(v);
  }
}

static int eltgrid(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : g > 8192 ? 8192 : g);
}

static hipError_t gemm(const GemmArgs& g, hipStream_t st) {
  dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT);
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

}  // namespace aa

using namespace aa;

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {
constexpr int kIn = 256, kH = 256, kOutP = 64;
constexpr int kNF = AA_MLP_FEATURES, kNO = AA_MLP_OUTPUTS;
constexpr int kLayers = 4;
const int kDin[kLayers] = {kIn, kH, kH, kH};
const int kDout[kLayers] = {kH, kH, kH, kOutP};

int64_t param_count() {
  int64_t s = 0;
  for (int l = 0; l < kLayers; ++l) s += (int64_t)kDin[l] * kDout[l] + kDout[l];
  return s;
}
size_t al(size_t x) { return (x + 255) / 256 * 256; }
}  // namespace

struct aa_mlp;
static aa_status mlp_reset_state(aa_mlp* n);

struct aa_mlp {
  int max_batch = 0;
  hipStream_t stream = nullptr;
  int64_t P = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // packed W0 b0 W1 b1 ...
  uint16_t* pb = nullptr;                                          // BF16 copy of p
  uint16_t* xb = nullptr;                                          // [B x 256]
  float* z[kLayers] = {};                                          // pre-activations
  uint16_t* h[kLayers] = {};                                       // h[l] = input of layer l (l >= 1)
  float *dz = nullptr, *dh = nullptr;
  uint16_t* dzb = nullptr;
  float* colpart = nullptr;  // kColSplit x 256 bias-gradient partial sums
  int last_batch = 0;
  int64_t t = 0;  // Adam steps taken
  int64_t off_w[kLayers], off_b[kLayers];
};

// Zero gradients and Adam moments, refresh the BF16 weights (after an
// initialization or a load of the master weights).
static aa_status mlp_reset_state(aa_mlp* n) {
  const hipStream_t st = n->stream;
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_fillf, dim3(eltgrid(n->P)), dim3(256), 0, st, n->g, n->P, 0.f);
  hipLaunchKernelGGL(k_fillf, dim3(eltgrid(n->P)), dim3(256), 0, st, n->m, n->P, 0.f);
  hipLaunchKernelGGL(k_fillf, dim3(eltgrid(n->P)), dim3(256), 0, st, n->v, n->P, 0.f);
  hipLaunchKernelGGL(k_to_bf16, dim3(eltgrid(n->P)), dim3(256), 0, st, n->p, n->pb, n->P);
  n->t = 0;
  return hipGetLastError() == hipSuccess ? AA_OK : AA_EHIP;
}

namespace aa {
hipStream_t mlp_stream(const aa_mlp* n) { return n->stream; }
int mlp_max_batch(const aa_mlp* n) { return n->max_batch; }
}  // namespace aa

extern "C" {

aa_status aa_mlp_workspace_size(int max_batch, size_t* bytes) {
  if (max_batch < 1 || max_batch > (1 << 20) || !bytes) return AA_EINVAL;
  const int64_t P = param_count();
  const size_t B = (size_t)max_batch;
  size_t s = 4 * al(sizeof(float) * P) + al(sizeof(uint16_t) * P);
  s += al(sizeof(uint16_t) * B * kIn);
  s += 3 * al(sizeof(float) * B * kH) + al(sizeof(float) * B * kOutP);
  s += 3 * al(sizeof(uint16_t) * B * kH);
  s += 2 * al(sizeof(float) * B * kH) + al(sizeof(uint16_t) * B * kH);
  s += al(sizeof(float) * kColSplit * kH);
  *bytes = s;
  return AA_OK;
}

aa_status aa_mlp_init(aa_mlp** out, int max_batch, uint64_t seed, void* d_ws, size_t bytes,
                      void* stream) {
  if (!out) return AA_EINVAL;
  *out = nullptr;
  size_t need = 0;
  if (aa_mlp_workspace_size(max_batch, &need) != AA_OK) return AA_EINVAL;
  if (!d_ws || ((uintptr_t)d_ws % 256) != 0) return AA_EINVAL;
  if (bytes < need) return AA_ENOSPACE;
  aa_mlp* n = new (std::nothrow) aa_mlp();
  if (!n) return AA_EINVAL;
  n->max_batch = max_batch;
  n->stream = (hipStream_t)stream;
  n->P = param_count();
  char* base = (char*)d_ws;
  size_t o = 0;
  const size_t B = (size_t)max_batch;
  auto take = [&](size_t sz) {
    char* r = base + o;
    o += al(sz);
    return r;
  };
  n->p = (float*)take(sizeof(float) * n->P);
  n->g = (float*)take(sizeof(float) * n->P);
  n->m = (float*)take(sizeof(float) * n->P);
  n->v = (float*)take(sizeof(float) * n->P);
  n->pb = (uint16_t*)take(sizeof(uint16_t) * n->P);
  n->xb = (uint16_t*)take(sizeof(uint16_t) * B * kIn);
  for (int l = 0; l < kLayers; ++l) n->z[l] = (float*)take(sizeof(float) * B * kDout[l]);
  for (int l = 1; l < kLayers; ++l) n->h[l] = (uint16_t*)take(sizeof(uint16_t) * B * kH);
  n->dz = (float*)take(sizeof(float) * B * kH);
  n->dh = (float*)take(sizeof(float) * B * kH);
  n->dzb = (uint16_t*)take(sizeof(uint16_t) * B * kH);
  n->colpart = (float*)take(sizeof(float) * kColSplit * kH);
  int64_t off = 0;
  for (int l = 0; l < kLayers; ++l) {
    n->off_w[l] = off;
    off += (int64_t)kDin[l] * kDout[l];
    n->off_b[l] = off;
    off += kDout[l];
  }
  aa_status s = aa_mlp_reseed(n, seed);
  if (s != AA_OK) {
    delete n;
    return s;
  }
  *out = n;
  return AA_OK;
}

aa_status aa_mlp_reseed(aa_mlp* n, uint64_t seed) {
  if (!n) return AA_EINVAL;
  const hipStream_t st = n->stream;
  hipLaunchKernelGGL(k_fillf, dim3(eltgrid(n->P)), dim3(256), 0, st, n->p, n->P, 0.f);
  for (int l = 0; l < kLayers - 1; ++l) {
    const int fin = l == 0 ? kNF : kH;
    const uint64_t sb = sm64_mix_host(sm64_mix_host(seed) + (uint64_t)l);
    hipLaunchKernelGGL(k_init_layer, dim3(eltgrid((int64_t)kDin[l] * kDout[l])), dim3(256), 0,
                       st, n->p + n->off_w[l], kDin[l], kDout[l], fin, kDout[l], sb,
                       sqrtf(2.0f / (float)fin));
  }
  // last layer: zero weights, beta-logit bias +4
  hipLaunchKernelGGL(k_fillf, dim3(1), dim3(64), 0, st, n->p + n->off_b[kLayers - 1] + (kNO - 1),
                     (int64_t)1, 4.0f);
  return mlp_reset_state(n);
}

aa_status aa_mlp_set_params(aa_mlp* n, const float* h) {
  if (!n || !h) return AA_EINVAL;
  if (hipMemcpyAsync(n->p, h, sizeof(float) * n->P, hipMemcpyHostToDevice, n->stream) !=
          hipSuccess ||
      hipStreamSynchronize(n->stream) != hipSuccess)
    return AA_EHIP;
  return mlp_reset_state(n);
}

aa_status aa_mlp_get_params(aa_mlp* n, float* h) {
  if (!n || !h) return AA_EINVAL;
  if (hipMemcpyAsync(h, n->p, sizeof(float) * n->P, hipMemcpyDeviceToHost, n->stream) !=
          hipSuccess ||
      hipStreamSynchronize(n->stream) != hipSuccess)
    return AA_EHIP;
  return AA_OK;
}

aa_status aa_mlp_get_grads(aa_mlp* n, float* h) {
  if (!n || !h) return AA_EINVAL;
  if (hipMemcpyAsync(h, n->g, sizeof(float) * n->P, hipMemcpyDeviceToHost, n->stream) !=
          hipSuccess ||
      hipStreamSynchronize(n->stream) != hipSuccess)
    return AA_EHIP;
  return AA_OK;
}

int64_t aa_mlp_param_count(void) { return param_count(); }

aa_status aa_mlp_forward(aa_mlp* n, int batch, const float* x, float* out) {
  if (!n || !x || batch < 1 || batch > n->max_batch) return AA_EINVAL;
  const hipStream_t st = n->stream;
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_cast_pad, dim3(eltgrid((int64_t)batch * kIn)), dim3(256), 0, st, x, kNF,
                     kNF, n->xb, kIn, batch);
  for (int l = 0; l < kLayers; ++l) {
    GemmArgs g{};
    g.a = l == 0 ? n->xb : n->h[l];
    g.sa0 = kDin[l];
    g.sa1 = 1;
    g.b = n->pb + n->off_w[l];
    g.sb0 = kDout[l];
    g.sb1 = 1;
    g.c = n->z[l];
    g.ldc = kDout[l];
    g.bias = n->p + n->off_b[l];
    g.M = batch;
    g.N = kDout[l];
    g.K = kDin[l];
    if (gemm(g, st) != hipSuccess) return AA_EHIP;
    if (l < kLayers - 1)
      hipLaunchKernelGGL(k_gelu_bf16, dim3(eltgrid((int64_t)batch * kH)), dim3(256), 0, st,
                         n->z[l], n->h[l + 1], (int64_t)batch * kH);
  }
  if (out)
    hipLaunchKernelGGL(k_take_out, dim3(eltgrid((int64_t)batch * kNO)), dim3(256), 0, st,
                       n->z[kLayers - 1], kOutP, out, batch, kNO);
  n->last_batch = batch;
  return hipGetLastError() == hipSuccess ? AA_OK : AA_EHIP;
}

aa_status aa_mlp_backward(aa_mlp* n, int batch, const float* dout) {
  if (!n || !dout || batch < 1 || batch != n->last_batch) return AA_EINVAL;
  const hipStream_t st = n->stream;
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  // dz of the output layer: [B x 64], live columns 0..20
  hipLaunchKernelGGL(k_pad_out, dim3(eltgrid((int64_t)batch * kOutP)), dim3(256), 0, st, dout,
                     kNO, n->dz, n->dzb, kOutP, batch);
  for (int l = kLayers - 1; l >= 0; --l) {
    const int din = kDin[l], dout_l = kDout[l];
    // dW_l += H_l^T dZ_l   (M = din, N = dout, K = batch)
    GemmArgs gw{};
    gw.a = l == 0 ? n->xb : n->h[l];
    gw.sa0 = 1;
    gw.sa1 = din;
    gw.b = n->dzb;
    gw.sb0 = dout_l;
    gw.sb1 = 1;
    gw.c = n->g + n->off_w[l];
    gw.ldc = dout_l;
    gw.M = din;
    gw.N = dout_l;
    gw.K = batch;
    gw.accumulate = 1;
    if (gemm(gw, st) != hipSuccess) return AA_EHIP;
    hipLaunchKernelGGL(k_colsum_part, dim3((dout_l + 63) / 64, kColSplit), dim3(256), 0, st,
                       n->dz, batch, dout_l, n->colpart);
    hipLaunchKernelGGL(k_colsum_fin, dim3((dout_l + 255) / 256), dim3(256), 0, st, n->colpart,
                       dout_l, n->g + n->off_b[l]);
    if (l == 0) break;
    // dH = dZ_l W_l^T   (M = batch, N = din, K = dout)
    GemmArgs gh{};
    gh.a = n->dzb;
    gh.sa0 = dout_l;
    gh.sa1 = 1;
    gh.b = n->pb + n->off_w[l];
    gh.sb0 = 1;
    gh.sb1 = dout_l;
    gh.c = n->dh;
    gh.ldc = din;
    gh.M = batch;
    gh.N = din;
    gh.K = dout_l;
    if (gemm(gh, st) != hipSuccess) return AA_EHIP;
    hipLaunchKernelGGL(k_gelu_back, dim3(eltgrid((int64_t)batch * kH)), dim3(256), 0, st, n->dh,
                       n->z[l - 1], n->dz, n->dzb, (int64_t)batch * kH);
  }
  return hipGetLastError() == hipSuccess ? AA_OK : AA_EHIP;
}

aa_status aa_mlp_adam(aa_mlp* n, float lr, float b1, float b2, float eps) {
  if (!n || !(lr >= 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
    return AA_EINVAL;
  n->t += 1;
  const float c1 = 1.f - powf(b1, (float)n->t), c2 = 1.f - powf(b2, (float)n->t);
  (void)hipGetLastError();  // drop a stale error left by an earlier call
  hipLaunchKernelGGL(k_adam, dim3(eltgrid(n->P)), dim3(256), 0, n->stream, n->p, n->g, n->m, n->v,
                     n->pb, n->P, lr, b1, b2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? AA_OK : AA_EHIP;
}

aa_status aa_mlp_destroy(aa_mlp* n) {
  delete n;
  return AA_OK;
}

}  // extern "C"
