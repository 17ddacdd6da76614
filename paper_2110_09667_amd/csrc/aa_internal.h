// aa_internal.h -- definitions shared by the kernel and host translation units
// of the Anderson-acceleration library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/aa.h"

namespace aa {

constexpr int kWG = 256;             // threads per workgroup (4 wave64s)
constexpr int kWaves = kWG / 64;
#ifndef AA_PAIRS
#define AA_PAIRS 2
#endif
constexpr int kPairs = AA_PAIRS;     // row pairs (16-byte loads) per lane per tile
constexpr int kTile = kWG * 2 * kPairs;  // rows per tile in streaming passes
constexpr int kMaxCols = AA_MAX_COLS;
constexpr int kMaxRed = 3 * kMaxCols + 4;  // reductions of one streaming pass
constexpr int kMaxPairs = (kMaxCols - 1) * (kMaxCols - 2) / 2;  // Gram after delete
constexpr int kMaxRedAll = kMaxPairs > kMaxRed ? kMaxPairs : kMaxRed;
constexpr int kFinWG = 1024;         // threads of the finalize kernel

// Scalar slots in the small device block.
// S_RHO, S_RKK: the lagged DCGS-2's divisors of its update pass (the norm of
// the reorthogonalized previous column and the new column's norm).
enum Scal : int { S_RES = 0, S_RES0 = 1, S_STEP = 2, S_RHO = 3, S_RKK = 4, S_COUNT = 8 };

// What the last-arriving workgroup does with the reduced values.
enum TailOp : int {
  TAIL_NONE = 0,
  TAIL_STORE,     // coef0[t] = red[t], t < count
  TAIL_MGS_R,     // R[row, k] = red[0]
  TAIL_NORM,      // R[k, k] = sqrt(red[idx]); breakdown check
  TAIL_CGS2_S,    // coef0 = s = red[0:k]
  TAIL_CGS2_Z,    // coef1 = z = red[0:k]; R[0:k-1, k] = s + z
  TAIL_ICWY,      // T row k-1 from red[k:2k-1]; forward solve; R col, coef0
  TAIL_DCGS2,     // R col k = red[0:k]; s = red[k:2k-1] -> coef1; R col k-1 fix
  TAIL_RHS,       // c = red[0:k]; back substitution -> gamma
  TAIL_RES,       // scal[S_RES] = red[0]
  TAIL_FIRST,     // scal[S_RES0] = scal[S_RES] = red[0], scal[S_STEP] = red[1]
  TAIL_STEP,      // scal[S_STEP] = red[0]
  TAIL_GRAM,      // T strict lower from pair sums
  TAIL_GRAM_ADD,  // pairs of [Q v (f)]: T refresh (gram_t), then the QRAdd's
                  // first-pass tail `inner` on the rearranged values (finalize)
  TAIL_DCGS2_LAG  // lagged DCGS-2: reorthogonalize and normalize the previous
                  // column, project the new one (R, coef0, coef1, S_RHO, S_RKK)
};

// Stop state of an AA iteration on the device (single-instance contexts).
// done: 0 running; AA_STOPPED_TEST (the stopping test held at the start of
// iteration `iter`, with k columns and window m_i); AA_STOPPED_BREAKDOWN (a
// breakdown in iteration `iter`); AA_STOPPED_CAP (the iteration cap).
struct StopState {
  int done;
  int k;
  int m_i;
  int pad;
  int64_t iter;
  int64_t cur;  // index i of the iteration the device is in (graph-safe count)
};

// Device-resident small dense state (pointers into the workspace).
struct Small {
  double* R;        // cap x cap, column-major
  double* T;        // cap x cap, column-major, unit lower (ICWY)
  double* coef0;    // cap
  double* coef1;    // cap
  double* gamma;    // cap
  double* givens;   // 2 * cap: cosines then sines
  double* scal;     // S_COUNT scalars
  int* status;      // latched aa_status
  double* partials; // reduction partials, [nred][grid]
  int cap;
  int64_t npart;    // doubles the partials buffer holds (0: not stated; the
                    // finalize then sums the partials in one workgroup)
  // AA step launches only (null otherwise): once done is set or a breakdown
  // is latched in status, every kernel of the step returns at once, and the
  // x update writes x_next = x (or G(x) in the step that broke down)
  StopState* stop;
};

enum StopMode : int { kStopNone = 0, kStopResidual = 1, kStopStep = 2 };

// Breakdown: the new column's R_kk at most this multiple of eps times the
// norm of its R column (the column numerically in the span of the window).
constexpr double kBreakdownRel = 64.0 * 2.220446049250313e-16;

// Whether the AA iteration this launch belongs to has ended.
__device__ __forceinline__ bool aa_stopped(const Small& sm) {
  return sm.stop != nullptr && (sm.stop->done != 0 || *sm.status != AA_OK);
}

struct Tail {
  int op;
  int k;        // columns in Q when the pass runs
  int row;      // TAIL_MGS_R: R row
  int count;    // TAIL_STORE: values
  int idx;      // TAIL_NORM: index of the squared norm in red[]
  int reorth;   // TAIL_DCGS2
  int literal;  // TAIL_DCGS2
  int rhs;      // R gamma = Q^T f folded into the QRAdd passes (see aa_step)
  int zoff;     // first QRAdd pass with rhs: index of Q^T f in red[]
  int inner;    // TAIL_GRAM_ADD: the QRAdd first-pass tail to run afterwards
  int gram_t;   // TAIL_GRAM_ADD: also refresh T from the Gram (ICWY)
  // TAIL_RES in an AA step: the stopping test (Alg. 1, reading A2) at the
  // start of the iteration, with k columns and window m_i (host values)
  int stop_mode;     // kStopNone, kStopResidual, kStopStep
  double stop_tol;
  int m_i;
};

// ---- streaming passes -------------------------------------------------------

// red[j] = Q_j^T x (j < nx); red[nx + j] = Q_j^T y (j < ny);
// red[nx + ny + j] = Q_j^T z (j < nz); red[nx + ny + nz] = x^T x (xx), then
// x^T z (xz, needs nz > 0)
struct DotsArgs {
  const double* Q; int64_t ldq; int64_t n;
  const double* x; int nx;
  const double* y; int ny;
  int xx;
  const double* z; int nz;
  int xz;
};

// out = v - sum_{j0 <= j < j0+nc} Q_j (c1[j] + c2[j]) evaluated as
// (v - Q c1) - Q c2; optional fused dot Q_{dotcol}^T out and out^T out.
// DCGS-2 mode (dcgs2_p >= 0): with p = dcgs2_p, first
//   q'_p = q_p - sum_{j<p} Q_j s[j]   (written back to column p if reorth),
// then out = v - sum_{j<p} Q_j c1[j] - q'_p c1[p].
struct UpdArgs {
  const double* Q; int64_t ldq; int64_t n;
  double* Qw;            // writable alias of Q (DCGS-2 writes column p)
  const double* v;
  double* out;           // may be null (no write) or alias v
  int j0, nc;
  const double* c1;      // device coefficients, indexed by absolute column
  const double* c2;      // may be null
  int dotcol;            // -1: none
  int nrm;               // 1: add out^T out
  int dcgs2_p;           // -1: off
  int reorth;
  const double* s;       // DCGS-2 reorthogonalization coefficients
  const double* rhsv;    // may be null: add out^T rhsv after the norm
  // lagged DCGS-2 (DCGS-2 mode): divide q'_p by *pdiv before use and the
  // output by *odiv (device scalars; null: no division)
  const double* pdiv;
  const double* odiv;
  // 1: walk the row tiles from the last to the first.  A pass that follows
  // another over the same columns runs the other way, so its first tiles are
  // the previous pass's last ones, still in the Infinity Cache.
  int rev;
};

struct Cgs2bArgs {       // y = v - Q s (registers), red[j] = Q_j^T y
  const double* Q; int64_t ldq; int64_t n;
  const double* v; int k;
  const double* s;
  int rev;               // 1: row tiles last to first (as UpdArgs::rev)
};

struct RotArgs {         // Givens sweep over k columns (+ ICWY Gram of k-1)
  double* Q; int64_t ldq; int64_t n; int k;
  const double* givens;
  int gram;
  // Gram only: naug vectors appended after the k-1 rotated columns (v, then
  // f), so the same contraction also yields Q^T v and Q^T f
  const double* v; const double* f; int naug;
  // Gram only, naug == 0: leave the last rotated column out of the Gram (its
  // row of T is recomputed by the QRAdd that follows, Alg. 4)
  int drop_last;
};

// Columns the Gram of a rotation pass contracts: the k-1 rotated columns
// (minus the last with drop_last), then the naug appended vectors.
__host__ __device__ inline int gram_cols(const RotArgs& a) {
  return a.k - 1 - a.drop_last + a.naug;
}

struct ScaleArgs {
  const double* in; double* out; int64_t n; const double* R; int kk; int cap;
  const StopState* stop; const int* status;  // AA step launches: skip once stopped
};

struct HistArgs {        // i >= 1: history formation; i == 0: first step
  const double* x; const double* g;
  double* W; double* f_prev; double* g_prev; double* dg;  // dg: ring slot
  double* x_next;        // first step only
  int64_t n; int first;
};

struct XupdArgs {
  const double* ring; int64_t ldq; int m; int slot0; int mi;
  const double* g; const double* x; double* x_next; int64_t n;
  const double* gamma;
};

// ---- batched / fused workgroup-level step (aa_batch.hip) ---------------------

// One AA instance processed by one workgroup.  Pointers into the workspace
// except x, f (caller's) and, for dim == 0, g (the caller's G(x)).
struct BInst {
  int64_t n, ld;          // length, leading dimension of Q / ring (even)
  int m;                  // window
  int dim;                // model map on an s^dim grid (1..3); 0: caller's g
  int64_t s;
  double h, omega, c;
  const double* f;        // model right-hand side
  double* x;              // iterate (updated in place)
  double* g;              // G(x) buffer (dim > 0) or the caller's G(x)
  double* f_prev; double* g_prev; double* W; double* Q; double* ring;
  double* xc; double* gc; // learned step: candidate and G(candidate) / adjoint work
  Small sm;               // R, T, coefficients, gamma, Givens, scalars, status
};

// Per-instance iteration state, updated on the device (layout of aa_batch_state).
struct BState {
  int64_t iter;           // index i of the next iteration
  int64_t conv_iter;      // iteration at which the instance stopped (-1: running)
  int k, m_i, active, status;
  double res_norm, res0_norm;
  int64_t g_evals, accepted;
  double loss;
  int pending, g_valid;
};

// Modes of the batched kernel.
enum BatchMode : int {
  BM_PLAIN = 0,   // a whole AA iteration
  BM_PHASE_A = 1, // up to R gamma = Q^T f_i, then the network features
  BM_GUARD = 2,   // learned candidate, guard, accept or plain step
  BM_TRAIN = 3    // plain step + loss gradient w.r.t. the network outputs
};
constexpr int kFeat = AA_MLP_FEATURES;   // network inputs per instance
constexpr int kOuts = AA_MLP_OUTPUTS;    // network outputs per instance
constexpr int kWin = kOuts - 1;          // window the features are padded to
static_assert(sizeof(BState) == sizeof(aa_batch_state), "BState mirrors aa_batch_state");

struct BatchArgs {
  BInst* inst; BState* state; const int* order; int count;
  unsigned* counter;      // work counter, reset before every launch
  int variant; unsigned flags;
  double tol; int64_t max_iter;
  // fused single-instance step (ov_iter >= 0): instance 0 only, with the
  // caller's x, G(x), x_next and the host's iteration index and column count
  const double* ox; const double* og; double* oxn;
  int64_t ov_iter; int ov_k;
  int mode;               // BatchMode
  const int* skip;        // plain mode: instances the persistent kernel leaves out
                          // (advanced on the grid-wide passes instead); may be null
  int stop_mode;          // fused single-instance step: the stopping test
  double stop_tol;
  float* feat;            // [count x kFeat] network inputs (phase A)
  const float* out;       // [count x kOuts] network outputs (guard / train)
  float* dout;            // [count x kOuts] loss gradient (train)
  float dscale;           // scale of dout (1 / count)
};

// stage_cols: largest number of columns the Gram staging holds (0: none);
// dynamic LDS = max(kbucket^2, gram_lds_doubles(stage_cols)) doubles.
// pairs: row pairs per lane per tile of the batched kernel's passes (4 or 2:
// two builds of aa_batch.hip, the autotuner's tile dimension)
hipError_t launch_batch(const BatchArgs&, int grid, int kbucket, bool gram, int stage_cols,
                        hipStream_t, int pairs = 4);
namespace p4 {
hipError_t launch_batch(const BatchArgs&, int grid, int kbucket, bool gram, int stage_cols,
                        hipStream_t);
}
namespace p2 {
hipError_t launch_batch(const BatchArgs&, int grid, int kbucket, bool gram, int stage_cols,
                        hipStream_t);
}
// Staged Gram columns and whether the batched kernel needs its Gram
// instantiation, for a window of up to mmax columns, variant and flags.
int batch_stage_cols(int mmax, int variant, unsigned flags);
bool batch_needs_gram(int variant, unsigned flags);
hipStream_t mlp_stream(const aa_mlp*);
int mlp_max_batch(const aa_mlp*);
hipError_t launch_batch_reset(unsigned* counter, hipStream_t);

// A single-instance context over a batched instance's memory (Q, history,
// small block), with a shared partials buffer and its own stop state: the
// batch's split path runs a large instance's iterations on the grid-wide
// passes.  Counters are the instance's (iteration, columns, window); tol and
// max_iter the batch's (the instance stops at the start of iteration i with
// ||f_i|| <= tol ||f_0|| or i >= max_iter).
aa_ctx* view_create(const BInst& I, int variant, unsigned flags, double* partials,
                    StopState* stop, int64_t iter, int k, int m_i, double tol, int64_t max_iter,
                    hipStream_t st);
void view_counters(const aa_ctx* c, int64_t* iter, int* k, int* m_i);
void view_destroy(aa_ctx* c);
hipError_t launch_set_int(int* p, int64_t n, int v, hipStream_t);
// The batched state of a split instance from its stop state and small block.
hipError_t launch_split_state(BState* st, const StopState* stop, const Small& sm, int k, int m_i,
                              hipStream_t);
hipError_t launch_batch_init(BInst* inst, int count, hipStream_t);

// launchers (aa_kernels.hip)
// Profiling hook: while set, the next finalize launch records this event on
// its stream first (separating a pass from its finalize kernel).
void set_profile_mid(hipEvent_t e);
bool profile_mid_used();

hipError_t launch_dots(const DotsArgs&, const Small&, const Tail&, int grid, hipStream_t);
hipError_t launch_update(const UpdArgs&, const Small&, const Tail&, int grid, hipStream_t);
hipError_t launch_cgs2b(const Cgs2bArgs&, const Small&, const Tail&, int grid, hipStream_t);
// transform: also rotate ICWY's T like the columns (AA_ICWY_T_TRANSFORM)
hipError_t launch_givens(const Small&, int k, hipStream_t, bool transform = false);
hipError_t launch_rotate(const RotArgs&, const Small&, const Tail&, int grid, hipStream_t);
hipError_t launch_scale(const ScaleArgs&, const Small&, hipStream_t);
hipError_t launch_history(const HistArgs&, const Small&, const Tail&, int grid, hipStream_t);
hipError_t launch_xupdate(const XupdArgs&, const Small&, const Tail&, int grid, hipStream_t);
hipError_t launch_init_small(const Small&, hipStream_t);
// (reads, writes) in {(1,0), (4,0), (8,0), (1,1), (2,1), (3,1), (8,1), (1,2)}
hipError_t launch_probe(int reads, int writes, const double* src, int64_t ld, double* dst,
                        int64_t n, double* sink, int grid, hipStream_t);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t);
hipError_t launch_stop_cap(StopState* stop, int k, int m_i, const double* x, double* xn,
                           int64_t n, hipStream_t);

// problems and generators (aa_problems.hip)
hipError_t launch_stencil(int dim, int64_t s, double h, double omega, double c,
                          const double* f, const double* u, double* out, hipStream_t);
// the EM map of Sec. 5.3; work: 6 x min(ceil(N / 256), 1024) doubles
hipError_t launch_em(const double alpha[3], const double sigma[3], const double* x, int64_t N,
                     const double* u, double* out, int64_t n, double* work, hipStream_t);
hipError_t launch_fill_uniform(double* out, int64_t n, uint64_t seed, uint64_t stream_id,
                               uint64_t offset, double lo, double hi, hipStream_t);
hipError_t launch_fill_normal(double* out, int64_t n, uint64_t seed, uint64_t stream_id,
                              uint64_t offset, hipStream_t);

}  // namespace aa
