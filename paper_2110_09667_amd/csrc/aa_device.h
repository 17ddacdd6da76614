// aa_device.h -- device helpers shared by the grid-wide passes and the
// workgroup-level (batched) passes: wavefront reductions and the 16-byte row
// loads of the streaming passes.
#pragma once

#include "aa_internal.h"

namespace aa {

// ---------------------------------------------------------------------------
// wavefront reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum N per-lane values across the 64 lanes at once (N a power of two, <= 64).
// Butterfly with halving: at the step of offset h, a lane keeps the half of
// its values selected by lane bit h and adds its partner's copy of that half.
// After log2(N) steps lane l holds column (l mod N) summed over the lanes that
// share its low bits; the remaining xor steps finish the sum.  N - 1 +
// 6 - log2(N) shuffles instead of 6 N.
template <int H, int N>
__device__ __forceinline__ void halve_step(double (&v)[N], int lane) {
  if constexpr (H >= 1) {
    const bool upper = (lane & H) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double keep = upper ? v[i + H] : v[i];
      const double send = upper ? v[i] : v[i + H];
      v[i] = keep + __shfl_xor(send, H, 64);
    }
    halve_step<H / 2, N>(v, lane);
  }
}

template <int N>
__device__ __forceinline__ double multi_reduce(double (&v)[N]) {
  const int lane = threadIdx.x & 63;
  halve_step<N / 2, N>(v, lane);
  double r = v[0];
#pragma unroll
  for (int o = N; o < 64; o <<= 1) r += __shfl_xor(r, o, 64);
  return r;
}

// ---------------------------------------------------------------------------
// row loads for the streaming passes: each lane owns kPairs pairs of
// consecutive rows (16-byte loads), pair i at rows b2 + 2 i kWG + {0, 1}.
// Full tiles use non-temporal loads (AA_NT_LOAD): the streamed columns are
// far larger than the caches and are not re-read within a pass, and marking
// them streaming measurably raises the sustained read bandwidth.
// ---------------------------------------------------------------------------

// AA_STREAMING (default 1): the passes stream data far larger than the
// caches, so full tiles use non-temporal loads and the rotation sweep
// non-temporal stores.  (Measured also for the batched kernel, whose 4096
// instances together far exceed the caches: 36.4 ms per iteration with them,
// 37.2 ms with ordinary loads and stores.)  Defining it to 0 before including
// this header restores ordinary accesses.
#ifndef AA_STREAMING
#define AA_STREAMING 1
#endif
#ifndef AA_NT_LOAD
#define AA_NT_LOAD AA_STREAMING
#endif
// AA_NT_STORE (default 1): the passes' vector stores (history, x update,
// scale, the batched step) are non-temporal too.  Ordinary stores leave the
// caches full of dirty lines whose write-back then shares HBM with the next
// pass's reads: with non-temporal stores the 256^3 recycle iteration at m = 20
// runs 2-5 % faster for every variant (ICWY 3.46 -> 3.32 ms).  The update
// pass's output, which the scale pass (or MGS's next update) reads at once,
// keeps ordinary stores (AA_NT_STORE_UPDATE 0: non-temporal there cost MGS
// 2 % and the QRAdd's scale pass 3 %).
#ifndef AA_NT_STORE_UPDATE
#define AA_NT_STORE_UPDATE 0
#endif
#ifndef AA_NT_STORE
#define AA_NT_STORE 1
#endif

typedef double f64x2 __attribute__((ext_vector_type(2)));

// One streamed 16-byte pair.
__device__ __forceinline__ f64x2 ld2v(const double2* p) {
#if AA_NT_LOAD
  return __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p));
#else
  const double2 v = *p;
  f64x2 r;
  r.x = v.x;
  r.y = v.y;
  return r;
#endif
}

// Store one 16-byte pair that no later pass of this call reads back soon
// (non-temporal: the written columns far exceed the caches).
__device__ __forceinline__ void st2v_stream(f64x2 v, double* p) {
#if AA_STREAMING
  __builtin_nontemporal_store(v, reinterpret_cast<f64x2*>(p));
#else
  *reinterpret_cast<f64x2*>(p) = v;
#endif
}

// Store one streamed value (the row-per-thread rotation sweep).
__device__ __forceinline__ void st1_stream(double v, double* p) {
#if AA_STREAMING
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}

// One streamed value (the row-per-thread sweeps).
__device__ __forceinline__ double ld1(const double* p) {
#if AA_NT_LOAD
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

template <bool FULL>
__device__ __forceinline__ void ld2(double2 (&r)[kPairs], const double* __restrict__ p,
                                    int64_t b2, int64_t n) {
#pragma unroll
  for (int i = 0; i < kPairs; ++i) {
    const int64_t row = b2 + (int64_t)i * 2 * kWG;
    if (FULL) {
#if AA_NT_LOAD
      const f64x2 v = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p + row));
      r[i] = make_double2(v.x, v.y);
#else
      r[i] = *reinterpret_cast<const double2*>(p + row);
#endif
    } else {
      r[i].x = row < n ? p[row] : 0.0;
      r[i].y = row + 1 < n ? p[row + 1] : 0.0;
    }
  }
}

template <bool FULL, bool NT = AA_NT_STORE != 0>
__device__ __forceinline__ void st2(const double2 (&r)[kPairs], double* p, int64_t b2,
                                    int64_t n) {
#pragma unroll
  for (int i = 0; i < kPairs; ++i) {
    const int64_t row = b2 + (int64_t)i * 2 * kWG;
    if (FULL) {
      if constexpr (NT) {
        f64x2 v;
        v.x = r[i].x;
        v.y = r[i].y;
        __builtin_nontemporal_store(v, reinterpret_cast<f64x2*>(p + row));
      } else {
        *reinterpret_cast<double2*>(p + row) = r[i];
      }
    } else {
      if (row < n) p[row] = r[i].x;
      if (row + 1 < n) p[row + 1] = r[i].y;
    }
  }
}

__device__ __forceinline__ void zero2(double2 (&r)[kPairs]) {
#pragma unroll
  for (int i = 0; i < kPairs; ++i) r[i] = make_double2(0.0, 0.0);
}

__device__ __forceinline__ double dot2(const double2 (&a)[kPairs], const double2 (&b)[kPairs]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kPairs; ++i) {
    s = fma(a[i].x, b[i].x, s);
    s = fma(a[i].y, b[i].y, s);
  }
  return s;
}

// acc += q * c
__device__ __forceinline__ void axpy2(double2 (&acc)[kPairs], const double2 (&q)[kPairs],
                                      double c) {
#pragma unroll
  for (int i = 0; i < kPairs; ++i) {
    acc[i].x = fma(q[i].x, c, acc[i].x);
    acc[i].y = fma(q[i].y, c, acc[i].y);
  }
}

#ifndef AA_GROUP
#define AA_GROUP 4
#endif
constexpr int kGroup = AA_GROUP;  // Q columns loaded together (kGroup * kPairs loads in flight)

// SplitMix64 (Steele, Lea, Flood 2014): output function of z + golden gamma;
// the library's seeded streams evaluate it at a per-stream origin plus i.
__host__ __device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline uint64_t sm64_mix_host(uint64_t z) { return sm64_mix(z); }

__device__ __forceinline__ double u01(uint64_t z) {
  return (double)(sm64_mix(z) >> 11) * 0x1.0p-53;
}

// Standard normal from counter pair (2e, 2e + 1) of a stream: Box-Muller,
// cosine branch.
__device__ __forceinline__ double normal_at(uint64_t base, uint64_t e) {
  const double u1 = u01(base + 2 * e), u2 = u01(base + 2 * e + 1);
  return sqrt(-2.0 * log1p(-u1)) * cos(6.283185307179586476925286766559 * u2);
}

}  // namespace aa
