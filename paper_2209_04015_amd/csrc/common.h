// Shared device/host helpers for the phaseless-AFQMC walker-step library.
// gfx950 (CDNA4) only: 64-wide wavefronts, MFMA matrix cores, 160 KB LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

#define AFQMC_WAVE 64

static inline int round_up(int x, int m) { return (x + m - 1) / m * m; }
static inline int ceil_div(int x, int m) { return (x + m - 1) / m; }

// ---------------------------------------------------------------------------
// complex helpers (double2 = re, im)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
// a^-1
__device__ __forceinline__ double2 cinv(double2 a) {
  double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}
// complex log: log|a| + i arg(a)
__device__ __forceinline__ double2 clog(double2 a) {
  return make_double2(0.5 * log(a.x * a.x + a.y * a.y), atan2(a.y, a.x));
}

// ---------------------------------------------------------------------------
// wave / block reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, AFQMC_WAVE);
  return v;
}
__device__ __forceinline__ double2 wave_sum2(double2 v) {
  v.x = wave_sum(v.x);
  v.y = wave_sum(v.y);
  return v;
}

// Sum over the whole block of a double2; result valid in every thread.
// `red` must hold blockDim.x / 64 double2 entries.
__device__ __forceinline__ double2 block_sum2(double2 v, double2* red) {
  v = wave_sum2(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  for (int w = 0; w < nw; ++w) s = cadd(s, red[w]);  // fixed order: deterministic
  return s;
}

// Status-word bits are the AFQMC_STATUS_* values of the public header.
#include "../../include/afqmc.h"
