// Hi/lo split contraction on the 16-bit matrix cores of gfx950.
//
// An FP32 operand x (after a per-row power-of-two scale s, exact) is stored
// as two 16-bit numbers hi = h(s x), lo = h(s x - hi).  The product of two
// split operands keeps three MFMA terms, a_hi b_hi + a_hi b_lo + a_lo b_hi
// (the dropped a_lo b_lo is below the rounding of the FP32 accumulator for
// FP16 and at 2^-16 relative for BF16), accumulated in FP32 by
// v_mfma_f32_16x16x32_{bf16,f16}.
//
// Lane layout of v_mfma_f32_16x16x32_*: lane l supplies row (or column)
// l%16 and the eight consecutive k values 8*(l/16) .. 8*(l/16)+7 of a 32-wide
// k chunk as one 16-byte LDS read; the output fragment is the same as the
// FP32 16x16 MFMA (lane l holds rows 4*(l/16)+r, column l%16).
#pragma once

#include "common.h"

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));

struct HalfBF16 {
  using raw_t = unsigned short;
  using vec8 = bf16x8_t;
  static constexpr bool SCALED = false;  // FP32 exponent range: no row scaling
  __device__ __forceinline__ static floatx4 mma(vec8 a, vec8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static raw_t from_float(float x) {
    __bf16 h = (__bf16)x;  // round to nearest even
    return __builtin_bit_cast(raw_t, h);
  }
  __device__ __forceinline__ static float to_float(raw_t r) {
    return (float)__builtin_bit_cast(__bf16, r);
  }
};

struct HalfF16 {
  using raw_t = unsigned short;
  using vec8 = f16x8_t;
  static constexpr bool SCALED = true;   // 5-bit exponent: rows scaled by powers of two
  __device__ __forceinline__ static floatx4 mma(vec8 a, vec8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static raw_t from_float(float x) {
    _Float16 h = (_Float16)x;
    return __builtin_bit_cast(raw_t, h);
  }
  __device__ __forceinline__ static float to_float(raw_t r) {
    return (float)__builtin_bit_cast(_Float16, r);
  }
};

// Power-of-two row scale that puts the row maximum in [2^13, 2^14) (FP16), or 1.
template <class H>
__device__ __forceinline__ float split_row_scale(float rowmax) {
  if constexpr (!H::SCALED) {
    return 1.0f;
  } else {
    if (!(rowmax > 0.f) || !isfinite(rowmax)) return 1.0f;
    const int e = ilogbf(rowmax);  // rowmax in [2^e, 2^(e+1))
    return ldexpf(1.0f, 13 - e);
  }
}

// LDS footprint (16-bit elements) of one staged tile set (A_hi, A_lo, B_hi, B_lo).
template <int BM, int BN, int BK>
struct SplitLds {
  static constexpr int LD = BK + 8;  // one 16-byte pad slot per row
  static constexpr int ELEMS = 2 * (BM + BN) * LD;
  static constexpr int BYTES = ELEMS * 2;
};

// Main loop of C[BM x BN] = A B^T with split operands.
// Prob supplies (row, k) -> 16-byte vectors of 8 raw 16-bit values:
//   uint4 load_a(int m, int k, int part) const   part 0 = hi, 1 = lo
//   uint4 load_b(int n, int k, int part) const
// returning zeros outside the problem.  k is a multiple of 8; kdim of 32.
// PIPE as in mfma_tile.h: 0 no prefetch, 1 register prefetch, 2 + double-buffered LDS.
template <class H, int BM, int BN, int BK, int WM, int WN, class Prob, int PIPE = 2>
__device__ __forceinline__ void split_tile_mainloop(const Prob& prob, int kdim,
                                                    floatx4 (&acc)[BM / WM / 16][BN / WN / 16],
                                                    unsigned short* lds) {
  constexpr int NT = WM * WN * 64;
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  constexpr int LD = SplitLds<BM, BN, BK>::LD;
  constexpr int STAGE = SplitLds<BM, BN, BK>::ELEMS;
  constexpr int KV = BK / 8;                // 16-byte vectors per row per part
  constexpr int VA = 2 * BM * KV;           // hi and lo
  constexpr int VB = 2 * BN * KV;
  constexpr int NA = (VA + NT - 1) / NT;
  constexpr int NB = (VB + NT - 1) / NT;
  static_assert(BK % 32 == 0, "BK must be a multiple of 32");
  using vec8 = typename H::vec8;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid / WN;
  const int wn = wid % WN;
  const int lrow = lane & 15;
  const int lk = 8 * (lane >> 4);

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  uint4 ra[NA], rb[NB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int v = tid + t * NT;
      ra[t] = make_uint4(0, 0, 0, 0);
      if (v < VA) {
        const int part = v / (BM * KV), w = v % (BM * KV);
        const int r = w / KV, k = k0 + (w % KV) * 8;
        if (k < kdim) ra[t] = prob.load_a(r, k, part);
      }
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int v = tid + t * NT;
      rb[t] = make_uint4(0, 0, 0, 0);
      if (v < VB) {
        const int part = v / (BN * KV), w = v % (BN * KV);
        const int r = w / KV, k = k0 + (w % KV) * 8;
        if (k < kdim) rb[t] = prob.load_b(r, k, part);
      }
    }
  };
  // stage layout: A_hi [BM][LD], A_lo [BM][LD], B_hi [BN][LD], B_lo [BN][LD]
  auto stash = [&](unsigned short* s) {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int v = tid + t * NT;
      if (v < VA) {
        const int part = v / (BM * KV), w = v % (BM * KV);
        const int r = w / KV, k = (w % KV) * 8;
        *reinterpret_cast<uint4*>(s + (part * BM + r) * LD + k) = ra[t];
      }
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int v = tid + t * NT;
      if (v < VB) {
        const int part = v / (BN * KV), w = v % (BN * KV);
        const int r = w / KV, k = (w % KV) * 8;
        *reinterpret_cast<uint4*>(s + (2 * BM + part * BN + r) * LD + k) = rb[t];
      }
    }
  };
  auto compute = [&](const unsigned short* s, int k0) {
#pragma unroll
    for (int kc = 0; kc < BK; kc += 32) {
      if (k0 + kc >= kdim) break;
      vec8 ah[FM], al[FM];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int r = wm * (BM / WM) + i * 16 + lrow;
        ah[i] = __builtin_bit_cast(vec8, *reinterpret_cast<const uint4*>(s + r * LD + kc + lk));
        al[i] = __builtin_bit_cast(vec8, *reinterpret_cast<const uint4*>(s + (BM + r) * LD + kc + lk));
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int r = wn * (BN / WN) + j * 16 + lrow;
        const vec8 bh = __builtin_bit_cast(vec8, *reinterpret_cast<const uint4*>(s + (2 * BM + r) * LD + kc + lk));
        const vec8 bl = __builtin_bit_cast(vec8, *reinterpret_cast<const uint4*>(s + (2 * BM + BN + r) * LD + kc + lk));
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          acc[i][j] = H::mma(al[i], bh, acc[i][j]);
          acc[i][j] = H::mma(ah[i], bl, acc[i][j]);
          acc[i][j] = H::mma(ah[i], bh, acc[i][j]);
        }
      }
    }
  };

  if constexpr (PIPE == 0) {
    for (int k0 = 0; k0 < kdim; k0 += BK) {
      fetch(k0);
      __syncthreads();
      stash(lds);
      __syncthreads();
      compute(lds, k0);
    }
  } else if constexpr (PIPE == 1) {
    fetch(0);
    for (int k0 = 0; k0 < kdim; k0 += BK) {
      __syncthreads();
      stash(lds);
      __syncthreads();
      if (k0 + BK < kdim) fetch(k0 + BK);
      compute(lds, k0);
    }
  } else {
    fetch(0);
    __syncthreads();
    stash(lds);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < kdim; k0 += BK) {
      const bool more = k0 + BK < kdim;
      if (more) fetch(k0 + BK);
      compute(lds + cur * STAGE, k0);
      if (more) stash(lds + (cur ^ 1) * STAGE);
      __syncthreads();
      cur ^= 1;
    }
  }
}
