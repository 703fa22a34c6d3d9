// Hi/lo split contraction on the 16-bit matrix cores of gfx950.
//
// An FP32 operand x (after a per-row power-of-two scale s, exact) is stored
// as two 16-bit numbers hi = h(s x), lo = h(s x - hi).  The product of two
// split operands keeps three MFMA terms, a_hi b_hi + a_hi b_lo + a_lo b_hi
// (the dropped a_lo b_lo is below the rounding of the FP32 accumulator for
// FP16 and at 2^-16 relative for BF16), accumulated in FP32 by
// v_mfma_f32_16x16x32_{bf16,f16}.
//
// Operand rows in memory: for every block of 32 contraction indices, 32 hi
// values then the 32 matching lo values (128 bytes, one cache line), so one
// k step of a tile reads whole lines.
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
// The scale stops at 2^127, the largest finite power of two: rows whose
// maximum lies below 2^-114 come out below 2^13 (their hi / lo parts may fall
// under the FP16 normal range, at magnitudes far below every other term).
template <class H>
__device__ __forceinline__ float split_row_scale(float rowmax) {
  if constexpr (!H::SCALED) {
    return 1.0f;
  } else {
    if (!(rowmax > 0.f) || !isfinite(rowmax)) return 1.0f;
    const int k = 13 - ilogbf(rowmax);  // rowmax in [2^(13-k), 2^(14-k))
    return ldexpf(1.0f, k < 127 ? k : 127);
  }
}

// Half-precision elements per k block in memory (32 hi + 32 lo).
constexpr int SPLIT_KB = 64;
// LDS row of one staged k block: 64 halves plus one 16-byte pad slot, so
// that the 16-byte fragment reads of 8 consecutive rows fall in 8 distinct
// bank groups.
constexpr int SPLIT_SLD = SPLIT_KB + 8;

template <int BM, int BN>
struct SplitStage {
  static constexpr int BYTES = (BM + BN) * SPLIT_SLD * 2;
};

// Byte offset that lies outside every operand buffer: a bounds-checked
// buffer load from it returns zeros.
constexpr int SPLIT_ROW_NONE = 0x7fffffff;

// Power-of-two exponent e putting 2^e b in [2^13, 2^14) (0 for b zero, not
// finite or not positive; at most 64): the scale of a split VHS, from a
// bound b on the magnitudes of a walker's VHS entries.  The VHS build and
// the propagation that reads its split rows take it from the same bound.
__device__ __forceinline__ int vhs_split_exp(float b) {
  if (!(b > 0.f) || !isfinite(b)) return 0;
  const int e = 13 - ilogbf(b);
  return e < 64 ? e : 64;
}

// Buffer resource over n_bytes (< 2^31) of split rows: raw (stride 0),
// bounds-checked loads.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t split_rsrc(const void* base, int n_bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n_bytes, 0x00020000);
}

// Main loop of C[BM x BN] = A B^T with split operands, one k block (32
// contraction indices) per stage, the next DEPTH blocks prefetched into
// registers while the matrix cores work on the current one (DEPTH 2 keeps
// two blocks of loads in flight, for long contractions whose loads come
// from beyond the L2).
//   a_rsrc / b_rsrc: buffer resources over the operand rows;
//   a_off[t] / b_off[t]: byte offset of the 16-byte chunk this thread stages
//   in slot t for the first k block, or SPLIT_ROW_NONE for rows outside the
//   problem (the bounds check stages zeros).  k block kb lies kb * 128 bytes
//   further (scalar offset).
// Thread tid stages chunk tid % 8 of rows tid / 8 + 32 t.
template <class H, int BM, int BN, int WM, int WN, int DEPTH = 1>
__device__ __forceinline__ void split_tile_mainloop(__amdgpu_buffer_rsrc_t a_rsrc, __amdgpu_buffer_rsrc_t b_rsrc,
                                                    const int (&a_off)[BM * 8 / (WM * WN * 64)],
                                                    const int (&b_off)[BN * 8 / (WM * WN * 64)],
                                                    int nkb, floatx4 (&acc)[BM / WM / 16][BN / WN / 16],
                                                    unsigned short* lds) {
  constexpr int NT = WM * WN * 64;
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  constexpr int NA = BM * 8 / NT;
  constexpr int NB = BN * 8 / NT;
  static_assert(BM * 8 % NT == 0 && BN * 8 % NT == 0, "rows must split evenly over the threads");
  using vec8 = typename H::vec8;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid / WN;
  const int wn = wid % WN;
  const int lrow = lane & 15;
  const int lk = 8 * (lane >> 4);
  const int srow = tid >> 3, schunk = tid & 7;

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  uint4 ra[DEPTH][NA], rb[DEPTH][NB];
  // k block kb into register set s (a block past the last one reads rows of
  // the same buffers or, past their end, zeros: never staged)
  auto fetch = [&](int s, int kb) {
    const int o = kb * (SPLIT_KB * 2);
#pragma unroll
    for (int t = 0; t < NA; ++t)
      ra[s][t] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(a_rsrc, a_off[t], o, 0));
#pragma unroll
    for (int t = 0; t < NB; ++t)
      rb[s][t] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(b_rsrc, b_off[t], o, 0));
  };
  auto stash = [&](int s) {
#pragma unroll
    for (int t = 0; t < NA; ++t)
      *reinterpret_cast<uint4*>(lds + (srow + t * (NT / 8)) * SPLIT_SLD + schunk * 8) = ra[s][t];
#pragma unroll
    for (int t = 0; t < NB; ++t)
      *reinterpret_cast<uint4*>(lds + (BM + srow + t * (NT / 8)) * SPLIT_SLD + schunk * 8) = rb[s][t];
  };
  // The B fragments of column block j + 1 are read before the matrix-core
  // work of block j is issued, so their LDS latency is covered by it.
  auto compute = [&]() {
    vec8 ah[FM], al[FM];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const unsigned short* r = lds + (wm * (BM / WM) + i * 16 + lrow) * SPLIT_SLD + lk;
      ah[i] = __builtin_bit_cast(vec8, *reinterpret_cast<const uint4*>(r));
      al[i] = __builtin_bit_cast(vec8, *reinterpret_cast<const uint4*>(r + 32));
    }
    auto bfrag = [&](int j, vec8& bh, vec8& bl) {
      const unsigned short* r = lds + (BM + wn * (BN / WN) + j * 16 + lrow) * SPLIT_SLD + lk;
      bh = __builtin_bit_cast(vec8, *reinterpret_cast<const uint4*>(r));
      bl = __builtin_bit_cast(vec8, *reinterpret_cast<const uint4*>(r + 32));
    };
    vec8 bh[2], bl[2];
    bfrag(0, bh[0], bl[0]);
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      if (j + 1 < FN) bfrag(j + 1, bh[(j + 1) & 1], bl[(j + 1) & 1]);
      __builtin_amdgcn_sched_barrier(0);  // keep those reads ahead of this block's MFMAs
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        acc[i][j] = H::mma(al[i], bh[j & 1], acc[i][j]);
        acc[i][j] = H::mma(ah[i], bl[j & 1], acc[i][j]);
        acc[i][j] = H::mma(ah[i], bh[j & 1], acc[i][j]);
      }
    }
  };

  if constexpr (DEPTH == 1) {
    fetch(0, 0);
    for (int kb = 0; kb < nkb; ++kb) {
      if (kb) __syncthreads();  // every wave is done with the previous stage
      stash(0);
      __syncthreads();
      if (kb + 1 < nkb) fetch(0, kb + 1);
      compute();
    }
  } else {
    static_assert(DEPTH == 2, "prefetch depth 1 or 2");
    // straight-line pairs of blocks with unconditional fetches, so that the
    // wait before each stash leaves the other set's loads in flight
    fetch(0, 0);
    fetch(1, 1);
    for (int kb = 0; kb < nkb; kb += 2) {
      if (kb) __syncthreads();
      stash(0);
      __syncthreads();
      fetch(0, kb + 2);
      compute();
      if (kb + 1 >= nkb) break;
      __syncthreads();
      stash(1);
      __syncthreads();
      fetch(1, kb + 3);
      compute();
    }
  }
}
