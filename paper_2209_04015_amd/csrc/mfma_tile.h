// LDS-staged MFMA tile engine for gfx950.
//
// One workgroup computes a BM x BN tile of C = A B^T over a contraction of
// length kdim.  A is read row-wise with k contiguous (m-major); B is read
// either the same way (n-major, k contiguous) or k-major (n contiguous) and
// transposed into LDS on the way in.  Every contraction of the walker step
// (force bias, VHS build, Taylor products, one-body half steps, exchange)
// instantiates this engine with its own operand loaders and epilogue.
//
// MFMA shapes: v_mfma_f32_16x16x4_f32 (FP32) and v_mfma_f64_16x16x4_f64
// (FP64).  Both are fed 16 consecutive k per LDS step: lane l reads the
// four contiguous k values kc + 4*(l/16) + {0..3} with one 16-byte (FP32)
// or two 16-byte (FP64) LDS reads, and issues four MFMAs, one per offset s.
// Within each MFMA the lanes that share l/16 supply A and B at the same k, so
// the sum over the 16 k values is exact whatever the order.
//
// Output fragment layout.  The hardware places register r of lane l at
//   FP32: row 4*(l/16) + r        FP64: row (l/16) + 4*r      (column l%16)
// of each 16 x 16 block.  The engine loads the A rows of an FP64 tile into
// LDS in the permuted order logical_row(), so that for both types lane l
// holds the LOGICAL rows
//   C[m_base + 4*(l/16) + r][n_base + l%16],  r = 0..3,
// and every epilogue is written once for that layout.
#pragma once

#include "common.h"

template <typename T> struct MF;

template <> struct MF<float> {
  using acc_t = floatx4;
  using vec_t = float4;
  static constexpr int VEC = 4;  // elements per 16-byte vector
  __device__ __forceinline__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ __forceinline__ static vec_t vzero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  // LDS row r of an A tile holds logical row logical_row(r)
  __device__ __forceinline__ static int logical_row(int r) { return r; }
};

template <> struct MF<double> {
  using acc_t = doublex4;
  using vec_t = double2;
  static constexpr int VEC = 2;
  __device__ __forceinline__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ __forceinline__ static vec_t vzero() { return make_double2(0.0, 0.0); }
  // within each 16-row block: hardware row g + 4 r  <->  logical row 4 g + r
  __device__ __forceinline__ static int logical_row(int r) {
    return (r & ~15) | ((r & 3) << 2) | ((r >> 2) & 3);
  }
};

__device__ __forceinline__ float vget(const float4& v, int e) {
  return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}
__device__ __forceinline__ double vget(const double2& v, int e) { return e == 0 ? v.x : v.y; }

// LDS footprint (in elements of T) of one staged A+B tile pair.
template <typename T, int BM, int BN, int BK>
struct TileLds {
  static constexpr int PAD = 16 / (int)sizeof(T);  // one 16-byte slot per row
  static constexpr int LD = BK + PAD;
  static constexpr int ELEMS = (BM + BN) * LD;
  static constexpr int BYTES = ELEMS * (int)sizeof(T);
};

// Main loop.  With PIPE 2 the LDS holds two staged tile pairs (2 x TileLds
// bytes): the next tile is written into the idle buffer after the MFMAs of
// the current one, so each K step needs one barrier instead of two.
// Prob supplies
//   vec_t load_a(int batch, int m, int k) const      (m-major A, k contiguous)
//   vec_t load_b(int batch, int n, int k) const      (n-major B)        if !B_KMAJOR
//   vec_t load_b_km(int batch, int k, int n) const   (k-major B, n contiguous) if B_KMAJOR
// and must return zeros for m or n outside its problem.  k >= kdim is zero-filled here.
// PIPE: 0 = no prefetch (load, stage, compute: fewest registers, for two
// workgroups per CU that cover each other's memory waits), 1 = the next tile
// is prefetched into registers during the MFMAs, 2 = 1 plus double-buffered LDS.
template <typename T, int BM, int BN, int BK, int WM, int WN, bool B_KMAJOR, class Prob,
          int PIPE = 1>
__device__ __forceinline__ void mfma_tile_mainloop(
    const Prob& prob, int batch, int m0, int n0, int kdim,
    typename MF<T>::acc_t (&acc)[BM / WM / 16][BN / WN / 16], T* lds) {
  using M = MF<T>;
  using vec_t = typename M::vec_t;
  constexpr int VEC = M::VEC;
  constexpr int NT = WM * WN * 64;
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  constexpr int LD = TileLds<T, BM, BN, BK>::LD;
  constexpr int VA = BM * BK / VEC;  // vectors per A tile
  constexpr int VB = BN * BK / VEC;
  constexpr int NA = (VA + NT - 1) / NT;
  // k-major B is moved in VEC x VEC blocks (VEC k rows of VEC n values),
  // transposed in registers and stored as vectors along k
  constexpr int KBLK = BK / VEC, NBLK = BN / VEC;
  constexpr int VBB = B_KMAJOR ? KBLK * NBLK : VB;
  constexpr int NB = (VBB + NT - 1) / NT;
  constexpr int RB = B_KMAJOR ? VEC : 1;  // vectors held per block
  static_assert(BK % 16 == 0, "BK must be a multiple of 16");
  static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "tile/wave mismatch");

  T* As = lds;
  T* Bs = lds + BM * LD;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid / WN;
  const int wn = wid % WN;
  const int lrow = lane & 15;
  const int lk = 4 * (lane >> 4);

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = M::zero();

  vec_t ra[NA], rb[NB][RB];

  auto fetch = [&](int k0) {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int v = tid + t * NT;
      ra[t] = M::vzero();
      if (v < VA) {
        const int r = v / (BK / VEC);
        const int k = k0 + (v % (BK / VEC)) * VEC;
        if (k < kdim) ra[t] = prob.load_a(batch, m0 + M::logical_row(r), k);
      }
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int v = tid + t * NT;
#pragma unroll
      for (int e = 0; e < RB; ++e) rb[t][e] = M::vzero();
      if (v < VBB) {
        if constexpr (!B_KMAJOR) {
          const int r = v / (BK / VEC);
          const int k = k0 + (v % (BK / VEC)) * VEC;
          if (k < kdim) rb[t][0] = prob.load_b(batch, n0 + r, k);
        } else {
          const int kb = v % KBLK, nb = v / KBLK;
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            const int k = k0 + kb * VEC + e;
            if (k < kdim) rb[t][e] = prob.load_b_km(batch, k, n0 + nb * VEC);
          }
        }
      }
    }
  };
  auto stash = [&](T* As, T* Bs) {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int v = tid + t * NT;
      if (v < VA) {
        const int r = v / (BK / VEC);
        const int k = (v % (BK / VEC)) * VEC;
        *reinterpret_cast<vec_t*>(As + r * LD + k) = ra[t];
      }
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int v = tid + t * NT;
      if (v < VBB) {
        if constexpr (!B_KMAJOR) {
          const int r = v / (BK / VEC);
          const int k = (v % (BK / VEC)) * VEC;
          *reinterpret_cast<vec_t*>(Bs + r * LD + k) = rb[t][0];
        } else {
          const int kb = v % KBLK, nb = v / KBLK;
#pragma unroll
          for (int c = 0; c < VEC; ++c) {
            vec_t w;
            if constexpr (VEC == 4) {
              w = make_float4(vget(rb[t][0], c), vget(rb[t][1], c), vget(rb[t][2], c), vget(rb[t][3], c));
            } else {
              w = make_double2(vget(rb[t][0], c), vget(rb[t][1], c));
            }
            *reinterpret_cast<vec_t*>(Bs + (nb * VEC + c) * LD + kb * VEC) = w;
          }
        }
      }
    }
  };

  auto compute = [&](const T* Asb, const T* Bsb, int k0) {
#pragma unroll
    for (int kc = 0; kc < BK; kc += 16) {
      if (k0 + kc >= kdim) break;  // zero-padded tail: no MFMA work
      T a[FM][4], b[FN][4];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const T* p = Asb + (wm * (BM / WM) + i * 16 + lrow) * LD + kc + lk;
        if constexpr (VEC == 4) {
          const float4 x = *reinterpret_cast<const float4*>(p);
          a[i][0] = x.x; a[i][1] = x.y; a[i][2] = x.z; a[i][3] = x.w;
        } else {
          const double2 x = *reinterpret_cast<const double2*>(p);
          const double2 y = *reinterpret_cast<const double2*>(p + 2);
          a[i][0] = x.x; a[i][1] = x.y; a[i][2] = y.x; a[i][3] = y.y;
        }
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const T* p = Bsb + (wn * (BN / WN) + j * 16 + lrow) * LD + kc + lk;
        if constexpr (VEC == 4) {
          const float4 x = *reinterpret_cast<const float4*>(p);
          b[j][0] = x.x; b[j][1] = x.y; b[j][2] = x.z; b[j][3] = x.w;
        } else {
          const double2 x = *reinterpret_cast<const double2*>(p);
          const double2 y = *reinterpret_cast<const double2*>(p + 2);
          b[j][0] = x.x; b[j][1] = x.y; b[j][2] = y.x; b[j][3] = y.y;
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[i][j] = M::mma(a[i][s], b[j][s], acc[i][j]);
    }
  };

  if constexpr (PIPE == 0) {
    for (int k0 = 0; k0 < kdim; k0 += BK) {
      fetch(k0);
      __syncthreads();
      stash(As, Bs);
      __syncthreads();
      compute(As, Bs, k0);
    }
  } else if constexpr (PIPE == 1) {
    fetch(0);
    for (int k0 = 0; k0 < kdim; k0 += BK) {
      __syncthreads();
      stash(As, Bs);
      __syncthreads();
      if (k0 + BK < kdim) fetch(k0 + BK);
      compute(As, Bs, k0);
    }
  } else {
    constexpr int STAGE = (BM + BN) * LD;
    fetch(0);
    __syncthreads();  // LDS may still be read by a previous use of the buffer
    stash(As, Bs);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < kdim; k0 += BK) {
      const bool more = k0 + BK < kdim;
      if (more) fetch(k0 + BK);
      compute(lds + cur * STAGE, lds + cur * STAGE + BM * LD, k0);
      if (more) stash(lds + (cur ^ 1) * STAGE, lds + (cur ^ 1) * STAGE + BM * LD);
      __syncthreads();
      cur ^= 1;
    }
  }
}
