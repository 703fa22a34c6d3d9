// The propagation phi' = P T6(VHS) P phi of Eq. Bx (symmetric split, Taylor
// series of the exponential truncated after the 6th-order term) in one launch
// per step, on the 16-bit split matrix cores (FP16X3).
//
// One workgroup owns one (walker, spin): its 2 n_s real orbital columns never
// leave the chip between the first one-body half step and the last.  The
// series is evaluated by Horner's rule,
//   v_{K+1} = t0,  v_k = t0 + VHS v_{k+1} / k  (k = K .. 1),  T_K(VHS) t0 = v_1,
// with t0 = P phi; it equals the sum of the terms VHS^k t0 / k! up to
// rounding.  v (hi/lo fp16 pairs, the B operand of every product) and t0
// (FP32) live in LDS; the walker's FP32 VHS rows are streamed from memory
// straight into registers and split there (the scale from max |VHS| of the
// finished build), once per order, with no LDS staging and no barrier inside
// a product.  The two spins of a walker get workgroup ids 8 apart, so they
// run on one XCD and the second stream of the VHS rows comes from its L2.
//
// Lanes and fragments (v_mfma_f32_16x16x32_f16): eight waves, two per SIMD
// (one wave per SIMD issues matrix instructions too slowly to keep the
// matrix core busy); wave w owns the 16-row tiles w + 8 i of the output and
// every column tile (it streams those VHS rows itself); a 16-wide column
// tile holds orbitals j0 .. j0+7, lanes n < 8 the real parts and lanes
// n >= 8 the imaginary parts (comp = n / 8).
// LDS layouts, per orbital j:
//   v: 16-byte chunks per four rows q: Re v[q..q+3][j] then Im v[q..q+3][j]
//      (fp16; one plane of hi parts, one of lo parts);
//   t0: one FP32 plane per component, rows q contiguous.
// B operands:
//   VHS step, k = (q, re|im) interleaved: B[(j,re)] = (Re v, -Im v) pairs,
//   B[(j,im)] = (Im v, Re v) pairs, built from one chunk with v_perm (the
//   selector per lane) and a sign flip of the high halves for comp 0;
//   P step, k = q: the lane's component of eight consecutive q, two 8-byte
//   reads.
// Scales: one power of two per (walker, spin) and operand (max |phi|, max
// |t0|, max |v_k|; max |VHS| of the walker, recorded by the VHS build) and
// one for P, exact and undone in each epilogue.

#include <cmath>
#include <cstring>

#include "common.h"
#include "kernels.h"
#include "split_tile.h"

namespace {

constexpr int PF_RG = 8;                     // row groups: two waves per SIMD
constexpr int PF_CG = 1;                     // column groups
constexpr int PF_WAVES = PF_RG * PF_CG;
constexpr int PF_NT = PF_WAVES * 64;
constexpr int PF_FM = 3;                     // row tiles per wave
constexpr int PF_MAX_RT = 20;                // 20 row tiles: N <= 320 (the LDS bound)
constexpr int PF_MAX_CT = 4;                 // 4 column tiles: n_s <= 32

// column tiles per wave
template <int CT>
struct PfCols {
  static constexpr int W = (CT + PF_CG - 1) / PF_CG;
};

struct PropFusedArgs {
  double2* phi_a;                // [W][N][na] in / out
  double2* phi_b;                // [W][N][nb] in / out
  const float* vhs;              // [W][N][ldV] interleaved complex
  const unsigned* vmax;          // [W] max |VHS| (float bits)
  const unsigned short* psplit;  // [QP][nkbP][64] P split, scaled by 2^pexp
  int W, N, na, nb, ldV, RT, QP, QCH, TQS, nkbP, order, pexp, nspin;
  float sa;                      // the walker's VHS scale (set per workgroup)
};

__device__ __forceinline__ float pf_block_max(float v, float* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  __syncthreads();  // earlier readers of red are done (and every wave is past its product)
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = red[0];
#pragma unroll
  for (int w = 1; w < PF_WAVES; ++w) r = fmaxf(r, red[w]);
  return r;
}

// power-of-two scale putting m in [2^13, 2^14), as an exponent
__device__ __forceinline__ int pf_scale_exp(float m) {
  if (!(m > 0.f) || !isfinite(m)) return 0;
  return 13 - ilogbf(m);
}

// hi and lo fp16 halves of four values, packed two per word
__device__ __forceinline__ void pf_split4(float x0, float x1, float x2, float x3, uint2& hi, uint2& lo) {
  const float x[4] = {x0, x1, x2, x3};
  unsigned short h[4], l[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const _Float16 a = (_Float16)x[e];
    h[e] = __builtin_bit_cast(unsigned short, a);
    l[e] = __builtin_bit_cast(unsigned short, (_Float16)(x[e] - (float)a));
  }
  hi = make_uint2((unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16));
  lo = make_uint2((unsigned)l[0] | ((unsigned)l[1] << 16), (unsigned)l[2] | ((unsigned)l[3] << 16));
}

// The three products of column tile t for the wave's nv real row tiles (nv
// is wave-uniform: scalar branches).  Each product kind is issued for all
// row tiles before the next, so that dependent MFMAs on one accumulator are
// several instructions apart.
template <int CW>
__device__ __forceinline__ void pf_mma_tiles(floatx4 (&acc)[PF_FM][CW], const f16x8_t (&ah)[PF_FM],
                                             const f16x8_t (&al)[PF_FM], const f16x8_t& bh, const f16x8_t& bl,
                                             int t, int nv) {
#pragma unroll
  for (int i = 0; i < PF_FM; ++i)
    if (i < nv) acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], bh, acc[i][t], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < PF_FM; ++i)
    if (i < nv) acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bl, acc[i][t], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < PF_FM; ++i)
    if (i < nv) acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bh, acc[i][t], 0, 0, 0);
}

struct PfCtx {
  int lane, wid, lrow, kg;  // kg = lane / 16
  int rg, cg;               // the wave's row group (row tiles rg + PF_RG i) and column group
  int nv;                   // the wave's real row tiles
  int jl, comp;             // this lane's column: orbital offset in a tile, re (0) / im (1)
};

template <int CW>
__device__ __forceinline__ void pf_zero(floatx4 (&acc)[PF_FM][CW]) {
#pragma unroll
  for (int i = 0; i < PF_FM; ++i)
#pragma unroll
    for (int t = 0; t < CW; ++t) acc[i][t] = floatx4{0.f, 0.f, 0.f, 0.f};
}

// first orbital of the wave's column tile t, or -1 past the walker's tiles
template <int CT>
__device__ __forceinline__ int pf_col0(const PfCtx& c, int t) {
  const int tg = c.cg * PfCols<CT>::W + t;
  return tg < CT ? 8 * tg : -1;
}

// acc = P v (k = q), v from the LDS planes
template <int CT>
__device__ __forceinline__ void pf_product_p(const PropFusedArgs& p, const PfCtx& c, const uint4* u_hi,
                                             const uint4* u_lo, floatx4 (&acc)[PF_FM][PfCols<CT>::W]) {
  constexpr int CW = PfCols<CT>::W;
  pf_zero<CW>(acc);
  // A rows of this lane: byte offsets of its 16-byte chunks in the first k
  // block (bounds-checked loads: a block past the last reads zeros or rows
  // that are never used)
  const __amdgpu_buffer_rsrc_t prs = split_rsrc(p.psplit, p.QP * p.nkbP * SPLIT_KB * 2);
  int arow[PF_FM];
#pragma unroll
  for (int i = 0; i < PF_FM; ++i) {
    const int rt = c.rg + PF_RG * i;
    arow[i] = rt < p.RT ? (((rt * 16 + c.lrow) * p.nkbP * SPLIT_KB) + 8 * c.kg) * 2 : SPLIT_ROW_NONE;
  }
  uint4 pa_h[PF_FM], pa_l[PF_FM];
  auto fetch = [&](int kb) {
#pragma unroll
    for (int i = 0; i < PF_FM; ++i) {
      pa_h[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(prs, arow[i], kb * 128, 0));
      pa_l[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(prs, arow[i], kb * 128 + 64, 0));
    }
  };
  fetch(0);
  for (int kb = 0; kb < p.nkbP; ++kb) {
    f16x8_t ah[PF_FM], al[PF_FM];
#pragma unroll
    for (int i = 0; i < PF_FM; ++i) {
      ah[i] = __builtin_bit_cast(f16x8_t, pa_h[i]);
      al[i] = __builtin_bit_cast(f16x8_t, pa_l[i]);
    }
    fetch(kb + 1);  // unconditional (see above), so the wait counts stay exact
    const int ch = 8 * kb + 2 * c.kg;  // first of the two chunks of q0 .. q0+7
    const bool qok = 4 * ch < p.QP;
#pragma unroll
    for (int t = 0; t < CW; ++t) {
      const int j0 = pf_col0<CT>(c, t);
      if (j0 < 0) break;  // uniform
      uint4 hw = make_uint4(0u, 0u, 0u, 0u), lw = hw;
      if (qok) {
        const int o = (j0 + c.jl) * p.QCH + ch;
        const uint2* h = reinterpret_cast<const uint2*>(u_hi + o) + c.comp;
        const uint2* l = reinterpret_cast<const uint2*>(u_lo + o) + c.comp;
        const uint2 h0 = h[0], h1 = h[2], l0 = l[0], l1 = l[2];  // chunks ch and ch + 1
        hw = make_uint4(h0.x, h0.y, h1.x, h1.y);
        lw = make_uint4(l0.x, l0.y, l1.x, l1.y);
      }
      pf_mma_tiles<CW>(acc, ah, al, __builtin_bit_cast(f16x8_t, hw), __builtin_bit_cast(f16x8_t, lw), t, c.nv);
    }
  }
}

// acc = VHS v (k = (q, re|im)), the VHS rows streamed from memory into
// registers and split there with the walker's power-of-two scale p.sa
template <int CT>
__device__ __forceinline__ void pf_product_v(const PropFusedArgs& p, const PfCtx& c, __amdgpu_buffer_rsrc_t vrs,
                                             const uint4* u_hi, const uint4* u_lo,
                                             floatx4 (&acc)[PF_FM][PfCols<CT>::W]) {
  constexpr int CW = PfCols<CT>::W;
  pf_zero<CW>(acc);
  // byte offsets of this lane's 8 floats of the first k block; rows past N
  // (and past the tiles) lie outside the buffer and read as zeros
  int aoff[PF_FM];
#pragma unroll
  for (int i = 0; i < PF_FM; ++i) {
    const int rt = c.rg + PF_RG * i;
    aoff[i] = rt < p.RT ? ((rt * 16 + c.lrow) * p.ldV + 8 * c.kg) * 4 : SPLIT_ROW_NONE;
  }
  // per-lane v_perm selectors: (Re, Im) or (Im, Re) pairs of q0+m, and the
  // sign flip of the high halves for the real-part columns
  const unsigned sel0 = c.comp ? 0x01000504u : 0x05040100u;
  const unsigned sel1 = c.comp ? 0x03020706u : 0x07060302u;
  const unsigned flip = c.comp ? 0u : 0x80000000u;
  auto bop = [&](const uint4& d) {  // d = (re0 re1, re2 re3, im0 im1, im2 im3)
    return __builtin_bit_cast(f16x8_t,
                              make_uint4(__builtin_amdgcn_perm(d.z, d.x, sel0) ^ flip,
                                         __builtin_amdgcn_perm(d.z, d.x, sel1) ^ flip,
                                         __builtin_amdgcn_perm(d.w, d.y, sel0) ^ flip,
                                         __builtin_amdgcn_perm(d.w, d.y, sel1) ^ flip));
  };
  int ob[CW];  // the wave's column tiles: first LDS chunk of orbital j0 + jl (or none)
#pragma unroll
  for (int t = 0; t < CW; ++t) {
    const int j0 = pf_col0<CT>(c, t);
    ob[t] = j0 < 0 ? -1 : (j0 + c.jl) * p.QCH + c.kg;
  }
  const int nkb = p.RT;
  float4 ra[2][PF_FM][2];
  auto fetch = [&](int s, int kb) {
#pragma unroll
    for (int i = 0; i < PF_FM; ++i) {
      ra[s][i][0] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(vrs, aoff[i], kb * 128, 0));
      ra[s][i][1] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(vrs, aoff[i], kb * 128 + 16, 0));
    }
  };
  auto compute = [&](int s, int kb) {
    f16x8_t ah[PF_FM], al[PF_FM];
#pragma unroll
    for (int i = 0; i < PF_FM; ++i) {
      const float x[8] = {ra[s][i][0].x * p.sa, ra[s][i][0].y * p.sa, ra[s][i][0].z * p.sa, ra[s][i][0].w * p.sa,
                          ra[s][i][1].x * p.sa, ra[s][i][1].y * p.sa, ra[s][i][1].z * p.sa, ra[s][i][1].w * p.sa};
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const _Float16 h = (_Float16)x[e];
        ah[i][e] = h;
        al[i][e] = (_Float16)(x[e] - (float)h);
      }
    }
#pragma unroll
    for (int t = 0; t < CW; ++t) {
      if (ob[t] < 0) break;  // uniform
      const uint4 dh = u_hi[ob[t] + 4 * kb], dl = u_lo[ob[t] + 4 * kb];
      pf_mma_tiles<CW>(acc, ah, al, bop(dh), bop(dl), t, c.nv);
    }
  };
  // two k blocks of loads in flight: fetch kb + 2 while working on kb.  The
  // fetches are unconditional (past the last block they read the next rows
  // or, past the buffer, zeros; never used), so that every wait leaves the
  // other set's loads in flight.
  fetch(0, 0);
  fetch(1, 1);
  int kb = 0;
  // The scheduling barriers keep each set's loads after the work that reads
  // the set before them, so that no wait covers the other set.
  for (; kb + 2 <= nkb; kb += 2) {  // one regular body: the waits stay exact across the back edge
    compute(0, kb);
    __builtin_amdgcn_sched_barrier(0);
    fetch(0, kb + 2);
    __builtin_amdgcn_sched_barrier(0);
    compute(1, kb + 1);
    __builtin_amdgcn_sched_barrier(0);
    fetch(1, kb + 3);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (kb < nkb) compute(0, kb);
}

// v (values of the accumulator layout, scaled by 2^e) into the LDS planes:
// each lane stores its component of four rows, hi and lo
template <int CT>
__device__ __forceinline__ void pf_store_v(const PropFusedArgs& p, const PfCtx& c,
                                           const floatx4 (&v)[PF_FM][PfCols<CT>::W], int e, uint4* u_hi,
                                           uint4* u_lo) {
  constexpr int CW = PfCols<CT>::W;
#pragma unroll
  for (int i = 0; i < PF_FM; ++i) {
    const int rt = c.rg + PF_RG * i;
    if (rt >= p.RT) break;  // uniform: a wave's real tiles come first
    const int ch = rt * 4 + c.kg;
#pragma unroll
    for (int t = 0; t < CW; ++t) {
      const int j0 = pf_col0<CT>(c, t);
      if (j0 < 0) break;  // uniform
      uint2 hw, lw;
      pf_split4(ldexpf(v[i][t][0], e), ldexpf(v[i][t][1], e), ldexpf(v[i][t][2], e), ldexpf(v[i][t][3], e), hw,
                lw);
      const int o = (j0 + c.jl) * p.QCH + ch;
      reinterpret_cast<uint2*>(u_hi + o)[c.comp] = hw;
      reinterpret_cast<uint2*>(u_lo + o)[c.comp] = lw;
    }
  }
}

template <int CT>
__global__ __launch_bounds__(PF_NT, 1) void prop_fused_kernel(PropFusedArgs p) {
  constexpr int CW = PfCols<CT>::W;
  extern __shared__ __attribute__((aligned(16))) uint4 pf_lds[];
  constexpr int JC = 8 * CT;
  uint4* u_hi = pf_lds;                                          // [JC][QCH] chunks
  uint4* u_lo = u_hi + JC * p.QCH;
  float* t0p = reinterpret_cast<float*>(u_lo + JC * p.QCH);     // [2][JC][TQS]
  float* red = t0p + 2 * JC * p.TQS;                             // [PF_WAVES] doubles or floats
  // (walker, spin): the two spins of a walker 8 ids apart (one XCD)
  int z, sp;
  if (p.nspin == 2) {
    z = (blockIdx.x >> 4) * 8 + (blockIdx.x & 7);
    sp = (blockIdx.x >> 3) & 1;
  } else {
    z = blockIdx.x;
    sp = 0;
  }
  if (z >= p.W) return;  // uniform: the padding ids of the last group of eight
  const int ns = sp ? p.nb : p.na;
  double2* ph = sp ? p.phi_b + (size_t)z * p.N * p.nb : p.phi_a + (size_t)z * p.N * p.na;
  const int tid = threadIdx.x;
  PfCtx c;
  c.lane = tid & 63;
  c.wid = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: scalar branches on tiles
  c.rg = c.wid % PF_RG;
  c.cg = c.wid / PF_RG;
  c.nv = c.rg < p.RT ? min(PF_FM, (p.RT - 1 - c.rg) / PF_RG + 1) : 0;
  c.lrow = c.lane & 15;
  c.kg = c.lane >> 4;
  c.jl = c.lane & 7;
  c.comp = (c.lane >> 3) & 1;

  // ---- phi into LDS, scaled by 2^e (the scale taken in FP64, so that any
  // FP64 walker fits the fp16 range) ----
  double dm = 0.0;
  for (int e = tid; e < p.N * ns; e += PF_NT) {
    const double2 x = ph[e];
    dm = fmax(dm, fmax(fabs(x.x), fabs(x.y)));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o, 64));
  if (c.lane == 0) reinterpret_cast<double*>(red)[c.wid] = dm;
  __syncthreads();
  dm = reinterpret_cast<const double*>(red)[0];
#pragma unroll
  for (int w = 1; w < PF_WAVES; ++w) dm = fmax(dm, reinterpret_cast<const double*>(red)[w]);
  int es = (dm > 0.0 && isfinite(dm)) ? 13 - ilogb(dm) : 0;
  const int nch = p.QP / 4;
  for (int e = tid; e < JC * nch; e += PF_NT) {
    const int j = e % JC, ch = e / JC;
    float re[4], im[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = 4 * ch + r;
      double2 x = make_double2(0.0, 0.0);
      if (q < p.N && j < ns) x = ph[(size_t)q * ns + j];
      re[r] = (float)ldexp(x.x, es);
      im[r] = (float)ldexp(x.y, es);
    }
    uint2 rh, rl, ih, il;
    pf_split4(re[0], re[1], re[2], re[3], rh, rl);
    pf_split4(im[0], im[1], im[2], im[3], ih, il);
    u_hi[j * p.QCH + ch] = make_uint4(rh.x, rh.y, ih.x, ih.y);
    u_lo[j * p.QCH + ch] = make_uint4(rl.x, rl.y, il.x, il.y);
  }
  __syncthreads();

  floatx4 acc[PF_FM][CW];
  // t0 of the lane's fragment (i, t): component comp, orbital j0 + jl, rows q0 .. q0+3
  auto t0_at = [&](int i, int j0) -> float4* {
    const int q0 = (c.rg + PF_RG * i) * 16 + 4 * c.kg;
    return reinterpret_cast<float4*>(t0p + (c.comp * JC + j0 + c.jl) * p.TQS + q0);
  };

  // ---- t0 = P phi ----
  pf_product_p<CT>(p, c, u_hi, u_lo, acc);
  float m = 0.f;
  {
    const int ex = -(es + p.pexp);
#pragma unroll
    for (int i = 0; i < PF_FM; ++i) {
      if (c.rg + PF_RG * i >= p.RT) break;  // uniform
#pragma unroll
      for (int t = 0; t < CW; ++t) {
        const int j0 = pf_col0<CT>(c, t);
        if (j0 < 0) break;  // uniform
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc[i][t][r] = ldexpf(acc[i][t][r], ex);
          m = fmaxf(m, fabsf(acc[i][t][r]));
        }
        *t0_at(i, j0) = make_float4(acc[i][t][0], acc[i][t][1], acc[i][t][2], acc[i][t][3]);
      }
    }
  }
  es = pf_scale_exp(pf_block_max(m, red));  // every wave is past its product: v may be overwritten
  pf_store_v<CT>(p, c, acc, es, u_hi, u_lo);
  __syncthreads();

  // ---- Horner: v = t0 + VHS v / k, k = order .. 1 ----
  const int sa_exp = pf_scale_exp(__uint_as_float(p.vmax[z]));  // the scale of the split VHS rows
  p.sa = ldexpf(1.f, sa_exp);
  const __amdgpu_buffer_rsrc_t vrs = split_rsrc(p.vhs + (size_t)z * p.N * p.ldV, p.N * p.ldV * 4);
  for (int k = p.order; k >= 1; --k) {
    pf_product_v<CT>(p, c, vrs, u_hi, u_lo, acc);
    const int ex = -(es + sa_exp);
    const float rk = 1.f / (float)k;
    m = 0.f;
#pragma unroll
    for (int i = 0; i < PF_FM; ++i) {
      if (c.rg + PF_RG * i >= p.RT) break;  // uniform
#pragma unroll
      for (int t = 0; t < CW; ++t) {
        const int j0 = pf_col0<CT>(c, t);
        if (j0 < 0) break;  // uniform
        const float4 b = *t0_at(i, j0);
        acc[i][t][0] = b.x + ldexpf(acc[i][t][0] * rk, ex);
        acc[i][t][1] = b.y + ldexpf(acc[i][t][1] * rk, ex);
        acc[i][t][2] = b.z + ldexpf(acc[i][t][2] * rk, ex);
        acc[i][t][3] = b.w + ldexpf(acc[i][t][3] * rk, ex);
#pragma unroll
        for (int r = 0; r < 4; ++r) m = fmaxf(m, fabsf(acc[i][t][r]));
      }
    }
    es = pf_scale_exp(pf_block_max(m, red));
    pf_store_v<CT>(p, c, acc, es, u_hi, u_lo);
    __syncthreads();
  }

  // ---- phi' = P v ----
  pf_product_p<CT>(p, c, u_hi, u_lo, acc);
  const int ex = -(es + p.pexp);
  double* out = reinterpret_cast<double*>(ph);
#pragma unroll
  for (int i = 0; i < PF_FM; ++i) {
    const int rt = c.rg + PF_RG * i;
    if (rt >= p.RT) break;  // uniform
#pragma unroll
    for (int t = 0; t < CW; ++t) {
      const int j0 = pf_col0<CT>(c, t);
      if (j0 < 0) break;  // uniform
      const int j = j0 + c.jl;
      if (j >= ns) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = rt * 16 + 4 * c.kg + r;
        if (q < p.N) out[((size_t)q * ns + j) * 2 + c.comp] = ldexp((double)acc[i][t][r], ex);
      }
    }
  }
}

// P split into hi/lo fp16 rows of 32-wide k blocks, scaled by 2^pexp; rows
// and k past N are zero.  One thread per (row, k block, k of 32).
__global__ void psplit_kernel(const double* __restrict__ P, int N, int ldP, int QP, int nkbP, int pexp,
                              unsigned short* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= QP * nkbP * 32) return;
  const int row = e / (nkbP * 32), kk = e - row * (nkbP * 32);
  const int kb = kk >> 5, k = kk & 31;
  const int q = kb * 32 + k;
  const float x = (row < N && q < N) ? (float)ldexp(P[(size_t)row * ldP + q], pexp) : 0.f;
  const _Float16 h = (_Float16)x;
  const _Float16 l = (_Float16)(x - (float)h);
  unsigned short* dst = out + ((size_t)row * nkbP + kb) * SPLIT_KB;
  dst[k] = __builtin_bit_cast(unsigned short, h);
  dst[32 + k] = __builtin_bit_cast(unsigned short, l);
}

__global__ void pmax_kernel(const double* __restrict__ P, int N, int ldP, unsigned* __restrict__ out) {
  float m = 0.f;
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int r = e / N, q = e - r * N;
    m = fmaxf(m, fabsf((float)P[(size_t)r * ldP + q]));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

const void* prop_kernel_of(int ct) {
  switch (ct) {
    case 1: return reinterpret_cast<const void*>(prop_fused_kernel<1>);
    case 2: return reinterpret_cast<const void*>(prop_fused_kernel<2>);
    case 3: return reinterpret_cast<const void*>(prop_fused_kernel<3>);
    default: return reinterpret_cast<const void*>(prop_fused_kernel<4>);
  }
}

}  // namespace

PropFusedGeom prop_fused_geom(const StepDims& d) {
  PropFusedGeom g{};
  g.RT = ceil_div(d.N, 16);
  g.QP = 16 * g.RT;
  g.QCH = g.QP / 4 + 1;  // one pad chunk per row: consecutive orbitals' chunks fall in distinct bank groups
  g.TQS = g.QP + 4;
  g.CT = ceil_div(2 * (d.na > d.nb ? d.na : d.nb), 16);
  g.nkbP = ceil_div(d.N, 32);
  const size_t jc = 8 * (size_t)g.CT;
  g.lds_bytes = 2 * jc * g.QCH * 16 + 2 * jc * g.TQS * 4 + PF_WAVES * 8;
  g.psplit_halves = (size_t)g.QP * g.nkbP * SPLIT_KB;
  g.ok = g.RT <= PF_MAX_RT && g.CT >= 1 && g.CT <= PF_MAX_CT && g.lds_bytes <= 160 * 1024 && d.ldV % 32 == 0 &&
         d.ldV >= 32 * g.RT;
  return g;
}

hipError_t setup_prop_fused(const StepDims& d, const double* P, unsigned short* psplit, unsigned* pmax_scratch,
                            int* pexp_host, hipStream_t s) {
  const PropFusedGeom g = prop_fused_geom(d);
  hipError_t e = hipMemsetAsync(pmax_scratch, 0, sizeof(unsigned), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pmax_kernel, dim3(1), dim3(1024), 0, s, P, d.N, d.ldP, pmax_scratch);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  unsigned bits = 0;
  if ((e = hipMemcpyAsync(&bits, pmax_scratch, sizeof bits, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  float m;
  memcpy(&m, &bits, sizeof m);
  const int pexp = (m > 0.f && std::isfinite(m)) ? 13 - ilogbf(m) : 0;
  *pexp_host = pexp;
  const int n = g.QP * g.nkbP * 32;
  hipLaunchKernelGGL(psplit_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, P, d.N, d.ldP, g.QP, g.nkbP, pexp,
                     psplit);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipFuncSetAttribute(prop_kernel_of(g.CT), hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds_bytes);
}

hipError_t launch_prop_fused(const StepDims& d, int W, double2* phi_a, double2* phi_b, const float* vhs,
                             const unsigned* vmax, const unsigned short* psplit, int pexp, int order,
                             hipStream_t s) {
  if (W == 0) return hipSuccess;
  const PropFusedGeom g = prop_fused_geom(d);
  if (!g.ok) return hipErrorInvalidValue;
  const int nspin = d.nb > 0 ? 2 : 1;
  PropFusedArgs p{phi_a, phi_b, vhs, vmax, psplit, W, d.N, d.na, d.nb, d.ldV, g.RT, g.QP, g.QCH, g.TQS,
                  g.nkbP, order, pexp, nspin, 1.f};
  const dim3 grid((unsigned)(nspin == 2 ? ceil_div(W, 8) * 16 : W)), block(PF_NT);
  switch (g.CT) {
    case 1: hipLaunchKernelGGL(prop_fused_kernel<1>, grid, block, g.lds_bytes, s, p); break;
    case 2: hipLaunchKernelGGL(prop_fused_kernel<2>, grid, block, g.lds_bytes, s, p); break;
    case 3: hipLaunchKernelGGL(prop_fused_kernel<3>, grid, block, g.lds_bytes, s, p); break;
    default: hipLaunchKernelGGL(prop_fused_kernel<4>, grid, block, g.lds_bytes, s, p); break;
  }
  return hipGetLastError();
}
