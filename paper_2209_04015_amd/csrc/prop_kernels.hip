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
// (FP32) live in LDS; the walker's VHS rows, already split by the VHS build
// (each entry as fp16 hi and lo (Re, Im) pairs, scaled by a power of two
// from a bound on the walker's |VHS|), are streamed from memory straight
// into the A registers,
// once per order, with no LDS staging and no barrier inside a product.  The
// two spins of a walker get workgroup ids 8 apart, so they run on one XCD
// and the second stream of the VHS rows comes from its L2.
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
// |t0|, max |v_k|; the walker's |VHS| bound for the VHS rows) and one for
// P, exact and undone in each epilogue.

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
  const float* vhs;              // [W][N][ldV / 2] entries of fp16 (hi Re, hi Im, lo Re, lo Im)
  const unsigned* vbound;        // [W] |VHS| bound (float bits): the scale of the split rows
  const unsigned short* psplit;  // [QP][nkbP][64] P split, scaled by 2^pexp
  int W, N, na, nb, ldV, RT, QP, QCH, TQS, nkbP, order, pexp, nspin;
};

// Maximum over the workgroup.  Every earlier reader of red has passed a
// barrier since (the one that follows each store of v), so the writes need
// no barrier of their own; the one barrier here also puts every wave past
// the product whose results it reduces, so v may be overwritten after it.
__device__ __forceinline__ float pf_block_max(float v, float* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
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

// The three products of column tile t for the wave's NV real row tiles (a
// compile-time count: the products of a wave are one straight run of MFMAs,
// with no branch among them).  Each product kind is issued for all row
// tiles before the next, so that dependent MFMAs on one accumulator are
// several instructions apart.
template <int CW, int NV>
__device__ __forceinline__ void pf_mma_tiles(floatx4 (&acc)[PF_FM][CW], const f16x8_t (&ah)[PF_FM],
                                             const f16x8_t (&al)[PF_FM], const f16x8_t& bh, const f16x8_t& bl,
                                             int t) {
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], bh, acc[i][t], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bl, acc[i][t], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bh, acc[i][t], 0, 0, 0);
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
  const int tg = (PF_CG > 1 ? c.cg * PfCols<CT>::W : 0) + t;  // one column group: known at compile time
  return tg < CT ? 8 * tg : -1;
}

// acc = P v (k = q), v from the LDS planes, for the wave's NV row tiles
template <int CT, int NV>
__device__ __forceinline__ void pf_product_p_nv(const PropFusedArgs& p, const PfCtx& c, const uint4* u_hi,
                                                const uint4* u_lo, floatx4 (&acc)[PF_FM][PfCols<CT>::W]) {
  constexpr int CW = PfCols<CT>::W;
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
    for (int i = 0; i < NV; ++i) {
      pa_h[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(prs, arow[i], kb * 128, 0));
      pa_l[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(prs, arow[i], kb * 128 + 64, 0));
    }
  };
  fetch(0);
  for (int kb = 0; kb < p.nkbP; ++kb) {
    f16x8_t ah[PF_FM], al[PF_FM];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      ah[i] = __builtin_bit_cast(f16x8_t, pa_h[i]);
      al[i] = __builtin_bit_cast(f16x8_t, pa_l[i]);
    }
    fetch(kb + 1);  // unconditional (see above), so the wait counts stay exact
    // first of the two chunks of q0 .. q0+7; chunks past the rows read
    // chunk 0 (in bounds) and are replaced by zeros
    const int ch = 8 * kb + 2 * c.kg;
    const bool qok = 4 * ch < p.QP;
    const int chs = qok ? ch : 0;
#pragma unroll
    for (int t = 0; t < CW; ++t) {
      const int j0 = pf_col0<CT>(c, t);
      if (j0 < 0) break;  // compile time
      const int o = (j0 + c.jl) * p.QCH + chs;
      const uint2* h = reinterpret_cast<const uint2*>(u_hi + o) + c.comp;
      const uint2* l = reinterpret_cast<const uint2*>(u_lo + o) + c.comp;
      const uint2 h0 = h[0], h1 = h[2], l0 = l[0], l1 = l[2];  // chunks ch and ch + 1
      const uint4 hw = qok ? make_uint4(h0.x, h0.y, h1.x, h1.y) : make_uint4(0u, 0u, 0u, 0u);
      const uint4 lw = qok ? make_uint4(l0.x, l0.y, l1.x, l1.y) : make_uint4(0u, 0u, 0u, 0u);
      pf_mma_tiles<CW, NV>(acc, ah, al, __builtin_bit_cast(f16x8_t, hw), __builtin_bit_cast(f16x8_t, lw), t);
    }
  }
}

// acc = P v for the wave's real row tiles (one straight-line loop per count)
template <int CT>
__device__ __forceinline__ void pf_product_p(const PropFusedArgs& p, const PfCtx& c, const uint4* u_hi,
                                             const uint4* u_lo, floatx4 (&acc)[PF_FM][PfCols<CT>::W]) {
  pf_zero<PfCols<CT>::W>(acc);
  static_assert(PF_FM == 3, "one case per row-tile count");
  switch (c.nv) {  // wave-uniform
    case 3: pf_product_p_nv<CT, 3>(p, c, u_hi, u_lo, acc); break;
    case 2: pf_product_p_nv<CT, 2>(p, c, u_hi, u_lo, acc); break;
    case 1: pf_product_p_nv<CT, 1>(p, c, u_hi, u_lo, acc); break;
    default: break;
  }
}

// four 32-bit words as a native vector (whole-register selects between two
// of them stay in registers)
typedef unsigned pf_u32x4 __attribute__((ext_vector_type(4)));

// k blocks of VHS rows in flight per wave (a third set spills)
constexpr int PF_DEPTH = 2;

// The wave's split VHS operands of PF_DEPTH k blocks (per row tile the
// lane's four entries q0 .. q0+3, 32 contiguous bytes: hi and lo (Re, Im)
// words alternate), loaded ahead of the products that use them.
// Successive passes over the rows (one per Horner order) alternate the
// direction of k, so that each pass starts on the blocks the previous one
// read last, the ones most likely still in the L2.
struct PfVhsStream {
  pf_u32x4 r0[PF_DEPTH][PF_FM], r1[PF_DEPTH][PF_FM];  // entries q0, q0+1 and q0+2, q0+3
  int aoff[PF_FM];  // byte offsets of the lane's entries in k block 0
  int nkb;          // k blocks
  int nkbe;         // positions per pass: k blocks rounded up to a multiple of PF_DEPTH (set s holds position s mod PF_DEPTH)
  int dir;          // direction of the current pass: 0 ascending k blocks, 1 descending
};

// k block at position pos of a pass in direction dir (positions past the
// count are phantoms: never computed)
__device__ __forceinline__ int pf_block_at(const PfVhsStream& v, int pos, int dir) {
  return (dir && pos < v.nkb) ? v.nkb - 1 - pos : pos;
}

// set s <- position pos of the current pass (positions past its end: of the
// next pass, in the other direction); phantom blocks and rows past the tiles
// read in-bounds data or, past the buffer, zeros, and are never used
__device__ __forceinline__ void pf_vhs_fetch(PfVhsStream& v, __amdgpu_buffer_rsrc_t vrs, int s, int pos) {
  const int kb = pos >= v.nkbe ? pf_block_at(v, pos - v.nkbe, v.dir ^ 1) : pf_block_at(v, pos, v.dir);
#pragma unroll
  for (int i = 0; i < PF_FM; ++i) {
    v.r0[s][i] = __builtin_bit_cast(pf_u32x4, __builtin_amdgcn_raw_buffer_load_b128(vrs, v.aoff[i], kb * 128, 0));
    v.r1[s][i] = __builtin_bit_cast(pf_u32x4, __builtin_amdgcn_raw_buffer_load_b128(vrs, v.aoff[i], kb * 128 + 16, 0));
  }
}

// acc = VHS v (k = (q, re|im)), the split VHS rows streamed from memory into
// the A registers.  On entry set s of the stream holds (or is loading) the
// block at position s of this pass; every block is fetched PF_DEPTH
// positions ahead, wrapping into the next pass, so that on exit the sets
// hold the first blocks of the next one, already in flight across the
// epilogue and its barriers.
template <int CT, int NV>
__device__ __forceinline__ void pf_product_v_nv(const PropFusedArgs& p, const PfCtx& c, __amdgpu_buffer_rsrc_t vrs,
                                                PfVhsStream& vs, const uint4* u_hi, const uint4* u_lo,
                                                floatx4 (&acc)[PF_FM][PfCols<CT>::W]) {
  constexpr int CW = PfCols<CT>::W;
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
  static_assert(PF_CG == 1, "every wave holds every column tile");
  int ob[CW];  // the wave's column tiles: first LDS chunk of orbital j0 + jl
#pragma unroll
  for (int t = 0; t < CW; ++t) ob[t] = (pf_col0<CT>(c, t) + c.jl) * p.QCH + c.kg;
  const int nkb = p.RT;
  auto compute = [&](int s, int pos) {
    const int kb = pf_block_at(vs, pos, vs.dir);
    if (NV == 0) return;
    f16x8_t ah[PF_FM], al[PF_FM];
#pragma unroll
    for (int i = 0; i < NV; ++i) {  // the hi words and the lo words of the four entries
      ah[i] = __builtin_bit_cast(f16x8_t, __builtin_shufflevector(vs.r0[s][i], vs.r1[s][i], 0, 2, 4, 6));
      al[i] = __builtin_bit_cast(f16x8_t, __builtin_shufflevector(vs.r0[s][i], vs.r1[s][i], 1, 3, 5, 7));
    }
#pragma unroll
    for (int t = 0; t < CW; ++t) {
      const uint4 dh = u_hi[ob[t] + 4 * kb], dl = u_lo[ob[t] + 4 * kb];
      pf_mma_tiles<CW, NV>(acc, ah, al, bop(dh), bop(dl), t);
    }
  };
  // The fetches are unconditional, so that every wait leaves the other sets'
  // loads in flight; the scheduling barriers keep each set's loads after the
  // work that reads the set before them.
  for (int kb = 0; kb < vs.nkbe; kb += PF_DEPTH) {  // one regular body: the waits stay exact across the back edge
#pragma unroll
    for (int s = 0; s < PF_DEPTH; ++s) {
      if (kb + s < nkb) compute(s, kb + s);  // uniform: phantom blocks past the count are skipped
      __builtin_amdgcn_sched_barrier(0);
      pf_vhs_fetch(vs, vrs, s, kb + s + PF_DEPTH);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  vs.dir ^= 1;
}

// acc = VHS v for the wave's real row tiles (one straight-line loop per
// count; a wave with none still keeps its VHS stream in step)
template <int CT>
__device__ __forceinline__ void pf_product_v(const PropFusedArgs& p, const PfCtx& c, __amdgpu_buffer_rsrc_t vrs,
                                             PfVhsStream& vs, const uint4* u_hi, const uint4* u_lo,
                                             floatx4 (&acc)[PF_FM][PfCols<CT>::W]) {
  pf_zero<PfCols<CT>::W>(acc);
  static_assert(PF_FM == 3, "one case per row-tile count");
  switch (c.nv) {  // wave-uniform
    case 3: pf_product_v_nv<CT, 3>(p, c, vrs, vs, u_hi, u_lo, acc); break;
    case 2: pf_product_v_nv<CT, 2>(p, c, vrs, vs, u_hi, u_lo, acc); break;
    case 1: pf_product_v_nv<CT, 1>(p, c, vrs, vs, u_hi, u_lo, acc); break;
    default: pf_product_v_nv<CT, 0>(p, c, vrs, vs, u_hi, u_lo, acc); break;
  }
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

  // ---- the walker's VHS stream ----
  const int sa_exp = vhs_split_exp(__uint_as_float(p.vbound[z]));  // the scale of the split VHS rows
  const __amdgpu_buffer_rsrc_t vrs = split_rsrc(p.vhs + (size_t)z * p.N * p.ldV, p.N * p.ldV * 4);
  PfVhsStream vs;
  vs.nkb = p.RT;
  vs.nkbe = (p.RT + PF_DEPTH - 1) / PF_DEPTH * PF_DEPTH;
  vs.dir = 0;
#pragma unroll
  for (int i = 0; i < PF_FM; ++i) {
    const int rt = c.rg + PF_RG * i;
    // rows past N (and past the tiles) lie outside the buffer and read as zeros
    vs.aoff[i] = rt < p.RT ? ((rt * 16 + c.lrow) * p.ldV + 8 * c.kg) * 4 : SPLIT_ROW_NONE;
  }

  // ---- phi into LDS, scaled by 2^e (the scale taken in FP64, so that any
  // FP64 walker fits the fp16 range).  One pass: each thread loads its items
  // (four rows of one orbital) at once, then the block maximum, then the
  // split. ----
  constexpr int PHI_IT = (8 * CT * 4 * PF_MAX_RT + PF_NT - 1) / PF_NT;
  const int nch = p.QP / 4;
  double2 xv[PHI_IT][4];
  double dm = 0.0;
#pragma unroll
  for (int it = 0; it < PHI_IT; ++it) {
    const int e = tid + it * PF_NT;
    const int j = e % JC, ch = e / JC;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = 4 * ch + r;
      xv[it][r] = (ch < nch && q < p.N && j < ns) ? ph[(size_t)q * ns + j] : make_double2(0.0, 0.0);
    }
  }
#pragma unroll
  for (int it = 0; it < PHI_IT; ++it)
#pragma unroll
    for (int r = 0; r < 4; ++r) dm = fmax(dm, fmax(fabs(xv[it][r].x), fabs(xv[it][r].y)));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o, 64));
  if (c.lane == 0) reinterpret_cast<double*>(red)[c.wid] = dm;
  __syncthreads();
  dm = reinterpret_cast<const double*>(red)[0];
#pragma unroll
  for (int w = 1; w < PF_WAVES; ++w) dm = fmax(dm, reinterpret_cast<const double*>(red)[w]);
  int es = (dm > 0.0 && isfinite(dm)) ? 13 - ilogb(dm) : 0;
#pragma unroll
  for (int it = 0; it < PHI_IT; ++it) {
    const int e = tid + it * PF_NT;
    const int j = e % JC, ch = e / JC;
    if (ch >= nch) break;  // the items of later passes lie further out
    float re[4], im[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      re[r] = (float)ldexp(xv[it][r].x, es);
      im[r] = (float)ldexp(xv[it][r].y, es);
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

  // ---- t0 = P phi, the first k blocks of the VHS rows in flight ----
#pragma unroll
  for (int s = 0; s < PF_DEPTH; ++s) pf_vhs_fetch(vs, vrs, s, s);
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
  for (int k = p.order; k >= 1; --k) {
    pf_product_v<CT>(p, c, vrs, vs, u_hi, u_lo, acc);
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
                             const unsigned* vbound, const unsigned short* psplit, int pexp, int order,
                             hipStream_t s) {
  if (W == 0) return hipSuccess;
  const PropFusedGeom g = prop_fused_geom(d);
  if (!g.ok) return hipErrorInvalidValue;
  const int nspin = d.nb > 0 ? 2 : 1;
  PropFusedArgs p{phi_a, phi_b, vhs, vbound, psplit, W, d.N, d.na, d.nb, d.ldV, g.RT, g.QP, g.QCH, g.TQS,
                  g.nkbP, order, pexp, nspin};
  const dim3 grid((unsigned)(nspin == 2 ? ceil_div(W, 8) * 16 : W)), block(PF_NT);
  switch (g.CT) {
    case 1: hipLaunchKernelGGL(prop_fused_kernel<1>, grid, block, g.lds_bytes, s, p); break;
    case 2: hipLaunchKernelGGL(prop_fused_kernel<2>, grid, block, g.lds_bytes, s, p); break;
    case 3: hipLaunchKernelGGL(prop_fused_kernel<3>, grid, block, g.lds_bytes, s, p); break;
    default: hipLaunchKernelGGL(prop_fused_kernel<4>, grid, block, g.lds_bytes, s, p); break;
  }
  return hipGetLastError();
}
