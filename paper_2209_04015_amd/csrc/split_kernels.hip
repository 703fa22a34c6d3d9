// Exchange energy with hi/lo split operands on the 16-bit matrix cores
// (mixed modes AFQMC_BF16X3 and AFQMC_FP16X3).  Same algorithm as the FP32 /
// FP64 exchange kernel (Sec. III.C direct algorithm, T never leaves the chip);
// only the operand format and the MFMA differ.

#include <math.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "split_tile.h"
#include "tile_order.h"
#include "exchange_tri.h"
#include "exchange_pair.h"

// ---------------------------------------------------------------------------
// Row splitting: src rows (FP32, stride ld_src, ncols valid) -> split rows of
// ldh (multiple of 32) contraction indices, stored per block of 32 as 32 hi
// then 32 lo values (2 * ldh halves per row, zero padded), plus the inverse
// of the power-of-two row scale (the factor that restores a product).  One
// wave per row.
// ---------------------------------------------------------------------------
template <class H>
__global__ __launch_bounds__(256) void split_rows_kernel(long nrows, int ncols, const float* __restrict__ src,
                                                         int ld_src, unsigned short* __restrict__ dst,
                                                         int ldh, float* __restrict__ unscale) {
  // each lane holds two neighbouring columns of every 128-column chunk: the
  // row is loaded once (all loads in flight together), and the hi and lo
  // halves of the pair leave as 4-byte words
  constexpr int CHUNKS = 1024 / 128;  // rows of up to 1024 split columns (ldh < 1024 here)
  const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nrows) return;
  const float* s = src + row * ld_src;
  float x0[CHUNKS], x1[CHUNKS];
  float m = 0.f;
#pragma unroll
  for (int t = 0; t < CHUNKS; ++t) {
    const int c = 128 * t + 2 * lane;
    x0[t] = c < ncols ? s[c] : 0.f;
    x1[t] = c + 1 < ncols ? s[c + 1] : 0.f;
    m = fmaxf(m, fmaxf(fabsf(x0[t]), fabsf(x1[t])));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  const float sc = split_row_scale<H>(m);
  unsigned* d = reinterpret_cast<unsigned*>(dst + row * 2 * ldh);
#pragma unroll
  for (int t = 0; t < CHUNKS; ++t) {
    const int c = 128 * t + 2 * lane;  // even: the pair lies in one 32-column block
    if (c >= ldh) break;
    const float a = x0[t] * sc, b = x1[t] * sc;
    const unsigned short ah = H::from_float(a), bh = H::from_float(b);
    const unsigned short al = H::from_float(a - H::to_float(ah)), bl = H::from_float(b - H::to_float(bh));
    const int w = ((c >> 5) * SPLIT_KB + (c & 31)) >> 1;  // 4-byte word of the hi pair
    d[w] = (unsigned)ah | ((unsigned)bh << 16);
    d[w + 16] = (unsigned)al | ((unsigned)bl << 16);  // the lo pair, 32 halves further
  }
  if (lane == 0) unscale[row] = 1.0f / sc;  // power of two: exact
}

// The same for wide rows, one workgroup (four waves) per row: the fields of
// a step are only 2 W rows of K, too few waves for a wave per row.
template <class H>
__global__ __launch_bounds__(256) void split_rows_wide_kernel(int ncols, const float* __restrict__ src, int ld_src,
                                                              unsigned short* __restrict__ dst, int ldh,
                                                              float* __restrict__ unscale) {
  __shared__ float red[4];
  const long row = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const float* s = src + row * ld_src;
  float m = 0.f;
  for (int c = tid; c < ncols; c += 256) m = fmaxf(m, fabsf(s[c]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if (lane == 0) red[wid] = m;
  __syncthreads();
  m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  const float sc = split_row_scale<H>(m);
  unsigned short* d = dst + row * 2 * ldh;
  for (int c = tid; c < ldh; c += 256) {
    const float x = c < ncols ? s[c] * sc : 0.f;
    const unsigned short xh = H::from_float(x);
    unsigned short* b = d + (c >> 5) * SPLIT_KB + (c & 31);
    b[0] = xh;
    b[32] = H::from_float(x - H::to_float(xh));
  }
  if (tid == 0) unscale[row] = 1.0f / sc;  // power of two: exact
}

template <class H>
hipError_t launch_split_rows(long nrows, int ncols, const float* src, int ld_src, unsigned short* dst,
                             int ldh, float* unscale, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  if (ldh % 32 != 0 || ldh < ncols) return hipErrorInvalidValue;
  if (ncols >= 1024 || ldh > 1024)  // the one-wave kernel holds up to 1024 split columns
    hipLaunchKernelGGL(split_rows_wide_kernel<H>, dim3((unsigned)nrows), dim3(256), 0, s, ncols, src, ld_src, dst,
                       ldh, unscale);
  else
    hipLaunchKernelGGL(split_rows_kernel<H>, dim3((unsigned)((nrows + 3) / 4)), dim3(256), 0, s, nrows,
                       ncols, src, ld_src, dst, ldh, unscale);
  return hipGetLastError();
}

hipError_t launch_split_rows_mode(int mode, long nrows, int ncols, const float* src, int ld_src,
                                  unsigned short* dst, int ldh, float* unscale, hipStream_t s) {
  return mode == SPLIT_BF16 ? launch_split_rows<HalfBF16>(nrows, ncols, src, ld_src, dst, ldh, unscale, s)
                            : launch_split_rows<HalfF16>(nrows, ncols, src, ld_src, dst, ldh, unscale, s);
}

// ---------------------------------------------------------------------------
// Shift and split in one pass (Eq. of the optimal force bias, Sec. II.B): for
// the split VHS build, which reads only the split rows of the shifted fields.
// Per walker z: xbar = -i sqrt(dt) vbias, xs = x - xbar rounded to FP32, the
// sum a_z = sum_g (x xbar - xbar^2 / 2), and the |VHS| bound
// sqrt(dt) max(sum_g |Re xs_g| m_g, sum_g |Im xs_g| m_g) (1 + 2^-9) into slot
// 1 of tmax (every slot zeroed first), each summed in the same order as the
// FP32 shift kernel; rows 2 z (Re xs) and 2 z + 1 (Im xs) leave as split rows
// with their row scales, as the row split of that kernel's output would
// store them.  One workgroup of eight waves per walker, the row in registers
// (K <= SHIFT_SPLIT_NT KI).
// ---------------------------------------------------------------------------
constexpr int SHIFT_SPLIT_NT = 512;
constexpr int SHIFT_SPLIT_KI = 8;
template <class H>
__global__ __launch_bounds__(SHIFT_SPLIT_NT) void shift_split_kernel(int K, const double2* __restrict__ vbias,
                                                          const double* __restrict__ x_base,
                                                          const int* __restrict__ ctr, long x_step,
                                                          unsigned short* __restrict__ xs_split, int ldhK,
                                                          float* __restrict__ xs_unscale, double2* __restrict__ a,
                                                          unsigned* __restrict__ tmax, int tslots, int tstride,
                                                          double sdt, const float* __restrict__ lmax) {
  constexpr int KI = SHIFT_SPLIT_KI, NT = SHIFT_SPLIT_NT, NW = NT / 64;
  __shared__ double2 red[NW];
  __shared__ float fred[2][NW];
  const int z = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const double* x = x_base + (ctr ? (size_t)ctr[0] * x_step : 0);
  double2 acc = make_double2(0.0, 0.0);
  double2 bnd = make_double2(0.0, 0.0);
  float re[KI], im[KI];
  float mre = 0.f, mim = 0.f;
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int g = tid + NT * i;
    re[i] = 0.f;
    im[i] = 0.f;
    if (g < K) {
      const double2 v = vbias[(size_t)z * K + g];
      const double2 xb = make_double2(sdt * v.y, -sdt * v.x);
      const double xv = x[(size_t)z * K + g];
      re[i] = (float)(xv - xb.x);
      im[i] = (float)(-xb.y);
      acc.x += xv * xb.x - 0.5 * (xb.x * xb.x - xb.y * xb.y);
      acc.y += xv * xb.y - xb.x * xb.y;
      if (lmax) {
        const double m = lmax[g];
        bnd.x += fabs((double)re[i]) * m;
        bnd.y += fabs((double)im[i]) * m;
      }
      mre = fmaxf(mre, fabsf(re[i]));
      mim = fmaxf(mim, fabsf(im[i]));
    }
  }
  const double2 sum = block_sum2(acc, red);
  const double2 b = lmax ? block_sum2(bnd, red) : bnd;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mre = fmaxf(mre, __shfl_xor(mre, o, 64));
    mim = fmaxf(mim, __shfl_xor(mim, o, 64));
  }
  if (lane == 0) {
    fred[0][wid] = mre;
    fred[1][wid] = mim;
  }
  __syncthreads();
  mre = fred[0][0];
  mim = fred[1][0];
#pragma unroll
  for (int w = 1; w < NW; ++w) {
    mre = fmaxf(mre, fred[0][w]);
    mim = fmaxf(mim, fred[1][w]);
  }
  const float sre = split_row_scale<H>(mre), sim = split_row_scale<H>(mim);
  unsigned short* dre = xs_split + (size_t)(2 * z) * 2 * ldhK;
  unsigned short* dim = dre + 2 * ldhK;
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int c = tid + NT * i;
    if (c >= ldhK) break;
    const int o = (c >> 5) * SPLIT_KB + (c & 31);
    const float u = re[i] * sre, v = im[i] * sim;
    const unsigned short uh = H::from_float(u), vh = H::from_float(v);
    dre[o] = uh;
    dre[o + 32] = H::from_float(u - H::to_float(uh));
    dim[o] = vh;
    dim[o + 32] = H::from_float(v - H::to_float(vh));
  }
  if (tid == 0) {
    xs_unscale[2 * z] = 1.0f / sre;  // powers of two: exact
    xs_unscale[2 * z + 1] = 1.0f / sim;
    a[z] = sum;
    for (int t = 0; t < tslots; ++t) tmax[(size_t)t * tstride + z] = 0u;  // running maxima of this step
    // |VHS| bound (slot 1): both parts of VHS = i sqrt(dt) sum_g xs_g L_g are
    // at most sqrt(dt) sum_g |xs part| max|L_g|; the margin covers the
    // rounding of the FP32 sums of the split build
    if (lmax) tmax[(size_t)tstride + z] = __float_as_uint((float)(sdt * fmax(b.x, b.y) * (1.0 + 0x1p-9)));
  }
}

bool shift_split_fits(int ldhK) { return ldhK <= SHIFT_SPLIT_NT * SHIFT_SPLIT_KI; }

hipError_t launch_shift_split(int mode, const StepDims& d, int W, const double2* vbias, const double* x,
                              const int* ctr, long x_step, unsigned short* xs_split, float* xs_unscale, double2* a,
                              unsigned* tmax, int tslots, int tstride, double sdt, const float* lmax,
                              hipStream_t s) {
  if (W == 0) return hipSuccess;
  if (d.ldhK % 32 != 0 || d.ldhK < d.K || !shift_split_fits(d.ldhK)) return hipErrorInvalidValue;
  if (mode == SPLIT_BF16)
    hipLaunchKernelGGL(shift_split_kernel<HalfBF16>, dim3(W), dim3(SHIFT_SPLIT_NT), 0, s, d.K, vbias, x, ctr, x_step,
                       xs_split, d.ldhK, xs_unscale, a, tmax, tslots, tstride, sdt, lmax);
  else
    hipLaunchKernelGGL(shift_split_kernel<HalfF16>, dim3(W), dim3(SHIFT_SPLIT_NT), 0, s, d.K, vbias, x, ctr, x_step,
                       xs_split, d.ldhK, xs_unscale, a, tmax, tslots, tstride, sdt, lmax);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exchange on split operands.
// ---------------------------------------------------------------------------
// 4-wave workgroups of 2 x 2 wave tiles; register prefetch of the next k
// block, one LDS stage; WPE workgroups per CU (two by default), so that one
// workgroup's epilogue runs beside another's matrix-core work.
template <int BM_, int BN_, int WPE_ = 2>
struct SplitCfgT {
  static constexpr int BM = BM_, BN = BN_, WM = 2, WN = 2, GS = 8;
  static constexpr int NT = WM * WN * 64;
  static constexpr int NA = BM * 8 / NT, NB = BN * 8 / NT;
  static constexpr int WAVES_PER_EU = WPE_;
  static_assert(BM % 32 == 0 && BN % 32 == 0, "whole fragments and staging rows");
};
using ExSplitCfg = SplitCfgT<160, 160>;
// The pair exchange and the VHS build: 128 x 128 tiles at three workgroups
// per CU (more tiles in flight hide each one's first loads and epilogue:
// 0.49 -> 0.47 ms and 0.72 -> 0.70 ms per step at n290), and narrow walker
// tiles (autotuner candidates for systems with few walkers): 32 walkers per
// pair-exchange tile, 32 walkers per VHS tile.  Both pair shapes have the
// row-tile height the pair tables are built for, both VHS shapes the width
// of a VHS pair block.
using ExPairWideCfg = SplitCfgT<128, 128, 3>;
using ExPairNarrowCfg = SplitCfgT<128, 64, 3>;
static_assert(ExPairWideCfg::BM == ExPairNarrowCfg::BM, "one row-tile height for the pair tables");
using VhsWideCfg = SplitCfgT<128, 128, 3>;
using VhsNarrowCfg = SplitCfgT<64, 128>;

struct ExSplitArgs {
  const unsigned short* a;  // Lh split rows of this spin: [K][nmax][2 ldh] halves
  const float* a_unscale;   // [K][nmax]
  const unsigned short* b;  // theta split rows: [W][re|im][spin][nmax][2 ldh] halves
  const float* b_unscale;   // [W][re|im][spin][nmax]
  int K, W, n, nmax, rowb, sp, G, Z, nkb;  // rowb: bytes per split row
};

// Static LDS of a workgroup (base address 0, so offsets fold into the LDS
// instructions): the operand stage, or the triangles and column sums, then
// the scale table at the end.  64 KB: two workgroups per CU.
constexpr int EXS_LDS_BYTES = 64 * 1024;
constexpr int EXS_TAB_OFF = EXS_LDS_BYTES - (ExSplitCfg::BM + ExSplitCfg::BN) * (int)sizeof(float);
static_assert(SplitStage<ExSplitCfg::BM, ExSplitCfg::BN>::BYTES <= EXS_TAB_OFF, "operand stage fits");
static_assert(4 * ExSplitCfg::WM * ExSplitCfg::BN * 16 <= EXS_TAB_OFF, "column sums fit");

// Walker slots per epilogue pass (0 if one slot does not fit).
static int exs_walkers_per_pass(int G, int Z, int n) {
  const int per = ex_tri_block(G, n) * (int)sizeof(float2);
  const int zp = (EXS_TAB_OFF - ex_tri_area_bytes(0, G, n)) / per;
  return zp < Z ? zp : Z;
}

template <class H>
__global__ __launch_bounds__(ExSplitCfg::NT, ExSplitCfg::WAVES_PER_EU) void exchange_split_kernel(
    ExSplitArgs p, double2* __restrict__ part, int ntg, int nwt, int zpp, int gs) {
  using C = ExSplitCfg;
  int gt, wt;
  if (!xcd_tile(blockIdx.x, ntg, nwt, gs, gt, wt)) return;
  __shared__ __attribute__((aligned(16))) char exs_lds[EXS_LDS_BYTES];
  const int tid = threadIdx.x;
  const int schunk = tid & 7, srow = tid >> 3;
  const int n = p.n, n2 = 2 * n;
  const float rn = 1.0f / (float)n, rn2 = 1.0f / (float)n2;
  // operand rows of this tile: buffers from the tile's first Cholesky vector
  // and first walker; rows staged by this thread as byte offsets in them
  const int g0 = gt * p.G, z0 = wt * p.Z;
  const int ng = min(p.G, p.K - g0), nz = min(p.Z, p.W - z0);
  const __amdgpu_buffer_rsrc_t a_rsrc =
      split_rsrc(p.a + (size_t)g0 * p.nmax * (p.rowb / 2), ng * p.nmax * p.rowb);
  const __amdgpu_buffer_rsrc_t b_rsrc =
      split_rsrc(p.b + (size_t)z0 * 4 * p.nmax * (p.rowb / 2), nz * 4 * p.nmax * p.rowb);
  int a_off[C::NA], b_off[C::NB];
#pragma unroll
  for (int t = 0; t < C::NA; ++t) {
    const int r = srow + t * (C::NT / 8);
    const int gl = ex_div(r, rn);
    a_off[t] = gl < ng ? (gl * p.nmax + (r - gl * n)) * p.rowb + schunk * 16 : SPLIT_ROW_NONE;
  }
#pragma unroll
  for (int t = 0; t < C::NB; ++t) {
    const int c = srow + t * (C::NT / 8);
    const int zt = ex_div(c, rn2);
    const int o = c - zt * n2;
    const int comp = o >= n ? 1 : 0;
    b_off[t] = zt < nz ? (((zt * 2 + comp) * 2 + p.sp) * p.nmax + (o - comp * n)) * p.rowb + schunk * 16
                       : SPLIT_ROW_NONE;
  }
  // operand scale factors of tile row / column tid, used by the epilogue
  float pre_row = 0.f, pre_col = 0.f;
  if constexpr (H::SCALED) {
    if (tid < C::BM) {
      const int gl = ex_div(tid, rn);
      const int g = gt * p.G + gl;
      if (gl < p.G && g < p.K) pre_row = p.a_unscale[(size_t)g * p.nmax + (tid - gl * n)];
    }
    if (tid < C::BN) {
      const int zt = ex_div(tid, rn2);
      const int o = tid - zt * n2;
      const int comp = o >= n ? 1 : 0;
      const int z = wt * p.Z + zt;
      if (zt < p.Z && z < p.W)
        pre_col = p.b_unscale[(((size_t)z * 2 + comp) * 2 + p.sp) * p.nmax + (o - comp * n)];
    }
  }
  floatx4 acc[C::BM / C::WM / 16][C::BN / C::WN / 16];
  split_tile_mainloop<H, C::BM, C::BN, C::WM, C::WN>(a_rsrc, b_rsrc, a_off, b_off, p.nkb, acc,
                                                    reinterpret_cast<unsigned short*>(exs_lds));
  const ExTriGeom q{n, p.G, p.Z, p.K, p.W, gt, wt, p.nmax, p.sp, ntg};
  exchange_tri_epilogue<C::BM, C::BN, C::WM, C::WN, H::SCALED>(acc, exs_lds, EXS_TAB_OFF, zpp, q, pre_row,
                                                               pre_col, part);
}

ExTile exchange_split_tile(int n) {
  ExTile t;
  t.G = n > 0 ? ExSplitCfg::BM / n : 0;
  t.Z = n > 0 ? ExSplitCfg::BN / (2 * n) : 0;
  return t;
}

hipError_t launch_exchange_split(int mode, const StepDims& d, int W, const unsigned short* lh,
                                 const float* lh_unscale, const unsigned short* th, const float* th_unscale,
                                 double2* part, int sp, int* ntg_out, hipStream_t s, int gs) {
  using C = ExSplitCfg;
  if (gs < 1) gs = C::GS;
  const ExTile t = exchange_split_tile(d.nmax);
  if (t.G < 1 || t.Z < 1 || d.ldh % 32 != 0) return hipErrorInvalidValue;
  const int ntg = ceil_div(d.K, t.G);
  const int nwt = ceil_div(W, t.Z);
  *ntg_out = ntg;
  const int n = sp == 0 ? d.na : d.nb;
  if (n == 0 || W == 0) return hipSuccess;
  const int rowb = 2 * d.ldh * 2;
  // per-tile buffers (G Cholesky vectors, Z walkers) below 2^31 bytes
  if ((double)t.G * d.nmax * rowb >= (double)SPLIT_ROW_NONE ||
      (double)t.Z * 4 * d.nmax * rowb >= (double)SPLIT_ROW_NONE)
    return hipErrorInvalidValue;
  const size_t sblk = (size_t)d.K * d.nmax;
  ExSplitArgs p{lh + sp * sblk * 2 * d.ldh, lh_unscale + sp * sblk, th, th_unscale, d.K, W, n, d.nmax, rowb,
                sp, t.G, t.Z, d.ldh / 32};
  const int zpp = exs_walkers_per_pass(t.G, t.Z, n);
  if (zpp < 1) return hipErrorInvalidValue;
  const int per = ceil_div(ntg * nwt, 8);
  if (mode == SPLIT_BF16)
    hipLaunchKernelGGL(exchange_split_kernel<HalfBF16>, dim3(8 * per), dim3(C::NT), 0, s, p, part, ntg, nwt,
                       zpp, gs);
  else
    hipLaunchKernelGGL(exchange_split_kernel<HalfF16>, dim3(8 * per), dim3(C::NT), 0, s, p, part, ntg, nwt,
                       zpp, gs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exchange through pair integrals on split operands (exchange_pair.h).  Row
// tile rt of group i: A = pair-integral split rows (j, p) of group i,
// B = theta split rows (z, re|im, spin, i) of the tile's 80 walkers,
// contraction over the orbital q.  Same stage, tile and XCD order as the
// direct split exchange; the epilogue is the Hadamard product with theta.
// ---------------------------------------------------------------------------
struct PairSplitArgs {
  const unsigned short* v;   // pair-integral split rows of this spin: [rows][2 ldh] halves
  const float* v_unscale;    // [rows]
  const unsigned short* th;  // theta split rows: [W][re|im][spin][nmax][2 ldh] halves
  const float* th_unscale;   // [W][re|im][spin][nmax]
  const float* theta;        // FP32 planar theta [W][re|im][spin][nmax][ldN]
  const PairTab* tab;        // this spin's row-tile tables
  int W, n, Np, nmax, ldN, rowb, sp, nkb, ntiles;
};

template <class H, class C>
__global__ __launch_bounds__(C::NT, C::WAVES_PER_EU) void exchange_pair_split_kernel(
    PairSplitArgs p, double2* __restrict__ part, int ntg, int nwt, int gs) {
  // the operand stage, then (epilogue) the column sums, in LDS sized for the
  // shape (three workgroups of the wide shape fit a CU)
  constexpr int PAIR_LDS = SplitStage<C::BM, C::BN>::BYTES > 4 * C::WM * C::BN * 16 ? SplitStage<C::BM, C::BN>::BYTES
                                                                                    : 4 * C::WM * C::BN * 16;
  int rt, wt;
  if (!xcd_tile(blockIdx.x, ntg, nwt, gs, rt, wt)) return;
  const int z0 = wt * (C::BN / 2);
  double2* out = part + ((size_t)p.sp * ntg + rt) * p.W;
  if (rt >= p.ntiles) {
    exchange_pair_zero<C::BN>(z0, p.W, out);
    return;
  }
  __shared__ __attribute__((aligned(16))) char exs_lds[PAIR_LDS];
  const int tid = threadIdx.x;
  const int schunk = tid & 7, srow = tid >> 3;
  const int i = pair_group(p.tab, p.n, rt);
  const int lr0 = (rt - p.tab->start[i]) * C::BM;
  const int R = (p.n - i) * p.Np;
  const int vb = p.tab->vbase[i];
  const int nr = min(C::BM, R - lr0);
  const int nz = min(C::BN / 2, p.W - z0);
  // buffers from the tile's first pair-integral row and first walker
  const __amdgpu_buffer_rsrc_t a_rsrc = split_rsrc(p.v + (size_t)(vb + lr0) * (p.rowb / 2), nr * p.rowb);
  const __amdgpu_buffer_rsrc_t b_rsrc =
      split_rsrc(p.th + (size_t)z0 * 4 * p.nmax * (p.rowb / 2), nz * 4 * p.nmax * p.rowb);
  int a_off[C::NA], b_off[C::NB];
#pragma unroll
  for (int t = 0; t < C::NA; ++t) {
    const int r = srow + t * (C::NT / 8);
    a_off[t] = r < nr ? r * p.rowb + schunk * 16 : SPLIT_ROW_NONE;
  }
#pragma unroll
  for (int t = 0; t < C::NB; ++t) {
    const int c = srow + t * (C::NT / 8);
    const int zt = c >> 1, comp = c & 1;
    b_off[t] = zt < nz ? (((zt * 2 + comp) * 2 + p.sp) * p.nmax + i) * p.rowb + schunk * 16 : SPLIT_ROW_NONE;
  }
  floatx4 acc[C::BM / C::WM / 16][C::BN / C::WN / 16];
  split_tile_mainloop<H, C::BM, C::BN, C::WM, C::WN>(a_rsrc, b_rsrc, a_off, b_off, p.nkb, acc,
                                                    reinterpret_cast<unsigned short*>(exs_lds));
  exchange_pair_epilogue<C::BM, C::BN, C::WM, C::WN, H::SCALED>(acc, exs_lds, i, lr0, R, p.Np, vb, z0, p.W, p.sp,
                                                                p.nmax, p.ldN, p.theta, p.v_unscale, p.th_unscale,
                                                                out);
}

int exchange_pair_split_rows() { return ExPairWideCfg::BM; }

template <class C>
static hipError_t launch_exchange_pair_split_t(int mode, const StepDims& d, int W, const PairLaunch& pl,
                                               const unsigned short* v, const float* v_unscale,
                                               const unsigned short* th, const float* th_unscale, const float* theta,
                                               double2* part, int sp, hipStream_t s, int gs) {
  if (gs < 1) gs = C::GS;
  const int n = sp == 0 ? d.na : d.nb;
  if (W == 0 || pl.ntg == 0) return hipSuccess;
  if (d.ldh % 32 != 0 || n > PAIR_MAX_N) return hipErrorInvalidValue;
  const int rowb = 2 * d.ldh * 2;
  const int Np = (d.N + 3) & ~3;
  // per-tile buffers below 2^31 bytes
  if ((double)C::BM * rowb >= (double)SPLIT_ROW_NONE ||
      (double)(C::BN / 2) * 4 * d.nmax * rowb >= (double)SPLIT_ROW_NONE)
    return hipErrorInvalidValue;
  const int nwt = ceil_div(2 * W, C::BN);
  PairSplitArgs p{v + (size_t)pl.vrow0 * 2 * d.ldh, v_unscale + pl.vrow0, th, th_unscale, theta, pl.tab,
                  W, n, Np, d.nmax, d.ldN, rowb, sp, d.ldh / 32, n > 0 ? pl.ntiles : 0};
  const int per = ceil_div(pl.ntg * nwt, 8);
  if (mode == SPLIT_BF16)
    hipLaunchKernelGGL((exchange_pair_split_kernel<HalfBF16, C>), dim3(8 * per), dim3(C::NT), 0, s, p, part, pl.ntg,
                       nwt, gs);
  else
    hipLaunchKernelGGL((exchange_pair_split_kernel<HalfF16, C>), dim3(8 * per), dim3(C::NT), 0, s, p, part, pl.ntg,
                       nwt, gs);
  return hipGetLastError();
}

hipError_t launch_exchange_pair_split(int mode, const StepDims& d, int W, const PairLaunch& pl,
                                      const unsigned short* v, const float* v_unscale, const unsigned short* th,
                                      const float* th_unscale, const float* theta, double2* part, int sp,
                                      hipStream_t s, int gs, int tile) {
  if (tile == SPLIT_TILE_NARROW)
    return launch_exchange_pair_split_t<ExPairNarrowCfg>(mode, d, W, pl, v, v_unscale, th, th_unscale, theta, part,
                                                         sp, s, gs);
  return launch_exchange_pair_split_t<ExPairWideCfg>(mode, d, W, pl, v, v_unscale, th, th_unscale, theta, part, sp,
                                                     s, gs);
}

// ---------------------------------------------------------------------------
// VHS build on split operands (Eq. of the propagator: VHS_z = i sqrt(dt)
// sum_g xs_zg L_g): C[(z, re|im)][pq] = sum_g xs[z][re|im][g] LT[pq][g] over
// the packed p <= q triangle, mirrored on store.  A = xs split rows (2 W),
// B = packed L split rows (N (N + 1) / 2), contraction over the Cholesky
// index.
// ---------------------------------------------------------------------------
// VHS blocks: the orbital pairs are packed in blocks of VB_P rows p by VB_Q
// columns q (one 128-column tile per block; blocks that touch the upper
// triangle q >= p, pairs outside the matrix or below the diagonal are zero
// rows and are not stored).  The tile's values go through LDS, so that both
// halves leave as contiguous runs: (p, q) rows of VB_Q pairs (64 bytes) and
// the mirror (q, p) rows of VB_P pairs (full 128-byte lines).
constexpr int VB_P = 16, VB_Q = 8;
// walkers per LDS pass of the store (the waves of one row half), and the LDS
template <class C>
struct VhsLds {
  static_assert(VB_P * VB_Q == C::BN, "one block per tile");
  static constexpr int ZPASS = C::BM / 2 / C::WM;
  static constexpr int BYTES = SplitStage<C::BM, C::BN>::BYTES > ZPASS * C::BN * 8 ? SplitStage<C::BM, C::BN>::BYTES
                                                                                    : ZPASS * C::BN * 8;
};

struct VhsSplitArgs {
  const unsigned short* a;  // xs split rows [2 W][2 ldhK]
  const float* a_unscale;   // [2 W]
  const unsigned short* b;  // block-packed L split rows [nblk * 160][2 ldhK]
  const float* b_unscale;   // [nblk * 160]
  const int2* blk;          // [nblk] (P, Q): rows p = VB_P P + i, columns q = VB_Q Q + j
  float* vhs;               // [W][N][ldV] complex interleaved
  unsigned* vmax;           // [W] FP32 output: max |VHS| (atomic), or null; split output: |VHS| bound (read)
  int W, nblk, N, ldV, rowb, nkb;
  float sdt;
  int split_out;            // 1: fp16 (hi Re, hi Im, lo Re, lo Im) per entry, scaled by 2^vhs_split_exp(bound)
};

template <class H, class C>
__global__ __launch_bounds__(C::NT, C::WAVES_PER_EU) void vhs_split_kernel(VhsSplitArgs p, int ntn, int ntm) {
  constexpr int FM = C::BM / C::WM / 16, FN = C::BN / C::WN / 16;
  constexpr int VHS_LDS_BYTES = VhsLds<C>::BYTES, VHS_ZPASS = VhsLds<C>::ZPASS;
  int tn, tm;  // consecutive tiles on one XCD share the packed-L tile
  if (!xcd_tile(blockIdx.x, ntn, ntm, 1, tn, tm)) return;
  __shared__ __attribute__((aligned(16))) unsigned short vs_lds[VHS_LDS_BYTES / 2];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid / C::WN, wn = wid % C::WN;
  const int m0 = tm * C::BM, n0 = tn * C::BN;
  const int nm = min(C::BM, 2 * p.W - m0);
  // rows past nm fall outside the tile buffer: staged as zeros
  const __amdgpu_buffer_rsrc_t a_rsrc = split_rsrc(p.a + (size_t)m0 * (p.rowb / 2), nm * p.rowb);
  const __amdgpu_buffer_rsrc_t b_rsrc = split_rsrc(p.b + (size_t)n0 * (p.rowb / 2), C::BN * p.rowb);
  int a_off[C::NA], b_off[C::NB];
#pragma unroll
  for (int t = 0; t < C::NA; ++t) a_off[t] = ((tid >> 3) + t * (C::NT / 8)) * p.rowb + (tid & 7) * 16;
#pragma unroll
  for (int t = 0; t < C::NB; ++t) b_off[t] = ((tid >> 3) + t * (C::NT / 8)) * p.rowb + (tid & 7) * 16;
  floatx4 acc[FM][FN];
  split_tile_mainloop<H, C::BM, C::BN, C::WM, C::WN>(a_rsrc, b_rsrc, a_off, b_off, p.nkb, acc, vs_lds);

  // values v = i sqrt(dt) (C_re + i C_im), rows m = 2 z + (re|im): each
  // lane's 4 consecutive rows are 2 whole walkers; per-walker maxima
  float cs[FN];
#pragma unroll
  for (int f = 0; f < FN; ++f)
    cs[f] = H::SCALED ? p.b_unscale[n0 + wn * (C::BN / C::WN) + f * 16 + (lane & 15)] : 1.0f;
  float2 val[FM][FN][2];
  float wmax[FM][2];
#pragma unroll
  for (int fi = 0; fi < FM; ++fi) {
    const int mb = m0 + wm * (C::BM / C::WM) + fi * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int z = (mb >> 1) + h;
      const bool ok = z < p.W;
      const float ur = ok && H::SCALED ? p.a_unscale[2 * z] : 1.0f;
      const float ui = ok && H::SCALED ? p.a_unscale[2 * z + 1] : 1.0f;
      float m = 0.f;
#pragma unroll
      for (int f = 0; f < FN; ++f) {  // powers of two: exact
        const float cr = acc[fi][f][2 * h] * ur * cs[f], ci = acc[fi][f][2 * h + 1] * ui * cs[f];
        val[fi][f][h] = make_float2(-p.sdt * ci, p.sdt * cr);
        m = fmaxf(m, fmaxf(fabsf(val[fi][f][h].x), fabsf(val[fi][f][h].y)));
      }
      wmax[fi][h] = m;
    }
  }
  // split output: each walker's values times its power-of-two scale, as the
  // 8 bytes (hi Re, hi Im, lo Re, lo Im) in fp16, stored where the FP32
  // (Re, Im) pair would be
  float zsc[FM][2];
#pragma unroll
  for (int fi = 0; fi < FM; ++fi)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int z = ((m0 + wm * (C::BM / C::WM) + fi * 16 + 4 * (lane >> 4)) >> 1) + h;
      zsc[fi][h] = p.split_out && z < p.W ? ldexpf(1.f, vhs_split_exp(__uint_as_float(p.vmax[z]))) : 1.f;
    }
  // stores: one row half of walkers at a time through LDS [walker][pair]
  // (8 bytes per entry in either form, moved as they are)
  const int2 PQ = p.blk[tn];
  const int pb0 = VB_P * PQ.x, qb0 = VB_Q * PQ.y;
  float2* sv = reinterpret_cast<float2*>(vs_lds);
  uint2* su = reinterpret_cast<uint2*>(vs_lds);
  for (int half = 0; half < C::WM; ++half) {
    __syncthreads();  // main loop (or the previous pass) done with the LDS
    if (wm == half) {
#pragma unroll
      for (int fi = 0; fi < FM; ++fi)
#pragma unroll
        for (int f = 0; f < FN; ++f)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int zl = ((fi * 16 + 4 * (lane >> 4)) >> 1) + h;  // walker within the half
            const int o = zl * C::BN + wn * (C::BN / C::WN) + f * 16 + (lane & 15);
            if (p.split_out) {
              const float yr = val[fi][f][h].x * zsc[fi][h], yi = val[fi][f][h].y * zsc[fi][h];
              const _Float16 hr = (_Float16)yr, hi_ = (_Float16)yi;
              const _Float16 lr = (_Float16)(yr - (float)hr), li = (_Float16)(yi - (float)hi_);
              su[o] = make_uint2((unsigned)__builtin_bit_cast(unsigned short, hr) |
                                     ((unsigned)__builtin_bit_cast(unsigned short, hi_) << 16),
                                 (unsigned)__builtin_bit_cast(unsigned short, lr) |
                                     ((unsigned)__builtin_bit_cast(unsigned short, li) << 16));
            } else {
              sv[o] = val[fi][f][h];
            }
          }
    }
    __syncthreads();
    const int zh = (m0 >> 1) + half * VHS_ZPASS;
    // (p, q), q >= p: consecutive threads on consecutive q
    for (int e = tid; e < VHS_ZPASS * C::BN; e += C::NT) {
      const int zl = e / C::BN, c = e - zl * C::BN;
      const int pp = c / VB_Q, qq = c - pp * VB_Q;
      const int z = zh + zl, pr = pb0 + pp, qc = qb0 + qq;
      if (z < p.W && pr < p.N && qc < p.N && qc >= pr)
        *reinterpret_cast<float2*>(p.vhs + ((size_t)z * p.N + pr) * p.ldV + 2 * qc) = sv[e];
    }
    // mirror (q, p), q > p: consecutive threads on consecutive p
    for (int e = tid; e < VHS_ZPASS * C::BN; e += C::NT) {
      const int zl = e / C::BN, c = e - zl * C::BN;
      const int qq = c / VB_P, pp = c - qq * VB_P;
      const int z = zh + zl, pr = pb0 + pp, qc = qb0 + qq;
      if (z < p.W && pr < p.N && qc < p.N && qc > pr)
        *reinterpret_cast<float2*>(p.vhs + ((size_t)z * p.N + qc) * p.ldV + 2 * pr) = sv[zl * C::BN + pp * VB_Q + qq];
    }
  }
  if (p.vmax && !p.split_out) {  // per walker: over the 16 lanes holding its rows, then one atomic
#pragma unroll
    for (int fi = 0; fi < FM; ++fi)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float m = wmax[fi][h];
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
        const int z = ((m0 + wm * (C::BM / C::WM) + fi * 16 + 4 * (lane >> 4)) >> 1) + h;
        if ((lane & 15) == 0 && z < p.W) atomicMax(p.vmax + z, __float_as_uint(m));
      }
  }
}

// (P, Q) of the VHS blocks that touch the upper triangle of an N x N matrix.
std::vector<int2> vhs_split_blocks(int N) {
  std::vector<int2> b;
  for (int P = 0; VB_P * P < N; ++P)
    for (int Q = 0; VB_Q * Q < N; ++Q)
      if (VB_Q * Q + VB_Q - 1 >= VB_P * P) b.push_back(make_int2(P, Q));
  return b;
}

// Orbital pair (p, q) of each packed row in block order, (-1, -1) for rows
// outside the matrix or below the diagonal.
std::vector<int2> vhs_split_pairs(int N, const std::vector<int2>& blk) {
  std::vector<int2> pq;
  pq.reserve(blk.size() * VB_P * VB_Q);
  for (const int2& b : blk)
    for (int i = 0; i < VB_P; ++i)
      for (int j = 0; j < VB_Q; ++j) {
        const int pr = VB_P * b.x + i, qc = VB_Q * b.y + j;
        pq.push_back(pr < N && qc < N && qc >= pr ? make_int2(pr, qc) : make_int2(-1, -1));
      }
  return pq;
}

template <class C>
static hipError_t launch_vhs_split_t(int mode, const StepDims& d, int W, const unsigned short* xs,
                                     const float* xs_unscale, const unsigned short* lt, const float* lt_unscale,
                                     const int2* blk, int nblk, float* vhs, unsigned* vmax, bool split_out,
                                     double sdt, hipStream_t s) {
  if (W == 0) return hipSuccess;
  if (d.ldhK % 32 != 0) return hipErrorInvalidValue;
  const int rowb = 2 * d.ldhK * 2;
  if ((double)(C::BM > C::BN ? C::BM : C::BN) * rowb >= (double)SPLIT_ROW_NONE) return hipErrorInvalidValue;
  const int ntm = ceil_div(2 * W, C::BM), ntn = nblk;
  if (split_out && !vmax) return hipErrorInvalidValue;
  VhsSplitArgs p{xs,     xs_unscale, lt,   lt_unscale, blk,           vhs,        vmax,
                 W,      nblk,       d.N,  d.ldV,      rowb,          d.ldhK / 32, (float)sdt,
                 split_out ? 1 : 0};
  const int per = ceil_div(ntm * ntn, 8);
  if (mode == SPLIT_BF16)
    hipLaunchKernelGGL((vhs_split_kernel<HalfBF16, C>), dim3(8 * per), dim3(C::NT), 0, s, p, ntn, ntm);
  else
    hipLaunchKernelGGL((vhs_split_kernel<HalfF16, C>), dim3(8 * per), dim3(C::NT), 0, s, p, ntn, ntm);
  return hipGetLastError();
}

hipError_t launch_vhs_split(int mode, const StepDims& d, int W, const unsigned short* xs, const float* xs_unscale,
                            const unsigned short* lt, const float* lt_unscale, const int2* blk, int nblk, float* vhs,
                            unsigned* vmax, bool split_out, double sdt, hipStream_t s, int tile) {
  if (tile == SPLIT_TILE_NARROW)
    return launch_vhs_split_t<VhsNarrowCfg>(mode, d, W, xs, xs_unscale, lt, lt_unscale, blk, nblk, vhs, vmax,
                                            split_out, sdt, s);
  return launch_vhs_split_t<VhsWideCfg>(mode, d, W, xs, xs_unscale, lt, lt_unscale, blk, nblk, vhs, vmax, split_out,
                                        sdt, s);
}

// ---------------------------------------------------------------------------
// Taylor term on split operands (the exp(VHS) of Eq. Bx truncated after the
// 6th-order term): t_k = VHS t_{k-1} / k for one walker per tile column, as a real GEMM
// over k = (q, re|im) interleaved:
//   A[p][2q + c]         = VHS_pq (c = 0 real, 1 imaginary part)
//   B[(j, re)][2q, 2q+1] = ( Re t_qj, -Im t_qj)
//   B[(j, im)][2q, 2q+1] = ( Im t_qj,  Re t_qj)
// so that C[p][(j, re|im)] = (VHS t)_pj.  Both operands are read in FP32 (the
// first term in FP64 from the accumulator) and split in registers with a
// per-walker power-of-two scale from running maxima (per-walker unsigned
// bit patterns of non-negative floats): max |VHS|, max |t_{k-1}|; each
// launch records max |t_k| for the next.
// ---------------------------------------------------------------------------
struct TaylorSplitCfg {
  static constexpr int BM = 160, BN = 128, WM = 2, WN = 2;
  static constexpr int NT = WM * WN * 64;
  static constexpr int FM = BM / WM / 16, FN = BN / WN / 16;
  static constexpr int NA = BM * 8 / NT;   // float4 of A per thread per k block
  static constexpr int NB = 16 * BN / 4 / NT;  // float4 of t per thread per k block (16 q values)
};

struct TaylorSplitArgs {
  const float* vhs;         // [W][N][ldV] complex interleaved
  const float* t_in;        // [W][N][ncolp] t_{k-1} (k >= 2)
  const double* acc;        // [W][N][ncolp] FP64 one-body product: operand of the first term
  float* t_out;             // [W][N][ncolp] t_k
  const unsigned* max_a;    // [W] max |VHS|
  const unsigned* max_b;    // [W] max |operand term|
  unsigned* max_out;        // [W] max |t_k| (atomic)
  int N, ldV, ncolp, ncol, ntm, ntn, nkb;
  double inv_k;
};

template <class H>
__device__ __forceinline__ float split_scale_of(unsigned bits) {
  return split_row_scale<H>(__uint_as_float(bits));
}

// hi/lo of four scaled values as two 8-byte halves vectors
template <class H>
__device__ __forceinline__ void split4(float4 v, float s, uint2& hi, uint2& lo) {
  const float x[4] = {v.x * s, v.y * s, v.z * s, v.w * s};
  unsigned short h[4], l[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    h[e] = H::from_float(x[e]);
    l[e] = H::from_float(x[e] - H::to_float(h[e]));
  }
  hi = make_uint2((unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16));
  lo = make_uint2((unsigned)l[0] | ((unsigned)l[1] << 16), (unsigned)l[2] | ((unsigned)l[3] << 16));
}
template <class H>
__device__ __forceinline__ void split2(float a, float b, unsigned& hi, unsigned& lo) {
  const unsigned short ha = H::from_float(a), hb = H::from_float(b);
  const unsigned short la = H::from_float(a - H::to_float(ha)), lb = H::from_float(b - H::to_float(hb));
  hi = (unsigned)ha | ((unsigned)hb << 16);
  lo = (unsigned)la | ((unsigned)lb << 16);
}

// LDS row of a Taylor stage: two k blocks (hi 32 | lo 32 each) and a 16-byte
// pad; 272-byte rows put the fragment reads of 8 consecutive rows in 8
// distinct bank groups.
constexpr int TS_SLD = 2 * SPLIT_KB + 8;

template <class H, bool FIRST>
__global__ __launch_bounds__(TaylorSplitCfg::NT, 2) void taylor_split_kernel(TaylorSplitArgs p) {
  using C = TaylorSplitCfg;
  using vec8 = typename H::vec8;
  __shared__ __attribute__((aligned(16))) unsigned short ts_lds[(C::BM + C::BN) * TS_SLD];
  const int tiles = p.ntm * p.ntn;
  const int z = blockIdx.x / tiles;
  const int tr = blockIdx.x - z * tiles;
  const int tm = tr % p.ntm, tn = tr / p.ntm;
  const int m0 = tm * C::BM, n0 = tn * C::BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid / C::WN, wn = wid % C::WN;
  const int lrow = lane & 15, lk = 8 * (lane >> 4);
  const float sa = split_scale_of<H>(p.max_a[z]);
  const float sb = split_scale_of<H>(p.max_b[z]);
  const size_t tz = (size_t)z * p.N * p.ncolp;
  // per-walker bounds-checked buffers: rows past N (and the B columns past
  // ncol, given an out-of-range offset) load as zeros; ldV is a multiple of
  // 32, so every k block lies inside its (zero-padded) VHS row
  constexpr int esz = FIRST ? 8 : 4;  // bytes per B element
  const __amdgpu_buffer_rsrc_t a_rsrc = split_rsrc(p.vhs + (size_t)z * p.N * p.ldV, p.N * p.ldV * 4);
  const __amdgpu_buffer_rsrc_t b_rsrc =
      FIRST ? split_rsrc(p.acc + tz, p.N * p.ncolp * 8) : split_rsrc(p.t_in + tz, p.N * p.ncolp * 4);
  // A: thread stages float4 chunk (tid % 8) of rows tid / 8 + 32 t
  // B: thread stages float4 u = tid + NT t of the 16 x BN / 4 block, q
  // fastest, so that the lanes of a wave store consecutive k of one row
  // (distinct LDS banks)
  int a_off[C::NA], b_off[C::NB];
#pragma unroll
  for (int t = 0; t < C::NA; ++t)
    a_off[t] = ((m0 + (tid >> 3) + t * (C::NT / 8)) * p.ldV + 4 * (tid & 7)) * 4;
#pragma unroll
  for (int t = 0; t < C::NB; ++t) {
    const int u = tid + t * C::NT;
    const int col = n0 + 4 * (u >> 4);
    b_off[t] = col < p.ncol ? ((u & 15) * p.ncolp + col) * esz : SPLIT_ROW_NONE;
  }

  floatx4 acc[C::FM][C::FN];
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  // one stage = k blocks 2 ks and 2 ks + 1, fetched a whole stage ahead
  const int nks = (p.nkb + 1) / 2;
  float4 ra[2][C::NA], rb[2][C::NB];
  auto fetch = [&](int ks) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kb = 2 * ks + h;
      if (kb >= p.nkb) break;  // uniform
#pragma unroll
      for (int t = 0; t < C::NA; ++t)
        ra[h][t] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(a_rsrc, a_off[t], kb * 128, 0));
      const int bo = kb * 16 * p.ncolp * esz;
#pragma unroll
      for (int t = 0; t < C::NB; ++t) {
        if constexpr (FIRST) {
          const double2 x0 =
              __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(b_rsrc, b_off[t], bo, 0));
          const double2 x1 =
              __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(b_rsrc, b_off[t], bo + 16, 0));
          rb[h][t] = make_float4((float)x0.x, (float)x0.y, (float)x1.x, (float)x1.y);
        } else {
          rb[h][t] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(b_rsrc, b_off[t], bo, 0));
        }
      }
    }
  };
  auto stash = [&](int ks) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (2 * ks + h >= p.nkb) break;  // uniform
#pragma unroll
      for (int t = 0; t < C::NA; ++t) {
        uint2 hi, lo;
        split4<H>(ra[h][t], sa, hi, lo);
        unsigned short* row = ts_lds + ((tid >> 3) + t * (C::NT / 8)) * TS_SLD + h * SPLIT_KB + 4 * (tid & 7);
        *reinterpret_cast<uint2*>(row) = hi;
        *reinterpret_cast<uint2*>(row + 32) = lo;
      }
#pragma unroll
      for (int t = 0; t < C::NB; ++t) {
        const int u = tid + t * C::NT;
        const int kk = 2 * (u & 15);  // k offset of q in this block
        const int c = 4 * (u >> 4);   // first of the 4 columns (2 complex)
        const float4 v = rb[h][t];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float re = (e ? v.z : v.x) * sb, im = (e ? v.w : v.y) * sb;
          unsigned hi, lo;
          unsigned short* r0 = ts_lds + (C::BM + c + 2 * e) * TS_SLD + h * SPLIT_KB + kk;
          split2<H>(re, -im, hi, lo);  // (j, re) row
          *reinterpret_cast<unsigned*>(r0) = hi;
          *reinterpret_cast<unsigned*>(r0 + 32) = lo;
          split2<H>(im, re, hi, lo);   // (j, im) row
          *reinterpret_cast<unsigned*>(r0 + TS_SLD) = hi;
          *reinterpret_cast<unsigned*>(r0 + TS_SLD + 32) = lo;
        }
      }
    }
  };
  auto compute = [&](int ks) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (2 * ks + h >= p.nkb) break;  // uniform
      vec8 ah[C::FM], al[C::FM];
#pragma unroll
      for (int i = 0; i < C::FM; ++i) {
        const unsigned short* r = ts_lds + (wm * (C::BM / C::WM) + i * 16 + lrow) * TS_SLD + h * SPLIT_KB + lk;
        ah[i] = __builtin_bit_cast(vec8, *reinterpret_cast<const uint4*>(r));
        al[i] = __builtin_bit_cast(vec8, *reinterpret_cast<const uint4*>(r + 32));
      }
#pragma unroll
      for (int j = 0; j < C::FN; ++j) {
        const unsigned short* r =
            ts_lds + (C::BM + wn * (C::BN / C::WN) + j * 16 + lrow) * TS_SLD + h * SPLIT_KB + lk;
        const vec8 bh = __builtin_bit_cast(vec8, *reinterpret_cast<const uint4*>(r));
        const vec8 bl = __builtin_bit_cast(vec8, *reinterpret_cast<const uint4*>(r + 32));
#pragma unroll
        for (int i = 0; i < C::FM; ++i) {
          acc[i][j] = H::mma(al[i], bh, acc[i][j]);
          acc[i][j] = H::mma(ah[i], bl, acc[i][j]);
          acc[i][j] = H::mma(ah[i], bh, acc[i][j]);
        }
      }
    }
  };
  fetch(0);
  for (int ks = 0; ks < nks; ++ks) {
    if (ks) __syncthreads();  // every wave is done with the previous stage
    stash(ks);
    __syncthreads();
    if (ks + 1 < nks) fetch(ks + 1);
    compute(ks);
  }

  // t_k = C / (sa sb k), stored alone: the terms are summed into the
  // accumulator once, after the last order
  const double unscale = p.inv_k / ((double)sa * (double)sb);
  float vmax = 0.f;
#pragma unroll
  for (int i = 0; i < C::FM; ++i)
#pragma unroll
    for (int j = 0; j < C::FN; ++j) {
      const int col = n0 + wn * (C::BN / C::WN) + j * 16 + (lane & 15);
      const int mb = m0 + wm * (C::BM / C::WM) + i * 16 + 4 * (lane >> 4);
      if (col >= p.ncol) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mb + r;
        if (row >= p.N) continue;
        const size_t o = tz + (size_t)row * p.ncolp + col;
        const float tv = (float)((double)acc[i][j][r] * unscale);
        p.t_out[o] = tv;
        vmax = fmaxf(vmax, fabsf(tv));
      }
    }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o, 64));
  if (lane == 0) atomicMax(p.max_out + z, __float_as_uint(vmax));
}

// acc += t_1 + ... + t_order in FP64, in order (terms of stride n)
// Four consecutive elements per thread (16-byte term loads, two 16-byte
// accumulator loads and stores); n is a multiple of 4 (ncolp is).
__global__ __launch_bounds__(256) void taylor_split_sum_kernel(size_t n4, int order, const float* __restrict__ t,
                                                               double* __restrict__ acc) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n4) return;
  double2* a2 = reinterpret_cast<double2*>(acc) + 2 * e;
  double2 a = a2[0], b = a2[1];
  for (int k = 0; k < order; ++k) {
    const float4 v = reinterpret_cast<const float4*>(t)[(size_t)k * n4 + e];
    a.x += (double)v.x;
    a.y += (double)v.y;
    b.x += (double)v.z;
    b.y += (double)v.w;
  }
  a2[0] = a;
  a2[1] = b;
}

hipError_t launch_taylor_split_sum(const StepDims& d, int W, int order, const float* terms, double* acc,
                                   hipStream_t s) {
  if (W == 0) return hipSuccess;
  if (order > 32 || d.ncolp % 4 != 0) return hipErrorInvalidValue;
  const size_t n4 = (size_t)W * d.N * d.ncolp / 4;
  hipLaunchKernelGGL(taylor_split_sum_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, n4, order,
                     terms, acc);
  return hipGetLastError();
}

// One Taylor order k of the split path (FP16X3 / BF16X3 operands).  tmax has
// order + 2 slots of stride tstride: 0 max |P phi|, 1 max |VHS|, 1 + k max |t_k|.
hipError_t launch_taylor_split(int mode, const StepDims& d, int W, const float* vhs, const float* t_in,
                               float* t_out, const double* acc, unsigned* tmax, int tstride, int k,
                               hipStream_t s) {
  using C = TaylorSplitCfg;
  if (W == 0) return hipSuccess;
  const int ntm = ceil_div(d.N, C::BM), ntn = ceil_div(d.ncol, C::BN);
  const bool first = k == 1;
  TaylorSplitArgs p{vhs, t_in, acc, t_out, tmax + tstride, tmax + (first ? 0 : k) * (size_t)tstride,
                    tmax + (size_t)(1 + k) * tstride, d.N, d.ldV, d.ncolp, d.ncol, ntm, ntn,
                    ceil_div(2 * d.N, 32), 1.0 / k};
  const dim3 grid((unsigned)(W * ntm * ntn));
  if (mode == SPLIT_BF16) {
    if (first)
      hipLaunchKernelGGL((taylor_split_kernel<HalfBF16, true>), grid, dim3(C::NT), 0, s, p);
    else
      hipLaunchKernelGGL((taylor_split_kernel<HalfBF16, false>), grid, dim3(C::NT), 0, s, p);
  } else {
    if (first)
      hipLaunchKernelGGL((taylor_split_kernel<HalfF16, true>), grid, dim3(C::NT), 0, s, p);
    else
      hipLaunchKernelGGL((taylor_split_kernel<HalfF16, false>), grid, dim3(C::NT), 0, s, p);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Force bias on split operands (Eq. of the optimal force bias, Sec. II.B):
// vbias[z][g] = sum_{spin, i, p} Lh[spin][g][i][p] theta[z][re|im][spin][i][p],
// one GEMM over k = (spin, i, p).  Its operands carry one power-of-two scale
// per contraction row: per Cholesky vector g for Lh, per (walker, re|im) for
// theta (the per-row scales of the exchange operands vary along this k).
// ---------------------------------------------------------------------------

// Block split: block b holds rows r = s nsub + i (s < nspl, i < nsub) taken
// from source row s * S1 + b * S2 + i; one scale for the whole block.  Output
// rows b * nspl * nsub + r of 2 ldh halves (as split_rows_kernel).
// eight waves per block: 2 W blocks of 2 n rows are few rows per wave
constexpr int SPLIT_BLOCKS_NT = 512;
template <class H>
__global__ __launch_bounds__(SPLIT_BLOCKS_NT) void split_blocks_kernel(int nspl, int nsub, int ncols, const float* __restrict__ src,
                                                           int ld_src, long S1, long S2, unsigned short* __restrict__ dst,
                                                           int ldh, float* __restrict__ unscale) {
  constexpr int NW = SPLIT_BLOCKS_NT / 64;
  __shared__ float red[NW];
  const int b = blockIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int rows = nspl * nsub;
  float m = 0.f;
  for (int r = wid; r < rows; r += NW) {
    const int sp = r / nsub, i = r - sp * nsub;
    const float* srow = src + ((long)sp * S1 + (long)b * S2 + i) * ld_src;
    for (int c = lane; c < ncols; c += 64) m = fmaxf(m, fabsf(srow[c]));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if (lane == 0) red[wid] = m;
  __syncthreads();
  m = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) m = fmaxf(m, red[w]);
  const float sc = split_row_scale<H>(m);
  for (int r = wid; r < rows; r += NW) {
    const int sp = r / nsub, i = r - sp * nsub;
    const float* srow = src + ((long)sp * S1 + (long)b * S2 + i) * ld_src;
    unsigned short* d = dst + ((long)b * rows + r) * 2 * ldh;
    for (int c = lane; c < ldh; c += 64) {
      const float x = c < ncols ? srow[c] * sc : 0.f;
      const unsigned short xh = H::from_float(x);
      unsigned short* o = d + (c >> 5) * SPLIT_KB + (c & 31);
      o[0] = xh;
      o[32] = H::from_float(x - H::to_float(xh));
    }
  }
  if (threadIdx.x == 0) unscale[b] = 1.0f / sc;  // power of two: exact
}

hipError_t launch_split_blocks_mode(int mode, int nblocks, int nspl, int nsub, int ncols, const float* src, int ld_src,
                                    long S1, long S2, unsigned short* dst, int ldh, float* unscale, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  if (ldh % 32 != 0 || ldh < ncols) return hipErrorInvalidValue;
  if (mode == SPLIT_BF16)
    hipLaunchKernelGGL(split_blocks_kernel<HalfBF16>, dim3(nblocks), dim3(SPLIT_BLOCKS_NT), 0, s, nspl, nsub, ncols, src, ld_src,
                       S1, S2, dst, ldh, unscale);
  else
    hipLaunchKernelGGL(split_blocks_kernel<HalfF16>, dim3(nblocks), dim3(SPLIT_BLOCKS_NT), 0, s, nspl, nsub, ncols, src, ld_src,
                       S1, S2, dst, ldh, unscale);
  return hipGetLastError();
}

// Both splits of consecutive rows in one pass, for theta when the force
// bias and the exchange take it in the same step: block b is rows
// b * rows .. b * rows + rows - 1 (rows contiguous, stride ld_src), split once
// with the block's scale (as split_blocks_kernel with S1 = nsub, S2 = rows)
// into dst_blk and once with each row's own scale (as split_rows_kernel) into
// dst_row, both at output row b * rows + r.  The source is read once, held
// in registers (two neighbouring columns of every 128-column chunk per lane,
// SPLIT_BOTH_RPW rows per wave), and the hi / lo pairs leave as 4-byte
// words.  Every value written equals what the two separate kernels write.
constexpr int SPLIT_BOTH_NT = 512;
constexpr int SPLIT_BOTH_RPW = 8;  // blocks of up to 64 rows
constexpr int SPLIT_BOTH_CH = 3;   // rows of up to 384 split columns
template <class H>
__global__ __launch_bounds__(SPLIT_BOTH_NT) void split_both_kernel(int rows, int ncols, const float* __restrict__ src,
                                                                   int ld_src, int ldh,
                                                                   unsigned short* __restrict__ dst_blk,
                                                                   float* __restrict__ unscale_blk,
                                                                   unsigned short* __restrict__ dst_row,
                                                                   float* __restrict__ unscale_row) {
  constexpr int NW = SPLIT_BOTH_NT / 64;
  constexpr int RPW = SPLIT_BOTH_RPW, CH = SPLIT_BOTH_CH;
  __shared__ float red[NW];
  const int b = blockIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  float x0[RPW][CH], x1[RPW][CH], rm[RPW];
#pragma unroll
  for (int j = 0; j < RPW; ++j) {
    const int r = wid + NW * j;
    const float* s = src + ((long)b * rows + r) * ld_src;
    float mr = 0.f;
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int c = 128 * t + 2 * lane;
      x0[j][t] = r < rows && c < ncols ? s[c] : 0.f;
      x1[j][t] = r < rows && c + 1 < ncols ? s[c + 1] : 0.f;
      mr = fmaxf(mr, fmaxf(fabsf(x0[j][t]), fabsf(x1[j][t])));
    }
    rm[j] = mr;
  }
  float m = 0.f;
#pragma unroll
  for (int j = 0; j < RPW; ++j) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) rm[j] = fmaxf(rm[j], __shfl_xor(rm[j], o, 64));
    m = fmaxf(m, rm[j]);
  }
  if (lane == 0) red[wid] = m;
  __syncthreads();
  m = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) m = fmaxf(m, red[w]);
  const float sb = split_row_scale<H>(m);
  auto put = [&](unsigned* d, int w, float a, float c) {
    const unsigned short ah = H::from_float(a), ch = H::from_float(c);
    const unsigned short al = H::from_float(a - H::to_float(ah)), cl = H::from_float(c - H::to_float(ch));
    d[w] = (unsigned)ah | ((unsigned)ch << 16);
    d[w + 16] = (unsigned)al | ((unsigned)cl << 16);  // the lo pair, 32 halves further
  };
#pragma unroll
  for (int j = 0; j < RPW; ++j) {
    const int r = wid + NW * j;
    if (r >= rows) break;
    const float sr = split_row_scale<H>(rm[j]);
    const long o = ((long)b * rows + r) * 2 * ldh;
    unsigned* db = reinterpret_cast<unsigned*>(dst_blk + o);
    unsigned* dr = reinterpret_cast<unsigned*>(dst_row + o);
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int c = 128 * t + 2 * lane;  // even: the pair lies in one 32-column block
      if (c >= ldh) break;
      const int w = ((c >> 5) * SPLIT_KB + (c & 31)) >> 1;  // 4-byte word of the hi pair
      put(db, w, x0[j][t] * sb, x1[j][t] * sb);
      put(dr, w, x0[j][t] * sr, x1[j][t] * sr);
    }
    if (lane == 0) unscale_row[(long)b * rows + r] = 1.0f / sr;  // powers of two: exact
  }
  if (threadIdx.x == 0) unscale_blk[b] = 1.0f / sb;
}

bool split_both_fits(int rows, int ldh) {
  return rows <= SPLIT_BOTH_NT / 64 * SPLIT_BOTH_RPW && ldh <= 128 * SPLIT_BOTH_CH;
}

hipError_t launch_split_both_mode(int mode, int nblocks, int rows, int ncols, const float* src, int ld_src,
                                  int ldh, unsigned short* dst_blk, float* unscale_blk, unsigned short* dst_row,
                                  float* unscale_row, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  if (ldh % 32 != 0 || ldh < ncols || !split_both_fits(rows, ldh)) return hipErrorInvalidValue;
  if (mode == SPLIT_BF16)
    hipLaunchKernelGGL(split_both_kernel<HalfBF16>, dim3(nblocks), dim3(SPLIT_BOTH_NT), 0, s, rows, ncols, src,
                       ld_src, ldh, dst_blk, unscale_blk, dst_row, unscale_row);
  else
    hipLaunchKernelGGL(split_both_kernel<HalfF16>, dim3(nblocks), dim3(SPLIT_BOTH_NT), 0, s, rows, ncols, src,
                       ld_src, ldh, dst_blk, unscale_blk, dst_row, unscale_row);
  return hipGetLastError();
}

// C_c[(z, re|im)][g] over the k blocks of chunk c: A = theta block-split rows
// (2 W), B = Lh block-split rows (K), both 2 nmax sub-rows of 2 ldh halves.

struct FbSplitArgs {
  const unsigned short* a;  // theta [2 W][2][nmax][2 ldh]
  const unsigned short* b;  // Lh [K][2][nmax][2 ldh]
  float* part;              // [chunks][2 W][K]
  int W, K, rowb, nkb, kchunk;  // rowb: bytes per block row; k blocks per chunk
};

// 128 x 128 tiles at three workgroups per CU, as the pair exchange and the
// VHS build (0.295 -> 0.266 ms per step at n290 against 160 x 160 at two)
using FbCfg = SplitCfgT<128, 128, 3>;

template <class H>
__global__ __launch_bounds__(FbCfg::NT, FbCfg::WAVES_PER_EU) void fb_split_kernel(FbSplitArgs p, int ntm, int ntn,
                                                                                 int per8) {
  using C = FbCfg;
  constexpr int FM = C::BM / C::WM / 16, FN = C::BN / C::WN / 16;
  __shared__ __attribute__((aligned(16))) unsigned short fs_lds[SplitStage<C::BM, C::BN>::BYTES / 2];
  const int ch = blockIdx.x / per8;  // k chunk; per8 is a multiple of 8, so block % 8 stays the XCD
  int tm, tn;  // consecutive tiles on one XCD share the Lh tile
  if (!xcd_tile(blockIdx.x - ch * per8, ntn, ntm, 1, tn, tm)) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid / C::WN, wn = wid % C::WN;
  const int m0 = tm * C::BM, n0 = tn * C::BN;
  const int nm = min(C::BM, 2 * p.W - m0), nn = min(C::BN, p.K - n0);
  const int kb0 = ch * p.kchunk;
  const int nkb = min(p.kchunk, p.nkb - kb0);
  const __amdgpu_buffer_rsrc_t a_rsrc = split_rsrc(p.a + (size_t)m0 * (p.rowb / 2), nm * p.rowb);
  const __amdgpu_buffer_rsrc_t b_rsrc = split_rsrc(p.b + (size_t)n0 * (p.rowb / 2), nn * p.rowb);
  int a_off[C::NA], b_off[C::NB];
#pragma unroll
  for (int t = 0; t < C::NA; ++t) a_off[t] = ((tid >> 3) + t * (C::NT / 8)) * p.rowb + kb0 * 128 + (tid & 7) * 16;
#pragma unroll
  for (int t = 0; t < C::NB; ++t) b_off[t] = ((tid >> 3) + t * (C::NT / 8)) * p.rowb + kb0 * 128 + (tid & 7) * 16;
  floatx4 acc[FM][FN];
  split_tile_mainloop<H, C::BM, C::BN, C::WM, C::WN>(a_rsrc, b_rsrc, a_off, b_off, nkb, acc, fs_lds);
  float* out = p.part + (size_t)ch * 2 * p.W * p.K;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * (C::BN / C::WN) + j * 16 + (lane & 15);
      const int mb = m0 + wm * (C::BM / C::WM) + i * 16 + 4 * (lane >> 4);
      if (col >= p.K) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (mb + r < 2 * p.W) out[(size_t)(mb + r) * p.K + col] = acc[i][j][r];
    }
}

// vbias[z][g] = sum over chunks (fixed order) x the two unscale factors
__global__ void fb_split_reduce_kernel(int W, int K, int chunks, const float* __restrict__ part,
                                       const float* __restrict__ th_unscale, const float* __restrict__ lh_unscale,
                                       double2* __restrict__ vbias) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)W * K) return;
  const int z = (int)(e / K), g = (int)(e - (size_t)z * K);
  const size_t cs = (size_t)2 * W * K;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < chunks; ++c) {
    re += (double)part[c * cs + (size_t)(2 * z) * K + g];
    im += (double)part[c * cs + (size_t)(2 * z + 1) * K + g];
  }
  const double ul = (double)lh_unscale[g];
  vbias[e] = make_double2(re * (double)th_unscale[2 * z] * ul, im * (double)th_unscale[2 * z + 1] * ul);
}

// Number of k chunks.  The kernel runs two workgroups per CU (LDS and VGPRs
// allow no more), 512 at a time on the 256 CUs, and every workgroup of a
// launch does the same work, so the time goes as rounds x work per workgroup:
// ceil(c tiles / 512) / c for c chunks.  The smallest minimiser up to
// FB_SPLIT_CHUNKS is taken (n290, 512 walkers: 133 tiles, 7 chunks in two
// rounds instead of 4 chunks in two rounds of which the second is 4% full).
static int fb_split_chunks(int tiles, int nkb) {
  constexpr int SLOTS = FbCfg::WAVES_PER_EU * 256;
  int best = 1;
  long bn = 1, bd = 1;  // best cost as the fraction bn / bd
  for (int c = 2; c <= FB_SPLIT_CHUNKS && c <= nkb; ++c) {
    const long rounds = ((long)tiles * c + SLOTS - 1) / SLOTS;
    if (rounds * bd < bn * c) {  // rounds / c < bn / bd
      best = c;
      bn = rounds;
      bd = c;
    }
  }
  return best;
}

// C = A B^T over split rows of rowb bytes (nkb k blocks), A rows (z, re|im)
// (2 W), B rows g (K); vbias[z][g] = the chunks' sum x a_unscale x b_unscale.
static hipError_t launch_fb_split_rows(int mode, int W, int K, int rowb, int nkb, const unsigned short* a,
                                       const float* a_unscale, const unsigned short* b, const float* b_unscale,
                                       float* part, double2* vbias, hipStream_t s) {
  using C = FbCfg;
  if (W == 0) return hipSuccess;
  if ((double)C::BM * rowb >= (double)SPLIT_ROW_NONE || (double)C::BN * rowb >= (double)SPLIT_ROW_NONE)
    return hipErrorInvalidValue;
  const int ntm = ceil_div(2 * W, C::BM), ntn = ceil_div(K, C::BN);
  const int kchunk = ceil_div(nkb, fb_split_chunks(ntm * ntn, nkb));
  const int chunks = ceil_div(nkb, kchunk);  // every chunk holds at least one k block
  FbSplitArgs p{a, b, part, W, K, rowb, nkb, kchunk};
  const int per = ceil_div(ntm * ntn, 8);
  const dim3 grid((unsigned)(chunks * 8 * per));
  if (mode == SPLIT_BF16)
    hipLaunchKernelGGL(fb_split_kernel<HalfBF16>, grid, dim3(C::NT), 0, s, p, ntm, ntn, 8 * per);
  else
    hipLaunchKernelGGL(fb_split_kernel<HalfF16>, grid, dim3(C::NT), 0, s, p, ntm, ntn, 8 * per);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t n = (size_t)W * K;
  hipLaunchKernelGGL(fb_split_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, K, chunks,
                     part, a_unscale, b_unscale, vbias);
  return hipGetLastError();
}

hipError_t launch_force_bias_split(int mode, const StepDims& d, int W, const unsigned short* th, const float* th_unscale,
                                   const unsigned short* lh, const float* lh_unscale, float* part, double2* vbias,
                                   hipStream_t s) {
  const int rowb = 2 * d.nmax * 2 * d.ldh * 2;  // (spin, i) sub-rows of 2 ldh halves
  const int nkb = 2 * d.nmax * (d.ldh / 32);
  return launch_fb_split_rows(mode, W, d.K, rowb, nkb, th, th_unscale, lh, lh_unscale, part, vbias, s);
}

// ---------------------------------------------------------------------------
// Multi-determinant force bias on the split engine (FP16X3):
// vbias_g = sum over pairs c = (p <= q) of Gsym[z][c] L_g[p][q] with the
// symmetrised Green's function rows of the walkers (A) against the packed L
// transposed, one split row per Cholesky vector g (B).
// ---------------------------------------------------------------------------

__device__ __forceinline__ float block_max256(float v, float* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// dst[g] = split row of L_g over the pair index (row-major upper triangle),
// scale per g; one workgroup per g
template <class H>
__global__ __launch_bounds__(256) void split_lt_transposed_kernel(int N, int npk, int ldh, const int2* __restrict__ pq,
                                                                  const double* __restrict__ L,
                                                                  unsigned short* __restrict__ dst,
                                                                  float* __restrict__ unscale) {
  __shared__ float red[4];
  const int g = blockIdx.x, tid = threadIdx.x;
  const double* Lg = L + (size_t)g * N * N;
  float m = 0.f;
  for (int c = tid; c < npk; c += 256) {
    const int2 ab = pq[c];
    m = fmaxf(m, fabsf((float)Lg[(size_t)ab.x * N + ab.y]));
  }
  m = block_max256(m, red);
  const float sc = split_row_scale<H>(m);
  unsigned short* d = dst + (size_t)g * 2 * ldh;
  for (int c = tid; c < ldh; c += 256) {
    float x = 0.f;
    if (c < npk) {
      const int2 ab = pq[c];
      x = (float)Lg[(size_t)ab.x * N + ab.y] * sc;
    }
    const unsigned short xh = H::from_float(x);
    unsigned short* o = d + (c >> 5) * SPLIT_KB + (c & 31);
    o[0] = xh;
    o[32] = H::from_float(x - H::to_float(xh));
  }
  if (tid == 0) unscale[g] = 1.0f / sc;
}

hipError_t setup_split_lt_transposed(int mode, int K, int N, int npk, int ldh, const int2* pq, const double* L,
                                     unsigned short* dst, float* unscale, hipStream_t s) {
  if (ldh % 32 != 0 || ldh < npk) return hipErrorInvalidValue;
  if (mode == SPLIT_BF16)
    hipLaunchKernelGGL(split_lt_transposed_kernel<HalfBF16>, dim3(K), dim3(256), 0, s, N, npk, ldh, pq, L, dst,
                       unscale);
  else
    hipLaunchKernelGGL(split_lt_transposed_kernel<HalfF16>, dim3(K), dim3(256), 0, s, N, npk, ldh, pq, L, dst,
                       unscale);
  return hipGetLastError();
}

// Row r of `data` (ldh floats, the first ncols meaningful) becomes, in place,
// the split row of 2 ldh halves (the same bytes), scale per row; one
// workgroup per row.  Every value is read (for the maximum) before the
// barrier inside block_max256; after it each k block (32 floats, 128 bytes)
// is read by one half-wave, one float per lane in a single load, and then
// overwritten by the same half-wave with its 32 hi and 32 lo halves.
template <class H>
__global__ __launch_bounds__(256) void split_rows_inplace_kernel(int ncols, int ldh, float* __restrict__ data,
                                                                 float* __restrict__ unscale) {
  __shared__ float red[4];
  const int r = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  float* row = data + (size_t)r * ldh;
  float m = 0.f;
  for (int c = tid; c < ncols; c += 256) m = fmaxf(m, fabsf(row[c]));
  m = block_max256(m, red);
  const float sc = split_row_scale<H>(m);
  unsigned short* d = reinterpret_cast<unsigned short*>(row);
  const int nkb = ldh / 32, i = lane & 31;
  for (int kb = 2 * wid + (lane >> 5); kb < nkb; kb += 8) {
    const int c = kb * 32 + i;
    const float x = c < ncols ? row[c] * sc : 0.f;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the block's read stays ahead of its overwrite
    const unsigned short xh = H::from_float(x);
    d[kb * SPLIT_KB + i] = xh;
    d[kb * SPLIT_KB + 32 + i] = H::from_float(x - H::to_float(xh));
  }
  if (tid == 0) unscale[r] = 1.0f / sc;
}

__global__ void zero_fill_kernel(float* __restrict__ p, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    p[e] = 0.f;
}

hipError_t launch_msd_fb_split(int mode, int W, int K, int npk, int ldh, float* gs, float* gs_unscale,
                               const unsigned short* lts, const float* lts_unscale, float* part, double2* vbias,
                               hipStream_t s) {
  if (W == 0) return hipSuccess;
  if (ldh % 32 != 0 || ldh < npk) return hipErrorInvalidValue;
  if (mode == SPLIT_BF16)
    hipLaunchKernelGGL(split_rows_inplace_kernel<HalfBF16>, dim3(2 * W), dim3(256), 0, s, npk, ldh, gs, gs_unscale);
  else
    hipLaunchKernelGGL(split_rows_inplace_kernel<HalfF16>, dim3(2 * W), dim3(256), 0, s, npk, ldh, gs, gs_unscale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_fb_split_rows(mode, W, K, 4 * ldh, ldh / 32, reinterpret_cast<const unsigned short*>(gs),
                                 gs_unscale, lts, lts_unscale, part, vbias, s)) != hipSuccess)
    return e;
  // gs lives in the VHS workspace, whose rows the split propagation kernels
  // read up to their zero padding: leave the rows zero (a fill kernel, no
  // memset node under graph capture); gs_unscale follows gs
  const size_t n = (size_t)2 * W * (ldh + 1);
  hipLaunchKernelGGL(zero_fill_kernel, dim3((unsigned)std::min<size_t>((n + 255) / 256, 8192)), dim3(256), 0, s, gs,
                     n);
  return hipGetLastError();
}
