// Exchange energy with hi/lo split operands on the 16-bit matrix cores
// (mixed modes AFQMC_BF16X3 and AFQMC_FP16X3).  Same algorithm as the FP32 /
// FP64 exchange kernel (Sec. III.C direct algorithm, T never leaves the chip);
// only the operand format and the MFMA differ.

#include <math.h>

#include "common.h"
#include "kernels.h"
#include "split_tile.h"
#include "tile_order.h"
#include "exchange_epilogue.h"

// ---------------------------------------------------------------------------
// Row splitting: src rows (FP32, stride ld_src, ncols valid) -> hi/lo rows
// (stride ld_dst, zero padded) and the power-of-two row scale.  One wave per row.
// ---------------------------------------------------------------------------
template <class H>
__global__ __launch_bounds__(256) void split_rows_kernel(long nrows, int ncols, const float* __restrict__ src,
                                                         int ld_src, unsigned short* __restrict__ hi,
                                                         unsigned short* __restrict__ lo, int ld_dst,
                                                         float* __restrict__ scale) {
  const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nrows) return;
  const float* s = src + row * ld_src;
  float m = 0.f;
  for (int c = lane; c < ncols; c += 64) m = fmaxf(m, fabsf(s[c]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  const float sc = split_row_scale<H>(m);
  unsigned short* h = hi + row * ld_dst;
  unsigned short* l = lo + row * ld_dst;
  for (int c = lane; c < ld_dst; c += 64) {
    const float x = c < ncols ? s[c] * sc : 0.f;
    const unsigned short xh = H::from_float(x);
    h[c] = xh;
    l[c] = H::from_float(x - H::to_float(xh));
  }
  if (lane == 0) scale[row] = sc;
}

template <class H>
hipError_t launch_split_rows(long nrows, int ncols, const float* src, int ld_src, unsigned short* hi,
                             unsigned short* lo, int ld_dst, float* scale, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  hipLaunchKernelGGL(split_rows_kernel<H>, dim3((unsigned)((nrows + 3) / 4)), dim3(256), 0, s, nrows,
                     ncols, src, ld_src, hi, lo, ld_dst, scale);
  return hipGetLastError();
}

hipError_t launch_split_rows_mode(int mode, long nrows, int ncols, const float* src, int ld_src,
                                  unsigned short* hi, unsigned short* lo, int ld_dst, float* scale,
                                  hipStream_t s) {
  return mode == SPLIT_BF16 ? launch_split_rows<HalfBF16>(nrows, ncols, src, ld_src, hi, lo, ld_dst, scale, s)
                            : launch_split_rows<HalfF16>(nrows, ncols, src, ld_src, hi, lo, ld_dst, scale, s);
}

// ---------------------------------------------------------------------------
// Exchange on split operands.
// ---------------------------------------------------------------------------
// 4-wave workgroups, single-buffered LDS under 80 KB: two workgroups per CU.
struct ExSplitCfg {
  static constexpr int BM = 192, BN = 160, BK = 32, WM = 2, WN = 2, GS = 8;
  static constexpr int PIPE = 0;
  static constexpr bool DBUF = false;
  static constexpr int WAVES_PER_EU = 2;
};

struct ExSplitProb {
  const unsigned short* a_hi;  // spin block [K][nmax][ldh]
  const unsigned short* a_lo;
  const float* a_scale;        // spin block [K][nmax]
  const unsigned short* b_hi;  // theta [W][re|im][spin][nmax][ldh]
  const unsigned short* b_lo;
  const float* b_scale;        // [W][re|im][spin][nmax]
  int K, W, n, nmax, ldh, sp, G, Z;
  int gt, wt;
  __device__ uint4 load_a(int r, int k, int part) const {
    if (r >= G * n) return make_uint4(0, 0, 0, 0);
    const int g = gt * G + r / n;
    if (g >= K) return make_uint4(0, 0, 0, 0);
    const unsigned short* base = part ? a_lo : a_hi;
    return *reinterpret_cast<const uint4*>(base + ((size_t)g * nmax + r % n) * ldh + k);
  }
  __device__ size_t b_row(int c) const {  // -1 if outside
    const int n2 = 2 * n;
    const int z = wt * Z + c / n2;
    const int cc = c % n2;
    const int comp = cc >= n ? 1 : 0;
    const int j = cc - comp * n;
    return (((size_t)z * 2 + comp) * 2 + sp) * nmax + j;
  }
  __device__ uint4 load_b(int c, int k, int part) const {
    if (c >= Z * 2 * n) return make_uint4(0, 0, 0, 0);
    if (wt * Z + c / (2 * n) >= W) return make_uint4(0, 0, 0, 0);
    const unsigned short* base = part ? b_lo : b_hi;
    return *reinterpret_cast<const uint4*>(base + b_row(c) * ldh + k);
  }
};

constexpr size_t EXS_EPI_BUDGET = 64 * 1024;

static int exs_walkers_per_pass(int G, int Z, int n) {
  const size_t per = (size_t)G * n * (2 * n + 1) * sizeof(float);
  int zp = (int)(EXS_EPI_BUDGET / per);
  const int slots = 64 / (ExSplitCfg::WM * ExSplitCfg::WN);
  if (zp > slots) zp = slots;
  if (zp < 1) zp = 1;
  return zp < Z ? zp : Z;
}

static size_t exs_tab_off(int G, int Z, int n) {
  using C = ExSplitCfg;
  const size_t stage = (C::DBUF ? 2 : 1) * (size_t)SplitLds<C::BM, C::BN, C::BK>::BYTES;
  const size_t epi = (size_t)exs_walkers_per_pass(G, Z, n) * G * n * (2 * n + 1) * sizeof(float);
  return (stage > epi ? stage : epi + 15) / 16 * 16;
}
static size_t exs_lds_bytes(int G, int Z, int n) {
  return exs_tab_off(G, Z, n) + EX_TAB_BYTES + EX_RED_BYTES;
}

template <class H>
__global__ __launch_bounds__(ExSplitCfg::WM* ExSplitCfg::WN * 64, ExSplitCfg::WAVES_PER_EU) void exchange_split_kernel(
    ExSplitProb p0, double2* __restrict__ part, int ntg, int nwt, int tab_off, int zpp, int gs) {
  using C = ExSplitCfg;
  constexpr int BM = C::BM, BN = C::BN, BK = C::BK, WM = C::WM, WN = C::WN;
  ExSplitProb p = p0;
  if (!xcd_tile(blockIdx.x, ntg, nwt, gs, p.gt, p.wt)) return;
  extern __shared__ double2 exs_lds_raw[];
  floatx4 acc[BM / WM / 16][BN / WN / 16];
  split_tile_mainloop<H, BM, BN, BK, WM, WN, ExSplitProb, C::PIPE>(
      p, p.ldh, acc, reinterpret_cast<unsigned short*>(exs_lds_raw));
  const ExTileGeom q{p.n, p.G, p.Z, p.K, p.W, p.gt, p.wt};
  const float* as = p.a_scale;
  const float* bs = p.b_scale;
  const int nmax = p.nmax, sp = p.sp;
  auto rscale = [as, nmax](int g, int i) { return as[(size_t)g * nmax + i]; };
  auto cscale = [bs, nmax, sp](int z, int comp, int j) {
    return bs[(((size_t)z * 2 + comp) * 2 + sp) * nmax + j];
  };
  exchange_epilogue<float, floatx4, BM, BN, WM, WN>(acc, reinterpret_cast<char*>(exs_lds_raw), tab_off,
                                                   tab_off + EX_TAB_BYTES, q, zpp, H::SCALED, rscale,
                                                   cscale, part, p.sp, ntg);
}

ExTile exchange_split_tile(int n) {
  ExTile t;
  t.G = n > 0 ? ExSplitCfg::BM / n : 0;
  t.Z = n > 0 ? ExSplitCfg::BN / (2 * n) : 0;
  return t;
}

hipError_t launch_exchange_split(int mode, const StepDims& d, int W, const unsigned short* lh_hi,
                                 const unsigned short* lh_lo, const float* lh_scale,
                                 const unsigned short* th_hi, const unsigned short* th_lo,
                                 const float* th_scale, double2* part, int sp, int* ntg_out,
                                 hipStream_t s, int gs) {
  using C = ExSplitCfg;
  if (gs < 1) gs = C::GS;
  const ExTile t = exchange_split_tile(d.nmax);
  if (t.G < 1 || t.Z < 1) return hipErrorInvalidValue;
  const int ntg = ceil_div(d.K, t.G);
  const int nwt = ceil_div(W, t.Z);
  *ntg_out = ntg;
  const int n = sp == 0 ? d.na : d.nb;
  if (n == 0) return hipSuccess;
  const size_t sblk = (size_t)d.K * d.nmax;
  ExSplitProb p{lh_hi + sp * sblk * d.ldh, lh_lo + sp * sblk * d.ldh, lh_scale + sp * sblk,
                th_hi, th_lo, th_scale, d.K, W, n, d.nmax, d.ldh, sp, t.G, t.Z, 0, 0};
  const size_t lds = exs_lds_bytes(t.G, t.Z, n);
  const int tab_off = (int)exs_tab_off(t.G, t.Z, n);
  const int zpp = exs_walkers_per_pass(t.G, t.Z, n);
  const int per = ceil_div(ntg * nwt, 8);
  if (mode == SPLIT_BF16)
    hipLaunchKernelGGL(exchange_split_kernel<HalfBF16>, dim3(8 * per), dim3(C::WM * C::WN * 64), lds, s,
                       p, part, ntg, nwt, tab_off, zpp, gs);
  else
    hipLaunchKernelGGL(exchange_split_kernel<HalfF16>, dim3(8 * per), dim3(C::WM * C::WN * 64), lds, s,
                       p, part, ntg, nwt, tab_off, zpp, gs);
  return hipGetLastError();
}

hipError_t set_split_kernel_attributes() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(exchange_split_kernel<HalfBF16>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(exchange_split_kernel<HalfF16>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}
