// Exchange energy with hi/lo split operands on the 16-bit matrix cores
// (mixed modes AFQMC_BF16X3 and AFQMC_FP16X3).  Same algorithm as the FP32 /
// FP64 exchange kernel (Sec. III.C direct algorithm, T never leaves the chip);
// only the operand format and the MFMA differ.

#include <math.h>

#include "common.h"
#include "kernels.h"
#include "split_tile.h"
#include "tile_order.h"
#include "exchange_tri.h"

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
  const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nrows) return;
  const float* s = src + row * ld_src;
  float m = 0.f;
  for (int c = lane; c < ncols; c += 64) m = fmaxf(m, fabsf(s[c]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  const float sc = split_row_scale<H>(m);
  unsigned short* d = dst + row * 2 * ldh;
  for (int c = lane; c < ldh; c += 64) {
    const float x = c < ncols ? s[c] * sc : 0.f;
    const unsigned short xh = H::from_float(x);
    unsigned short* b = d + (c >> 5) * SPLIT_KB + (c & 31);
    b[0] = xh;
    b[32] = H::from_float(x - H::to_float(xh));
  }
  if (lane == 0) unscale[row] = 1.0f / sc;  // power of two: exact
}

template <class H>
hipError_t launch_split_rows(long nrows, int ncols, const float* src, int ld_src, unsigned short* dst,
                             int ldh, float* unscale, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  if (ldh % 32 != 0 || ldh < ncols) return hipErrorInvalidValue;
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
// Exchange on split operands.
// ---------------------------------------------------------------------------
// 4-wave workgroups of 80 x 80 wave tiles; register prefetch of the next k
// block, one LDS stage; two workgroups per CU, so that one workgroup's
// epilogue runs beside the other's matrix-core work.
struct ExSplitCfg {
  static constexpr int BM = 160, BN = 160, WM = 2, WN = 2, GS = 8;
  static constexpr int NT = WM * WN * 64;
  static constexpr int NA = BM * 8 / NT, NB = BN * 8 / NT;
  static constexpr int WAVES_PER_EU = 2;
};

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
// VHS build on split operands (Eq. of the propagator: VHS_z = i sqrt(dt)
// sum_g xs_zg L_g): C[(z, re|im)][pq] = sum_g xs[z][re|im][g] LT[pq][g] over
// the packed p <= q triangle, mirrored on store.  A = xs split rows (2 W),
// B = packed L split rows (N (N + 1) / 2), contraction over the Cholesky
// index.
// ---------------------------------------------------------------------------
struct VhsSplitArgs {
  const unsigned short* a;  // xs split rows [2 W][2 ldhK]
  const float* a_unscale;   // [2 W]
  const unsigned short* b;  // LT split rows [Npk][2 ldhK]
  const float* b_unscale;   // [Npk]
  const int2* pq;           // packed index -> (p, q)
  float* vhs;               // [W][N][ldV] complex interleaved
  int W, Npk, N, ldV, rowb, nkb;
  float sdt;
};

template <class H>
__global__ __launch_bounds__(ExSplitCfg::NT, ExSplitCfg::WAVES_PER_EU) void vhs_split_kernel(VhsSplitArgs p,
                                                                                             int ntn, int ntm) {
  using C = ExSplitCfg;
  constexpr int FM = C::BM / C::WM / 16, FN = C::BN / C::WN / 16;
  int tn, tm;  // consecutive tiles on one XCD share the packed-L tile
  if (!xcd_tile(blockIdx.x, ntn, ntm, 1, tn, tm)) return;
  __shared__ __attribute__((aligned(16))) unsigned short vs_lds[SplitStage<C::BM, C::BN>::BYTES / 2];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid / C::WN, wn = wid % C::WN;
  const int m0 = tm * C::BM, n0 = tn * C::BN;
  const int nm = min(C::BM, 2 * p.W - m0), nn = min(C::BN, p.Npk - n0);
  // rows past nm / nn fall outside the tile buffers: staged as zeros
  const __amdgpu_buffer_rsrc_t a_rsrc = split_rsrc(p.a + (size_t)m0 * (p.rowb / 2), nm * p.rowb);
  const __amdgpu_buffer_rsrc_t b_rsrc = split_rsrc(p.b + (size_t)n0 * (p.rowb / 2), nn * p.rowb);
  int a_off[C::NA], b_off[C::NB];
#pragma unroll
  for (int t = 0; t < C::NA; ++t) a_off[t] = ((tid >> 3) + t * (C::NT / 8)) * p.rowb + (tid & 7) * 16;
#pragma unroll
  for (int t = 0; t < C::NB; ++t) b_off[t] = ((tid >> 3) + t * (C::NT / 8)) * p.rowb + (tid & 7) * 16;
  floatx4 acc[FM][FN];
  split_tile_mainloop<H, C::BM, C::BN, C::WM, C::WN>(a_rsrc, b_rsrc, a_off, b_off, p.nkb, acc, vs_lds);
  // rows m = 2 z + (re|im): each lane's 4 consecutive rows are 2 whole walkers
#pragma unroll
  for (int f = 0; f < FN; ++f) {
    const int col = n0 + wn * (C::BN / C::WN) + f * 16 + (lane & 15);
    if (col >= p.Npk) continue;
    const int2 ij = p.pq[col];
    const float cs = H::SCALED ? p.b_unscale[col] : 1.0f;
#pragma unroll
    for (int fi = 0; fi < FM; ++fi) {
      const int mb = m0 + wm * (C::BM / C::WM) + fi * 16 + 4 * (lane >> 4);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int z = (mb >> 1) + h;
        if (z >= p.W) continue;
        float cr = acc[fi][f][2 * h], ci = acc[fi][f][2 * h + 1];
        if (H::SCALED) {  // powers of two: exact
          cr *= p.a_unscale[2 * z] * cs;
          ci *= p.a_unscale[2 * z + 1] * cs;
        }
        const float2 v = make_float2(-p.sdt * ci, p.sdt * cr);
        *reinterpret_cast<float2*>(p.vhs + ((size_t)z * p.N + ij.x) * p.ldV + 2 * ij.y) = v;
        if (ij.x != ij.y) *reinterpret_cast<float2*>(p.vhs + ((size_t)z * p.N + ij.y) * p.ldV + 2 * ij.x) = v;
      }
    }
  }
}

hipError_t launch_vhs_split(int mode, const StepDims& d, int W, const unsigned short* xs, const float* xs_unscale,
                            const unsigned short* lt, const float* lt_unscale, const int2* pq, float* vhs,
                            double sdt, hipStream_t s) {
  using C = ExSplitCfg;
  if (W == 0) return hipSuccess;
  if (d.ldhK % 32 != 0) return hipErrorInvalidValue;
  const int rowb = 2 * d.ldhK * 2;
  if ((double)C::BM * rowb >= (double)SPLIT_ROW_NONE) return hipErrorInvalidValue;
  const int ntm = ceil_div(2 * W, C::BM), ntn = ceil_div(d.Npk, C::BN);
  VhsSplitArgs p{xs, xs_unscale, lt, lt_unscale, pq, vhs, W, d.Npk, d.N, d.ldV, rowb, d.ldhK / 32, (float)sdt};
  const int per = ceil_div(ntm * ntn, 8);
  if (mode == SPLIT_BF16)
    hipLaunchKernelGGL(vhs_split_kernel<HalfBF16>, dim3(8 * per), dim3(C::NT), 0, s, p, ntn, ntm);
  else
    hipLaunchKernelGGL(vhs_split_kernel<HalfF16>, dim3(8 * per), dim3(C::NT), 0, s, p, ntn, ntm);
  return hipGetLastError();
}
