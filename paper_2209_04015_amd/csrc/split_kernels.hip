// Exchange energy with hi/lo split operands on the 16-bit matrix cores
// (mixed modes AFQMC_BF16X3 and AFQMC_FP16X3).  Same algorithm as the FP32 /
// FP64 exchange kernel (Sec. III.C direct algorithm, T never leaves the chip);
// only the operand format and the MFMA differ.

#include <math.h>

#include "common.h"
#include "kernels.h"
#include "split_tile.h"
#include "tile_order.h"

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
struct ExSplitCfg {
  static constexpr int BM = 192, BN = 160, BK = 32, WM = 4, WN = 2, GS = 8;
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

constexpr size_t EXS_EPI_BUDGET = 150 * 1024;

static int exs_walkers_per_pass(int G, int Z, int n) {
  const size_t per = (size_t)G * n * (2 * n + 1) * sizeof(float);
  int zp = (int)(EXS_EPI_BUDGET / per);
  const int slots = 64 / (ExSplitCfg::WM * ExSplitCfg::WN);
  if (zp > slots) zp = slots;
  if (zp < 1) zp = 1;
  return zp < Z ? zp : Z;
}

static size_t exs_lds_bytes(int G, int Z, int n) {
  using C = ExSplitCfg;
  const size_t stage = 2 * (size_t)SplitLds<C::BM, C::BN, C::BK>::BYTES;
  const size_t epi = (size_t)exs_walkers_per_pass(G, Z, n) * G * n * (2 * n + 1) * sizeof(float);
  return (stage > epi ? stage : epi) + 64 * sizeof(double2);
}

template <class H>
__global__ __launch_bounds__(ExSplitCfg::WM* ExSplitCfg::WN * 64) void exchange_split_kernel(
    ExSplitProb p0, double2* __restrict__ part, int ntg, int nwt, int red_off, int zpp) {
  using C = ExSplitCfg;
  constexpr int BM = C::BM, BN = C::BN, BK = C::BK, WM = C::WM, WN = C::WN;
  constexpr int NT = WM * WN * 64;
  ExSplitProb p = p0;
  if (!xcd_tile(blockIdx.x, ntg, nwt, C::GS, p.gt, p.wt)) return;
  extern __shared__ double2 exs_lds_raw[];
  floatx4 acc[BM / WM / 16][BN / WN / 16];
  split_tile_mainloop<H, BM, BN, BK, WM, WN>(p, p.ldh, acc,
                                             reinterpret_cast<unsigned short*>(exs_lds_raw));

  float* lds = reinterpret_cast<float*>(exs_lds_raw);
  const int n = p.n, n2 = 2 * n, TS = n2 + 1;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / WN, wn = wid % WN;
  const int rows = p.G * n;
  const int blk = rows * TS;
  const int nn = n * n;
  constexpr int NWAVE = NT / 64;
  double2* red = reinterpret_cast<double2*>(reinterpret_cast<char*>(exs_lds_raw) + red_off);
  for (int z0 = 0; z0 < p.Z; z0 += zpp) {
    const int zn = min(zpp, p.Z - z0);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BM / WM / 16; ++i)
#pragma unroll
      for (int j = 0; j < BN / WN / 16; ++j) {
        const int mb = wm * (BM / WM) + i * 16 + 4 * (lane >> 4);
        const int cg = wn * (BN / WN) + j * 16 + (lane & 15);
        const int c = cg - z0 * n2;
        if (c < 0 || c >= zn * n2) continue;
        if (p.wt * p.Z + cg / n2 >= p.W) continue;
        const int zz = c / n2, col = c - zz * n2;
        const float cs = 1.0f / p.b_scale[p.b_row(cg)];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = mb + r;
          if (row >= rows) continue;
          const int g = p.gt * p.G + row / n;
          const float rs = g < p.K ? 1.0f / p.a_scale[(size_t)g * p.nmax + row % n] : 0.f;
          lds[zz * blk + row * TS + col] = acc[i][j][r] * rs * cs;  // exact: powers of two
        }
      }
    __syncthreads();
    for (int zz = 0; zz < zn; ++zz) {
      const float* tb = lds + zz * blk;
      double2 s = make_double2(0.0, 0.0);
      for (int e = threadIdx.x; e < p.G * nn; e += NT) {
        const int g = e / nn, ij = e % nn, i = ij / n, j = ij % n;
        const float* ri = tb + (g * n + i) * TS;
        const float* rj = tb + (g * n + j) * TS;
        const double ar = ri[j], ai = ri[n + j];
        const double br = rj[i], bi = rj[n + i];
        s.x += ar * br - ai * bi;
        s.y += ar * bi + ai * br;
      }
      s = wave_sum2(s);
      if (lane == 0) red[zz * NWAVE + wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < zn) {
      const int z = p.wt * p.Z + z0 + threadIdx.x;
      if (z < p.W) {
        double2 t = make_double2(0.0, 0.0);
        for (int w = 0; w < NWAVE; ++w) t = cadd(t, red[threadIdx.x * NWAVE + w]);
        part[((size_t)p.sp * ntg + p.gt) * p.W + z] = t;
      }
    }
  }
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
                                 hipStream_t s) {
  using C = ExSplitCfg;
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
  const int red_off = (int)(lds - 64 * sizeof(double2));
  const int zpp = exs_walkers_per_pass(t.G, t.Z, n);
  const int per = ceil_div(ntg * nwt, 8);
  if (mode == SPLIT_BF16)
    hipLaunchKernelGGL(exchange_split_kernel<HalfBF16>, dim3(8 * per), dim3(C::WM * C::WN * 64), lds, s,
                       p, part, ntg, nwt, red_off, zpp);
  else
    hipLaunchKernelGGL(exchange_split_kernel<HalfF16>, dim3(8 * per), dim3(C::WM * C::WN * 64), lds, s,
                       p, part, ntg, nwt, red_off, zpp);
  return hipGetLastError();
}

hipError_t set_split_kernel_attributes() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(exchange_split_kernel<HalfBF16>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(exchange_split_kernel<HalfF16>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}
