// Kernels of one phaseless-AFQMC walker step (arXiv 2209.04015, Secs. II.B and III).
//
// Working precision T is double (FP64 path) or float (mixed path: the
// contractions run on FP32 MFMA; overlaps, inverses, weights, QR, the
// one-body half steps and every energy accumulation stay FP64).

#include <math.h>

#include "common.h"
#include "kernels.h"
#include "mfma_tile.h"
#include "tile_order.h"
#include "exchange_epilogue.h"

template <typename T> struct Cplx;
template <> struct Cplx<float> { using t = float2; };
template <> struct Cplx<double> { using t = double2; };

// ===========================================================================
// Green's function: S = PhiT^T phi, log det S, theta = phi S^-1, E1 = tr(hh theta)
// (Sec. III.A overlap; Eq. halfgf; one-body energy of Sec. III.C)
//
// One workgroup per (walker, spin).  S is built from 32-row chunks of phi
// staged in LDS; the inverse comes from Gauss-Jordan elimination with
// partial pivoting on [S | I] in LDS, which also yields log det S as the sum
// of the complex logs of the pivots plus i pi per row swap.
// ===========================================================================

// 16-row chunks and at most 128 VGPRs (4 waves per SIMD): at n = 26, four
// workgroups fit on a CU, so 512 walkers x 2 spins run in one round
// (0.33 -> 0.26 ms per call at n290 against 32-row chunks and 168 VGPRs)
#ifndef GF_CHUNK_ROWS
#define GF_CHUNK_ROWS 16
#endif
#ifndef GF_WPE
#define GF_WPE 4
#endif
constexpr int GF_THREADS = 256;
constexpr int GF_CHUNK = GF_CHUNK_ROWS;
// Instances by the bound NB on the electrons per spin (32 or 45): 2 x 2
// blocks of S per thread, ceil(NB / 2)^2 <= GF_SBLK * 256, and walker-chunk
// entries per thread
template <int NB>
struct GfBound {
  static constexpr int SBLK = ((NB + 1) / 2 * ((NB + 1) / 2) + GF_THREADS - 1) / GF_THREADS;
  static constexpr int LD = (GF_CHUNK * NB + GF_THREADS - 1) / GF_THREADS;
  static constexpr bool PREFETCH = NB <= 32;  // the larger instance has no registers to spare
};

static size_t gf_lds_bytes(int n) {
  return (size_t)n * 2 * n * sizeof(double2)       // [S | I]
         + (size_t)GF_CHUNK * n * sizeof(double2)  // phi chunk
         + (size_t)GF_CHUNK * n * sizeof(double)   // PhiT chunk
         + (size_t)n * sizeof(double2)             // elimination factors
         + 8 * sizeof(double2) + 16;               // reductions, pivot
}

template <typename T, int NB>
__global__ __launch_bounds__(GF_THREADS) __attribute__((amdgpu_waves_per_eu(GF_WPE))) void gf_kernel(
    StepDims d, const double2* __restrict__ phi_a, const double2* __restrict__ phi_b,
    const double* __restrict__ phiT, const double* __restrict__ hh, T* __restrict__ theta,
    double2* __restrict__ logdet, double2* __restrict__ e1, int* __restrict__ status) {
  extern __shared__ double2 gf_lds[];
  constexpr int GF_SBLK = GfBound<NB>::SBLK, GF_LD = GfBound<NB>::LD;
  const int z = blockIdx.x;
  const int sp = blockIdx.y;
  const int n = sp == 0 ? d.na : d.nb;
  const int N = d.N;
  const int tid = threadIdx.x;
  const int n2 = 2 * n;
  double2* aug = gf_lds;                               // n x 2n
  double2* ch = aug + n * n2;                          // CHUNK x n
  double* tch = reinterpret_cast<double*>(ch + GF_CHUNK * n);  // CHUNK x n
  double2* fac = reinterpret_cast<double2*>(tch + GF_CHUNK * n);
  double2* red = fac + n;
  int* sh_piv = reinterpret_cast<int*>(red + 8);

  if (n == 0) {
    if (tid == 0) {
      logdet[2 * z + sp] = make_double2(0.0, 0.0);
      if (e1) e1[2 * z + sp] = make_double2(0.0, 0.0);
    }
    return;
  }
  const double2* phi = (sp == 0 ? phi_a : phi_b) + (size_t)z * N * n;
  const double* pT = phiT + (size_t)sp * N * d.nmax;

  // ---- S = PhiT^T phi: each thread owns 2 x 2 blocks of entries, so four LDS
  // reads (two PhiT values, two phi values) feed four products ----
  const int nbk = (n + 1) >> 1;  // blocks per side (a last odd row / column is clamped, not stored)
  double2 sacc[GF_SBLK][4];
#pragma unroll
  for (int b = 0; b < GF_SBLK; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) sacc[b][q] = make_double2(0.0, 0.0);
  // the walker's chunk after the current one is loaded into registers while
  // the current one is worked on (entry e of chunk p0: row p0 + e / n,
  // orbital e % n); the trial's rows, shared by every walker, come from the
  // L2 when the chunk is stored
  typedef double d2v __attribute__((ext_vector_type(2)));  // a native vector: kept in registers
  d2v pf[GF_LD];
  auto load_chunk = [&](int p0) {
    if (!GfBound<NB>::PREFETCH) return;
    const int cnt = p0 < N ? min(GF_CHUNK, N - p0) * n : 0;
#pragma unroll
    for (int b = 0; b < GF_LD; ++b) {
      const int e = tid + b * GF_THREADS;
      pf[b] = e < cnt ? *reinterpret_cast<const d2v*>(phi + (size_t)p0 * n + e) : d2v{0.0, 0.0};
    }
  };
  auto store_chunk = [&](int p0, bool with_trial) {
    const int cnt = min(GF_CHUNK, N - p0) * n;
    if (GfBound<NB>::PREFETCH) {
#pragma unroll
      for (int b = 0; b < GF_LD; ++b) {
        const int e = tid + b * GF_THREADS;
        if (e < cnt) {
          ch[e] = make_double2(pf[b].x, pf[b].y);
          if (with_trial) tch[e] = pT[(size_t)(p0 + e / n) * d.nmax + e % n];
        }
      }
    } else {
#pragma unroll 1
      for (int e = tid; e < cnt; e += GF_THREADS) {
        ch[e] = phi[(size_t)p0 * n + e];
        if (with_trial) tch[e] = pT[(size_t)(p0 + e / n) * d.nmax + e % n];
      }
    }
  };
  load_chunk(0);
  for (int p0 = 0; p0 < N; p0 += GF_CHUNK) {
    const int rows = min(GF_CHUNK, N - p0);
    __syncthreads();
    store_chunk(p0, true);
    load_chunk(p0 + GF_CHUNK);
    __syncthreads();
#pragma unroll
    for (int b = 0; b < GF_SBLK; ++b) {
      const int e = tid + b * GF_THREADS;
      if (e < nbk * nbk) {
        const int bi = e / nbk, bj = e - bi * nbk;
        const int i0 = 2 * bi, j0 = 2 * bj;
        const int i1 = min(i0 + 1, n - 1), j1 = min(j0 + 1, n - 1);
        double2 s00 = make_double2(0.0, 0.0), s01 = s00, s10 = s00, s11 = s00;
        for (int pr = 0; pr < rows; ++pr) {
          const double t0 = tch[pr * n + i0], t1 = tch[pr * n + i1];
          const double2 f0 = ch[pr * n + j0], f1 = ch[pr * n + j1];
          s00.x = fma(t0, f0.x, s00.x);
          s00.y = fma(t0, f0.y, s00.y);
          s01.x = fma(t0, f1.x, s01.x);
          s01.y = fma(t0, f1.y, s01.y);
          s10.x = fma(t1, f0.x, s10.x);
          s10.y = fma(t1, f0.y, s10.y);
          s11.x = fma(t1, f1.x, s11.x);
          s11.y = fma(t1, f1.y, s11.y);
        }
        sacc[b][0] = cadd(sacc[b][0], s00);
        sacc[b][1] = cadd(sacc[b][1], s01);
        sacc[b][2] = cadd(sacc[b][2], s10);
        sacc[b][3] = cadd(sacc[b][3], s11);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < GF_SBLK; ++b) {
    const int e = tid + b * GF_THREADS;
    if (e < nbk * nbk) {
      const int bi = e / nbk, bj = e - bi * nbk;
      const int i0 = 2 * bi, j0 = 2 * bj;
      aug[i0 * n2 + j0] = sacc[b][0];
      if (j0 + 1 < n) aug[i0 * n2 + j0 + 1] = sacc[b][1];
      if (i0 + 1 < n) aug[(i0 + 1) * n2 + j0] = sacc[b][2];
      if (i0 + 1 < n && j0 + 1 < n) aug[(i0 + 1) * n2 + j0 + 1] = sacc[b][3];
    }
  }
  for (int e = tid; e < n * n; e += GF_THREADS) {
    const int i = e / n, j = e % n;
    aug[i * n2 + n + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();

  // ---- Gauss-Jordan with partial pivoting ----
  double2 ld = make_double2(0.0, 0.0);  // meaningful in thread 0
  bool singular = false;
  for (int k = 0; k < n; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < n; i += 64) {
        const double v = cabs2(aug[i * n2 + k]);
        if (v > best) { best = v; bi = i; }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) *sh_piv = bi;
    }
    __syncthreads();
    const int piv = *sh_piv;
    if (piv != k) {
      for (int c = tid; c < n2; c += GF_THREADS) {
        const double2 t = aug[k * n2 + c];
        aug[k * n2 + c] = aug[piv * n2 + c];
        aug[piv * n2 + c] = t;
      }
      if (tid == 0) ld.y += M_PI;
    }
    __syncthreads();
    double2 pv = aug[k * n2 + k];
    if (cabs2(pv) == 0.0) {
      singular = true;
      pv = make_double2(1.0, 0.0);
    }
    if (tid == 0) ld = cadd(ld, clog(pv));
    const double2 ipv = cinv(pv);
    for (int i = tid; i < n; i += GF_THREADS) fac[i] = aug[i * n2 + k];
    __syncthreads();
    for (int c = tid; c < n2; c += GF_THREADS) aug[k * n2 + c] = cmul(aug[k * n2 + c], ipv);
    __syncthreads();
    for (int e = tid; e < n * n2; e += GF_THREADS) {
      const int i = e / n2, c = e % n2;
      if (i != k) aug[e] = csub(aug[e], cmul(fac[i], aug[k * n2 + c]));
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (singular) {
      ld = make_double2(-INFINITY, 0.0);
      atomicOr(status, AFQMC_STATUS_SINGULAR);
    }
    logdet[2 * z + sp] = ld;
  }

  // ---- theta = phi S^-1 and E1 = sum_{j,p} hh[j][p] theta[p][j] ----
  const double* hs = hh + (size_t)sp * d.nmax * N;
  double2 eacc = make_double2(0.0, 0.0);
  const size_t plane = (size_t)d.nmax * d.ldN;
  T* th_re = theta ? theta + ((size_t)(2 * z + 0) * 2 + sp) * plane : nullptr;
  T* th_im = theta ? theta + ((size_t)(2 * z + 1) * 2 + sp) * plane : nullptr;
  load_chunk(0);
  for (int p0 = 0; p0 < N; p0 += GF_CHUNK) {
    const int rows = min(GF_CHUNK, N - p0);
    __syncthreads();
    store_chunk(p0, false);
    load_chunk(p0 + GF_CHUNK);
    __syncthreads();
    // 2 x 2 blocks of outputs (two rows of the chunk, two columns): four LDS
    // reads feed four products; consecutive threads take consecutive row pairs
    const int nbp = (rows + 1) >> 1, nbj = (n + 1) >> 1;
    for (int e = tid; e < nbp * nbj; e += GF_THREADS) {
      const int bj = e / nbp, bp = e - bj * nbp;
      const int j0 = 2 * bj, j1 = min(j0 + 1, n - 1);
      const int q0 = 2 * bp, q1 = min(q0 + 1, rows - 1);
      // the one-body weights of the four outputs, loaded ahead of the products
      double hv[4] = {0.0, 0.0, 0.0, 0.0};
      if (GfBound<NB>::PREFETCH) {
        hv[0] = hs[(size_t)j0 * N + p0 + q0];
        hv[1] = hs[(size_t)j1 * N + p0 + q0];
        hv[2] = hs[(size_t)j0 * N + p0 + q1];
        hv[3] = hs[(size_t)j1 * N + p0 + q1];
      }
      double2 t00 = make_double2(0.0, 0.0), t01 = t00, t10 = t00, t11 = t00;
      if (!singular) {
        for (int k = 0; k < n; ++k) {
          const double2 a0 = ch[q0 * n + k], a1 = ch[q1 * n + k];
          const double2 b0 = aug[k * n2 + n + j0], b1 = aug[k * n2 + n + j1];
          t00 = cadd(t00, cmul(a0, b0));
          t01 = cadd(t01, cmul(a0, b1));
          t10 = cadd(t10, cmul(a1, b0));
          t11 = cadd(t11, cmul(a1, b1));
        }
      }
      const double2 tv[4] = {t00, t01, t10, t11};
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        const int j = j0 + (o & 1), q = q0 + (o >> 1);
        if (j >= n || q >= rows) continue;
        const int p = p0 + q;
        const double2 t = tv[o];
        const double h = GfBound<NB>::PREFETCH ? hv[o] : hs[(size_t)j * N + p];
        eacc.x += h * t.x;
        eacc.y += h * t.y;
        if (theta) {
          th_re[(size_t)j * d.ldN + p] = (T)t.x;
          th_im[(size_t)j * d.ldN + p] = (T)t.y;
        }
      }
    }
  }
  if (e1) {
    const double2 s = block_sum2(eacc, red);
    if (tid == 0) e1[2 * z + sp] = s;
  }
}

template <typename T>
hipError_t launch_gf(const StepDims& d, int W, const double2* phi_a, const double2* phi_b,
                     const double* phiT, const double* hh, T* theta, double2* logdet,
                     double2* e1, int* status, hipStream_t s) {
  const size_t lds = gf_lds_bytes(d.nmax);
  if (d.nmax <= 32)
    hipLaunchKernelGGL((gf_kernel<T, 32>), dim3(W, 2), dim3(GF_THREADS), lds, s, d, phi_a, phi_b, phiT, hh, theta,
                       logdet, e1, status);
  else
    hipLaunchKernelGGL((gf_kernel<T, 45>), dim3(W, 2), dim3(GF_THREADS), lds, s, d, phi_a, phi_b, phiT, hh, theta,
                       logdet, e1, status);
  return hipGetLastError();
}
template hipError_t launch_gf<float>(const StepDims&, int, const double2*, const double2*,
                                     const double*, const double*, float*, double2*, double2*,
                                     int*, hipStream_t);
template hipError_t launch_gf<double>(const StepDims&, int, const double2*, const double2*,
                                      const double*, const double*, double*, double2*, double2*,
                                      int*, hipStream_t);

// ===========================================================================
// Force bias: vbias[z][g] = sum_s sum_{j,p} Lh^s[g][j][p] theta^s_z[p][j] (Eq. rfb)
// A GEMM over all walkers at once with the real Lh as A (rows g) and the
// planar real and imaginary parts of theta as B (rows (z, re|im)), so Lh is
// never converted to complex.
// ===========================================================================

template <typename T>
struct FbProb {
  using vec_t = typename MF<T>::vec_t;
  const T* Lh;
  const T* theta;
  int K, W;
  int plane;  // nmax * ldN
  __device__ vec_t load_a(int, int g, int k) const {
    if (g >= K) return MF<T>::vzero();
    const int s = k >= plane ? 1 : 0;
    const int rest = k - s * plane;
    return *reinterpret_cast<const vec_t*>(Lh + ((size_t)s * K + g) * plane + rest);
  }
  __device__ vec_t load_b(int, int col, int k) const {
    if (col >= 2 * W) return MF<T>::vzero();
    return *reinterpret_cast<const vec_t*>(theta + (size_t)col * 2 * plane + k);
  }
};

template <typename T, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(WM* WN * 64) void fb_kernel(FbProb<T> p, double2* __restrict__ vbias) {
  __shared__ __attribute__((aligned(16))) T lds[TileLds<T, BM, BN, BK>::ELEMS];
  typename MF<T>::acc_t acc[BM / WM / 16][BN / WN / 16];
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  mfma_tile_mainloop<T, BM, BN, BK, WM, WN, false>(p, 0, m0, n0, 2 * p.plane, acc, lds);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / WN, wn = wid % WN;
#pragma unroll
  for (int i = 0; i < BM / WM / 16; ++i)
#pragma unroll
    for (int j = 0; j < BN / WN / 16; ++j) {
      const int mb = m0 + wm * (BM / WM) + i * 16 + 4 * (lane >> 4);
      const int col = n0 + wn * (BN / WN) + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double v = (double)acc[i][j][r];
        const double o = __shfl_xor(v, 1, 64);
        const int g = mb + r;
        if ((col & 1) == 0 && g < p.K && (col >> 1) < p.W)
          vbias[(size_t)(col >> 1) * p.K + g] = make_double2(v, o);
      }
    }
}

template <typename T>
hipError_t launch_force_bias(const StepDims& d, int W, const T* Lh, const T* theta,
                             double2* vbias, hipStream_t s) {
  constexpr int BM = 64, BN = 64, BK = sizeof(T) == 4 ? 32 : 16, WM = 2, WN = 2;
  FbProb<T> p{Lh, theta, d.K, W, d.nmax * d.ldN};
  dim3 grid(ceil_div(d.K, BM), ceil_div(2 * W, BN));
  hipLaunchKernelGGL((fb_kernel<T, BM, BN, BK, WM, WN>), grid, dim3(WM * WN * 64), 0, s, p, vbias);
  return hipGetLastError();
}
template hipError_t launch_force_bias<float>(const StepDims&, int, const float*, const float*,
                                             double2*, hipStream_t);
template hipError_t launch_force_bias<double>(const StepDims&, int, const double*, const double*,
                                              double2*, hipStream_t);

// ===========================================================================
// Shift: xbar = -i sqrt(dt) vbias, xs = x - xbar, a_z = sum_g (x xbar - xbar^2/2)
// (Eq. import and the optimal force bias of Sec. II.B)
// ===========================================================================

// `ctr` (optional, device) selects the step inside a stacked field array:
// x = x_base + ctr[0] * x_step.  A captured graph replays one step many
// times with a counter it advances itself.
template <typename T>
__global__ __launch_bounds__(256) void shift_kernel(int K, int ldK, const double2* __restrict__ vbias,
                                                    const double* __restrict__ x_base,
                                                    const int* __restrict__ ctr, long x_step,
                                                    T* __restrict__ xs, double2* __restrict__ a,
                                                    unsigned* __restrict__ tmax, int tslots,
                                                    int tstride, double sdt, const float* __restrict__ lmax) {
  __shared__ double2 red[4];
  const int z = blockIdx.x;
  const double* x = x_base + (ctr ? (size_t)ctr[0] * x_step : 0);
  double2 acc = make_double2(0.0, 0.0);
  double2 bnd = make_double2(0.0, 0.0);  // sum_g |Re xs_g| m_g, sum_g |Im xs_g| m_g
  for (int g = threadIdx.x; g < K; g += 256) {
    const double2 v = vbias[(size_t)z * K + g];
    const double2 xb = make_double2(sdt * v.y, -sdt * v.x);
    const double xv = x[(size_t)z * K + g];
    const T re = (T)(xv - xb.x), im = (T)(-xb.y);
    xs[(size_t)(2 * z) * ldK + g] = re;
    xs[(size_t)(2 * z + 1) * ldK + g] = im;
    acc.x += xv * xb.x - 0.5 * (xb.x * xb.x - xb.y * xb.y);
    acc.y += xv * xb.y - xb.x * xb.y;
    if (lmax) {
      const double m = lmax[g];
      bnd.x += fabs((double)re) * m;
      bnd.y += fabs((double)im) * m;
    }
  }
  const double2 s = block_sum2(acc, red);
  const double2 b = lmax ? block_sum2(bnd, red) : bnd;
  if (threadIdx.x == 0) {
    a[z] = s;
    for (int t = 0; t < tslots; ++t) tmax[(size_t)t * tstride + z] = 0u;  // running maxima of this step
    // |VHS| bound of the walker (slot 1): both parts of VHS = i sqrt(dt)
    // sum_g xs_g L_g are at most sqrt(dt) sum_g |xs part| max|L_g|; the
    // margin covers the rounding of the FP32 sums of the split build
    if (lmax) tmax[(size_t)tstride + z] = __float_as_uint((float)(sdt * fmax(b.x, b.y) * (1.0 + 0x1p-9)));
  }
}

template <typename T>
hipError_t launch_shift(const StepDims& d, int W, const double2* vbias, const double* x, const int* ctr,
                        long x_step, T* xs, double2* a, unsigned* tmax, int tslots, int tstride, double sdt,
                        const float* lmax, hipStream_t s) {
  hipLaunchKernelGGL(shift_kernel<T>, dim3(W), dim3(256), 0, s, d.K, d.ldK, vbias, x, ctr, x_step, xs,
                     a, tmax, tslots, tstride, sdt, lmax);
  return hipGetLastError();
}
template hipError_t launch_shift<float>(const StepDims&, int, const double2*, const double*,
                                        const int*, long, float*, double2*, unsigned*, int, int, double,
                                        const float*, hipStream_t);
template hipError_t launch_shift<double>(const StepDims&, int, const double2*, const double*,
                                         const int*, long, double*, double2*, unsigned*, int, int,
                                         double, const float*, hipStream_t);

// m_g = max over (p, q) of |L_g[p][q]| (rounded up to FP32), one block per g
__global__ __launch_bounds__(256) void lmax_kernel(int NN, const double* __restrict__ L, float* __restrict__ out) {
  __shared__ double red[4];
  const int g = blockIdx.x;
  double m = 0.0;
  for (int e = threadIdx.x; e < NN; e += 256) m = fmax(m, fabs(L[(size_t)g * NN + e]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    out[g] = (float)(m * (1.0 + 0x1p-20));
  }
}

hipError_t setup_lmax(int K, int N, const double* L, float* lmax, hipStream_t s) {
  hipLaunchKernelGGL(lmax_kernel, dim3(K), dim3(256), 0, s, N * N, L, lmax);
  return hipGetLastError();
}

// ===========================================================================
// VHS build: VHS_z = i sqrt(dt) sum_g xs_zg L_g over the packed (p <= q)
// triangle, mirrored on store (the symmetric L_g make VHS complex symmetric).
// A = xs planar rows (z, re|im); B = packed L rows (p, q), K contiguous.
// ===========================================================================

template <typename T>
struct VhsProb {
  using vec_t = typename MF<T>::vec_t;
  const T* xs;
  const T* LT;
  int W, Npk, ldK;
  __device__ vec_t load_a(int, int m, int k) const {
    if (m >= 2 * W) return MF<T>::vzero();
    return *reinterpret_cast<const vec_t*>(xs + (size_t)m * ldK + k);
  }
  __device__ vec_t load_b(int, int n, int k) const {
    if (n >= Npk) return MF<T>::vzero();
    return *reinterpret_cast<const vec_t*>(LT + (size_t)n * ldK + k);
  }
};

template <typename T, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(WM* WN * 64) void vhs_kernel(VhsProb<T> p, const int2* __restrict__ pq,
                                                          T* __restrict__ vhs, int N, int ldV,
                                                          double sdt) {
  using C2 = typename Cplx<T>::t;
  __shared__ __attribute__((aligned(16))) T lds[TileLds<T, BM, BN, BK>::ELEMS];
  typename MF<T>::acc_t acc[BM / WM / 16][BN / WN / 16];
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  mfma_tile_mainloop<T, BM, BN, BK, WM, WN, false>(p, 0, m0, n0, p.ldK, acc, lds);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / WN, wn = wid % WN;
#pragma unroll
  for (int j = 0; j < BN / WN / 16; ++j) {
    const int col = n0 + wn * (BN / WN) + j * 16 + (lane & 15);
    if (col >= p.Npk) continue;
    const int2 ij = pq[col];
#pragma unroll
    for (int i = 0; i < BM / WM / 16; ++i) {
      const int mb = m0 + wm * (BM / WM) + i * 16 + 4 * (lane >> 4);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int z = (mb >> 1) + h;
        if (z >= p.W) continue;
        const double cr = (double)acc[i][j][2 * h], ci = (double)acc[i][j][2 * h + 1];
        C2 v;
        v.x = (T)(-sdt * ci);
        v.y = (T)(sdt * cr);
        *reinterpret_cast<C2*>(vhs + ((size_t)z * N + ij.x) * ldV + 2 * ij.y) = v;
        if (ij.x != ij.y) *reinterpret_cast<C2*>(vhs + ((size_t)z * N + ij.y) * ldV + 2 * ij.x) = v;
      }
    }
  }
}

template <typename T>
hipError_t launch_vhs(const StepDims& d, int W, const T* xs, const T* LT, const int2* pq, T* vhs,
                      double sdt, hipStream_t s) {
  constexpr int BM = 64, BN = 64, BK = sizeof(T) == 4 ? 32 : 16, WM = 2, WN = 2;
  VhsProb<T> p{xs, LT, W, d.Npk, d.ldK};
  dim3 grid(ceil_div(2 * W, BM), ceil_div(d.Npk, BN));
  hipLaunchKernelGGL((vhs_kernel<T, BM, BN, BK, WM, WN>), grid, dim3(WM * WN * 64), 0, s, p, pq,
                     vhs, d.N, d.ldV, sdt);
  return hipGetLastError();
}
template hipError_t launch_vhs<float>(const StepDims&, int, const float*, const float*, const int2*,
                                      float*, double, hipStream_t);
template hipError_t launch_vhs<double>(const StepDims&, int, const double*, const double*,
                                       const int2*, double*, double, hipStream_t);

// ===========================================================================
// One-body half step of the propagator B(x) of Eq. Bx, split symmetrically
// (P = exp(-dt (h' - mu) / 2) on each side of exp(VHS); the paper leaves the
// factorisation open):
// out_z = P in_z for every walker, both spins side by side as real columns.
// ===========================================================================

#ifndef PPHI_BM
#define PPHI_BM 64
#endif
#ifndef PPHI_BN
#define PPHI_BN 64
#endif
// k depth and pipelining per type (measured at n290, 512 walkers: FP32 one
// LDS stage of 64 k, 0.25 ms per half step; FP64 two stages of 16 k, 0.30 ms)
#ifndef PPHI_BK
#define PPHI_BK 16
#endif
#ifndef PPHI_BK_F32
#define PPHI_BK_F32 64
#endif
#ifndef PPHI_PIPE
#define PPHI_PIPE 2
#endif
#ifndef PPHI_PIPE_F32
#define PPHI_PIPE_F32 1
#endif

// The FP64 path multiplies on the FP64 matrix cores.  The FP32 and split
// paths, whose VHS and Taylor products already round to single precision,
// multiply on the FP32 matrix cores (twice the FP64 rate): operands are
// rounded to FP32 on the way into LDS, the products accumulate in FP32, and
// the result is stored back in FP64.
template <typename T>
struct PphiProb {
  using vec_t = typename MF<T>::vec_t;
  const double* P;
  int N, ldP, ncolp, na, nb;
  const double* in_a;  // mode 0
  const double* in_b;
  const double* acc;   // mode 1
  int mode;
  // two consecutive real columns (col even) of row q of walker z's operand
  __device__ double2 pair(int z, int q, int col) const {
    if (mode == 1) return *reinterpret_cast<const double2*>(acc + ((size_t)z * N + q) * ncolp + col);
    if (col < 2 * na) return *reinterpret_cast<const double2*>(in_a + ((size_t)z * N + q) * 2 * na + col);
    const int c = col - 2 * na;
    if (c >= 2 * nb) return make_double2(0.0, 0.0);
    return *reinterpret_cast<const double2*>(in_b + ((size_t)z * N + q) * 2 * nb + c);
  }
  // rows of P are zero-padded to ldP (a multiple of 16), so a vector that
  // starts below N stays inside its row
  __device__ vec_t load_a(int, int r, int k) const {
    if (r >= N) return MF<T>::vzero();
    const double2* src = reinterpret_cast<const double2*>(P + (size_t)r * ldP + k);
    if constexpr (sizeof(T) == 8) {
      return src[0];
    } else {
      const double2 u = src[0], v = src[1];
      return make_float4((float)u.x, (float)u.y, (float)v.x, (float)v.y);
    }
  }
  // ncolp is a multiple of 4 and 2 na is even, so each pair lies in one operand
  __device__ vec_t load_b_km(int z, int q, int col) const {
    if (q >= N || col >= ncolp) return MF<T>::vzero();
    if constexpr (sizeof(T) == 8) {
      return pair(z, q, col);
    } else {
      const double2 u = pair(z, q, col), v = pair(z, q, col + 2);
      return make_float4((float)u.x, (float)u.y, (float)v.x, (float)v.y);
    }
  }
};

// 1-D grid in XCD order: workgroups go to the 8 XCDs in turn (XCD = id mod 8)
// and the ntile tiles of a walker get ids of one residue, row tile fastest, so
// the row tiles that share a walker's column tile run together on one XCD and
// read it once into that XCD's L2.
template <typename T, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(WM* WN * 64) void pphi_kernel(PphiProb<T> p, int W, int mt, int ntile,
                                                           double* __restrict__ acc_out,
                                                           double2* __restrict__ out_a,
                                                           double2* __restrict__ out_b,
                                                           unsigned* __restrict__ tmax) {
  constexpr int PIPE = sizeof(T) == 4 ? PPHI_PIPE_F32 : PPHI_PIPE;
  __shared__ __attribute__((aligned(16))) T lds[(PIPE == 2 ? 2 : 1) * TileLds<T, BM, BN, BK>::ELEMS];
  typename MF<T>::acc_t acc[BM / WM / 16][BN / WN / 16];
  const int L = blockIdx.x;
  const int r8 = L >> 3, t = r8 % ntile;
  const int z = (L & 7) + 8 * (r8 / ntile);
  if (z >= W) return;  // whole workgroup, before any barrier
  const int m0 = (t % mt) * BM, n0 = (t / mt) * BN;
  mfma_tile_mainloop<T, BM, BN, BK, WM, WN, true, PphiProb<T>, PIPE>(p, z, m0, n0, p.N, acc, lds);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / WN, wn = wid % WN;
  const int ncol = 2 * (p.na + p.nb);
  float vmax = 0.f;
#pragma unroll
  for (int i = 0; i < BM / WM / 16; ++i)
#pragma unroll
    for (int j = 0; j < BN / WN / 16; ++j) {
      const int mb = m0 + wm * (BM / WM) + i * 16 + 4 * (lane >> 4);
      const int col = n0 + wn * (BN / WN) + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mb + r;
        if (row >= p.N || col >= ncol) continue;
        const double v = acc[i][j][r];
        if (p.mode == 0) {
          acc_out[((size_t)z * p.N + row) * p.ncolp + col] = v;
          vmax = fmaxf(vmax, (float)fabs(v));
        } else {
          double* dst;
          if (col < 2 * p.na)
            dst = reinterpret_cast<double*>(out_a) + ((size_t)z * p.N + row) * 2 * p.na + col;
          else
            dst = reinterpret_cast<double*>(out_b) + ((size_t)z * p.N + row) * 2 * p.nb + (col - 2 * p.na);
          *dst = v;
        }
      }
    }
  if (p.mode == 0 && tmax) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o, 64));
    if (lane == 0) atomicMax(tmax + z, __float_as_uint(vmax));
  }
}

template <typename T>
hipError_t launch_pphi(const StepDims& d, int W, const double* P, const double2* phi_a_in,
                       const double2* phi_b_in, double* acc, double2* phi_a_out,
                       double2* phi_b_out, unsigned* tmax, int mode, hipStream_t s) {
  PphiProb<T> p{P, d.N, d.ldP, d.ncolp, d.na, d.nb,
                reinterpret_cast<const double*>(phi_a_in), reinterpret_cast<const double*>(phi_b_in),
                acc, mode};
  // 64 x 64 tiles: many small workgroups per walker (larger tiles lower the occupancy)
  constexpr int BK = sizeof(T) == 4 ? PPHI_BK_F32 : PPHI_BK, WM = 2, WN = 2;
  constexpr int BM = PPHI_BM, BN = PPHI_BN;
  const int mt = ceil_div(d.N, BM), ntile = mt * ceil_div(d.ncolp, BN);
  const long nblk = (long)ntile * ceil_div(W, 8) * 8;
  hipLaunchKernelGGL((pphi_kernel<T, BM, BN, BK, WM, WN>), dim3((unsigned)nblk), dim3(WM * WN * 64), 0, s,
                     p, W, mt, ntile, acc, phi_a_out, phi_b_out, tmax);
  return hipGetLastError();
}
template hipError_t launch_pphi<float>(const StepDims&, int, const double*, const double2*,
                                       const double2*, double*, double2*, double2*, unsigned*, int,
                                       hipStream_t);
template hipError_t launch_pphi<double>(const StepDims&, int, const double*, const double2*,
                                        const double2*, double*, double2*, double2*, unsigned*, int,
                                        hipStream_t);

// ===========================================================================
// Taylor term: t_k = VHS t_{k-1} / k, acc += t_k (exp(VHS) of Eq. Bx
// truncated after the 6th-order term).
// Complex product as a real GEMM: A = VHS rows with interleaved (re, im)
// along the contraction, B rows (q, re|im) built on the fly from t:
//   row (q, re) = t[q][:]              (tr, ti pairs)
//   row (q, im) = t[q][:] with each pair (tr, ti) -> (-ti, tr)
// so that C[p][(j, re)] = sum Vr tr - Vi ti and C[p][(j, im)] = sum Vr ti + Vi tr.
// In the mixed path t is FP32 with a per-walker power-of-two scale taken
// from max |P phi| (exact; the FP64 accumulator holds unscaled values).
// ===========================================================================

template <typename T>
__device__ __forceinline__ double taylor_scale_exp(const unsigned* tmax, int z) {
  if constexpr (sizeof(T) == 8) {
    return 0.0;
  } else {
    const float m = __uint_as_float(tmax[z]);
    return (m > 0.f && isfinite(m)) ? (double)ilogbf(m) : 0.0;
  }
}

template <typename T>
struct TaylorProb {
  using vec_t = typename MF<T>::vec_t;
  const T* vhs;
  int N, ldV, ncolp;
  const double* acc;  // first term: FP64 source
  const T* t_in;
  const unsigned* tmax;
  int first;
  __device__ vec_t load_a(int z, int r, int k) const {
    if (r >= N) return MF<T>::vzero();
    return *reinterpret_cast<const vec_t*>(vhs + ((size_t)z * N + r) * ldV + k);
  }
  __device__ vec_t load_b_km(int z, int k, int col) const {
    const int q = k >> 1, c = k & 1;
    if (q >= N || col >= ncolp) return MF<T>::vzero();
    vec_t v;
    if (first) {
      const double sc = ldexp(1.0, -(int)taylor_scale_exp<T>(tmax, z));
      const double* src = acc + ((size_t)z * N + q) * ncolp + col;
      if constexpr (MF<T>::VEC == 4) {
        const double2 x0 = *reinterpret_cast<const double2*>(src);
        const double2 x1 = *reinterpret_cast<const double2*>(src + 2);
        v = make_float4((float)(x0.x * sc), (float)(x0.y * sc), (float)(x1.x * sc), (float)(x1.y * sc));
      } else {
        v = *reinterpret_cast<const double2*>(src);
      }
    } else {
      v = *reinterpret_cast<const vec_t*>(t_in + ((size_t)z * N + q) * ncolp + col);
    }
    if (c) {
      if constexpr (MF<T>::VEC == 4) {
        v = make_float4(-v.y, v.x, -v.w, v.z);
      } else {
        v = make_double2(-v.y, v.x);
      }
    }
    return v;
  }
};

template <typename T, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(WM* WN * 64) void taylor_kernel(TaylorProb<T> p, T* __restrict__ t_out,
                                                             double* __restrict__ acc_out, int ncol,
                                                             double inv_k, int add_prev,
                                                             int add_this) {
  __shared__ __attribute__((aligned(16))) T lds[TileLds<T, BM, BN, BK>::ELEMS];
  typename MF<T>::acc_t acc[BM / WM / 16][BN / WN / 16];
  const int z = blockIdx.z;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  mfma_tile_mainloop<T, BM, BN, BK, WM, WN, true>(p, z, m0, n0, p.ldV, acc, lds);
  const double unscale = ldexp(1.0, (int)taylor_scale_exp<T>(p.tmax, z));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / WN, wn = wid % WN;
#pragma unroll
  for (int i = 0; i < BM / WM / 16; ++i)
#pragma unroll
    for (int j = 0; j < BN / WN / 16; ++j) {
      const int mb = m0 + wm * (BM / WM) + i * 16 + 4 * (lane >> 4);
      const int col = n0 + wn * (BN / WN) + j * 16 + (lane & 15);
      if (col >= ncol) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mb + r;
        if (row >= p.N) continue;
        const double v = (double)acc[i][j][r] * inv_k;
        const size_t o = ((size_t)z * p.N + row) * p.ncolp + col;
        const T tv = (T)v;
        // The first term reads the accumulator as its operand, so no launch
        // writes the accumulator while reading it: launch k adds term k-1,
        // and the last launch also adds its own term.
        double add = 0.0;
        if (add_prev) add += (double)p.t_in[o];
        if (add_this) add += (double)tv;
        if (add_prev | add_this) acc_out[o] += add * unscale;
        t_out[o] = tv;
      }
    }
}

template <typename T>
__global__ void taylor_last_kernel(int W, int N, int ncolp, int ncol, const T* __restrict__ t,
                                   double* __restrict__ acc, const unsigned* __restrict__ tmax) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per = (size_t)N * ncolp;
  if (e >= per * W) return;
  const int z = (int)(e / per);
  if ((int)(e % ncolp) >= ncol) return;
  acc[e] += (double)t[e] * ldexp(1.0, (int)taylor_scale_exp<T>(tmax, z));
}

template <typename T>
hipError_t launch_taylor(const StepDims& d, int W, const T* vhs, const T* t_in, T* t_out,
                         double* acc, const unsigned* tmax, int k, int order, hipStream_t s) {
  constexpr int BK = sizeof(T) == 4 ? 32 : 16;
  TaylorProb<T> p{vhs, d.N, d.ldV, d.ncolp, acc, t_in, tmax, k == 1 ? 1 : 0};
  const int add_prev = k >= 2 ? 1 : 0;
  const int add_this = (k == order && k >= 2) ? 1 : 0;
  constexpr int BM = 64, BN = 64, WM = 2, WN = 2;
  dim3 grid(ceil_div(d.N, BM), ceil_div(d.ncolp, BN), W);
  hipLaunchKernelGGL((taylor_kernel<T, BM, BN, BK, WM, WN>), grid, dim3(WM * WN * 64), 0, s, p,
                     t_out, acc, d.ncol, 1.0 / k, add_prev, add_this);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !(k == order && k == 1)) return e;
  const size_t tot = (size_t)W * d.N * d.ncolp;
  hipLaunchKernelGGL(taylor_last_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     W, d.N, d.ncolp, d.ncol, t_out, acc, tmax);
  return hipGetLastError();
}
template hipError_t launch_taylor<float>(const StepDims&, int, const float*, const float*, float*,
                                         double*, const unsigned*, int, int, hipStream_t);
template hipError_t launch_taylor<double>(const StepDims&, int, const double*, const double*,
                                          double*, double*, const unsigned*, int, int, hipStream_t);

// ===========================================================================
// Weights (Eqs. import, ovl, ph, theta):
//   ln O_z = log<Psi_T|phi'> - log<Psi_T|phi>, theta_z = Im ln O_z,
//   log w += Re ln O_z + Re a_z + cst + ln max(0, cos theta_z)
// ===========================================================================

__global__ void weight_kernel(int W, const double2* __restrict__ logdet, const double* __restrict__ corr,
                              const double2* __restrict__ a, double2* __restrict__ log_ovlp,
                              double* __restrict__ log_w, double cst, int* __restrict__ status) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= W) return;
  const double2 l0 = logdet[2 * z], l1 = logdet[2 * z + 1];
  const double2 ld = cadd(l0, l1);
  const double c = corr ? corr[2 * z] + corr[2 * z + 1] : 0.0;
  const double2 lo = log_ovlp[z];
  const double lnr = ld.x + c - lo.x;
  const double lni = ld.y - lo.y;
  const double ct = cos(lni);
  const double lw0 = log_w[z];
  double lw;
  if (lw0 == -INFINITY || ld.x == -INFINITY || !(ct > 0.0)) {
    lw = -INFINITY;
  } else {
    lw = lw0 + lnr + a[z].x + cst + log(ct);
  }
  if (isnan(lw) || isnan(ld.x) || isnan(ld.y)) {
    atomicOr(status, AFQMC_STATUS_NONFINITE);
    lw = -INFINITY;
  }
  log_ovlp[z] = ld;
  log_w[z] = lw;
}

hipError_t launch_weight(int W, const double2* logdet, const double* corr, const double2* a,
                         double2* log_ovlp, double* log_w, double cst, int* status, hipStream_t s) {
  hipLaunchKernelGGL(weight_kernel, dim3(ceil_div(W, 256)), dim3(256), 0, s, W, logdet, corr, a,
                     log_ovlp, log_w, cst, status);
  return hipGetLastError();
}

__global__ void overlap_store_kernel(int W, const double2* __restrict__ logdet, double2* __restrict__ log_ovlp) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z < W) log_ovlp[z] = cadd(logdet[2 * z], logdet[2 * z + 1]);
}

hipError_t launch_overlap_store(int W, const double2* logdet, double2* log_ovlp, hipStream_t s) {
  hipLaunchKernelGGL(overlap_store_kernel, dim3(ceil_div(W, 256)), dim3(256), 0, s, W, logdet, log_ovlp);
  return hipGetLastError();
}

// ===========================================================================
// Exchange energy (Sec. III.C): E_K = -1/2 sum_s sum_g sum_ij T_ij T_ji,
// T^{s}_{z g} = Lh^s_g theta^s_z (n x n), formed tile by tile on MFMA and
// consumed in LDS without ever reaching HBM.  A workgroup owns G whole
// Cholesky blocks (rows (g, i)) and Z whole walkers (columns (z, re|im, j)),
// so every T_ij meets its partner T_ji inside the tile.  Per-tile partial
// sums go to part[s][g-tile][z] and are reduced in a fixed order later.
// ===========================================================================

template <typename T>
struct ExProb {
  using vec_t = typename MF<T>::vec_t;
  const T* Lh;      // spin block [K][nmax][ldN]
  const T* theta;
  int K, W, n, nmax, ldN, sp, G, Z;
  int gt, wt;       // this workgroup's Cholesky tile and walker tile
  __device__ vec_t load_a(int, int r, int k) const {
    if (r >= G * n) return MF<T>::vzero();
    const int g = gt * G + r / n;
    if (g >= K) return MF<T>::vzero();
    return *reinterpret_cast<const vec_t*>(Lh + ((size_t)g * nmax + r % n) * ldN + k);
  }
  __device__ vec_t load_b(int, int c, int k) const {
    const int n2 = 2 * n;
    if (c >= Z * n2) return MF<T>::vzero();
    const int z = wt * Z + c / n2;
    if (z >= W) return MF<T>::vzero();
    const int cc = c % n2;
    const int comp = cc >= n ? 1 : 0;
    const int j = cc - comp * n;
    return *reinterpret_cast<const vec_t*>(
        theta + (((size_t)z * 2 + comp) * 2 + sp) * (size_t)nmax * ldN + (size_t)j * ldN + k);
  }
};

// Tile shapes.  GS = Cholesky tiles per L2 group in the XCD-aware order (the
// A tiles of one group plus the walker tiles in flight fit one XCD's 4 MB L2).
template <typename T> struct ExCfg;
// FP32: 4-wave workgroups, single-buffered LDS under 80 KB and at most 256
// registers per wave, so two independent workgroups share a CU (their
// barriers do not line up, one computes while the other waits on memory).
// FP64: the 8-byte accumulators need 8 waves; one double-buffered workgroup per CU.
template <> struct ExCfg<float> {
  static constexpr int BM = 192, BN = 160, BK = 32, WM = 2, WN = 2, GS = 8;
  static constexpr int PIPE = 0;
  static constexpr bool DBUF = false;
  static constexpr int WAVES_PER_EU = 2;
  static constexpr size_t EPI_BUDGET = 72 * 1024;
};
template <> struct ExCfg<double> {
  static constexpr int BM = 192, BN = 160, BK = 16, WM = 4, WN = 2, GS = 4;
  static constexpr int PIPE = 2;
  static constexpr bool DBUF = true;
  static constexpr int WAVES_PER_EU = 2;
  static constexpr size_t EPI_BUDGET = 150 * 1024;
};

// Walkers whose T blocks go through LDS together in one epilogue pass.
template <typename T>
static int ex_walkers_per_pass(int G, int Z, int n) {
  const size_t per = (size_t)G * n * (2 * n + 1) * sizeof(T);
  int zp = (int)(ExCfg<T>::EPI_BUDGET / per);
  const int slots = 64 / (ExCfg<T>::WM * ExCfg<T>::WN);  // cross-wave reduction slots
  if (zp > slots) zp = slots;
  if (zp < 1) zp = 1;
  return zp < Z ? zp : Z;
}

// LDS: max(operand staging, T blocks of one epilogue pass), then the
// epilogue tables and the reduction slots.
template <typename T>
static size_t ex_tab_off(int G, int Z, int n) {
  using C = ExCfg<T>;
  const size_t stage = (C::DBUF ? 2 : 1) * (size_t)TileLds<T, C::BM, C::BN, C::BK>::BYTES;
  const size_t epi = (size_t)ex_walkers_per_pass<T>(G, Z, n) * G * n * (2 * n + 1) * sizeof(T);
  return (stage > epi ? stage : epi + 15) / 16 * 16;
}
template <typename T>
static size_t ex_lds_bytes(int G, int Z, int n) {
  return ex_tab_off<T>(G, Z, n) + EX_TAB_BYTES + EX_RED_BYTES;
}

template <typename T>
__global__ __launch_bounds__(ExCfg<T>::WM* ExCfg<T>::WN * 64, ExCfg<T>::WAVES_PER_EU) void exchange_kernel(
    ExProb<T> p0, double2* __restrict__ part, int ntg, int nwt, int tab_off, int zpp, int gs) {
  using C = ExCfg<T>;
  constexpr int BM = C::BM, BN = C::BN, BK = C::BK, WM = C::WM, WN = C::WN;
  ExProb<T> p = p0;
  if (!xcd_tile(blockIdx.x, ntg, nwt, gs, p.gt, p.wt)) return;
  extern __shared__ double2 ex_lds_raw[];
  T* lds = reinterpret_cast<T*>(ex_lds_raw);
  typename MF<T>::acc_t acc[BM / WM / 16][BN / WN / 16];
  mfma_tile_mainloop<T, BM, BN, BK, WM, WN, false, ExProb<T>, C::PIPE>(p, 0, 0, 0, p.ldN, acc, lds);
  const ExTileGeom q{p.n, p.G, p.Z, p.K, p.W, p.gt, p.wt};
  auto one3 = [](int, int, int) { return 1.0f; };
  auto one2 = [](int, int) { return 1.0f; };
  exchange_epilogue<T, typename MF<T>::acc_t, BM, BN, WM, WN>(
      acc, reinterpret_cast<char*>(ex_lds_raw), tab_off, tab_off + EX_TAB_BYTES, q, zpp, false, one2,
      one3, part, p.sp, ntg);
}

template <typename T>
ExTile exchange_tile(int n) {
  using C = ExCfg<T>;
  ExTile t;
  t.G = n > 0 ? C::BM / n : 0;
  t.Z = n > 0 ? C::BN / (2 * n) : 0;
  return t;
}
template ExTile exchange_tile<float>(int);
template ExTile exchange_tile<double>(int);

template <typename T>
hipError_t launch_exchange(const StepDims& d, int W, const T* Lh, const T* theta, double2* part,
                           int sp, int* ntg_out, hipStream_t s, int gs) {
  using C = ExCfg<T>;
  const ExTile t = exchange_tile<T>(d.nmax);
  if (t.G < 1 || t.Z < 1) return hipErrorInvalidValue;
  const int ntg = ceil_div(d.K, t.G);
  const int nwt = ceil_div(W, t.Z);
  *ntg_out = ntg;
  const int n = sp == 0 ? d.na : d.nb;
  if (n == 0) return hipSuccess;
  // A spin with fewer electrons reuses the tile shape of the larger one.
  ExProb<T> p{Lh + (size_t)sp * d.K * d.nmax * d.ldN, theta, d.K, W, n, d.nmax, d.ldN, sp, t.G, t.Z,
              0, 0};
  const size_t lds = ex_lds_bytes<T>(t.G, t.Z, n);
  const int tab_off = (int)ex_tab_off<T>(t.G, t.Z, n);
  const int zpp = ex_walkers_per_pass<T>(t.G, t.Z, n);
  if (zpp * (C::WM * C::WN) > 64) return hipErrorInvalidValue;  // reduction slots
  const int per = ceil_div(ntg * nwt, 8);
  if (gs < 1) gs = C::GS;
  hipLaunchKernelGGL(exchange_kernel<T>, dim3(8 * per), dim3(C::WM * C::WN * 64), lds, s, p, part,
                     ntg, nwt, tab_off, zpp, gs);
  return hipGetLastError();
}
template hipError_t launch_exchange<float>(const StepDims&, int, const float*, const float*,
                                           double2*, int, int*, hipStream_t, int);
template hipError_t launch_exchange<double>(const StepDims&, int, const double*, const double*,
                                            double2*, int, int*, hipStream_t, int);

// ===========================================================================
// Exchange through pair integrals (exchange_pair.h), FP32 / FP64 matrix
// cores: row tile rt of group i, A = pair-integral rows (j, p) of group i
// ([rows][ldN], working precision), B = theta rows (z, re|im, spin, i) of
// the tile's 80 walkers.  Tile shapes and XCD order as the direct exchange.
// ===========================================================================

template <typename T>
struct PairProb {
  using vec_t = typename MF<T>::vec_t;
  const T* V;      // this tile's first pair-integral row
  const T* theta;
  int W, nmax, ldN, sp, i, nr, z0;
  __device__ vec_t load_a(int, int r, int k) const {
    if (r >= nr) return MF<T>::vzero();
    return *reinterpret_cast<const vec_t*>(V + (size_t)r * ldN + k);
  }
  __device__ vec_t load_b(int, int c, int k) const {
    const int z = z0 + (c >> 1);
    if (z >= W) return MF<T>::vzero();
    return *reinterpret_cast<const vec_t*>(theta + (((size_t)z * 2 + (c & 1)) * 2 + sp) * (size_t)nmax * ldN +
                                           (size_t)i * ldN + k);
  }
};

template <typename T>
static size_t pair_lds_bytes() {
  using C = ExCfg<T>;
  const size_t stage = (C::DBUF ? 2 : 1) * (size_t)TileLds<T, C::BM, C::BN, C::BK>::BYTES;
  const size_t red = (size_t)4 * C::WM * C::BN * sizeof(double2);
  return stage > red ? stage : red;
}

template <typename T>
__global__ __launch_bounds__(ExCfg<T>::WM* ExCfg<T>::WN * 64, ExCfg<T>::WAVES_PER_EU) void exchange_pair_kernel(
    const T* __restrict__ V, const T* __restrict__ theta, const PairTab* __restrict__ tab, int n, int Np, int W,
    int nmax, int ldN, int sp, int ntiles, double2* __restrict__ part, int ntg, int nwt, int gs) {
  using C = ExCfg<T>;
  constexpr int BM = C::BM, BN = C::BN, BK = C::BK, WM = C::WM, WN = C::WN;
  int rt, wt;
  if (!xcd_tile(blockIdx.x, ntg, nwt, gs, rt, wt)) return;
  const int z0 = wt * (BN / 2);
  double2* out = part + ((size_t)sp * ntg + rt) * W;
  if (rt >= ntiles) {
    exchange_pair_zero<BN>(z0, W, out);
    return;
  }
  extern __shared__ double2 ex_lds_raw[];
  const int i = pair_group(tab, n, rt);
  const int lr0 = (rt - tab->start[i]) * BM;
  const int R = (n - i) * Np;
  const int vb = tab->vbase[i];
  const PairProb<T> p{V + (size_t)(vb + lr0) * ldN, theta, W, nmax, ldN, sp, i, min(BM, R - lr0), z0};
  typename MF<T>::acc_t acc[BM / WM / 16][BN / WN / 16];
  mfma_tile_mainloop<T, BM, BN, BK, WM, WN, false, PairProb<T>, C::PIPE>(p, 0, 0, 0, ldN, acc,
                                                                         reinterpret_cast<T*>(ex_lds_raw));
  exchange_pair_epilogue<BM, BN, WM, WN, false>(acc, reinterpret_cast<char*>(ex_lds_raw), i, lr0, R, Np, vb, z0,
                                                W, sp, nmax, ldN, theta, nullptr, nullptr, out);
}

template <typename T>
int exchange_pair_rows() {
  return ExCfg<T>::BM;
}
template int exchange_pair_rows<float>();
template int exchange_pair_rows<double>();

template <typename T>
hipError_t launch_exchange_pair(const StepDims& d, int W, const PairLaunch& pl, const T* v, const T* theta,
                                double2* part, int sp, hipStream_t s, int gs) {
  using C = ExCfg<T>;
  const int n = sp == 0 ? d.na : d.nb;
  if (W == 0 || pl.ntg == 0) return hipSuccess;
  if (n > PAIR_MAX_N) return hipErrorInvalidValue;
  const int nwt = ceil_div(2 * W, C::BN);
  const int per = ceil_div(pl.ntg * nwt, 8);
  if (gs < 1) gs = C::GS;
  hipLaunchKernelGGL(exchange_pair_kernel<T>, dim3(8 * per), dim3(C::WM * C::WN * 64), pair_lds_bytes<T>(), s,
                     v + (size_t)pl.vrow0 * d.ldN, theta, pl.tab, n, (d.N + 3) & ~3, W, d.nmax, d.ldN, sp,
                     n > 0 ? pl.ntiles : 0, part, pl.ntg, nwt, gs);
  return hipGetLastError();
}
template hipError_t launch_exchange_pair<float>(const StepDims&, int, const PairLaunch&, const float*, const float*,
                                                double2*, int, hipStream_t, int);
template hipError_t launch_exchange_pair<double>(const StepDims&, int, const PairLaunch&, const double*,
                                                 const double*, double2*, int, hipStream_t, int);

// ===========================================================================
// Energy assembly (Sec. III.C): E1 from the Green's function pass,
// EJ = 1/2 sum_g vbias_g^2, EK = -1/2 sum of the exchange partials.
// ===========================================================================

__global__ __launch_bounds__(256) void energy_kernel(int W, int K, int ntg, int nb_zero,
                                                     const double2* __restrict__ e1,
                                                     const double2* __restrict__ vbias,
                                                     const double2* __restrict__ part,
                                                     double2* __restrict__ e_base,
                                                     const int* __restrict__ ctr, long e_step) {
  __shared__ double2 red[4];
  // Workgroups go round the 8 XCDs in turn; the exchange partials of 8
  // neighbouring walkers share cache lines, so when the walker count is a
  // multiple of 8 each XCD takes a contiguous range of walkers (one L2 fetch
  // per line instead of one per XCD).
  const int nb = gridDim.x;
  const int z = (nb & 7) == 0 ? (int)(blockIdx.x & 7) * (nb >> 3) + (int)(blockIdx.x >> 3) : (int)blockIdx.x;
  double2* e_out = e_base + (ctr ? (size_t)ctr[0] * e_step : 0);
  // batches of EJ_BATCH loads in flight per thread; each thread still adds
  // its terms in increasing g
  constexpr int EJ_BATCH = 8;
  double2 ej = make_double2(0.0, 0.0);
  for (int g0 = threadIdx.x; g0 < K; g0 += 256 * EJ_BATCH) {
    double2 v[EJ_BATCH];
#pragma unroll
    for (int u = 0; u < EJ_BATCH; ++u) {
      const int g = g0 + 256 * u;
      v[u] = g < K ? vbias[(size_t)z * K + g] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < EJ_BATCH; ++u)
      if (g0 + 256 * u < K) ej = cadd(ej, cmul(v[u], v[u]));
  }
  ej = block_sum2(ej, red);
  double2 ek = make_double2(0.0, 0.0);
  const int nsp = nb_zero ? 1 : 2;
  // the partials of (spin, tile group) e sit at row e (sp ntg + t = e)
  for (int e0 = threadIdx.x; e0 < nsp * ntg; e0 += 256 * EJ_BATCH) {
    double2 v[EJ_BATCH];
#pragma unroll
    for (int u = 0; u < EJ_BATCH; ++u) {
      const int e = e0 + 256 * u;
      v[u] = e < nsp * ntg ? part[(size_t)e * W + z] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < EJ_BATCH; ++u)
      if (e0 + 256 * u < nsp * ntg) ek = cadd(ek, v[u]);
  }
  ek = block_sum2(ek, red);
  if (threadIdx.x == 0) {
    e_out[3 * z + 0] = cadd(e1[2 * z], e1[2 * z + 1]);
    e_out[3 * z + 1] = cscale(ej, 0.5);
    e_out[3 * z + 2] = cscale(ek, -0.5);
  }
}

hipError_t launch_energy(const StepDims& d, int W, const double2* e1, const double2* vbias,
                         const double2* part, int ntg, double2* e_out, const int* ctr, long e_step,
                         hipStream_t s) {
  hipLaunchKernelGGL(energy_kernel, dim3(W), dim3(256), 0, s, W, d.K, ntg, d.nb == 0 ? 1 : 0, e1,
                     vbias, part, e_out, ctr, e_step);
  return hipGetLastError();
}

__global__ void counter_advance_kernel(int* ctr) {
  if (threadIdx.x == 0) ctr[0] += 1;
}
__global__ void counter_set_kernel(int* ctr, int v) {
  if (threadIdx.x == 0) ctr[0] = v;
}
hipError_t launch_counter_advance(int* ctr, hipStream_t s) {
  hipLaunchKernelGGL(counter_advance_kernel, dim3(1), dim3(64), 0, s, ctr);
  return hipGetLastError();
}
hipError_t launch_counter_set(int* ctr, int v, hipStream_t s) {
  hipLaunchKernelGGL(counter_set_kernel, dim3(1), dim3(64), 0, s, ctr, v);
  return hipGetLastError();
}

// ===========================================================================
// Re-orthogonalisation of the walkers: phi = Q R with R upper triangular and
// a positive real diagonal (the unique such factorisation; Householder QR
// followed by the phases D = diag(R_ii / |R_ii|) gives the same Q and R),
// corr = sum ln R_ii.  Computed as Cholesky QR applied twice: S = A^H A,
// S = R^H R, A <- A R^{-1}; the second pass restores orthogonality to FP64
// rounding for any condition number below ~1e8, and R = R2 R1.  One
// workgroup per (walker, spin) holds the N x n block in LDS, column-major.
//   Gram: the real Gram matrix X^T X of X = [Re a_0, Im a_0, Re a_1, ...]
//     (N x 2n) on the FP64 matrix cores, one wave per 16 x 16 block of its
//     upper triangle; S_ij = G[2i][2j] + G[2i+1][2j+1]
//     + i (G[2i][2j+1] - G[2i+1][2j]) assembled across lanes.
//   Cholesky: every thread keeps up to QR_NPT entries (i <= j) of S in
//     registers; step k publishes row k (final once the previous steps are
//     applied) to LDS, and after one barrier every entry below it is reduced,
//     S_ij -= conj(S_ki) S_kj / S_kk; the square roots come at the end,
//     R_ij = S_ij / sqrt(S_ii).
//   A <- A R^{-1}: forward substitution, one row of A per thread held in
//     registers (the column count is a template bound), R read from LDS as
//     broadcasts.
// ===========================================================================

constexpr int QR_THREADS = 512;

// LDS column stride: N rounded up to 1 mod 8 complex doubles, so that one row
// of different columns spreads over the LDS banks
static __host__ __device__ inline int qr_col_stride(int N) { return N + ((9 - N % 8) % 8); }

// R rows are read QR_BPAD entries past the last row by the unrolled
// substitution (values unused): padding behind the n x n block
constexpr int QR_BPAD = 48;

// walker loads per thread issued together (one wait per batch)
constexpr int QR_LD_BATCH = 8;

size_t qr_lds_bytes_for(int N, int n) {
  return (size_t)n * qr_col_stride(N) * sizeof(double2) + ((size_t)n * n + QR_BPAD) * sizeof(double2) +
         n * sizeof(double) + 64;
}
size_t qr_lds_bytes(const StepDims& d) { return qr_lds_bytes_for(d.N, d.nmax); }

template <int NMAX>
__global__ __launch_bounds__(QR_THREADS) void qr_kernel(StepDims d, double2* __restrict__ phi_a,
                                                        double2* __restrict__ phi_b,
                                                        double* __restrict__ corr,
                                                        int* __restrict__ status) {
  extern __shared__ double2 qr_lds[];
  constexpr int NWAVE = QR_THREADS / 64;
  constexpr int NPT = (NMAX * (NMAX + 1) / 2 + QR_THREADS - 1) / QR_THREADS;
  const int z = blockIdx.x, sp = blockIdx.y;
  const int n = sp == 0 ? d.na : d.nb;
  const int N = d.N, Np = qr_col_stride(N);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (n == 0) {
    if (tid == 0) corr[2 * z + sp] = 0.0;
    return;
  }
  double2* A = qr_lds;                                  // A[j * Np + p]
  double2* B = A + (size_t)n * Np;                                // [n][n]: S, then the rows of R
  double* rinv = reinterpret_cast<double*>(B + n * n + QR_BPAD);  // 1 / R_jj
  const double* Ad = reinterpret_cast<const double*>(A);
  double2* phi = (sp == 0 ? phi_a : phi_b) + (size_t)z * N * n;

  // phi into LDS, QR_LD_BATCH loads per thread in flight at a time
  for (int e0 = 0; e0 < N * n; e0 += QR_LD_BATCH * QR_THREADS) {
    typedef double d2v __attribute__((ext_vector_type(2)));  // a native vector: kept in registers
    d2v v[QR_LD_BATCH];
#pragma unroll
    for (int b = 0; b < QR_LD_BATCH; ++b) {
      const int e = e0 + b * QR_THREADS + tid;
      v[b] = e < N * n ? *reinterpret_cast<const d2v*>(phi + e) : d2v{0.0, 0.0};
    }
#pragma unroll
    for (int b = 0; b < QR_LD_BATCH; ++b) {
      const int e = e0 + b * QR_THREADS + tid;
      if (e < N * n) {
        const int p = e / n, j = e - p * n;
        A[j * Np + p] = make_double2(v[b].x, v[b].y);
      }
    }
  }
  // this thread's Cholesky entries (i, j), i <= j, in row-major order
  const int npair = n * (n + 1) / 2;
  int ei[NPT], ej[NPT];
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    int r = tid + t * QR_THREADS, i = 0;
    if (r < npair) {
      while (r >= n - i) r -= n - i, ++i;
      ei[t] = i;
      ej[t] = i + r;
    } else {
      ei[t] = ej[t] = -1;
    }
  }
  bool failed = false;
  double lnr = 0.0;  // sum ln R_kk of both passes (thread 0)
  __syncthreads();

  const int nc = 2 * n, nbk = (nc + 15) / 16, nblk = nbk * (nbk + 1) / 2;
  for (int pass = 0; pass < 2; ++pass) {
    // ---- Gram: upper 16 x 16 blocks of X^T X, two k steps per iteration ----
    for (int b = wid; b < nblk; b += NWAVE) {
      int bi = 0, r = b;
      while (r >= nbk - bi) r -= nbk - bi, ++bi;
      const int bj = bi + r;
      const int c1 = 16 * bi + (lane & 15), c2 = 16 * bj + (lane & 15);
      const bool ok1 = c1 < nc, ok2 = c2 < nc;
      const int o1 = 2 * (c1 >> 1) * Np + (c1 & 1), o2 = 2 * (c2 >> 1) * Np + (c2 & 1);
      doublex4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
      for (int pb = 0; pb < N; pb += 8) {  // uniform trip count: the matrix instructions see every lane
        const int p0 = pb + (lane >> 4), p1 = p0 + 4;
        const double a0 = ok1 && p0 < N ? Ad[o1 + 2 * p0] : 0.0, b0 = ok2 && p0 < N ? Ad[o2 + 2 * p0] : 0.0;
        const double a1 = ok1 && p1 < N ? Ad[o1 + 2 * p1] : 0.0, b1 = ok2 && p1 < N ? Ad[o2 + 2 * p1] : 0.0;
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
      }
      // register r of lane l: G[16 bi + l / 16 + 4 r][16 bj + l % 16]
      const int g = lane >> 4, c = lane & 15;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const double v = acc0[rr] + acc1[rr];
        const double v01 = __shfl(v, lane + 1 < 64 ? lane + 1 : lane, 64);
        const double v10 = __shfl(v, lane + 16 < 64 ? lane + 16 : lane, 64);
        const double v11 = __shfl(v, lane + 17 < 64 ? lane + 17 : lane, 64);
        if (!(g & 1) && !(c & 1)) {
          const int i = (16 * bi + g + 4 * rr) >> 1, j = (16 * bj + c) >> 1;
          if (i <= j && j < n) B[i * n + j] = make_double2(v + v11, v01 - v10);
        }
      }
    }
    __syncthreads();
    // ---- Cholesky, entries in registers, one barrier per step ----
    double2 sv[NPT];
#pragma unroll
    for (int t = 0; t < NPT; ++t) sv[t] = ei[t] >= 0 ? B[ei[t] * n + ej[t]] : make_double2(0.0, 0.0);
    __syncthreads();  // every entry is read before rows are republished
    for (int k = 0; k < n; ++k) {
#pragma unroll
      for (int t = 0; t < NPT; ++t)
        if (ei[t] == k) B[k * n + ej[t]] = sv[t];
      __syncthreads();
      const double dk = B[k * n + k].x;
      if (!(dk > 0.0) || !isfinite(dk)) {  // a vanished column: every thread reads the same pivot
        failed = true;
        break;
      }
      const double idk = 1.0 / dk;
#pragma unroll
      for (int t = 0; t < NPT; ++t)
        if (ei[t] > k) sv[t] = csub(sv[t], cscale(cmul(cconj(B[k * n + ei[t]]), B[k * n + ej[t]]), idk));
    }
    if (failed) break;
    __syncthreads();
    if (tid < n) rinv[tid] = 1.0 / sqrt(B[tid * n + tid].x);
    if (wid == 0) {
      double l = lane < n ? 0.5 * log(B[lane * n + lane].x) : 0.0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
      lnr += l;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NPT; ++t)
      if (ei[t] >= 0 && ej[t] > ei[t]) B[ei[t] * n + ej[t]] = cscale(sv[t], rinv[ei[t]]);
    __syncthreads();
    // ---- A <- A R^{-1}: one row per thread, in registers; column i is
    // final once scaled, then removed from the later columns (their entries
    // past n use padding values and are never stored) ----
    for (int q = tid; q < N; q += QR_THREADS) {
      double2 a[NMAX];
#pragma unroll
      for (int j = 0; j < NMAX; ++j) a[j] = j < n ? A[(size_t)j * Np + q] : make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < NMAX; ++i) {
        if (i < n) {  // uniform
          const double2 qi = cscale(a[i], rinv[i]);
          a[i] = qi;
          const double2* Bi = B + i * n;
#pragma unroll
          for (int j = i + 1; j < NMAX; ++j) a[j] = csub(a[j], cmul(qi, Bi[j]));
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int j = 0; j < NMAX; ++j)
        if (j < n) A[(size_t)j * Np + q] = a[j];
    }
    __syncthreads();
  }

  if (failed) {  // rank-deficient walker: flagged, left as it is, weight ln 0
    if (tid == 0) {
      atomicOr(status, AFQMC_STATUS_QR_ZERO);
      corr[2 * z + sp] = -INFINITY;
    }
    return;
  }
  for (int e = tid; e < N * n; e += QR_THREADS) {
    const int p = e / n, j = e - p * n;
    phi[e] = A[j * Np + p];
  }
  if (tid == 0) corr[2 * z + sp] = lnr;
}

hipError_t launch_qr(const StepDims& d, int W, double2* phi_a, double2* phi_b, double* corr,
                     int* status, hipStream_t s) {
  const size_t lds = qr_lds_bytes(d);
  if (d.nmax <= 16)
    hipLaunchKernelGGL(qr_kernel<16>, dim3(W, 2), dim3(QR_THREADS), lds, s, d, phi_a, phi_b, corr, status);
  else if (d.nmax <= 32)
    hipLaunchKernelGGL(qr_kernel<32>, dim3(W, 2), dim3(QR_THREADS), lds, s, d, phi_a, phi_b, corr, status);
  else if (d.nmax <= 48)
    hipLaunchKernelGGL(qr_kernel<48>, dim3(W, 2), dim3(QR_THREADS), lds, s, d, phi_a, phi_b, corr, status);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// log overlap -= sum ln R_ii; a rank-deficient walker (corr = -inf from the
// QR) is discarded: log overlap +inf, weight 0 (log w = -inf), as the step's
// weight update does for it
__global__ void ortho_update_kernel(int W, const double* __restrict__ corr, double2* __restrict__ log_ovlp,
                                    double* __restrict__ log_w) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= W) return;
  const double c = corr[2 * z] + corr[2 * z + 1];
  log_ovlp[z].x -= c;
  if (!isfinite(c)) log_w[z] = -INFINITY;
}

hipError_t launch_ortho_update(int W, const double* corr, double2* log_ovlp, double* log_w, hipStream_t s) {
  hipLaunchKernelGGL(ortho_update_kernel, dim3(ceil_div(W, 256)), dim3(256), 0, s, W, corr, log_ovlp, log_w);
  return hipGetLastError();
}

hipError_t set_kernel_attributes(const StepDims& d) {
  hipError_t e;
  const int big = 160 * 1024;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(qr_kernel<16>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(qr_kernel<32>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(qr_kernel<48>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if (e != hipSuccess) return e;
  for (const void* f : {reinterpret_cast<const void*>(gf_kernel<float, 32>),
                        reinterpret_cast<const void*>(gf_kernel<float, 45>),
                        reinterpret_cast<const void*>(gf_kernel<double, 32>),
                        reinterpret_cast<const void*>(gf_kernel<double, 45>)}) {
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
  }
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(exchange_kernel<float>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(exchange_kernel<double>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(exchange_pair_kernel<float>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(exchange_pair_kernel<double>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)d;
  return e;
}
