// Step-independent setup of a Hamiltonian (run once per Hamiltonian, not timed).
//
//   h' = h1 - 1/2 sum_g L_g L_g        (rewrite of Eq. Habinitio with v_g = sum L_g a+ a)
//   mu = tr(h') / N
//   P  = exp(-dt (h' - mu) / 2)        (symmetric Trotter half step, scalar factored out)
//   Lh^s_g = PhiT_s^T L_g              (half-rotated Cholesky vectors, Sec. III.B)
//   hh^s   = PhiT_s^T h1
//   LT[(p<=q)][g] = L_g[p][q]          (packed triangle, Cholesky index contiguous)
//
// All arithmetic runs here on the device in FP64; P comes from scaling and
// squaring of a truncated Taylor series (no eigendecomposition needed).

#include <math.h>

#include "common.h"
#include "setup.h"

// ---------------------------------------------------------------------------
// Plain LDS-tiled FP64 GEMM for setup:  C[kc] = op(A) B over one K chunk.
//   amode 0: op(A) = A, A[r][k] at A[r * lda + k]
//   amode 1: op(A) = A^T, A[k][r] at A[k * lda + r]
//   amode 2: stacked blocks, A(r, k) = A[(k / lda) * lda * lda + r * lda + k % lda]
//            (the [K][N][N] Cholesky array read as L_g rows: sum over (g, col))
//   chunk kc covers k in [kc * kchunk, (kc + 1) * kchunk); C is [nchunk][M][ldc]
// ---------------------------------------------------------------------------
constexpr int ST = 16;

__global__ __launch_bounds__(ST* ST) void setup_gemm_kernel(int M, int N, int K, int transA,
                                                            const double* __restrict__ A, long lda,
                                                            const double* __restrict__ B, long ldb,
                                                            double* __restrict__ C, long ldc,
                                                            int kchunk) {
  __shared__ double As[ST][ST + 1], Bs[ST][ST + 1];
  const int tx = threadIdx.x % ST, ty = threadIdx.x / ST;
  const int row = blockIdx.x * ST + ty, col = blockIdx.y * ST + tx;
  const int kc = blockIdx.z;
  const int kbeg = kc * kchunk, kend = min(K, kbeg + kchunk);
  double acc = 0.0;
  for (int k0 = kbeg; k0 < kend; k0 += ST) {
    {
      const int r = blockIdx.x * ST + ty, k = k0 + tx;
      double v = 0.0;
      if (r < M && k < kend) {
        if (transA == 0) v = A[(long)r * lda + k];
        else if (transA == 1) v = A[(long)k * lda + r];
        else v = A[(long)(k / lda) * lda * lda + (long)r * lda + (k % lda)];
      }
      As[ty][tx] = v;
      const int kb = k0 + ty, c = blockIdx.y * ST + tx;
      double w = 0.0;
      if (kb < kend && c < N) w = B[(long)kb * ldb + c];
      Bs[ty][tx] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < ST; ++kk) acc += As[ty][kk] * Bs[kk][tx];
    __syncthreads();
  }
  if (row < M && col < N) C[(long)kc * M * ldc + (long)row * ldc + col] = acc;
}

__global__ void sum_chunks_kernel(int nchunk, long n, const double* __restrict__ part,
                                  double* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(long)c * n + e];
  out[e] = s;
}

hipError_t setup_gemm(int M, int N, int K, int transA, const double* A, long lda, const double* B,
                      long ldb, double* C, long ldc, double* scratch, int nchunk, hipStream_t s) {
  if (nchunk <= 1) {
    dim3 grid(ceil_div(M, ST), ceil_div(N, ST), 1);
    hipLaunchKernelGGL(setup_gemm_kernel, grid, dim3(ST * ST), 0, s, M, N, K, transA, A, lda, B,
                       ldb, C, ldc, K);
    return hipGetLastError();
  }
  const int kchunk = round_up(ceil_div(K, nchunk), ST);
  nchunk = ceil_div(K, kchunk);
  dim3 grid(ceil_div(M, ST), ceil_div(N, ST), nchunk);
  hipLaunchKernelGGL(setup_gemm_kernel, grid, dim3(ST * ST), 0, s, M, N, K, transA, A, lda, B,
                     ldb, scratch, (long)N, kchunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ldc != N) return hipErrorInvalidValue;
  const long n = (long)M * N;
  hipLaunchKernelGGL(sum_chunks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     nchunk, n, scratch, C);
  return hipGetLastError();
}

// h' = h1 - 1/2 LL ; out_scalar[0] = tr(h') (single block, fixed order)
__global__ __launch_bounds__(256) void hprime_kernel(int N, const double* __restrict__ h1,
                                                     const double* __restrict__ LL,
                                                     double* __restrict__ hp,
                                                     double* __restrict__ tr) {
  __shared__ double red[256];
  double t = 0.0;
  for (int e = threadIdx.x; e < N * N; e += 256) {
    const double v = h1[e] - 0.5 * LL[e];
    hp[e] = v;
    if (e / N == e % N) t += v;
  }
  red[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < 256; ++i) s += red[i];
    tr[0] = s;
  }
}

// A = c (h' - mu I); out[0] = max column abs sum of A (single block)
__global__ __launch_bounds__(256) void expm_arg_kernel(int N, const double* __restrict__ hp, double mu,
                                                       double c, double* __restrict__ A,
                                                       double* __restrict__ norm1) {
  __shared__ double red[256];
  double best = 0.0;
  for (int q = threadIdx.x; q < N; q += 256) {
    double s = 0.0;
    for (int p = 0; p < N; ++p) {
      const double v = c * (hp[p * N + q] - (p == q ? mu : 0.0));
      A[p * N + q] = v;
      s += fabs(v);
    }
    best = fmax(best, s);
  }
  red[threadIdx.x] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int i = 0; i < 256; ++i) m = fmax(m, red[i]);
    norm1[0] = m;
  }
}

// X = alpha X + I  (N x N)
__global__ void scale_add_identity_kernel(int N, double alpha, double* __restrict__ X) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * N) return;
  X[e] = alpha * X[e] + ((e / N == e % N) ? 1.0 : 0.0);
}

__global__ void scale_kernel(long n, double alpha, double* __restrict__ X) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) X[e] *= alpha;
}

__global__ void copy_pad_kernel(int rows, int cols, const double* __restrict__ src, int lds_,
                                double* __restrict__ dst, int ldd) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows * cols) return;
  const int r = (int)(e / cols), c = (int)(e % cols);
  dst[(long)r * ldd + c] = src[(long)r * lds_ + c];
}

hipError_t setup_hprime(int N, const double* h1, const double* LL, double* hp, double* tr,
                        hipStream_t s) {
  hipLaunchKernelGGL(hprime_kernel, dim3(1), dim3(256), 0, s, N, h1, LL, hp, tr);
  return hipGetLastError();
}

hipError_t setup_expm_arg(int N, const double* hp, double mu, double c, double* A, double* norm1,
                          hipStream_t s) {
  hipLaunchKernelGGL(expm_arg_kernel, dim3(1), dim3(256), 0, s, N, hp, mu, c, A, norm1);
  return hipGetLastError();
}

// exp(A) by scaling and squaring: B = A / 2^sq, R = sum_{k<=order} B^k / k! by
// Horner (R <- I + B R / k), then R <- R^2 sq times.  A, R, T are N x N.
hipError_t setup_expm(int N, double* A, int sq, int order, double* R, double* T, hipStream_t s) {
  const long nn = (long)N * N;
  const unsigned nb = (unsigned)((nn + 255) / 256);
  hipLaunchKernelGGL(scale_kernel, dim3(nb), dim3(256), 0, s, nn, ldexp(1.0, -sq), A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // R = I + B / order
  e = hipMemcpyAsync(R, A, nn * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scale_add_identity_kernel, dim3(nb), dim3(256), 0, s, N, 1.0 / order, R);
  for (int k = order - 1; k >= 1; --k) {
    e = setup_gemm(N, N, N, 0, A, N, R, N, T, N, nullptr, 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scale_add_identity_kernel, dim3(nb), dim3(256), 0, s, N, 1.0 / k, T);
    e = hipMemcpyAsync(R, T, nn * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  for (int i = 0; i < sq; ++i) {
    e = setup_gemm(N, N, N, 0, R, N, R, N, T, N, nullptr, 1, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(R, T, nn * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t setup_copy_pad(int rows, int cols, const double* src, int lds_, double* dst, int ldd,
                          hipStream_t s) {
  const long n = (long)rows * cols;
  hipLaunchKernelGGL(copy_pad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rows,
                     cols, src, lds_, dst, ldd);
  return hipGetLastError();
}

// Lh[s][g][j][p] (working precision, padded) from Y[(g, p)][j] = (L_g PhiT_s)[p][j]
template <typename T>
__global__ void pack_lh_kernel(int K, int N, int n, int nmax, int ldN, const double* __restrict__ Y,
                               T* __restrict__ Lh) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)K * n * N) return;
  const int p = (int)(e % N);
  const long r = e / N;
  const int j = (int)(r % n);
  const int g = (int)(r / n);
  Lh[((long)g * nmax + j) * ldN + p] = (T)Y[((long)g * N + p) * n + j];
}

template <typename T>
hipError_t setup_pack_lh(int K, int N, int n, int nmax, int ldN, const double* Y, T* Lh,
                         hipStream_t s) {
  const long tot = (long)K * n * N;
  hipLaunchKernelGGL(pack_lh_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, K, N,
                     n, nmax, ldN, Y, Lh);
  return hipGetLastError();
}
template hipError_t setup_pack_lh<float>(int, int, int, int, int, const double*, float*, hipStream_t);
template hipError_t setup_pack_lh<double>(int, int, int, int, int, const double*, double*, hipStream_t);

// LT[pq][g] = L[g][p][q] for the packed (p <= q) list; 32 x 32 tiles through LDS.
template <typename T>
__global__ __launch_bounds__(256) void pack_lt_kernel(int K, int N, int Npk, int ldK,
                                                      const int2* __restrict__ pq,
                                                      const double* __restrict__ L,
                                                      T* __restrict__ LT) {
  __shared__ T tile[32][33];
  const int pq0 = blockIdx.x * 32, g0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int g = g0 + r, c = pq0 + tx;
    T v = (T)0;
    if (g < K && c < Npk) {
      const int2 ij = pq[c];
      if (ij.x >= 0) v = (T)L[((long)g * N + ij.x) * N + ij.y];  // (-1, -1): a zero row
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int c = pq0 + r, g = g0 + tx;
    if (c < Npk && g < K) LT[(long)c * ldK + g] = tile[tx][r];
  }
}

template <typename T>
hipError_t setup_pack_lt(int K, int N, int Npk, int ldK, const int2* pq, const double* L, T* LT,
                         hipStream_t s) {
  dim3 grid(ceil_div(Npk, 32), ceil_div(K, 32));
  hipLaunchKernelGGL(pack_lt_kernel<T>, grid, dim3(256), 0, s, K, N, Npk, ldK, pq, L, LT);
  return hipGetLastError();
}
template hipError_t setup_pack_lt<float>(int, int, int, int, const int2*, const double*, float*, hipStream_t);
template hipError_t setup_pack_lt<double>(int, int, int, int, const int2*, const double*, double*, hipStream_t);

// hh[j][p] = sum_q PhiT[q][j] h1[q][p]   (PhiT stored [N][nmax])
__global__ void hh_kernel(int N, int n, int nmax, const double* __restrict__ phiT,
                          const double* __restrict__ h1, double* __restrict__ hh) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * N) return;
  const int j = e / N, p = e % N;
  double s = 0.0;
  for (int q = 0; q < N; ++q) s += phiT[q * nmax + j] * h1[q * N + p];
  hh[j * N + p] = s;
}

hipError_t setup_hh(int N, int n, int nmax, const double* phiT, const double* h1, double* hh,
                    hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(hh_kernel, dim3(ceil_div(n * N, 256)), dim3(256), 0, s, N, n, nmax, phiT, h1, hh);
  return hipGetLastError();
}

// walker = PhiT as complex, [N][n]
__global__ void trial_walker_kernel(int N, int n, int nmax, const double* __restrict__ phiT,
                                    double2* __restrict__ phi) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * n) return;
  const int p = e / n, j = e % n;
  phi[e] = make_double2(phiT[p * nmax + j], 0.0);
}

hipError_t setup_trial_walker(int N, int n, int nmax, const double* phiT, double2* phi,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(trial_walker_kernel, dim3(ceil_div(N * n, 256)), dim3(256), 0, s, N, n, nmax,
                     phiT, phi);
  return hipGetLastError();
}

// Pair integrals of one spin for the exchange through pair integrals: row
// (i, j >= i, p) of group i (groups in order of i, rows of a group in order
// of j then p < Np) holds c V_ij[p][q] over q < ldq, with
// V_ij[p][q] = C[p n + i][q n + j], C = Y^T Y the sum over Cholesky vectors
// of the half-rotated products (Y [K][N][n]), c = 2 for j > i and 1 for
// j = i; rows p >= N and columns q >= N are zero.
template <typename T>
__global__ __launch_bounds__(256) void pack_vpair_kernel(int N, int n, int Np, int ldq, long rows,
                                                         const double* __restrict__ C, T* __restrict__ V) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * ldq) return;
  const long v = e / ldq;
  const int q = (int)(e - v * ldq);
  const int blk = (int)(v / Np), p = (int)(v - (long)blk * Np);
  int i = 0;  // pair blocks before group i: i n - i (i - 1) / 2
  while (i + 1 < n && (i + 1) * n - (i + 1) * i / 2 <= blk) ++i;
  const int j = i + (blk - (i * n - i * (i - 1) / 2));
  double x = 0.0;
  if (p < N && q < N) x = (j > i ? 2.0 : 1.0) * C[((long)p * n + i) * ((long)N * n) + (long)q * n + j];
  V[e] = (T)x;
}

template <typename T>
hipError_t setup_pack_vpair(int N, int n, int Np, int ldq, long rows, const double* C, T* V, hipStream_t s) {
  const long tot = rows * ldq;
  hipLaunchKernelGGL(pack_vpair_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, N, n, Np, ldq,
                     rows, C, V);
  return hipGetLastError();
}
template hipError_t setup_pack_vpair<float>(int, int, int, int, long, const double*, float*, hipStream_t);
template hipError_t setup_pack_vpair<double>(int, int, int, int, long, const double*, double*, hipStream_t);
