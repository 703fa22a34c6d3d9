// Mixed estimators (Sec. IV.B): the full one-body Green's function of every
// walker (the input of any custom one-body mixed estimator), the mixed S^2,
// and the weighted walker mean that turns per-walker values into an
// ensemble estimate.  theta is the working-precision planar array of the
// Green's-function kernel, [W][re|im][spin][nmax][ldN] (row i = electron,
// column = orbital); the trial orbitals are FP64 [spin][N][nmax].  Every
// product is accumulated in FP64.

#include "common.h"
#include "kernels.h"

namespace {

constexpr int GF_ROWS = 16;   // rows p of G per thread
constexpr int GF_COLS = 256;  // columns q of G per workgroup (one per thread)

__device__ __forceinline__ double wabs_weight(double lw, double m) { return isfinite(lw) ? exp(lw - m) : 0.0; }

// G[z][s][p][q] = sum_i PhiT_s[p][i] theta_s[q][i]  (the paper's G_pq; rows
// p0 .. p0 + GF_ROWS - 1, column q per thread).  Grid: x = column blocks x
// row blocks, y = (walker - z0) * 2 + spin.
template <typename T>
__global__ __launch_bounds__(GF_COLS) void green_full_kernel(StepDims d, int z0, const T* __restrict__ theta,
                                                             const double* __restrict__ phiT,
                                                             double2* __restrict__ G) {
  const int nqb = (d.N + GF_COLS - 1) / GF_COLS;
  const int qb = blockIdx.x % nqb, pb = blockIdx.x / nqb;
  const int z = z0 + (int)(blockIdx.y >> 1), s = blockIdx.y & 1;
  const int q = qb * GF_COLS + threadIdx.x;
  const int p0 = pb * GF_ROWS;
  const int n = s ? d.nb : d.na;
  const T* tre = theta + ((size_t)(z * 2 + 0) * 2 + s) * d.nmax * d.ldN;
  const T* tim = theta + ((size_t)(z * 2 + 1) * 2 + s) * d.nmax * d.ldN;
  const double* ph = phiT + (size_t)s * d.N * d.nmax;
  double2 acc[GF_ROWS];
#pragma unroll
  for (int r = 0; r < GF_ROWS; ++r) acc[r] = make_double2(0.0, 0.0);
  if (q < d.N) {
    for (int i = 0; i < n; ++i) {
      const double a = (double)tre[(size_t)i * d.ldN + q], b = (double)tim[(size_t)i * d.ldN + q];
#pragma unroll
      for (int r = 0; r < GF_ROWS; ++r) {
        const int p = p0 + r < d.N ? p0 + r : d.N - 1;  // clamped rows are not stored
        const double f = ph[(size_t)p * d.nmax + i];
        acc[r].x = fma(f, a, acc[r].x);
        acc[r].y = fma(f, b, acc[r].y);
      }
    }
    double2* out = G + ((size_t)z * 2 + s) * d.N * d.N;
#pragma unroll
    for (int r = 0; r < GF_ROWS; ++r)
      if (p0 + r < d.N) out[(size_t)(p0 + r) * d.N + q] = acc[r];
  }
}

// s2[z] = nb + Ms (Ms + 1) - sum_{i < nb, j < na} X_ij Y_ji with
// X = theta_b^T PhiT_a (nb x na) and Y = theta_a^T PhiT_b (na x nb), i.e.
// minus the trace of G^a G^b.  One workgroup per walker, one (i, j) pair per
// thread and pass.
template <typename T>
__global__ __launch_bounds__(256) void s2_kernel(StepDims d, const T* __restrict__ theta,
                                                 const double* __restrict__ phiT, double2* __restrict__ s2) {
  __shared__ double2 red[4];
  const int z = blockIdx.x;
  const int na = d.na, nb = d.nb;
  const T* ta_re = theta + ((size_t)(z * 2 + 0) * 2 + 0) * d.nmax * d.ldN;
  const T* ta_im = theta + ((size_t)(z * 2 + 1) * 2 + 0) * d.nmax * d.ldN;
  const T* tb_re = theta + ((size_t)(z * 2 + 0) * 2 + 1) * d.nmax * d.ldN;
  const T* tb_im = theta + ((size_t)(z * 2 + 1) * 2 + 1) * d.nmax * d.ldN;
  const double* pa = phiT;
  const double* pbt = phiT + (size_t)d.N * d.nmax;
  double2 t = make_double2(0.0, 0.0);
  for (int e = threadIdx.x; e < na * nb; e += blockDim.x) {
    const int i = e / na, j = e - i * na;
    double2 x = make_double2(0.0, 0.0), y = make_double2(0.0, 0.0);
    for (int p = 0; p < d.N; ++p) {
      const double fa = pa[(size_t)p * d.nmax + j], fb = pbt[(size_t)p * d.nmax + i];
      x.x = fma((double)tb_re[(size_t)i * d.ldN + p], fa, x.x);
      x.y = fma((double)tb_im[(size_t)i * d.ldN + p], fa, x.y);
      y.x = fma((double)ta_re[(size_t)j * d.ldN + p], fb, y.x);
      y.y = fma((double)ta_im[(size_t)j * d.ldN + p], fb, y.y);
    }
    t = cadd(t, cmul(x, y));
  }
  t = block_sum2(t, red);
  if (threadIdx.x == 0) {
    const double ms = 0.5 * (na - nb);
    s2[z] = make_double2(nb + ms * (ms + 1.0) - t.x, -t.y);
  }
}

// out[2k], out[2k+1] = Re, Im of sum_z w_z v[z][k] / sum_z w_z; block k
// handles column k; block 0 also writes out[2m] = ln sum w, out[2m+1] =
// live walkers.  No live walker: NaN means, -inf, 0.
__global__ __launch_bounds__(1024) void weighted_mean_kernel(int nw, int m, const double* __restrict__ log_w,
                                                             const double2* __restrict__ v, double* __restrict__ out) {
  __shared__ double2 red[16];
  const int k = blockIdx.x, tid = threadIdx.x;
  double mx = -INFINITY;
  for (int z = tid; z < nw; z += blockDim.x) {
    const double lw = log_w[z];
    if (isfinite(lw)) mx = fmax(mx, lw);
  }
  // block max through the pair-sum helper's storage
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = make_double2(mx, 0.0);
  __syncthreads();
  mx = red[0].x;
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mx = fmax(mx, red[w].x);
  if (mx == -INFINITY) {  // uniform
    if (tid == 0) {
      out[2 * k] = NAN;
      out[2 * k + 1] = NAN;
      if (k == 0) {
        out[2 * m] = -INFINITY;
        out[2 * m + 1] = 0.0;
      }
    }
    return;
  }
  double2 num = make_double2(0.0, 0.0), dl = make_double2(0.0, 0.0);
  for (int z = tid; z < nw; z += blockDim.x) {
    const double w = wabs_weight(log_w[z], mx);
    if (w > 0.0) {
      num = cadd(num, cscale(v[(size_t)z * m + k], w));
      dl.x += w;
      dl.y += 1.0;
    }
  }
  num = block_sum2(num, red);
  dl = block_sum2(dl, red);
  if (tid == 0) {
    out[2 * k] = num.x / dl.x;
    out[2 * k + 1] = num.y / dl.x;
    if (k == 0) {
      out[2 * m] = mx + log(dl.x);
      out[2 * m + 1] = dl.y;
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_green_full(const StepDims& d, int W, const T* theta, const double* phiT, double2* G,
                             hipStream_t s) {
  const int nqb = (d.N + GF_COLS - 1) / GF_COLS, npb = (d.N + GF_ROWS - 1) / GF_ROWS;
  constexpr int ZCHUNK = 16384;  // walkers per launch (grid y = 2 per walker)
  for (int z0 = 0; z0 < W; z0 += ZCHUNK) {
    const int nz = W - z0 < ZCHUNK ? W - z0 : ZCHUNK;
    hipLaunchKernelGGL(green_full_kernel<T>, dim3(nqb * npb, 2 * nz), dim3(GF_COLS), 0, s, d, z0, theta, phiT, G);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_s2(const StepDims& d, int W, const T* theta, const double* phiT, double2* s2, hipStream_t s) {
  hipLaunchKernelGGL(s2_kernel<T>, dim3(W), dim3(256), 0, s, d, theta, phiT, s2);
  return hipGetLastError();
}

hipError_t launch_weighted_mean(int nw, int m, const double* log_w, const double2* v, double* out, hipStream_t s) {
  hipLaunchKernelGGL(weighted_mean_kernel, dim3(m), dim3(1024), 0, s, nw, m, log_w, v, out);
  return hipGetLastError();
}

template hipError_t launch_green_full<float>(const StepDims&, int, const float*, const double*, double2*, hipStream_t);
template hipError_t launch_green_full<double>(const StepDims&, int, const double*, const double*, double2*, hipStream_t);
template hipError_t launch_s2<float>(const StepDims&, int, const float*, const double*, double2*, hipStream_t);
template hipError_t launch_s2<double>(const StepDims&, int, const double*, const double*, double2*, hipStream_t);
