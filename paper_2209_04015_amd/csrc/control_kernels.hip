// Ensemble kernels around the walker step: the weighted global energy
// (Sec. III.C, the walker-averaged estimate) and population control by a
// comb (population control is named in Sec. I without an algorithm; the comb
// is this library's choice).  Both reduce over every walker of a call inside
// one workgroup, in a fixed order, so results do not depend on scheduling.
//
// Weights: w_z = exp(log_w_z - m) with m the largest finite log weight; a
// non-finite log weight (-inf for a discarded walker, NaN) counts as 0.

#include <mutex>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace {

constexpr int CT = 1024;       // threads of the single-workgroup kernels
constexpr int CW = CT / 64;    // their waves

__device__ __forceinline__ double rel_weight(double lw, double m) { return isfinite(lw) ? exp(lw - m) : 0.0; }

// Block-wide max; every thread gets the result.  red: CW entries.
template <typename V>
__device__ V block_max(V v, V* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const V t = __shfl_xor(v, o, 64);
    v = t > v ? t : v;
  }
  __syncthreads();  // earlier readers of red are done
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  V r = red[0];
  for (int w = 1; w < CW; ++w) r = red[w] > r ? red[w] : r;
  return r;
}

// Block-wide exclusive prefix sum over the threads in thread order; *total
// gets the sum of all.  red: CW entries.
template <typename V>
__device__ V block_exclusive_scan(V v, V* red, V* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  V inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const V t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  V exc = __shfl_up(inc, 1, 64);
  if (lane == 0) exc = V(0);
  __syncthreads();  // earlier readers of red are done
  if (lane == 63) red[wid] = inc;
  __syncthreads();
  V base = V(0), tot = V(0);
  for (int w = 0; w < CW; ++w) {
    if (w < wid) base += red[w];
    tot += red[w];
  }
  *total = tot;
  return base + exc;
}

// ---------------------------------------------------------------------------
// E = sum_z w_z E_L^z / sum_z w_z,  E_L^z = e[z][0] + e[z][1] + e[z][2].
// out = {Re E, Im E, ln sum_z w_z, live walkers}; {NaN, NaN, -inf, 0} when
// no walker is alive.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(CT) void global_energy_kernel(int nw, const double* __restrict__ log_w,
                                                           const double2* __restrict__ e, double* __restrict__ out) {
  __shared__ double redd[CW];
  __shared__ double2 red2[CW];
  const int tid = threadIdx.x;
  double m = -INFINITY;
  for (int z = tid; z < nw; z += CT) {
    const double v = log_w[z];
    if (isfinite(v)) m = fmax(m, v);
  }
  m = block_max(m, redd);
  if (m == -INFINITY) {  // uniform
    if (tid == 0) {
      out[0] = NAN;
      out[1] = NAN;
      out[2] = -INFINITY;
      out[3] = 0.0;
    }
    return;
  }
  double2 num = make_double2(0.0, 0.0), dl = make_double2(0.0, 0.0);
  for (int z = tid; z < nw; z += CT) {
    const double w = rel_weight(log_w[z], m);
    if (w > 0.0) {
      const double2 el = cadd(cadd(e[3 * z], e[3 * z + 1]), e[3 * z + 2]);
      num = cadd(num, cscale(el, w));
      dl.x += w;
      dl.y += 1.0;
    }
  }
  num = block_sum2(num, red2);
  dl = block_sum2(dl, red2);
  if (tid == 0) {
    out[0] = num.x / dl.x;
    out[1] = num.y / dl.x;
    out[2] = m + log(dl.x);
    out[3] = dl.y;
  }
}

// ---------------------------------------------------------------------------
// Comb.  Teeth t_k = (k + u) W / nw (k < nw, W = total weight); tooth k
// selects the first walker z whose inclusive cumulative weight C_z exceeds
// t_k (a tooth past C_{nw-1}, possible only through rounding, selects the
// last live walker).  A walker with c >= 1 teeth keeps its slot; its c - 1
// extra copies, in walker order, go to the slots of walkers with no tooth, in
// slot order.  parent[k] = the walker whose copy slot k holds afterwards
// (k itself for survivors).  Every log weight becomes m + ln(W / nw).
// Thread t owns the contiguous walkers [t per, (t + 1) per).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(CT) void comb_kernel(int nw, double u, double* __restrict__ log_w,
                                                  double* __restrict__ csum, int* __restrict__ cnt,
                                                  int* __restrict__ src, int* __restrict__ parent,
                                                  int* __restrict__ status) {
  __shared__ double redd[CW];
  __shared__ int redi[CW];
  const int tid = threadIdx.x;
  const int per = (nw + CT - 1) / CT;
  const int i0 = min(tid * per, nw), i1 = min(i0 + per, nw);

  double m = -INFINITY;
  for (int i = i0; i < i1; ++i) {
    const double v = log_w[i];
    if (isfinite(v)) m = fmax(m, v);
  }
  m = block_max(m, redd);
  if (m == -INFINITY) {  // uniform: no live walker, nothing moves
    for (int i = tid; i < nw; i += CT) parent[i] = i;
    if (tid == 0) atomicOr(status, AFQMC_STATUS_NO_LIVE);
    return;
  }

  // inclusive cumulative weights and the last live walker
  double s = 0.0;
  int last = -1;
  for (int i = i0; i < i1; ++i) {
    const double w = rel_weight(log_w[i], m);
    s += w;
    if (w > 0.0) last = i;
  }
  double tot;
  s = block_exclusive_scan(s, redd, &tot);
  for (int i = i0; i < i1; ++i) {
    s += rel_weight(log_w[i], m);
    csum[i] = s;
  }
  last = block_max(last, redi);
  for (int i = i0; i < i1; ++i) cnt[i] = 0;
  __syncthreads();  // csum and cnt complete for the workgroup
  const double wtot = csum[nw - 1];

  for (int k = tid; k < nw; k += CT) {
    const double t = ((double)k + u) * wtot / (double)nw;
    int lo = 0, hi = nw;  // first z in [lo, hi) with csum[z] > t, else hi = nw
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (csum[mid] > t)
        hi = mid;
      else
        lo = mid + 1;
    }
    atomicAdd(&cnt[lo < nw ? lo : last], 1);
  }
  __syncthreads();  // every tooth counted

  // ranks of the extra copies and of the freed slots
  int ne = 0, nz = 0;
  for (int i = i0; i < i1; ++i) {
    const int c = cnt[i];
    ne += c > 1 ? c - 1 : 0;
    nz += c == 0;
  }
  int te, tz;
  int re = block_exclusive_scan(ne, redi, &te);
  int rz = block_exclusive_scan(nz, redi, &tz);
  for (int i = i0; i < i1; ++i) {
    const int c = cnt[i];
    for (int r = 1; r < c; ++r) src[re++] = i;
    parent[i] = c > 0 ? i : -1 - rz++;
  }
  __syncthreads();  // src complete
  for (int i = i0; i < i1; ++i) {
    const int p = parent[i];
    if (p < 0) parent[i] = src[-1 - p];
  }
  const double nlw = m + log(wtot / (double)nw);
  for (int i = i0; i < i1; ++i) log_w[i] = nlw;
}

// Slot k <- walker parent[k] for the freed slots.  Sources are survivors,
// whose slots are never written, so the copies do not interfere.
//   ea, eb: complex elements of one walker's phi_a / phi_b (N na, N nb)
__global__ __launch_bounds__(256) void comb_copy_kernel(const int* __restrict__ parent, long ea, long eb,
                                                        double2* phi_a, double2* phi_b, double2* log_ovlp) {
  const int k = blockIdx.x;
  const int p = parent[k];
  if (p == k) return;
  const long tot = ea + eb;
  for (long i = (long)blockIdx.y * 256 + threadIdx.x; i < tot; i += (long)gridDim.y * 256) {
    if (i < ea)
      phi_a[(size_t)k * ea + i] = phi_a[(size_t)p * ea + i];
    else
      phi_b[(size_t)k * eb + (i - ea)] = phi_b[(size_t)p * eb + (i - ea)];
  }
  if (blockIdx.y == 0 && threadIdx.x == 0) log_ovlp[k] = log_ovlp[p];
}

}  // namespace

hipError_t launch_global_energy(int nw, const double* log_w, const double2* e, double* out, hipStream_t s) {
  hipLaunchKernelGGL(global_energy_kernel, dim3(1), dim3(CT), 0, s, nw, log_w, e, out);
  return hipGetLastError();
}

hipError_t launch_comb(const StepDims& d, int nw, double u, double2* phi_a, double2* phi_b, double2* log_ovlp,
                       double* log_w, double* csum, int* cnt, int* src, int* parent, int* status, hipStream_t s) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(comb_kernel, dim3(1), dim3(CT), 0, s, nw, u, log_w, csum, cnt, src, parent, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long ea = (long)d.N * d.na, eb = (long)d.N * d.nb;
  const int ychunks = (int)((ea + eb + 2047) / 2048);  // about 8 elements per thread
  hipLaunchKernelGGL(comb_copy_kernel, dim3(nw, ychunks), dim3(256), 0, s, parent, ea, eb,
                     phi_a, phi_b, log_ovlp);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free comb: csum double [MAX], cnt, src
// and parent int [MAX], one status int.  Every GPU the library runs on holds
// its own copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t COMB_CSUM_OFF = 0;
constexpr size_t COMB_CNT_OFF = COMB_CSUM_OFF + sizeof(double) * COMB_STATIC_MAX_WALKERS;
constexpr size_t COMB_SRC_OFF = COMB_CNT_OFF + sizeof(int) * COMB_STATIC_MAX_WALKERS;
constexpr size_t COMB_PARENT_OFF = COMB_SRC_OFF + sizeof(int) * COMB_STATIC_MAX_WALKERS;
constexpr size_t COMB_STATUS_OFF = COMB_PARENT_OFF + sizeof(int) * COMB_STATIC_MAX_WALKERS;
constexpr size_t COMB_SCRATCH_BYTES = COMB_STATUS_OFF + 256;

}  // namespace

static __device__ __align__(256) unsigned char scratch[COMB_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device ordinal; null until looked up

}  // namespace

hipError_t comb_static_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_comb_static(void* scratch_ptr, const StepDims& d, int nw, double u, double2* phi_a,
                              double2* phi_b, double2* log_ovlp, double* log_w, int* parent, int* status,
                              hipStream_t s) {
  if (nw <= 0) return hipSuccess;
  if (nw > COMB_STATIC_MAX_WALKERS || !scratch_ptr) return hipErrorInvalidValue;
  unsigned char* base = static_cast<unsigned char*>(scratch_ptr);
  return launch_comb(d, nw, u, phi_a, phi_b, log_ovlp, log_w, reinterpret_cast<double*>(base + COMB_CSUM_OFF),
                     reinterpret_cast<int*>(base + COMB_CNT_OFF), reinterpret_cast<int*>(base + COMB_SRC_OFF),
                     parent ? parent : reinterpret_cast<int*>(base + COMB_PARENT_OFF),
                     status ? status : reinterpret_cast<int*>(base + COMB_STATUS_OFF), s);
}
