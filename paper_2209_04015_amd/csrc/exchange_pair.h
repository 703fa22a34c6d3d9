// Exchange energy through pair integrals (Sec. III.C, the sum reordered).
//
// With T_g = Lh_g theta (n x n) and Theta[i][q] = theta[q][i],
//   sum_g sum_ij T_ij T_ji = sum_ij sum_pq V_ij[p][q] Theta[j][p] Theta[i][q],
//   V_ij[p][q] = sum_g Lh_g[i][p] Lh_g[j][q].
// V_ij[p][q] = V_ji[q][p], so the (i, j) and (j, i) terms are equal and only
// i <= j is kept, the i < j blocks stored times 2.  For one spin the pair
// integrals are rows (i, j >= i, p) over q; for a fixed i they are one GEMM
//   U[(j, p)][(z, c)] = sum_q V_ij[p][q] Theta_z[i][q]   (c = re | im)
// whose epilogue multiplies U by Theta_z[j][p] and sums over (j, p): a
// Hadamard product and a column reduction, no transposition.  The GEMM has
// n (n + 1) / 2 N rows and contraction N against K n rows and contraction N
// for the direct T, so it needs 2 K n / ((n + 1) N) times fewer products.
//
// Rows: group i holds the rows (j, p), j = i .. n-1, p < Np (N rounded up to
// 4, the extra rows zero), so a 4-row group of an MFMA fragment never
// straddles two j and its theta values are one aligned 16-byte load.
#pragma once

#include "common.h"

constexpr int PAIR_MAX_N = 48;  // electrons per spin supported by the pair tables

// Per-spin tables in device memory: start[i] = first row tile of group i
// (start[n] = row tiles of the spin), vbase[i] = first pair-integral row of
// group i.
struct PairTab {
  int start[PAIR_MAX_N + 1];
  int vbase[PAIR_MAX_N + 1];
};

// Group i of row tile rt (uniform across the workgroup).
__device__ __forceinline__ int pair_group(const PairTab* __restrict__ tab, int n, int rt) {
  int i = 0;
  while (i + 1 < n && tab->start[i + 1] <= rt) ++i;
  return i;
}

template <typename A>
struct PairAccT;
template <>
struct PairAccT<floatx4> {
  using T = float;
};
template <>
struct PairAccT<doublex4> {
  using T = double;
};

__device__ __forceinline__ void pair_load4(const float* p, float (&v)[4]) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  v[0] = t.x;
  v[1] = t.y;
  v[2] = t.z;
  v[3] = t.w;
}
__device__ __forceinline__ void pair_load4(const double* p, double (&v)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}

// The value of lane ^ 1 (a DPP quad permutation [1, 0, 3, 2]; every lane is
// active where it is used).
__device__ __forceinline__ float pair_from_neighbour(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_from_neighbour(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Epilogue of one tile (group i, local rows lr0 .. lr0 + BM - 1 of R, walker
// columns (z0 + c / 2, c % 2)).  acc holds U scaled by the operand row scales
// (SCALED: a_unscale per pair-integral row, b_unscale per theta split row;
// otherwise both 1 and unused).  Writes out[z] = sum over the tile's rows of U Theta_z[j][p] for the
// tile's walkers (fixed order: FP32 / FP64 over the four rows of a fragment,
// FP64 beyond).  theta: working-precision planar [W][re|im][spin][nmax][ldN],
// W * 4 * nmax * ldN < 2^31 elements.
template <int BM, int BN, int WM, int WN, bool SCALED, class AccV, class TT>
__device__ __forceinline__ void exchange_pair_epilogue(const AccV (&acc)[BM / WM / 16][BN / WN / 16],
                                                       char* lds_raw, int i, int lr0, int R, int Np, int vbase,
                                                       int z0, int W, int sp, int nmax, int ldN,
                                                       const TT* __restrict__ theta,
                                                       const float* __restrict__ a_unscale,
                                                       const float* __restrict__ b_unscale,
                                                       double2* __restrict__ out) {
  using AT = typename PairAccT<AccV>::T;
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid / WN, wn = wid % WN;
  const int comp = lane & 1;  // column (z, comp): every fragment column base is even
  const int plane = nmax * ldN;

  // Loads below stay after the main loop (their registers are not live
  // during it); the LDS is reused further down only after this barrier.
  __syncthreads();
  // per column: element offset of theta_re (theta_im is two planes further)
  // and the operand scale of its theta split row (0 outside the problem)
  int toff[FN];
  AT ub[FN];
#pragma unroll
  for (int f = 0; f < FN; ++f) {
    const int cl = wn * (BN / WN) + f * 16 + (lane & 15);
    const int z = z0 + (cl >> 1);
    const bool ok = z < W;
    const int zc = ok ? z : 0;  // stays inside the arrays; its weight is 0
    toff[f] = ((zc * 2 + 0) * 2 + sp) * plane;
    if constexpr (SCALED)
      ub[f] = ok ? (AT)b_unscale[((zc * 2 + comp) * 2 + sp) * nmax + i] : (AT)0;
    else
      ub[f] = ok ? (AT)1 : (AT)0;
  }
  double2 s[FN];
#pragma unroll
  for (int f = 0; f < FN; ++f) s[f] = make_double2(0.0, 0.0);

#pragma unroll
  for (int fi = 0; fi < FM; ++fi) {
    const int lr = lr0 + wm * (BM / WM) + fi * 16 + 4 * (lane >> 4);
    const bool rok = lr < R;
    const int lrc = rok ? lr : 0;
    const int jj = lrc / Np;  // j - i
    const int p = lrc - jj * Np;
    const int roff = (i + jj) * ldN + p;
    AT ua[4];
    if constexpr (SCALED) {
      float u4[4];
      pair_load4(a_unscale + vbase + lrc, u4);
#pragma unroll
      for (int r = 0; r < 4; ++r) ua[r] = rok ? (AT)u4[r] : (AT)0;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) ua[r] = rok ? (AT)1 : (AT)0;
    }
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      // the two lanes of a walker's columns (z, re) and (z, im) each load one
      // theta plane (re and im) and take the other from the neighbour
      TT mine[4], a[4], b[4];
      pair_load4(theta + (toff[f] + (comp ? 2 * plane : 0) + roff), mine);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const TT other = pair_from_neighbour(mine[r]);
        a[r] = comp ? other : mine[r];
        b[r] = comp ? mine[r] : other;
      }
      AT xr = 0, xi = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const AT u = acc[fi][f][r] * ua[r];
        xr = fma(u, (AT)a[r], xr);
        xi = fma(u, (AT)b[r], xi);
      }
      // column (z, re): U_re (Theta_re + i Theta_im); column (z, im): U_im (i Theta_re - Theta_im)
      const double vr = (double)(ub[f] * (comp ? -xi : xr));
      const double vi = (double)(ub[f] * (comp ? xr : xi));
      s[f].x += vr;
      s[f].y += vi;
    }
    // one row group at a time: its loads are not scheduled into the next
    // group's (keeps the epilogue inside the main loop's register budget)
    __builtin_amdgcn_sched_barrier(0);
  }

  // column sums through LDS: [4 row groups][WM][BN], then one thread per
  // walker adds the 4 WM entries of its two columns in a fixed order
  double2* colsum = reinterpret_cast<double2*>(lds_raw);
#pragma unroll
  for (int f = 0; f < FN; ++f)
    colsum[((lane >> 4) * WM + wm) * BN + wn * (BN / WN) + f * 16 + (lane & 15)] = s[f];
  __syncthreads();
  if (tid < BN / 2 && z0 + tid < W) {
    double2 t = make_double2(0.0, 0.0);
    for (int g = 0; g < 4 * WM; ++g) {
      t = cadd(t, colsum[g * BN + 2 * tid]);
      t = cadd(t, colsum[g * BN + 2 * tid + 1]);
    }
    out[z0 + tid] = t;
  }
}

// Zero partials of a row tile past this spin's tiles (the energy sum runs
// over the larger spin's tile count).
template <int BN>
__device__ __forceinline__ void exchange_pair_zero(int z0, int W, double2* __restrict__ out) {
  if (threadIdx.x < BN / 2 && z0 + (int)threadIdx.x < W) out[z0 + threadIdx.x] = make_double2(0.0, 0.0);
}
