// Single-pass exchange epilogue on the lower triangle of T (Sec. III.C,
// direct algorithm).  The accumulator tile holds T^{z,g}_{ij} for G whole
// Cholesky vectors (rows (g, i)) and Z whole walkers (columns
// (z, re|im, j)).  The exchange sum of one walker block is
//   sum_ij T_ij T_ji = sum_i T_ii^2 + 2 sum_{i<j} T_ij T_ji ,
// so only the lower triangle (i >= j, complex) goes through LDS: its owners
// store it, then the owners of i <= j read their partner T_ji from it and
// accumulate in FP64.  Per column (z, re|im, j) a thread keeps
//   x = sum w v P.re,  y = sum w v P.im   (v its own element, P = T_ji,
//   w = 2 off the diagonal, 1 on it),
// and for a walker Re = sum_re-columns x - sum_im-columns y,
// Im = sum_re-columns y + sum_im-columns x.
#pragma once

#include "common.h"

struct ExTriGeom {
  int n, G, Z, K, W, gt, wt, nmax, sp, ntg;
};

// Complex entries of one walker slot's triangles.
__host__ __device__ inline int ex_tri_block(int G, int n) { return G * (n * (n + 1) / 2); }

// floor(x / d) for 0 <= x < 2^16 and 1 <= d <= 2^16, with rinv = 1.0f / d.  The
// quotient (x + 1/2) / d sits at least 1/(2d) from an integer, far above the
// rounding of the single-precision product.
__device__ __forceinline__ int ex_div(int x, float rinv) {
  return (int)(((float)x + 0.5f) * rinv);
}

// Writes part[(sp * ntg + gt) * W + z] for the tile's walkers.  row_unscale(g,
// i) and col_unscale(z, comp, j) give the power-of-two factors that undo the
// operand scaling (used only if SCALED).  zpp walker slots per pass; LDS
// needs ex_tri_lds_bytes.  Both passes are branch-free (masked lanes store
// to a private dummy slot, or load a zero slot and weigh it by zero), so the
// LDS accesses of a row issue back to back.
__host__ __device__ inline int ex_tri_lds_bytes(int zpp, int G, int n, int WM, int BN) {
  const int tri = zpp * ex_tri_block(G, n) * 8 + 64 * 4 + 16;  // + dummy slot per lane, zero slot
  const int col = WM * BN * 16;
  return tri > col ? tri : col;
}

template <int BM, int BN, int WM, int WN, bool SCALED, class RowScale, class ColScale>
__device__ __forceinline__ void exchange_tri_epilogue(floatx4 (&acc)[BM / WM / 16][BN / WN / 16],
                                                      char* lds_raw, int zpp, const ExTriGeom& q,
                                                      RowScale row_unscale, ColScale col_unscale,
                                                      double2* __restrict__ part) {
  constexpr int NT = WM * WN * 64;
  constexpr int NWAVE = NT / 64;
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  constexpr int BIG = 1 << 20;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / WN, wn = wid % WN;
  const int n = q.n, n2 = 2 * n;
  const int tri = n * (n + 1) / 2;
  const int blk = q.G * tri;
  const float rn = 1.0f / (float)n, rn2 = 1.0f / (float)n2;
  const int rbase = wm * (BM / WM) + 4 * (lane >> 4);
  const unsigned dummy = (unsigned)(zpp * blk * 8 + lane * 4);  // byte offsets
  const unsigned zslot = (unsigned)(zpp * blk * 8 + 64 * 4);

  // this thread's columns
  int cz[FN], cj[FN], cc[FN];
#pragma unroll
  for (int f = 0; f < FN; ++f) {
    const int c = wn * (BN / WN) + f * 16 + (lane & 15);
    const int zt = ex_div(c, rn2);
    const int o = c - zt * n2;
    const int comp = o >= n ? 1 : 0;
    const int z = q.wt * q.Z + zt;
    cz[f] = (zt < q.Z && z < q.W) ? zt : BIG;  // outside every pass
    cj[f] = o - comp * n;
    cc[f] = comp;
  }
  if constexpr (SCALED) {  // true T = acc * row factor * column factor (powers of two: exact)
    float cs[FN];
#pragma unroll
    for (int f = 0; f < FN; ++f) cs[f] = cz[f] < BIG ? col_unscale(q.wt * q.Z + cz[f], cc[f], cj[f]) : 0.f;
#pragma unroll
    for (int fi = 0; fi < FM; ++fi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rbase + fi * 16 + r;
        const int gl = ex_div(row, rn);
        const int g = q.gt * q.G + gl;
        const float rs = (gl < q.G && g < q.K) ? row_unscale(g, row - gl * n) : 0.f;
#pragma unroll
        for (int f = 0; f < FN; ++f) acc[fi][f][r] *= rs * cs[f];
      }
  }
  double2 s[FN];
#pragma unroll
  for (int f = 0; f < FN; ++f) s[f] = make_double2(0.0, 0.0);

  for (int z0 = 0; z0 < q.Z; z0 += zpp) {
    // per pass and column: j bound for stores (i >= jw) and loads (i <= jr),
    // and the column's part of the LDS byte offsets
    int jw[FN], jr[FN];
    unsigned cw[FN], cr[FN];
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const int zl = cz[f] - z0;
      const bool in = zl >= 0 && zl < zpp;
      const int j = cj[f];
      jw[f] = in ? j : BIG;
      jr[f] = in ? j : -1;
      cw[f] = in ? (unsigned)(8 * (zl * blk + j) + 4 * cc[f]) : 0u;
      cr[f] = in ? (unsigned)(8 * (zl * blk + j * (j + 1) / 2)) : 0u;
    }
    // opaque per pass: keeps the per-row index arithmetic inside the pass
    // loop (hoisted, it would hold registers per element)
    int rb = rbase;
    asm volatile("" : "+v"(rb));
    __syncthreads();  // LDS free: main loop or previous pass done
    if (threadIdx.x == 0) *reinterpret_cast<float2*>(lds_raw + zslot) = make_float2(0.f, 0.f);
    // store the lower triangle (i >= j) of this pass's walker slots
#pragma unroll
    for (int fi = 0; fi < FM; ++fi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rb + fi * 16 + r;
        const int gl = ex_div(row, rn);
        const int i0 = row - gl * n;
        const bool ok = gl < q.G && q.gt * q.G + gl < q.K;
        const int i = ok ? i0 : -1;
        const unsigned rw = (unsigned)(8 * (gl * tri + i0 * (i0 + 1) / 2));
#pragma unroll
        for (int f = 0; f < FN; ++f) {
          const unsigned a = i >= jw[f] ? rw + cw[f] : dummy;
          *reinterpret_cast<float*>(lds_raw + a) = acc[fi][f][r];
        }
      }
    __syncthreads();
    // owners of i <= j pair with T_ji, weight 2 off the diagonal and 1 on it
    // (the common factor 2 is applied at the end)
#pragma unroll
    for (int fi = 0; fi < FM; ++fi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rb + fi * 16 + r;
        const int gl = ex_div(row, rn);
        const int i0 = row - gl * n;
        const bool ok = gl < q.G && q.gt * q.G + gl < q.K;
        const int i = ok ? i0 : BIG;
        const unsigned rr = (unsigned)(8 * (gl * tri + i0));
#pragma unroll
        for (int f = 0; f < FN; ++f) {
          const int d = jr[f] - i;  // > 0 above, 0 on, < 0 below the diagonal or masked
          const unsigned a = d >= 0 ? rr + cr[f] : zslot;
          const float2 p = *reinterpret_cast<const float2*>(lds_raw + a);
          const float t = (float)min(max(d, -1), 1);
          const float v = 0.5f * fmaf(acc[fi][f][r], t, acc[fi][f][r]);  // 0, acc/2 or acc: exact
          s[f].x = fma((double)v, (double)p.x, s[f].x);
          s[f].y = fma((double)v, (double)p.y, s[f].y);
        }
      }
  }

  // column sums over the four row groups of the wave, then over the WM waves
  __syncthreads();  // read passes done: LDS reused
  double2* colsum = reinterpret_cast<double2*>(lds_raw);  // [WM][BN]
#pragma unroll
  for (int f = 0; f < FN; ++f) {
    double2 v = s[f];
    v.x += __shfl_xor(v.x, 16, 64);
    v.y += __shfl_xor(v.y, 16, 64);
    v.x += __shfl_xor(v.x, 32, 64);
    v.y += __shfl_xor(v.y, 32, 64);
    if (lane < 16) colsum[wm * BN + wn * (BN / WN) + f * 16 + lane] = v;
  }
  __syncthreads();
  for (int zt = wid; zt < q.Z; zt += NWAVE) {
    const int z = q.wt * q.Z + zt;
    if (z >= q.W) break;
    double2 t = make_double2(0.0, 0.0);
    for (int w = 0; w < WM; ++w)
      for (int o = lane; o < n2; o += 64) {
        const double2 v = colsum[w * BN + zt * n2 + o];
        if (o < n) {
          t.x += v.x;
          t.y += v.y;
        } else {
          t.x -= v.y;
          t.y += v.x;
        }
      }
    t = wave_sum2(t);
    // weights above were 1 (off the diagonal) and 1/2 (on it) of the true 2 and 1
    if (lane == 0) part[((size_t)q.sp * q.ntg + q.gt) * q.W + z] = make_double2(2.0 * t.x, 2.0 * t.y);
  }
}
