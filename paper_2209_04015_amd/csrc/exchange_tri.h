// Single-pass exchange epilogue on the lower triangle of T (Sec. III.C,
// direct algorithm).  The accumulator tile holds T^{z,g}_{ij} for G whole
// Cholesky vectors (rows (g, i)) and Z whole walkers (columns
// (z, re|im, j)).  The exchange sum of one walker block is
//   sum_ij T_ij T_ji = sum_i T_ii^2 + 2 sum_{i<j} T_ij T_ji ,
// so only the lower triangle (i >= j, complex) goes through LDS: its owners
// store it, then the owners of i <= j read their partner T_ji from it and
// accumulate (FP32 FMAs over the 4 rows of a fragment, then FP64).  Per column (z, re|im, j) a thread keeps
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

// Small non-negative index products (operands below 2^23): full-rate 24-bit
// multiplies, and i (i + 1) / 2 by a shift.
__device__ __forceinline__ int ex_mul(int a, int b) { return (int)__umul24((unsigned)a, (unsigned)b); }
__device__ __forceinline__ int ex_tri(int i) { return (int)(__umul24((unsigned)i, (unsigned)(i + 1)) >> 1); }

// LDS of the epilogue: [triangles zpp * blk * 8][dummy slot per lane 256]
// [zero slot 16] ... [scale table (BM + BN) floats at tab_off]; the column
// sums [4 row groups][WM][BN] double2 reuse the start.  tab_off lies past the
// operand stage too, so the table can be filled while other waves still
// read the stage.
__host__ __device__ inline int ex_tri_area_bytes(int zpp, int G, int n) {
  return zpp * ex_tri_block(G, n) * 8 + 64 * 4 + 16;
}
__host__ __device__ inline int ex_tri_colsum_bytes(int WM, int BN) { return 4 * WM * BN * 16; }

// Writes part[(sp * ntg + gt) * W + z] for the tile's walkers.  If SCALED,
// pre_row / pre_col are this thread's entries of the scale table: the
// factors that undo the operand scaling for tile row threadIdx.x (if < BM)
// and tile column threadIdx.x (if < BN), 0 outside the problem.  zpp walker
// slots per pass.  Both passes are branch-free (masked lanes store to a
// private dummy slot, or load the zero slot), so the LDS accesses of a row
// issue back to back.
template <int BM, int BN, int WM, int WN, bool SCALED>
__device__ __forceinline__ void exchange_tri_epilogue(floatx4 (&acc)[BM / WM / 16][BN / WN / 16],
                                                      char* lds_raw, int tab_off, int zpp, const ExTriGeom& q,
                                                      float pre_row, float pre_col,
                                                      double2* __restrict__ part) {
  constexpr int NT = WM * WN * 64;
  constexpr int NWAVE = NT / 64;
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  constexpr int BIG = 1 << 20;
  static_assert(NT >= BM && NT >= BN, "one scale-table entry per thread");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int wm = wid / WN, wn = wid % WN;
  const int n = q.n, n2 = 2 * n;
  const int tri = n * (n + 1) / 2;
  const int blk = q.G * tri;
  const float rn = 1.0f / (float)n, rn2 = 1.0f / (float)n2;
  const int rbase = wm * (BM / WM) + 4 * (lane >> 4);
  const unsigned dummy = (unsigned)(zpp * blk * 8 + lane * 4);  // byte offsets
  const unsigned zslot = (unsigned)(zpp * blk * 8 + 64 * 4);
  float* tab = reinterpret_cast<float*>(lds_raw + tab_off);  // [BM] rows, [BN] columns

  if constexpr (SCALED) {
    if (tid < BM) tab[tid] = pre_row;
    if (tid < BN) tab[BM + tid] = pre_col;
  }
  // this thread's columns
  int cz[FN], cj[FN], cc[FN];
#pragma unroll
  for (int f = 0; f < FN; ++f) {
    const int c = wn * (BN / WN) + f * 16 + (lane & 15);
    const int zt = ex_div(c, rn2);
    const int o = c - ex_mul(zt, n2);
    const int comp = o >= n ? 1 : 0;
    const int z = ex_mul(q.wt, q.Z) + zt;
    cz[f] = (zt < q.Z && z < q.W) ? zt : BIG;  // outside every pass
    cj[f] = o - comp * n;
    cc[f] = comp;
  }
  // this thread's rows, one register each: bits 0-15 the row part of the
  // load offset, 8 (gl tri + i) (below 64 KB), bits 16-23 i + 1 (0 outside)
  unsigned rp[FM * 4];
#pragma unroll
  for (int fi = 0; fi < FM; ++fi)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rbase + fi * 16 + r;
      const int gl = ex_div(row, rn);
      const int i = row - ex_mul(gl, n);
      const bool ok = gl < q.G && ex_mul(q.gt, q.G) + gl < q.K;
      rp[fi * 4 + r] = (ok ? (unsigned)(8 * (ex_mul(gl, tri) + i)) : 0u) | ((ok ? (unsigned)(i + 1) : 0u) << 16);
    }
  double2 s[FN];
#pragma unroll
  for (int f = 0; f < FN; ++f) s[f] = make_double2(0.0, 0.0);

  __syncthreads();  // LDS free (main loop done), scale table filled
  if constexpr (SCALED) {  // true T = acc * row factor * column factor (powers of two: exact)
    float cs[FN];
#pragma unroll
    for (int f = 0; f < FN; ++f) cs[f] = tab[BM + wn * (BN / WN) + f * 16 + (lane & 15)];
#pragma unroll
    for (int fi = 0; fi < FM; ++fi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float rs = tab[rbase + fi * 16 + r];
#pragma unroll
        for (int f = 0; f < FN; ++f) acc[fi][f][r] *= rs * cs[f];
      }
  }

  for (int z0 = 0; z0 < q.Z; z0 += zpp) {
    // per pass and column: j bound for stores (i >= jw) and loads (i <= jr),
    // and the column's part of the LDS byte offsets
    // (in terms of i + 1 as packed in rp)
    int jw[FN], jr[FN];
    unsigned cw[FN], cr[FN];
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const int zl = cz[f] - z0;
      const bool in = zl >= 0 && zl < zpp;
      const int j = cj[f];
      jw[f] = in ? j + 1 : BIG;
      jr[f] = in ? j + 1 : -1;
      cw[f] = in ? (unsigned)(8 * (ex_mul(zl, blk) + j) + 4 * cc[f]) : 0u;
      cr[f] = in ? (unsigned)(8 * (ex_mul(zl, blk) + ex_tri(j))) : 0u;
    }
    // opaque per pass: the per-row values below stay inside the pass loop
    // (hoisted, they would take registers per row and column)
#pragma unroll
    for (int e = 0; e < FM * 4; ++e) asm volatile("" : "+v"(rp[e]));
    if (z0) __syncthreads();  // previous pass done with the LDS
    if (tid == 0) *reinterpret_cast<float2*>(lds_raw + zslot) = make_float2(0.f, 0.f);
    // store the lower triangle (i >= j) of this pass's walker slots
#pragma unroll
    for (int e = 0; e < FM * 4; ++e) {
      const int i1 = (int)(rp[e] >> 16);
      // 8 (gl tri + i (i + 1) / 2) = 8 (gl tri + i) + 4 i (i - 1)
      const unsigned rw = (rp[e] & 0xffffu) + 8u * (unsigned)ex_tri(i1 - 2);  // masked if i1 = 0
#pragma unroll
      for (int f = 0; f < FN; ++f) {
        const unsigned a = i1 >= jw[f] ? rw + cw[f] : dummy;  // i1 = 0 outside: never
        *reinterpret_cast<float*>(lds_raw + a) = acc[e >> 2][f][e & 3];
      }
    }
    __syncthreads();
    // halve the stored diagonal: below, every pair i < j counts once and the
    // total is doubled
    const int zn = min(zpp, q.Z - z0);
    for (int e = tid; e < zn * q.G * n; e += NT) {
      const int zg = ex_div(e, rn);
      const int i = e - ex_mul(zg, n);
      float2* d = reinterpret_cast<float2*>(lds_raw) + ex_mul(zg, tri) + ex_tri(i) + i;
      const float2 v = *d;
      *d = make_float2(0.5f * v.x, 0.5f * v.y);
    }
    __syncthreads();
    // owners of i <= j pair with T_ji: single-precision FMAs over the four
    // rows of a fragment, added to the double-precision column sums
#pragma unroll
    for (int fi = 0; fi < FM; ++fi) {
      float2 t[FN];
#pragma unroll
      for (int f = 0; f < FN; ++f) t[f] = make_float2(0.f, 0.f);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const unsigned pr = rp[fi * 4 + r];
        const int i1 = (int)(pr >> 16);
        const int ir = i1 > 0 ? i1 : BIG;
        const unsigned rr = pr & 0xffffu;
#pragma unroll
        for (int f = 0; f < FN; ++f) {
          const unsigned a = ir <= jr[f] ? rr + cr[f] : zslot;
          const float2 p = *reinterpret_cast<const float2*>(lds_raw + a);
          const float v = acc[fi][f][r];
          t[f].x = fmaf(v, p.x, t[f].x);
          t[f].y = fmaf(v, p.y, t[f].y);
        }
      }
#pragma unroll
      for (int f = 0; f < FN; ++f) {
        s[f].x += (double)t[f].x;
        s[f].y += (double)t[f].y;
      }
    }
  }

  // column sums: every lane's partial to LDS, then one wave per walker adds
  // the 4 row groups x WM waves x 2n columns of its block in a fixed order
  __syncthreads();  // read passes done: LDS reused
  double2* colsum = reinterpret_cast<double2*>(lds_raw);  // [4][WM][BN]
#pragma unroll
  for (int f = 0; f < FN; ++f)
    colsum[((lane >> 4) * WM + wm) * BN + wn * (BN / WN) + f * 16 + (lane & 15)] = s[f];
  __syncthreads();
  for (int zt = wid; zt < q.Z; zt += NWAVE) {
    const int z = q.wt * q.Z + zt;
    if (z >= q.W) break;
    double2 t = make_double2(0.0, 0.0);
    for (int o = lane; o < 4 * WM * n2; o += 64) {
      const int gw = ex_div(o, rn2);  // row group x wave
      const int cl = o - gw * n2;
      const double2 v = colsum[gw * BN + zt * n2 + cl];
      if (cl < n) {
        t.x += v.x;
        t.y += v.y;
      } else {
        t.x -= v.y;
        t.y += v.x;
      }
    }
    t = wave_sum2(t);
    if (lane == 0) part[((size_t)q.sp * q.ntg + q.gt) * q.W + z] = make_double2(2.0 * t.x, 2.0 * t.y);
  }
}
