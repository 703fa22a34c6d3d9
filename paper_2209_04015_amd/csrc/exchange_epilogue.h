// Epilogue shared by the exchange kernels (Sec. III.C, direct algorithm):
// the accumulator tile holds T^{z,g}_{ij} for G whole Cholesky blocks (rows
// (g, i)) and Z whole walkers (columns (z, re|im, j)); here T goes through LDS
// and every T_ij meets its partner T_ji.
//
// Decoding a row or column of the tile needs divisions by n and 2n; they are
// done once per tile into LDS tables, so the write pass does lookups only, and
// the pairing pass gives each thread one whole T row (one division per thread).
#pragma once

#include "common.h"

// LDS layout behind the T area: [row scale BM f32][col slot BN i16][col offset BN i16]
// [col scale BN f32] ... [reduction 64 double2].
constexpr int EX_TAB_BYTES = 4096;
constexpr int EX_RED_BYTES = 64 * 16;

struct ExTileGeom {
  int n, G, Z, K, W, gt, wt;
};

template <int BM, int BN>
struct ExTabs {
  float* rs;    // [BM] 1 / row scale, 0 for rows outside the problem
  short* slot;  // [BN] walker slot within the tile, -1 outside
  short* off;   // [BN] column within the walker block (re|im, j)
  float* cs;    // [BN] 1 / column scale
  __device__ ExTabs(char* base) {
    rs = reinterpret_cast<float*>(base);
    slot = reinterpret_cast<short*>(base + BM * 4);
    off = slot + BN;
    cs = reinterpret_cast<float*>(base + BM * 4 + BN * 4);
  }
};

// Fill the tables.  row_scale(g, i) and col_scale(z, comp, j) return the
// power-of-two scale of that operand row (1 when the operands are unscaled).
template <int BM, int BN, int NT, class RowScale, class ColScale>
__device__ __forceinline__ void exchange_tables(ExTabs<BM, BN> t, const ExTileGeom& q,
                                                RowScale row_scale, ColScale col_scale) {
  const int n2 = 2 * q.n;
  for (int r = threadIdx.x; r < BM; r += NT) {
    const int gl = r / q.n, i = r - gl * q.n;
    const int g = q.gt * q.G + gl;
    t.rs[r] = (gl < q.G && g < q.K) ? 1.0f / row_scale(g, i) : 0.0f;
  }
  for (int c = threadIdx.x; c < BN; c += NT) {
    const int zt = c / n2, o = c - zt * n2;
    const int z = q.wt * q.Z + zt;
    const bool ok = zt < q.Z && z < q.W;
    t.slot[c] = ok ? (short)zt : (short)-1;
    t.off[c] = (short)o;
    const int comp = o >= q.n ? 1 : 0;
    t.cs[c] = ok ? 1.0f / col_scale(z, comp, o - comp * q.n) : 0.0f;
  }
}

// Write pass of walkers [z0, z0 + zn) into lds[zz][row][col] (row stride TS).
template <typename E, typename Acc, int BM, int BN, int WM, int WN>
__device__ __forceinline__ void exchange_write(const Acc (&acc)[BM / WM / 16][BN / WN / 16], E* lds,
                                               ExTabs<BM, BN> t, int rows, int TS, int blk, int z0,
                                               int zn, bool scaled) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / WN, wn = wid % WN;
#pragma unroll
  for (int j = 0; j < BN / WN / 16; ++j) {
    const int c = wn * (BN / WN) + j * 16 + (lane & 15);
    const int zt = t.slot[c] - z0;
    if (zt < 0 || zt >= zn) continue;
    E* base = lds + zt * blk + t.off[c];
    const float cs = t.cs[c];
#pragma unroll
    for (int i = 0; i < BM / WM / 16; ++i) {
      const int mb = wm * (BM / WM) + i * 16 + 4 * (lane >> 4);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mb + r;
        if (row < rows) {
          E v = (E)acc[i][j][r];
          if (scaled) v *= (E)(t.rs[row] * cs);  // powers of two: exact
          base[row * TS] = v;
        }
      }
    }
  }
}

// Pairing pass for one walker block: sum over rows (g, i) and j of T_ij T_ji,
// one row per thread; returns this thread's share (FP64).
template <typename E>
__device__ __forceinline__ double2 exchange_pairs(const E* tb, int rows, int n, int TS) {
  double2 s = make_double2(0.0, 0.0);
  for (int row = threadIdx.x; row < rows; row += blockDim.x) {
    const int g = row / n, i = row - g * n;
    const E* ri = tb + row * TS;
    const E* rg = tb + g * n * TS;
    for (int j = 0; j < n; ++j) {
      const E* rj = rg + j * TS;
      const double ar = ri[j], ai = ri[n + j];
      const double br = rj[i], bi = rj[n + i];
      s.x += ar * br - ai * bi;
      s.y += ar * bi + ai * br;
    }
  }
  return s;
}

// Whole epilogue: tables, then passes of zpp walkers; writes
// part[(sp * ntg + gt) * W + z] for the tile's walkers.
template <typename E, typename Acc, int BM, int BN, int WM, int WN, class RowScale, class ColScale>
__device__ __forceinline__ void exchange_epilogue(const Acc (&acc)[BM / WM / 16][BN / WN / 16],
                                                  char* lds_raw, int tab_off, int red_off,
                                                  const ExTileGeom& q, int zpp, bool scaled,
                                                  RowScale row_scale, ColScale col_scale,
                                                  double2* __restrict__ part, int sp, int ntg) {
  constexpr int NT = WM * WN * 64;
  constexpr int NWAVE = NT / 64;
  const int n = q.n, n2 = 2 * n, TS = n2 + 1;
  const int rows = q.G * n;
  const int blk = rows * TS;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  E* lds = reinterpret_cast<E*>(lds_raw);
  ExTabs<BM, BN> t(lds_raw + tab_off);
  double2* red = reinterpret_cast<double2*>(lds_raw + red_off);
  __syncthreads();  // operand staging is done with the LDS
  exchange_tables<BM, BN, NT>(t, q, row_scale, col_scale);
  for (int z0 = 0; z0 < q.Z; z0 += zpp) {
    const int zn = min(zpp, q.Z - z0);
    __syncthreads();
    exchange_write<E, Acc, BM, BN, WM, WN>(acc, lds, t, rows, TS, blk, z0, zn, scaled);
    __syncthreads();
    for (int zz = 0; zz < zn; ++zz) {
      double2 s = exchange_pairs<E>(lds + zz * blk, rows, n, TS);
      s = wave_sum2(s);
      if (lane == 0) red[zz * NWAVE + wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < zn) {
      const int z = q.wt * q.Z + z0 + threadIdx.x;
      if (z < q.W) {
        double2 v = make_double2(0.0, 0.0);
        for (int w = 0; w < NWAVE; ++w) v = cadd(v, red[threadIdx.x * NWAVE + w]);  // fixed order
        part[((size_t)sp * ntg + q.gt) * q.W + z] = v;
      }
    }
  }
}
