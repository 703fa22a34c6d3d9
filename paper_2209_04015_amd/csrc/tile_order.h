// Workgroup -> tile order shared by the tiled kernels.
#pragma once

#include "common.h"

// Linear block id -> (Cholesky tile, walker tile).  Workgroups are handed to
// the 8 XCDs round-robin (XCD = id % 8); XCD x gets the contiguous tile range
// [x per, (x + 1) per) and walks it in groups of GS Cholesky tiles, Cholesky
// tile fastest, so consecutive workgroups on one XCD reuse its L2.
__device__ __forceinline__ bool xcd_tile(int L, int ntg, int nwt, int GS, int& gt, int& wt) {
  const int total = ntg * nwt;
  const int per = (total + 7) / 8;
  const int j = L >> 3;
  const int t = (L & 7) * per + j;
  if (j >= per || t >= total) return false;
  const int grp_tiles = GS * nwt;
  const int grp = t / grp_tiles, r = t % grp_tiles;
  const int rows = min(GS, ntg - grp * GS);
  wt = r / rows;
  gt = grp * GS + r % rows;
  return true;
}

