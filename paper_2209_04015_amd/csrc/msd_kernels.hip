// Multi-determinant trial: overlap and Green's function through the
// generalised Wick's theorem (Sec. III.A, Eqs. msdovlp and msdgf0; the MSD
// numerator of Eq. gf in Sec. III.B).
//
// Per spin, with orthogonal orbitals C = [C_occ | C_virt] and the reference
// psi_0 = C_occ, theta_0 = phi (C_occ^T phi)^-1 and Y = C_virt^T theta_0
// (virtual x occupied: the contractions of the intermediate of Eq. msdgf0).
// A determinant exciting holes h_m to particles q_m has, relative to psi_0,
// the overlap ratio det A with A[l][m] = Y[q_l][h_m].  With
//   s   = sum_a c_a det A^a_a det A^b_a           (overlap ratio, Eq. msdovlp)
//   M^s = sum_a c_a det A^{other spin}_a adj(A^s_a), scattered into
//         M^s[h_m][q_l] += adj[m][l]           (hole x virtual)
// the numerator of Eq. gf divided by <psi_0|phi> s collapses to
//   G_pq = sum_j theta_0[q][j] Q[p][j],
//   Q = C_occ (I - M Y / s)^T + C_virt (M / s)^T,
// a rank-n form like the single-determinant one with C_occ replaced by a
// walker-dependent Q.  The adjugate (cofactors) stays exact for singular A.
//
// Determinants are grouped by their per-spin excitation strings: det A and
// adj A are computed once per (walker, string) and the expansion enters
// only through sparse sums in a fixed order (no atomics: results are
// deterministic).

#include "common.h"
#include "kernels.h"
#include "mfma_tile.h"

namespace {

constexpr int KM = MSD_KMAX;
constexpr int KREG = 4;      // strings of rank <= KREG: cofactors in registers
constexpr int S_T = 64;      // strings per workgroup of the rank > KREG kernel (per-thread LDS)
constexpr int C_T = 256;     // strings per workgroup of the expansion sums

// ---------------------------------------------------------------------------
// Y^s_z[i][a] = sum_p theta_0[p][i] C_virt[p][a]: one FP64 MFMA GEMM per spin
// over all walkers, A = the theta_0 rows (walker, re | im, i) with p
// contiguous, B = C_virt (k-major, a contiguous).  Y is stored planar,
// yp[z][re | im][s][i][ldv], like theta.
// ---------------------------------------------------------------------------
struct MsdYProb {
  const double* theta;
  const double* cv;  // C_virt of the spin, [N][ldv]
  int rows;          // (walker, re | im, i) rows: 2 nz nmax
  int z0, s, nmax, ldN, ldv;
  __device__ double2 load_a(int, int r, int k) const {
    if (r >= rows) return make_double2(0.0, 0.0);
    const int zc = r / nmax, i = r - zc * nmax;  // zc = 2 (z - z0) + (re | im)
    const size_t plane = (size_t)nmax * ldN;
    return *reinterpret_cast<const double2*>(theta + ((size_t)(2 * z0 + zc) * 2 + s) * plane + (size_t)i * ldN + k);
  }
  __device__ double2 load_b_km(int, int k, int a) const {
    if (a >= ldv) return make_double2(0.0, 0.0);
    return *reinterpret_cast<const double2*>(cv + (size_t)k * ldv + a);
  }
};

constexpr int YBM = 64, YBN = 64, YBK = 16, YWM = 2, YWN = 2;

__global__ __launch_bounds__(YWM* YWN * 64) void msd_y_kernel(MsdDims m, MsdYProb p, double* __restrict__ yp) {
  __shared__ __attribute__((aligned(16))) double lds[TileLds<double, YBM, YBN, YBK>::ELEMS];
  MF<double>::acc_t acc[YBM / YWM / 16][YBN / YWN / 16];
  const int m0 = blockIdx.x * YBM, n0 = blockIdx.y * YBN;
  mfma_tile_mainloop<double, YBM, YBN, YBK, YWM, YWN, true>(p, 0, m0, n0, m.N, acc, lds);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / YWN, wn = wid % YWN;
  const int nv = m.nv[p.s];
  const size_t yplane = (size_t)m.nmax * m.ldv;
#pragma unroll
  for (int i = 0; i < YBM / YWM / 16; ++i)
#pragma unroll
    for (int j = 0; j < YBN / YWN / 16; ++j) {
      const int rb = m0 + wm * (YBM / YWM) + i * 16 + 4 * (lane >> 4);
      const int a = n0 + wn * (YBN / YWN) + j * 16 + (lane & 15);
      if (a >= nv) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rb + r;
        if (row >= p.rows) continue;
        const int zc = row / m.nmax, ii = row - zc * m.nmax;
        yp[((size_t)(2 * p.z0 + zc) * 2 + p.s) * yplane + (size_t)ii * m.ldv + a] = acc[i][j][r];
      }
    }
}

// complex Y^s_z[i][a] from the planar store
struct YView {
  const double* re;
  const double* im;
  int ldv;
  __device__ __forceinline__ double2 operator()(int i, int a) const {
    const size_t o = (size_t)i * ldv + a;
    return make_double2(re[o], im[o]);
  }
};
__device__ __forceinline__ YView y_view(const MsdDims& m, const double* yp, int z, int s) {
  const size_t yplane = (size_t)m.nmax * m.ldv;
  return YView{yp + ((size_t)(2 * z + 0) * 2 + s) * yplane, yp + ((size_t)(2 * z + 1) * 2 + s) * yplane, m.ldv};
}

// ---------------------------------------------------------------------------
// det and adjugate of one string's k x k matrix A, A[l][c] = Y[q_l][h_c];
// adj(A)[c][l] = (-1)^(l+c) det(A without row l, column c) is stored at
// sadj[aoff + c k + l].
// ---------------------------------------------------------------------------

__device__ __forceinline__ double2 cneg(double2 a) { return make_double2(-a.x, -a.y); }

template <int K>
struct SmallDet;
template <>
struct SmallDet<1> {
  static __device__ __forceinline__ double2 det(const double2 (&a)[1][1]) { return a[0][0]; }
};
template <>
struct SmallDet<2> {
  static __device__ __forceinline__ double2 det(const double2 (&a)[2][2]) {
    return csub(cmul(a[0][0], a[1][1]), cmul(a[0][1], a[1][0]));
  }
};
template <>
struct SmallDet<3> {
  static __device__ __forceinline__ double2 det(const double2 (&a)[3][3]) {
    const double2 c0 = csub(cmul(a[1][1], a[2][2]), cmul(a[1][2], a[2][1]));
    const double2 c1 = csub(cmul(a[1][0], a[2][2]), cmul(a[1][2], a[2][0]));
    const double2 c2 = csub(cmul(a[1][0], a[2][1]), cmul(a[1][1], a[2][0]));
    return cadd(csub(cmul(a[0][0], c0), cmul(a[0][1], c1)), cmul(a[0][2], c2));
  }
};

// Cofactors in registers (fully unrolled: every index is a constant).  ADJ
// false: only the row-0 cofactors of the Laplace expansion (det alone).
template <int K, bool ADJ>
__device__ __forceinline__ double2 det_adj_reg(const YView& Y, const int* holes, const int* parts,
                                               double2* __restrict__ adj) {
  double2 a[K][K];
  int h[K], q[K];
#pragma unroll
  for (int x = 0; x < K; ++x) {
    h[x] = holes[x];
    q[x] = parts[x];
  }
#pragma unroll
  for (int l = 0; l < K; ++l)
#pragma unroll
    for (int c = 0; c < K; ++c) a[l][c] = Y(h[c], q[l]);
  if constexpr (K == 1) {
    if constexpr (ADJ) adj[0] = make_double2(1.0, 0.0);
    return a[0][0];
  } else {
    double2 det = make_double2(0.0, 0.0);
#pragma unroll
    for (int l = 0; l < (ADJ ? K : 1); ++l)
#pragma unroll
      for (int c = 0; c < K; ++c) {
        double2 mi[K - 1][K - 1];
#pragma unroll
        for (int r = 0; r < K - 1; ++r)
#pragma unroll
          for (int x = 0; x < K - 1; ++x) mi[r][x] = a[r < l ? r : r + 1][x < c ? x : x + 1];
        double2 cof = SmallDet<K - 1>::det(mi);
        if ((l + c) & 1) cof = cneg(cof);
        if constexpr (ADJ) adj[c * K + l] = cof;
        if (l == 0) det = cadd(det, cmul(a[0][c], cof));  // Laplace along row 0
      }
    return det;
  }
}

// Strings of rank <= KREG, one thread per (walker, string).  The strings of
// a spin are sorted by rank, so a wave takes one branch except at the few
// rank boundaries.
template <bool ADJ>
__global__ __launch_bounds__(256) void msd_strings_kernel(MsdDims m, int z0, const int* __restrict__ srank,
                                                          const int* __restrict__ sorb,
                                                          const int* __restrict__ saoff,
                                                          const double* __restrict__ yp,
                                                          double2* __restrict__ sdet,
                                                          double2* __restrict__ sadj) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const int z = z0 + (int)blockIdx.y;
  if (u >= m.nstr_tot) return;
  const int k = srank[u];
  if (k > KREG) return;  // msd_strings_big_kernel
  const int s = u >= m.nstr[0] ? 1 : 0;
  const int* holes = sorb + (size_t)u * 2 * KM;
  const int* parts = holes + KM;
  const YView Y = y_view(m, yp, z, s);
  double2* adj = sadj + (size_t)z * m.nadj_tot + saoff[u];
  double2 det;
  switch (k) {
    case 1: det = det_adj_reg<1, ADJ>(Y, holes, parts, adj); break;
    case 2: det = det_adj_reg<2, ADJ>(Y, holes, parts, adj); break;
    case 3: det = det_adj_reg<3, ADJ>(Y, holes, parts, adj); break;
    case 4: det = det_adj_reg<4, ADJ>(Y, holes, parts, adj); break;
    default: det = make_double2(1.0, 0.0); break;  // the reference string
  }
  sdet[(size_t)z * m.nstr_tot + u] = det;
}

// Determinant of the k x k matrix in w (element e at w[e * S_T]) by Gaussian
// elimination with partial pivoting; w is overwritten.
__device__ double2 det_in_place(double2* w, int k) {
  double2 det = make_double2(1.0, 0.0);
  for (int c = 0; c < k; ++c) {
    int piv = c;
    double best = cabs2(w[(c * k + c) * S_T]);
    for (int r = c + 1; r < k; ++r) {
      const double v = cabs2(w[(r * k + c) * S_T]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
    if (best == 0.0) return make_double2(0.0, 0.0);
    if (piv != c) {
      for (int x = c; x < k; ++x) {
        const double2 t = w[(c * k + x) * S_T];
        w[(c * k + x) * S_T] = w[(piv * k + x) * S_T];
        w[(piv * k + x) * S_T] = t;
      }
      det = cneg(det);
    }
    const double2 pv = w[(c * k + c) * S_T];
    det = cmul(det, pv);
    const double2 ipv = cinv(pv);
    for (int r = c + 1; r < k; ++r) {
      const double2 f = cmul(w[(r * k + c) * S_T], ipv);
      for (int x = c + 1; x < k; ++x) w[(r * k + x) * S_T] = csub(w[(r * k + x) * S_T], cmul(f, w[(c * k + x) * S_T]));
    }
  }
  return det;
}

// Strings of rank KREG + 1 .. MSD_KMAX (the last ones of each spin after the
// sort): minors by pivoted elimination in per-thread LDS slots.
__global__ __launch_bounds__(S_T) void msd_strings_big_kernel(MsdDims m, int z0, const int* __restrict__ srank,
                                                              const int* __restrict__ sorb,
                                                              const int* __restrict__ saoff,
                                                              const double* __restrict__ yp,
                                                              double2* __restrict__ sdet,
                                                              double2* __restrict__ sadj, int want_adj) {
  // A and one minor per thread: (36 + 25) x 64 x 16 B = 62.5 KB
  __shared__ double2 lds_a[KM * KM * S_T];
  __shared__ double2 lds_w[(KM - 1) * (KM - 1) * S_T];
  const int lane = threadIdx.x;
  const int z = z0 + (int)(blockIdx.y >> 1), s = blockIdx.y & 1;
  const int loc = blockIdx.x * S_T + lane;
  if (loc >= m.nbig[s]) return;  // no barrier below: every thread works on its own LDS slots
  const int u = m.big0[s] + loc;
  const int k = srank[u];
  const int* holes = sorb + (size_t)u * 2 * KM;
  const int* parts = holes + KM;
  const YView Y = y_view(m, yp, z, s);
  double2* A = lds_a + lane;
  double2* Wk = lds_w + lane;
  for (int l = 0; l < k; ++l)
    for (int c = 0; c < k; ++c) A[(l * k + c) * S_T] = Y(holes[c], parts[l]);
  double2* adj = sadj + (size_t)z * m.nadj_tot + saoff[u];
  const int k1 = k - 1;
  for (int l = 0; l < (want_adj ? k : 0); ++l) {
    for (int c = 0; c < k; ++c) {
      int e = 0;
      for (int r = 0; r < k; ++r) {
        if (r == l) continue;
        for (int x = 0; x < k; ++x) {
          if (x == c) continue;
          Wk[e * S_T] = A[(r * k + x) * S_T];
          ++e;
        }
      }
      double2 minor = det_in_place(Wk, k1);
      if ((l + c) & 1) minor = cneg(minor);
      adj[c * k + l] = minor;
    }
  }
  sdet[(size_t)z * m.nstr_tot + u] = det_in_place(A, k);  // last: A is not needed afterwards
}

// ---------------------------------------------------------------------------
// Expansion sums: for a string u of spin s,
//   uw[u] = sum over determinants a with that string of c_a det A^{other}_a
// (CSR rows in increasing a).  A row can hold thousands of determinants (the
// reference string pairs with every excitation of the other spin), so rows
// are cut into tasks of at most MSD_TASK entries: msd_task_kernel sums each
// task, msd_combine_kernel adds a string's tasks in order and writes the
// workgroup's partial sum of det A_u uw[u] over its alpha strings;
// msd_ratio_kernel adds the partials of a walker in workgroup order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void msd_task_kernel(MsdDims m, int z0, const int* __restrict__ tbeg,
                                                       const double* __restrict__ ccoef,
                                                       const int* __restrict__ cstr,
                                                       const double2* __restrict__ sdet,
                                                       double2* __restrict__ tpart) {
  const int z = z0 + (int)blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m.ntask) return;
  const double2* dz = sdet + (size_t)z * m.nstr_tot;
  double2 acc = make_double2(0.0, 0.0);
  for (int e = tbeg[t]; e < tbeg[t + 1]; ++e) {
    const double2 d = dz[cstr[e]];
    acc.x = fma(ccoef[e], d.x, acc.x);
    acc.y = fma(ccoef[e], d.y, acc.y);
  }
  tpart[(size_t)z * m.ntask + t] = acc;
}

__global__ __launch_bounds__(C_T) void msd_combine_kernel(MsdDims m, int z0, const int* __restrict__ trow,
                                                          const double2* __restrict__ tpart,
                                                          const double2* __restrict__ sdet,
                                                          double2* __restrict__ uw,
                                                          double2* __restrict__ rpart) {
  __shared__ double2 red[C_T / 64];
  const int z = z0 + (int)blockIdx.y;
  const int u = blockIdx.x * C_T + threadIdx.x;
  double2 part = make_double2(0.0, 0.0);
  if (u < m.nstr_tot) {
    const double2* tz = tpart + (size_t)z * m.ntask;
    double2 acc = make_double2(0.0, 0.0);
    for (int t = trow[u]; t < trow[u + 1]; ++t) acc = cadd(acc, tz[t]);
    uw[(size_t)z * m.nstr_tot + u] = acc;
    if (u < m.nstr[0]) part = cmul(sdet[(size_t)z * m.nstr_tot + u], acc);
  }
  const double2 tot = block_sum2(part, red);
  if (threadIdx.x == 0) rpart[(size_t)z * gridDim.x + blockIdx.x] = tot;
}

__global__ void msd_ratio_kernel(int z0, int nz, int nblk, const double2* __restrict__ rpart,
                                 double2* __restrict__ ratio) {
  const int z = z0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (z >= z0 + nz) return;
  double2 t = make_double2(0.0, 0.0);
  for (int b = 0; b < nblk; ++b) t = cadd(t, rpart[(size_t)z * nblk + b]);
  ratio[z] = t;
}

// ---------------------------------------------------------------------------
// M^s[j][a] = sum over (string u, adjugate slot) entries of uw[u] adj_u[slot]
// (CSR per (j, a) entry of the spin, fixed order), divided by s_z and stored
// as the virtual columns of Zt: zt[z][re | im][s][j][n + a] (planar, theta's
// layout).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void msd_m_kernel(MsdDims m, int z0, const int* __restrict__ erow,
                                                    const int* __restrict__ estr, const int* __restrict__ eoff,
                                                    const double2* __restrict__ uw,
                                                    const double2* __restrict__ sadj,
                                                    const double2* __restrict__ ratio, double* __restrict__ zt) {
  const int z = z0 + (int)(blockIdx.y >> 1), s = blockIdx.y & 1;
  const int n = s ? m.nb : m.na, nv = m.nv[s];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nv) return;
  const int j = e / nv, a = e - j * nv;
  const int r = (s ? m.na * m.nv[0] : 0) + e;
  const double2* uz = uw + (size_t)z * m.nstr_tot;
  const double2* az = sadj + (size_t)z * m.nadj_tot;
  double2 acc = make_double2(0.0, 0.0);
  for (int x = erow[r]; x < erow[r + 1]; ++x) acc = cadd(acc, cmul(uz[estr[x]], az[eoff[x]]));
  acc = cmul(acc, cinv(ratio[z]));
  const size_t plane = (size_t)m.nmax * m.ldN;
  const size_t o = (size_t)j * m.ldN + n + a;
  zt[((size_t)(2 * z + 0) * 2 + s) * plane + o] = acc.x;
  zt[((size_t)(2 * z + 1) * 2 + s) * plane + o] = acc.y;
}

// ---------------------------------------------------------------------------
// Occupied columns of Zt: Zt[j][i] = delta_ji - sum_a Zt[j][n + a] Y[a][i]
// (= delta_ji - (M Y)[j][i] / s_z), one small real GEMM per (walker, spin)
// over k = (re | im, a): A row j = [Zr[j], Zi[j]] (virtual columns), B column
// 2i = [Yr[i], -Yi[i]] and 2i + 1 = [Yi[i], Yr[i]] (real and imaginary parts).
// ---------------------------------------------------------------------------
struct MsdZProb {
  const double* zt;
  const double* yp;
  int z0, nmax, ldN, ldv, na, nb, nv0, nv1;
  __device__ double2 load_a(int b, int j, int k) const {
    const int z = z0 + (b >> 1), s = b & 1;
    const int n = s ? nb : na, nv = s ? nv1 : nv0;
    const int c = k < ldv ? 0 : 1, a = k - c * ldv;
    if (j >= n) return make_double2(0.0, 0.0);
    const double* row = zt + ((size_t)(2 * z + c) * 2 + s) * nmax * ldN + (size_t)j * ldN + n;
    return make_double2(a < nv ? row[a] : 0.0, a + 1 < nv ? row[a + 1] : 0.0);
  }
  __device__ double2 load_b(int b, int col, int k) const {
    const int z = z0 + (b >> 1), s = b & 1;
    const int n = s ? nb : na;
    const int i = col >> 1, part = col & 1;
    const int c = k < ldv ? 0 : 1, a = k - c * ldv;  // a even, a + 1 < ldv (ldv a multiple of 4)
    if (i >= n) return make_double2(0.0, 0.0);
    const size_t yplane = (size_t)nmax * ldv;
    const double2 yr = *reinterpret_cast<const double2*>(yp + ((size_t)(2 * z + 0) * 2 + s) * yplane + (size_t)i * ldv + a);
    const double2 yi = *reinterpret_cast<const double2*>(yp + ((size_t)(2 * z + 1) * 2 + s) * yplane + (size_t)i * ldv + a);
    // Y entries a >= nv are zero (never written), so no guard is needed here
    if (part == 0) return c == 0 ? yr : make_double2(-yi.x, -yi.y);
    return c == 0 ? yi : yr;
  }
};

constexpr int ZBM = 64, ZBN = 64, ZBK = 16, ZWM = 2, ZWN = 2;

__global__ __launch_bounds__(ZWM* ZWN * 64) void msd_zocc_kernel(MsdDims m, MsdZProb p, double* __restrict__ zt) {
  __shared__ __attribute__((aligned(16))) double lds[TileLds<double, ZBM, ZBN, ZBK>::ELEMS];
  MF<double>::acc_t acc[ZBM / ZWM / 16][ZBN / ZWN / 16];
  const int b = blockIdx.z;
  const int m0 = blockIdx.x * ZBM, n0 = blockIdx.y * ZBN;
  mfma_tile_mainloop<double, ZBM, ZBN, ZBK, ZWM, ZWN, false>(p, b, m0, n0, 2 * m.ldv, acc, lds);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / ZWN, wn = wid % ZWN;
  const int z = p.z0 + (b >> 1), s = b & 1;
  const int n = s ? m.nb : m.na;
  const size_t plane = (size_t)m.nmax * m.ldN;
#pragma unroll
  for (int i = 0; i < ZBM / ZWM / 16; ++i)
#pragma unroll
    for (int jj = 0; jj < ZBN / ZWN / 16; ++jj) {
      const int jb = m0 + wm * (ZBM / ZWM) + i * 16 + 4 * (lane >> 4);
      const int col = n0 + wn * (ZBN / ZWN) + jj * 16 + (lane & 15);
      const int ii = col >> 1, part = col & 1;
      if (ii >= n) continue;
      double* dst = zt + ((size_t)(2 * z + part) * 2 + s) * plane + ii;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jb + r;
        if (j < n) dst[(size_t)j * m.ldN] = (part == 0 && j == ii ? 1.0 : 0.0) - acc[i][jj][r];
      }
    }
}

// ---------------------------------------------------------------------------
// Q[p][j] = sum_x C[p][x] Zt[j][x]: one FP64 MFMA GEMM per spin, A = C of
// the spin ([N][ldN], x contiguous), B = the Zt rows (walker, re | im, j).
// Q is stored planar, qp[z][re | im][s][p][ldq] (ldq = nmax rounded up to 2;
// columns j >= n stay zero).
// ---------------------------------------------------------------------------
struct MsdQProb {
  const double* cf;  // C of the spin, [N][ldN]
  const double* zt;
  int N, rows;       // B rows: 2 nz nmax
  int z0, s, nmax, ldN;
  __device__ double2 load_a(int, int p, int k) const {
    if (p >= N) return make_double2(0.0, 0.0);
    return *reinterpret_cast<const double2*>(cf + (size_t)p * ldN + k);
  }
  __device__ double2 load_b(int, int r, int k) const {
    if (r >= rows) return make_double2(0.0, 0.0);
    const int zc = r / nmax, j = r - zc * nmax;
    const size_t plane = (size_t)nmax * ldN;
    return *reinterpret_cast<const double2*>(zt + ((size_t)(2 * z0 + zc) * 2 + s) * plane + (size_t)j * ldN + k);
  }
};

constexpr int GBM = 64, GBN = 64, GBK = 16, GWM = 2, GWN = 2;

__global__ __launch_bounds__(GWM* GWN * 64) void msd_q_kernel(MsdDims m, MsdQProb p, double* __restrict__ qp) {
  __shared__ __attribute__((aligned(16))) double lds[TileLds<double, GBM, GBN, GBK>::ELEMS];
  MF<double>::acc_t acc[GBM / GWM / 16][GBN / GWN / 16];
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  mfma_tile_mainloop<double, GBM, GBN, GBK, GWM, GWN, false>(p, 0, m0, n0, m.N, acc, lds);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / GWN, wn = wid % GWN;
  const int n = p.s ? m.nb : m.na;
#pragma unroll
  for (int i = 0; i < GBM / GWM / 16; ++i)
#pragma unroll
    for (int jj = 0; jj < GBN / GWN / 16; ++jj) {
      const int pb = m0 + wm * (GBM / GWM) + i * 16 + 4 * (lane >> 4);
      const int col = n0 + wn * (GBN / GWN) + jj * 16 + (lane & 15);
      if (col >= p.rows) continue;
      const int zc = col / m.nmax, j = col - zc * m.nmax;
      if (j >= n) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = pb + r;
        if (row < m.N) qp[(((size_t)(2 * p.z0 + zc) * 2 + p.s) * m.N + row) * m.ldq + j] = acc[i][jj][r];
      }
    }
}

// ---------------------------------------------------------------------------
// G[z][s][p][q] = sum_j Q[p][j] theta_0[q][j] as a real GEMM per (walker,
// spin) over k = (re | im, j) (ldq values each): A row p = [Q_re[p], Q_im[p]],
// B column 2q = [theta_re[q], -theta_im[q]] (real part) and 2q + 1 =
// [theta_im[q], theta_re[q]] (imaginary part).  Output columns 2q, 2q + 1 are
// the real and imaginary parts of G[p][q], so the stores are contiguous.
// ---------------------------------------------------------------------------
struct MsdGProb {
  const double* qp;
  const double* theta;
  int N, nmax, ldN, ldq, z0;
  __device__ double2 load_a(int b, int p, int k) const {
    if (p >= N) return make_double2(0.0, 0.0);
    const int z = z0 + (b >> 1), s = b & 1;
    const int c = k < ldq ? 0 : 1, kk = k - c * ldq;
    return *reinterpret_cast<const double2*>(qp + (((size_t)(2 * z + c) * 2 + s) * N + p) * ldq + kk);
  }
  __device__ double2 load_b_km(int b, int k, int col) const {
    const int q = col >> 1;
    const int c = k < ldq ? 0 : 1, j = k - c * ldq;
    if (q >= N || j >= nmax) return make_double2(0.0, 0.0);
    const int z = z0 + (b >> 1), s = b & 1;
    const size_t plane = (size_t)nmax * ldN;
    const double tr = theta[((size_t)(2 * z + 0) * 2 + s) * plane + (size_t)j * ldN + q];
    const double ti = theta[((size_t)(2 * z + 1) * 2 + s) * plane + (size_t)j * ldN + q];
    return c == 0 ? make_double2(tr, ti) : make_double2(-ti, tr);
  }
};

// Workgroups are dispatched to the 8 XCDs in turn (XCD = linear id mod 8);
// the tiles of one (walker, spin) are given ids with the same residue, so
// its Q and theta are read into one XCD's L2 only.
constexpr int NXCD = 8;

__global__ __launch_bounds__(GWM* GWN * 64) void msd_green_kernel(MsdDims m, MsdGProb p, int nbatch, int mt, int ntile,
                                                                  double* __restrict__ G) {
  __shared__ __attribute__((aligned(16))) double lds[TileLds<double, GBM, GBN, GBK>::ELEMS];
  MF<double>::acc_t acc[GBM / GWM / 16][GBN / GWN / 16];
  const int L = blockIdx.x;
  const int xcd = L % NXCD, r = L / NXCD;
  const int t = r % ntile;
  const int b = xcd + NXCD * (r / ntile);
  if (b >= nbatch) return;  // whole workgroup, before any barrier
  const int m0 = (t % mt) * GBM, n0 = (t / mt) * GBN;
  mfma_tile_mainloop<double, GBM, GBN, GBK, GWM, GWN, true>(p, b, m0, n0, 2 * m.ldq, acc, lds);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / GWN, wn = wid % GWN;
  const int z = p.z0 + (b >> 1), s = b & 1;
  double* out = G + ((size_t)z * 2 + s) * m.N * 2 * m.N;
#pragma unroll
  for (int i = 0; i < GBM / GWM / 16; ++i)
#pragma unroll
    for (int jj = 0; jj < GBN / GWN / 16; ++jj) {
      const int pb = m0 + wm * (GBM / GWM) + i * 16 + 4 * (lane >> 4);
      const int col = n0 + wn * (GBN / GWN) + jj * 16 + (lane & 15);
      if (col >= 2 * m.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (pb + r < m.N) out[(size_t)(pb + r) * 2 * m.N + col] = acc[i][jj][r];
    }
}

// ---------------------------------------------------------------------------
// Force bias of the multi-determinant trial (Eq. fb with the MSD G):
//   vbias_g = sum_s sum_pq G^s_pq L_g,pq = sum_{p <= q} L_g,pq c_pq Gsym_pq,
//   Gsym = sum_s (G^s + G^s^T), c = 1 (p < q) or 1/2 (p = q),
// with G^s_pq = sum_j Q^s[p][j] theta_0^s[q][j], so that
//   Gsym_pq = sum_s sum_j (Q^s[p][j] theta^s[q][j] + theta^s[p][j] Q^s[q][j]).
// msd_gsym_kernel forms the packed c Gsym (upper triangle, the row order of
// the packed L) as one real GEMM per walker over
// k = (spin, half, re | im of the A factor, j): A row p = Q[p] (half 0) or
// theta[p] (half 1), B column 2q (+1) = the real (imaginary) part of the
// product with theta[q] (half 0) or Q[q] (half 1).  Tiles entirely below
// the diagonal are skipped.
// ---------------------------------------------------------------------------
struct MsdSProb {
  const double* qp;
  const double* theta;
  int N, nmax, ldN, ldq, z0;
  __device__ double2 load_a(int b, int p, int k) const {
    if (p >= N) return make_double2(0.0, 0.0);
    const int z = z0 + b;
    const int j = k % ldq, t = k / ldq;  // j even: ldq and k are even
    const int c = t & 1, h = (t >> 1) & 1, s = t >> 2;
    if (h == 0)
      return *reinterpret_cast<const double2*>(qp + (((size_t)(2 * z + c) * 2 + s) * N + p) * ldq + j);
    const double* th = theta + ((size_t)(2 * z + c) * 2 + s) * nmax * ldN + p;
    return make_double2(j < nmax ? th[(size_t)j * ldN] : 0.0, j + 1 < nmax ? th[(size_t)(j + 1) * ldN] : 0.0);
  }
  __device__ double2 load_b_km(int b, int k, int col) const {
    const int q = col >> 1;
    const int j = k % ldq, t = k / ldq;
    const int c = t & 1, h = (t >> 1) & 1, s = t >> 2;
    if (q >= N) return make_double2(0.0, 0.0);
    const int z = z0 + b;
    double br, bi;
    if (h == 0) {
      if (j >= nmax) return make_double2(0.0, 0.0);
      const size_t plane = (size_t)nmax * ldN;
      br = theta[((size_t)(2 * z + 0) * 2 + s) * plane + (size_t)j * ldN + q];
      bi = theta[((size_t)(2 * z + 1) * 2 + s) * plane + (size_t)j * ldN + q];
    } else {
      br = qp[(((size_t)(2 * z + 0) * 2 + s) * N + q) * ldq + j];
      bi = qp[(((size_t)(2 * z + 1) * 2 + s) * N + q) * ldq + j];
    }
    return c == 0 ? make_double2(br, bi) : make_double2(-bi, br);
  }
};

template <typename GT>
__global__ __launch_bounds__(GWM* GWN * 64) void msd_gsym_kernel(MsdDims m, MsdSProb p, int nz, int mt, int ntile,
                                                                 int ldpk, GT* __restrict__ gs) {
  __shared__ __attribute__((aligned(16))) double lds[TileLds<double, GBM, GBN, GBK>::ELEMS];
  MF<double>::acc_t acc[GBM / GWM / 16][GBN / GWN / 16];
  const int L = blockIdx.x;
  const int xcd = L % NXCD, r = L / NXCD;
  const int t = r % ntile;
  const int b = xcd + NXCD * (r / ntile);  // walker - z0: tiles of a walker on one XCD
  if (b >= nz) return;
  const int m0 = (t % mt) * GBM, n0 = (t / mt) * GBN;
  if (m0 > (n0 + GBN - 1) / 2) return;  // every p > every q of the tile
  mfma_tile_mainloop<double, GBM, GBN, GBK, GWM, GWN, true>(p, b, m0, n0, 8 * m.ldq, acc, lds);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / GWN, wn = wid % GWN;
  const int z = p.z0 + b;
  const int N = m.N;
#pragma unroll
  for (int i = 0; i < GBM / GWM / 16; ++i)
#pragma unroll
    for (int jj = 0; jj < GBN / GWN / 16; ++jj) {
      const int pb = m0 + wm * (GBM / GWM) + i * 16 + 4 * (lane >> 4);
      const int col = n0 + wn * (GBN / GWN) + jj * 16 + (lane & 15);
      const int q = col >> 1, part = col & 1;
      if (q >= N) continue;
      GT* dst = gs + (size_t)(2 * z + part) * ldpk;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int pp = pb + rr;
        if (pp > q) continue;
        const long idx = (long)pp * (2 * N - pp + 1) / 2 + (q - pp);  // row-major upper triangle
        dst[idx] = (GT)((pp == q ? 0.5 : 1.0) * acc[i][jj][rr]);
      }
    }
}

// vbias rows (z, re | im) = gs rows . packed L, split over the pair index into
// nsplit ranges of `chunk` pairs; partials fbp[split][2 z + c][ldK].  T is the
// type of both operands (FP64, or FP32 with the FP32 packed L of the mixed
// paths; accumulation in T on the matrix cores, partials summed in FP64).
template <typename T>
struct MsdFbProb {
  using vec_t = typename MF<T>::vec_t;
  static constexpr int VEC = MF<T>::VEC;
  const T* gs;
  const T* lt;
  int rows, ldpk, ldK, z0, chunk, npk;
  __device__ vec_t load_a(int split, int r, int k) const {
    if (r >= rows) return MF<T>::vzero();
    const int kk = split * chunk + k;
    const T* row = gs + (size_t)(2 * z0 + r) * ldpk;
    // entries past the packed triangle are not written (the scratch is reused): read as zero
    if (kk + VEC > npk) {
      T v[4] = {T(0), T(0), T(0), T(0)};
      for (int e = 0; e < VEC; ++e)
        if (kk + e < npk) v[e] = row[kk + e];
      if constexpr (VEC == 4)
        return make_float4(v[0], v[1], v[2], v[3]);
      else
        return make_double2(v[0], v[1]);
    }
    return *reinterpret_cast<const vec_t*>(row + kk);
  }
  __device__ vec_t load_b_km(int split, int k, int g) const {
    if (g >= ldK) return MF<T>::vzero();
    return *reinterpret_cast<const vec_t*>(lt + ((size_t)split * chunk + k) * ldK + g);
  }
};

template <typename T>
__global__ __launch_bounds__(GWM* GWN * 64) void msd_fb_kernel(MsdFbProb<T> p, int npk, int K, int W,
                                                               double* __restrict__ fbp) {
  constexpr int BK = sizeof(T) == 4 ? 32 : 16;
  __shared__ __attribute__((aligned(16))) T lds[TileLds<T, GBM, GBN, BK>::ELEMS];
  typename MF<T>::acc_t acc[GBM / GWM / 16][GBN / GWN / 16];
  const int split = blockIdx.z;
  const int k0 = split * p.chunk;
  const int kdim = npk - k0 < p.chunk ? npk - k0 : p.chunk;
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  mfma_tile_mainloop<T, GBM, GBN, BK, GWM, GWN, true>(p, split, m0, n0, kdim, acc, lds);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / GWN, wn = wid % GWN;
  double* out = fbp + (size_t)split * 2 * W * p.ldK;
#pragma unroll
  for (int i = 0; i < GBM / GWM / 16; ++i)
#pragma unroll
    for (int jj = 0; jj < GBN / GWN / 16; ++jj) {
      const int rb = m0 + wm * (GBM / GWM) + i * 16 + 4 * (lane >> 4);
      const int g = n0 + wn * (GBN / GWN) + jj * 16 + (lane & 15);
      if (g >= K) continue;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        if (rb + rr < p.rows) out[(size_t)(2 * p.z0 + rb + rr) * p.ldK + g] = (double)acc[i][jj][rr];
    }
}

// vbias[z][g] = sum over splits, in order, of the (re, im) partial rows
__global__ void msd_fb_reduce_kernel(int W, int K, int ldK, int nsplit, const double* __restrict__ fbp,
                                     double2* __restrict__ vbias) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)W * K) return;
  const int z = (int)(e / K), g = (int)(e - (long)z * K);
  double re = 0.0, im = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) {
    const double* o = fbp + (size_t)sp * 2 * W * ldK;
    re += o[(size_t)(2 * z) * ldK + g];
    im += o[(size_t)(2 * z + 1) * ldK + g];
  }
  vbias[e] = make_double2(re, im);
}

// log <Psi_T|phi_z> = log det S^a + log det S^b + log s_z
__global__ void msd_overlap_kernel(int W, const double2* __restrict__ logdet, const double2* __restrict__ ratio,
                                   double2* __restrict__ out, int* __restrict__ status) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= W) return;
  const double2 r = ratio[z];
  double2 lo = cadd(logdet[2 * z], logdet[2 * z + 1]);
  if (cabs2(r) == 0.0) {
    lo = make_double2(-INFINITY, 0.0);
    atomicOr(status, AFQMC_STATUS_SINGULAR);
  } else {
    lo = cadd(lo, clog(r));
  }
  out[z] = lo;
}

constexpr int ZCHUNK = 16384;  // walkers per launch (grid y, z <= 2 per walker)

}  // namespace

int msd_combine_blocks(const MsdDims& m) { return (m.nstr_tot + C_T - 1) / C_T; }

hipError_t launch_msd_ratio(const MsdDims& m, int W, const MsdTables& t, const double* theta, double* yp,
                            double2* sdet, double2* sadj, double2* tpart, double2* uw, double2* rpart,
                            double2* ratio, bool want_adj, hipStream_t s) {
  const int nblk = msd_combine_blocks(m);
  for (int z0 = 0; z0 < W; z0 += ZCHUNK) {
    const int nz = W - z0 < ZCHUNK ? W - z0 : ZCHUNK;
    hipError_t e;
    for (int sp = 0; sp < 2; ++sp) {
      if ((sp ? m.nb : m.na) == 0 || m.nv[sp] == 0) continue;
      MsdYProb p{theta, t.cvirt + (size_t)sp * m.N * m.ldv, 2 * nz * m.nmax, z0, sp, m.nmax, m.ldN, m.ldv};
      const dim3 grid((p.rows + YBM - 1) / YBM, (m.nv[sp] + YBN - 1) / YBN);
      hipLaunchKernelGGL(msd_y_kernel, grid, dim3(YWM * YWN * 64), 0, s, m, p, yp);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (want_adj)
      hipLaunchKernelGGL(msd_strings_kernel<true>, dim3((m.nstr_tot + 255) / 256, nz), dim3(256), 0, s, m, z0,
                         t.srank, t.sorb, t.saoff, yp, sdet, sadj);
    else
      hipLaunchKernelGGL(msd_strings_kernel<false>, dim3((m.nstr_tot + 255) / 256, nz), dim3(256), 0, s, m, z0,
                         t.srank, t.sorb, t.saoff, yp, sdet, sadj);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nbig = m.nbig[0] > m.nbig[1] ? m.nbig[0] : m.nbig[1];
    if (nbig > 0) {
      hipLaunchKernelGGL(msd_strings_big_kernel, dim3((nbig + S_T - 1) / S_T, 2 * nz), dim3(S_T), 0, s, m, z0,
                         t.srank, t.sorb, t.saoff, yp, sdet, sadj, want_adj ? 1 : 0);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(msd_task_kernel, dim3((m.ntask + 255) / 256, nz), dim3(256), 0, s, m, z0, t.tbeg, t.ccoef,
                       t.cstr, sdet, tpart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(msd_combine_kernel, dim3(nblk, nz), dim3(C_T), 0, s, m, z0, t.trow, tpart, sdet, uw, rpart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(msd_ratio_kernel, dim3((nz + 255) / 256), dim3(256), 0, s, z0, nz, nblk, rpart, ratio);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// (log <Psi_T|phi_z>, 0) pairs: the [W][2] per-spin layout the weight update reads
__global__ void msd_overlap_pairs_kernel(int W, const double2* __restrict__ logdet, const double2* __restrict__ ratio,
                                         double2* __restrict__ out, int* __restrict__ status) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= W) return;
  const double2 r = ratio[z];
  double2 lo = cadd(logdet[2 * z], logdet[2 * z + 1]);
  if (cabs2(r) == 0.0) {
    lo = make_double2(-INFINITY, 0.0);
    atomicOr(status, AFQMC_STATUS_SINGULAR);
  } else {
    lo = cadd(lo, clog(r));
  }
  out[2 * z] = lo;
  out[2 * z + 1] = make_double2(0.0, 0.0);
}

hipError_t launch_msd_overlap_pairs(int W, const double2* logdet, const double2* ratio, double2* out, int* status,
                                    hipStream_t s) {
  hipLaunchKernelGGL(msd_overlap_pairs_kernel, dim3((W + 255) / 256), dim3(256), 0, s, W, logdet, ratio, out,
                     status);
  return hipGetLastError();
}

hipError_t launch_msd_overlap_store(int W, const double2* logdet, const double2* ratio, double2* out, int* status,
                                    hipStream_t s) {
  hipLaunchKernelGGL(msd_overlap_kernel, dim3((W + 255) / 256), dim3(256), 0, s, W, logdet, ratio, out, status);
  return hipGetLastError();
}

hipError_t launch_msd_q(const MsdDims& m, int W, const MsdTables& t, const double* yp, const double2* sadj,
                        const double2* uw, const double2* ratio, double* zt, double* qp, hipStream_t s) {
  for (int z0 = 0; z0 < W; z0 += ZCHUNK) {
    const int nz = W - z0 < ZCHUNK ? W - z0 : ZCHUNK;
    const int nent = m.nmax * m.ldv;
    hipLaunchKernelGGL(msd_m_kernel, dim3((nent + 255) / 256, 2 * nz), dim3(256), 0, s, m, z0, t.erow, t.estr,
                       t.eoff, uw, sadj, ratio, zt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
      MsdZProb pz{zt, yp, z0, m.nmax, m.ldN, m.ldv, m.na, m.nb, m.nv[0], m.nv[1]};
      const dim3 grid((m.nmax + ZBM - 1) / ZBM, (2 * m.nmax + ZBN - 1) / ZBN, 2 * nz);
      hipLaunchKernelGGL(msd_zocc_kernel, grid, dim3(ZWM * ZWN * 64), 0, s, m, pz, zt);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int sp = 0; sp < 2; ++sp) {
      if ((sp ? m.nb : m.na) == 0) continue;
      MsdQProb p{t.cfull + (size_t)sp * m.N * m.ldN, zt, m.N, 2 * nz * m.nmax, z0, sp, m.nmax, m.ldN};
      const dim3 grid((m.N + GBM - 1) / GBM, (p.rows + GBN - 1) / GBN);
      hipLaunchKernelGGL(msd_q_kernel, grid, dim3(GWM * GWN * 64), 0, s, m, p, qp);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_msd_green(const MsdDims& m, int W, const MsdTables& t, const double* theta, const double* yp,
                            const double2* sadj, const double2* uw, const double2* ratio, double* zt, double* qp,
                            double2* G, hipStream_t s) {
  hipError_t e = launch_msd_q(m, W, t, yp, sadj, uw, ratio, zt, qp, s);
  if (e != hipSuccess) return e;
  for (int z0 = 0; z0 < W; z0 += ZCHUNK) {
    const int nz = W - z0 < ZCHUNK ? W - z0 : ZCHUNK;
    MsdGProb pg{qp, theta, m.N, m.nmax, m.ldN, m.ldq, z0};
    const int mt = (m.N + GBM - 1) / GBM, ntile = mt * ((2 * m.N + GBN - 1) / GBN);
    const int nbatch = 2 * nz, nbp = (nbatch + NXCD - 1) / NXCD * NXCD;
    hipLaunchKernelGGL(msd_green_kernel, dim3(ntile * nbp), dim3(GWM * GWN * 64), 0, s, m, pg, nbatch, mt, ntile,
                       reinterpret_cast<double*>(G));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

int msd_fb_splits(int W, int N, int K, int ldK, int ldpk, size_t gs_elem_bytes, size_t scratch_bytes) {
  const size_t gsb = (size_t)2 * W * ldpk * gs_elem_bytes, per = (size_t)2 * W * ldK * sizeof(double);
  if (scratch_bytes < gsb + per) return 0;
  size_t sp = (scratch_bytes - gsb) / per;
  const int npk = N * (N + 1) / 2;
  const int maxs = (npk + 255) / 256;  // at least 256 pairs per split
  if (sp > 8) sp = 8;
  if ((int)sp > maxs) sp = maxs;
  (void)K;
  return (int)sp;
}

template <typename T>
static hipError_t launch_msd_gsym(const MsdDims& m, int W, const double* theta, const double* qp, int ldpk, T* gs,
                                  hipStream_t s) {
  for (int z0 = 0; z0 < W; z0 += ZCHUNK) {
    const int nz = W - z0 < ZCHUNK ? W - z0 : ZCHUNK;
    MsdSProb ps{qp, theta, m.N, m.nmax, m.ldN, m.ldq, z0};
    const int mt = (m.N + GBM - 1) / GBM, ntile = mt * ((2 * m.N + GBN - 1) / GBN);
    const int nbp = (nz + NXCD - 1) / NXCD * NXCD;
    hipLaunchKernelGGL(msd_gsym_kernel<T>, dim3(ntile * nbp), dim3(GWM * GWN * 64), 0, s, m, ps, nz, mt, ntile, ldpk,
                       gs);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_msd_gsym_f32(const MsdDims& m, int W, const double* theta, const double* qp, int ldpk, float* gs,
                               hipStream_t s) {
  return launch_msd_gsym<float>(m, W, theta, qp, ldpk, gs, s);
}

template <typename T>
hipError_t launch_msd_force_bias(const MsdDims& m, int W, const double* theta, const double* qp, const T* lt, int K,
                                 int ldK, int ldpk, int nsplit, void* scratch, double2* vbias, hipStream_t s) {
  T* gs = reinterpret_cast<T*>(scratch);  // [W][2][ldpk]
  double* fbp = reinterpret_cast<double*>(gs + (size_t)2 * W * ldpk);  // [nsplit][2 W][ldK]
  const int npk = m.N * (m.N + 1) / 2;
  hipError_t e;
  if ((e = launch_msd_gsym<T>(m, W, theta, qp, ldpk, gs, s)) != hipSuccess) return e;
  // the pair range of each split is a multiple of 16 (whole k steps, aligned operand rows)
  int chunk = (npk + nsplit - 1) / nsplit;
  chunk = (chunk + 31) / 32 * 32;
  const int ns = (npk + chunk - 1) / chunk;
  for (int z0 = 0; z0 < W; z0 += ZCHUNK) {
    const int nz = W - z0 < ZCHUNK ? W - z0 : ZCHUNK;
    MsdFbProb<T> pf{gs, lt, 2 * nz, ldpk, ldK, z0, chunk, npk};
    const dim3 grid((2 * nz + GBM - 1) / GBM, (K + GBN - 1) / GBN, ns);
    hipLaunchKernelGGL(msd_fb_kernel<T>, grid, dim3(GWM * GWN * 64), 0, s, pf, npk, K, W, fbp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const long tot = (long)W * K;
  hipLaunchKernelGGL(msd_fb_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, W, K, ldK, ns, fbp,
                     vbias);
  return hipGetLastError();
}
template hipError_t launch_msd_force_bias<double>(const MsdDims&, int, const double*, const double*, const double*,
                                                  int, int, int, int, void*, double2*, hipStream_t);
template hipError_t launch_msd_force_bias<float>(const MsdDims&, int, const double*, const double*, const float*,
                                                 int, int, int, int, void*, double2*, hipStream_t);
