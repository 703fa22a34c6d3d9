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

namespace {

constexpr int Y_COLS = 256;  // virtual orbitals per workgroup (one per thread)
constexpr int Y_ROWS = 8;    // occupied orbitals per thread
constexpr int S_T = 64;      // strings per workgroup (per-thread LDS matrices)
constexpr int KM = MSD_KMAX;

// ---------------------------------------------------------------------------
// Y^s_z[i][a] = sum_p C_virt[p][a] theta_0[p][i]   (stored Yt[z][s][i][a])
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(Y_COLS) void msd_y_kernel(MsdDims m, int z0, const double* __restrict__ theta,
                                                       const double* __restrict__ cvirt,
                                                       double2* __restrict__ yt) {
  const int ncb = (m.ldv + Y_COLS - 1) / Y_COLS;
  const int cb = blockIdx.x % ncb, ib = blockIdx.x / ncb;
  const int z = z0 + (int)(blockIdx.y >> 1), s = blockIdx.y & 1;
  const int n = s ? m.nb : m.na, nv = m.nv[s];
  const int i0 = ib * Y_ROWS;
  const int a = cb * Y_COLS + threadIdx.x;
  if (i0 >= n || a >= nv) return;
  const size_t plane = (size_t)m.nmax * m.ldN;
  const double* tre = theta + ((size_t)(z * 2 + 0) * 2 + s) * plane;
  const double* tim = theta + ((size_t)(z * 2 + 1) * 2 + s) * plane;
  const double* cv = cvirt + (size_t)s * m.N * m.ldv;
  double2 acc[Y_ROWS];
#pragma unroll
  for (int r = 0; r < Y_ROWS; ++r) acc[r] = make_double2(0.0, 0.0);
  for (int p = 0; p < m.N; ++p) {
    const double c = cv[(size_t)p * m.ldv + a];
#pragma unroll
    for (int r = 0; r < Y_ROWS; ++r) {
      const int i = i0 + r < n ? i0 + r : n - 1;  // clamped rows are not stored
      acc[r].x = fma(c, tre[(size_t)i * m.ldN + p], acc[r].x);
      acc[r].y = fma(c, tim[(size_t)i * m.ldN + p], acc[r].y);
    }
  }
  double2* out = yt + ((size_t)z * 2 + s) * m.nmax * m.ldv;
#pragma unroll
  for (int r = 0; r < Y_ROWS; ++r)
    if (i0 + r < n) out[(size_t)(i0 + r) * m.ldv + a] = acc[r];
}

// ---------------------------------------------------------------------------
// det and adjugate of one string's k x k matrix A (per-thread LDS storage)
// ---------------------------------------------------------------------------

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
      det = make_double2(-det.x, -det.y);
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

// One thread per (walker, string): A[l][m] = Y[q_l][h_m]; sdet = det A,
// sadj[aoff + m k + l] = adj(A)[m][l] = (-1)^(l+m) det(A without row l, column m).
__global__ __launch_bounds__(S_T) void msd_strings_kernel(MsdDims m, int z0, const int* __restrict__ srank,
                                                          const int* __restrict__ sorb,
                                                          const int* __restrict__ saoff,
                                                          const double2* __restrict__ yt,
                                                          double2* __restrict__ sdet,
                                                          double2* __restrict__ sadj) {
  // A and one minor per thread: (36 + 25) x 64 x 16 B = 62.5 KB
  __shared__ double2 lds_a[KM * KM * S_T];
  __shared__ double2 lds_w[(KM - 1) * (KM - 1) * S_T];
  const int lane = threadIdx.x;
  const int u = blockIdx.x * S_T + lane;
  const int z = z0 + (int)blockIdx.y;
  if (u >= m.nstr_tot) return;  // no barrier below: every thread works on its own LDS slots
  const int s = u >= m.nstr[0] ? 1 : 0;
  const int k = srank[u];
  const int* holes = sorb + (size_t)u * 2 * KM;
  const int* parts = holes + KM;
  const double2* Y = yt + ((size_t)z * 2 + s) * m.nmax * m.ldv;
  double2* A = lds_a + lane;
  double2* Wk = lds_w + lane;
  for (int l = 0; l < k; ++l)
    for (int c = 0; c < k; ++c) A[(l * k + c) * S_T] = Y[(size_t)holes[c] * m.ldv + parts[l]];
  double2* adj = sadj + (size_t)z * m.nadj_tot + saoff[u];
  double2 det;
  if (k == 0) {
    det = make_double2(1.0, 0.0);
  } else if (k == 1) {
    det = A[0];
    adj[0] = make_double2(1.0, 0.0);
  } else if (k == 2) {
    const double2 a00 = A[0], a01 = A[S_T], a10 = A[2 * S_T], a11 = A[3 * S_T];
    det = csub(cmul(a00, a11), cmul(a01, a10));
    adj[0] = a11;                                     // [m=0][l=0]
    adj[1] = make_double2(-a01.x, -a01.y);            // [0][1]
    adj[2] = make_double2(-a10.x, -a10.y);            // [1][0]
    adj[3] = a00;                                     // [1][1]
  } else {
    const int k1 = k - 1;
    for (int l = 0; l < k; ++l) {
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
        if ((l + c) & 1) minor = make_double2(-minor.x, -minor.y);
        adj[c * k + l] = minor;
      }
    }
    det = det_in_place(A, k);  // last: A is not needed afterwards
  }
  sdet[(size_t)z * m.nstr_tot + u] = det;
}

// ---------------------------------------------------------------------------
// Expansion sums per walker (one workgroup): for a string u of spin s,
//   uw[u] = sum over determinants a with that string of c_a det A^{other}_a
// (CSR rows in increasing a), and s_z = sum_{alpha strings} det A_u uw[u].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void msd_combine_kernel(MsdDims m, int z0, const int* __restrict__ crow,
                                                          const double* __restrict__ ccoef,
                                                          const int* __restrict__ cstr,
                                                          const double2* __restrict__ sdet,
                                                          double2* __restrict__ uw,
                                                          double2* __restrict__ ratio) {
  __shared__ double2 red[8];
  const int z = z0 + (int)blockIdx.x;
  const double2* dz = sdet + (size_t)z * m.nstr_tot;
  double2* uz = uw + (size_t)z * m.nstr_tot;
  double2 part = make_double2(0.0, 0.0);
  for (int u = threadIdx.x; u < m.nstr_tot; u += blockDim.x) {
    double2 acc = make_double2(0.0, 0.0);
    for (int e = crow[u]; e < crow[u + 1]; ++e) {
      const double2 d = dz[cstr[e]];
      acc.x = fma(ccoef[e], d.x, acc.x);
      acc.y = fma(ccoef[e], d.y, acc.y);
    }
    uz[u] = acc;
    if (u < m.nstr[0]) part = cadd(part, cmul(dz[u], acc));
  }
  const double2 tot = block_sum2(part, red);
  if (threadIdx.x == 0) ratio[z] = tot;
}

// ---------------------------------------------------------------------------
// M^s[j][a] = sum over (string u, adjugate slot) entries of uw[u] adj_u[slot]
// (CSR per (a, j) entry of the spin, fixed order), stored Mt[z][s][a][j].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void msd_m_kernel(MsdDims m, int z0, const int* __restrict__ erow,
                                                    const int* __restrict__ estr, const int* __restrict__ eoff,
                                                    const double2* __restrict__ uw,
                                                    const double2* __restrict__ sadj,
                                                    double2* __restrict__ mt) {
  const int z = z0 + (int)(blockIdx.y >> 1), s = blockIdx.y & 1;
  const int n = s ? m.nb : m.na, nv = m.nv[s];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nv) return;
  const int a = e / n, j = e - a * n;
  const int r = (s ? m.na * m.nv[0] : 0) + e;
  const double2* uz = uw + (size_t)z * m.nstr_tot;
  const double2* az = sadj + (size_t)z * m.nadj_tot;
  double2 acc = make_double2(0.0, 0.0);
  for (int x = erow[r]; x < erow[r + 1]; ++x) acc = cadd(acc, cmul(uz[estr[x]], az[eoff[x]]));
  mt[(((size_t)z * 2 + s) * m.ldv + a) * m.nmax + j] = acc;
}

// ---------------------------------------------------------------------------
// Zocc[j][i] = delta_ji - (sum_a M[j][a] Y[a][i]) / s_z   (one workgroup per (walker, spin))
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void msd_zocc_kernel(MsdDims m, int z0, const double2* __restrict__ mt,
                                                       const double2* __restrict__ yt,
                                                       const double2* __restrict__ ratio,
                                                       double2* __restrict__ zocc) {
  const int z = z0 + (int)(blockIdx.x >> 1), s = blockIdx.x & 1;
  const int n = s ? m.nb : m.na, nv = m.nv[s];
  const double2 is = cinv(ratio[z]);
  const double2* M = mt + ((size_t)z * 2 + s) * m.ldv * m.nmax;
  const double2* Y = yt + ((size_t)z * 2 + s) * m.nmax * m.ldv;
  double2* Z = zocc + ((size_t)z * 2 + s) * m.nmax * m.nmax;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e - i * n;
    double2 acc = make_double2(0.0, 0.0);
    for (int a = 0; a < nv; ++a) acc = cadd(acc, cmul(M[(size_t)a * m.nmax + j], Y[(size_t)i * m.ldv + a]));
    const double2 t = cmul(acc, is);
    Z[(size_t)j * m.nmax + i] = make_double2((i == j ? 1.0 : 0.0) - t.x, -t.y);
  }
}

// ---------------------------------------------------------------------------
// Q[p][j] = sum_i C_occ[p][i] Zocc[j][i] + (sum_a C_virt[p][a] M[j][a]) / s_z
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void msd_q_kernel(MsdDims m, int z0, const double* __restrict__ cocc,
                                                    const double* __restrict__ cvirt,
                                                    const double2* __restrict__ zocc,
                                                    const double2* __restrict__ mt,
                                                    const double2* __restrict__ ratio,
                                                    double2* __restrict__ q) {
  const int z = z0 + (int)(blockIdx.y >> 1), s = blockIdx.y & 1;
  const int n = s ? m.nb : m.na, nv = m.nv[s];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.N * n) return;
  const int p = e / n, j = e - p * n;
  const double* co = cocc + (size_t)s * m.N * m.nmax + (size_t)p * m.nmax;
  const double* cv = cvirt + (size_t)s * m.N * m.ldv + (size_t)p * m.ldv;
  const double2* Z = zocc + ((size_t)z * 2 + s) * m.nmax * m.nmax + (size_t)j * m.nmax;
  const double2* M = mt + ((size_t)z * 2 + s) * m.ldv * m.nmax + j;
  double2 occ = make_double2(0.0, 0.0), vir = make_double2(0.0, 0.0);
  for (int i = 0; i < n; ++i) {
    occ.x = fma(co[i], Z[i].x, occ.x);
    occ.y = fma(co[i], Z[i].y, occ.y);
  }
  for (int a = 0; a < nv; ++a) {
    const double2 v = M[(size_t)a * m.nmax];
    vir.x = fma(cv[a], v.x, vir.x);
    vir.y = fma(cv[a], v.y, vir.y);
  }
  q[(((size_t)z * 2 + s) * m.N + p) * m.nmax + j] = cadd(occ, cmul(vir, cinv(ratio[z])));
}

// ---------------------------------------------------------------------------
// G[z][s][p][q] = sum_j theta_0[q][j] Q[p][j]
// ---------------------------------------------------------------------------
constexpr int G_ROWS = 16, G_COLS = 256;

__global__ __launch_bounds__(G_COLS) void msd_green_kernel(MsdDims m, int z0, const double* __restrict__ theta,
                                                           const double2* __restrict__ q,
                                                           double2* __restrict__ G) {
  const int nqb = (m.N + G_COLS - 1) / G_COLS;
  const int qb = blockIdx.x % nqb, pb = blockIdx.x / nqb;
  const int z = z0 + (int)(blockIdx.y >> 1), s = blockIdx.y & 1;
  const int n = s ? m.nb : m.na;
  const int c = qb * G_COLS + threadIdx.x;
  const int p0 = pb * G_ROWS;
  if (c >= m.N) return;
  const size_t plane = (size_t)m.nmax * m.ldN;
  const double* tre = theta + ((size_t)(z * 2 + 0) * 2 + s) * plane;
  const double* tim = theta + ((size_t)(z * 2 + 1) * 2 + s) * plane;
  const double2* Q = q + ((size_t)z * 2 + s) * m.N * m.nmax;
  double2 acc[G_ROWS];
#pragma unroll
  for (int r = 0; r < G_ROWS; ++r) acc[r] = make_double2(0.0, 0.0);
  for (int j = 0; j < n; ++j) {
    const double2 t = make_double2(tre[(size_t)j * m.ldN + c], tim[(size_t)j * m.ldN + c]);
#pragma unroll
    for (int r = 0; r < G_ROWS; ++r) {
      const int p = p0 + r < m.N ? p0 + r : m.N - 1;  // clamped rows are not stored
      acc[r] = cadd(acc[r], cmul(Q[(size_t)p * m.nmax + j], t));
    }
  }
  double2* out = G + ((size_t)z * 2 + s) * m.N * m.N;
#pragma unroll
  for (int r = 0; r < G_ROWS; ++r)
    if (p0 + r < m.N) out[(size_t)(p0 + r) * m.N + c] = acc[r];
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

constexpr int ZCHUNK = 16384;  // walkers per launch (grid y <= 2 per walker)

}  // namespace

hipError_t launch_msd_ratio(const MsdDims& m, int W, const MsdTables& t, const double* theta, double2* yt,
                            double2* sdet, double2* sadj, double2* uw, double2* ratio, hipStream_t s) {
  for (int z0 = 0; z0 < W; z0 += ZCHUNK) {
    const int nz = W - z0 < ZCHUNK ? W - z0 : ZCHUNK;
    const int ncb = (m.ldv + Y_COLS - 1) / Y_COLS, nib = (m.nmax + Y_ROWS - 1) / Y_ROWS;
    hipLaunchKernelGGL(msd_y_kernel, dim3(ncb * nib, 2 * nz), dim3(Y_COLS), 0, s, m, z0, theta, t.cvirt, yt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(msd_strings_kernel, dim3((m.nstr_tot + S_T - 1) / S_T, nz), dim3(S_T), 0, s, m, z0,
                       t.srank, t.sorb, t.saoff, yt, sdet, sadj);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(msd_combine_kernel, dim3(nz), dim3(256), 0, s, m, z0, t.crow, t.ccoef, t.cstr, sdet, uw,
                       ratio);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_msd_overlap_store(int W, const double2* logdet, const double2* ratio, double2* out, int* status,
                                    hipStream_t s) {
  hipLaunchKernelGGL(msd_overlap_kernel, dim3((W + 255) / 256), dim3(256), 0, s, W, logdet, ratio, out, status);
  return hipGetLastError();
}

hipError_t launch_msd_green(const MsdDims& m, int W, const MsdTables& t, const double* theta, const double2* yt,
                            const double2* sadj, const double2* uw, const double2* ratio, double2* mt,
                            double2* zocc, double2* q, double2* G, hipStream_t s) {
  for (int z0 = 0; z0 < W; z0 += ZCHUNK) {
    const int nz = W - z0 < ZCHUNK ? W - z0 : ZCHUNK;
    const int nent = m.nmax * m.ldv;
    hipLaunchKernelGGL(msd_m_kernel, dim3((nent + 255) / 256, 2 * nz), dim3(256), 0, s, m, z0, t.erow, t.estr,
                       t.eoff, uw, sadj, mt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(msd_zocc_kernel, dim3(2 * nz), dim3(256), 0, s, m, z0, mt, yt, ratio, zocc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(msd_q_kernel, dim3((m.N * m.nmax + 255) / 256, 2 * nz), dim3(256), 0, s, m, z0, t.cocc,
                       t.cvirt, zocc, mt, ratio, q);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nqb = (m.N + G_COLS - 1) / G_COLS, npb = (m.N + G_ROWS - 1) / G_ROWS;
    hipLaunchKernelGGL(msd_green_kernel, dim3(nqb * npb, 2 * nz), dim3(G_COLS), 0, s, m, z0, theta, q, G);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}
