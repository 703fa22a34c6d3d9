// Local energy of a walker against the multi-determinant trial (Sec. III.C:
// the one-body part from the expansion's Green's function, the two-body
// numerator through the generalised Wick's theorem of Sec. III.A), as the
// c_a <D_a|phi> weighted sum of the determinants' own local energies.
//
// Per spin, in the trial's orbital basis C (reference psi_0 = C_occ), with
// theta_0 = phi (C_occ^T phi)^-1 and Y = C_virt^T theta_0, a determinant that
// excites holes h_m to particles q_l has (relative to psi_0) the overlap
// ratio det A, A[l][m] = Y[q_l][h_m], and its half-rotated products
//   T^a_g = T_g - Delta_g,  Delta_g[h_m][:] = sum_l (A^-1)[m][l] R_g[q_l][:]
// where T_g = C_occ^T L_g theta_0 (n x n, the reference's), V_g = rows Q of
// C_virt^T L_g theta_0, and R_g = Y T_g - V_g (rows Q only).  Hence, with
// r_g = R_g[Q][H] (the active particles by the active holes, vector of
// length D = |Q| |H|), p_g = (R_g T_g)[Q][H], the adjugate F_u of a string
// scattered into (Q, H) and its overlap ratio d_u:
//   tr T^a_g       = tr T_g - <F_u, r_g> / d_u
//   tr T^a_g T^a_g = tr T_g T_g - 2 <F_u, p_g> / d_u + tr((adj R_s)^2) / d_u^2.
// Weighted by w_a = c_a d_alpha d_beta and summed over the expansion and
// over g, every term is one of
//   s sum_g J_g^2, s sum_g tr T_g T_g, <M, sum_g J_g r_g>, <M, sum_g p_g>,
//   sum_u (uw_u / d_u) F_u^T G F_u,  sum_a c_a F_alpha^T G^{ab} F_beta,
// with s = sum_a w_a, M = sum_u uw_u F_u (uw_u = sum over the determinants
// of string u of c_a det A^{other spin}), J_g = sum_s tr T^s_g and the Gram
// matrices G^{ss'} = sum_g r^s_g (r^s'_g)^T (D x D').  So the sum over the
// Cholesky vectors is taken once, by dense products (the Gram matrices on
// the FP64 matrix cores), and the expansion enters only through small
// per-string and per-determinant contractions with them; the cost of the
// g sum does not grow with the number of determinants.  The one-body part
// is the same linear form with h1 in place of L_g (block g = K).
//
// Numbers are FP64 throughout.  Where a string's determinant d_u is exactly
// zero (a walker exactly at the reference, say: Y = 0), its Coulomb and
// exchange quadratic terms diverge separately but their sum stays finite:
// with F = adj A, ((tr F R)^2 - tr (F R)^2) / d = 2 [t^2] det(A + t R), and
// the t^2 coefficient expands over pairs of columns (Laplace) into the
// complementary minors of A times 2 x 2 minors of R, whose sum over g is a
// difference of two Gram entries.  That sum is added to EJ for such a
// string (the split between EJ and EK is not defined there).

#include "common.h"
#include "kernels.h"
#include "mfma_tile.h"

namespace {

constexpr int KM = MSD_KMAX;
constexpr int RP_T = 256;  // threads of the per-(walker, Cholesky chunk) kernel
constexpr int CT_T = 256;  // threads of the contraction kernel

// ---------------------------------------------------------------------------
// U^s[z][g][c][r][j] = sum_p Lr^s[g][r][p] theta_0^s[z][c][j][p]: one FP64
// MFMA GEMM per spin over a chunk of walkers; rows (g, r) of the rotated
// vectors, columns (walker, re | im, j) of theta_0 (p contiguous in both).
// ---------------------------------------------------------------------------
struct MsdUProb {
  const double* lr;     // [K + 1][S][ldL]
  const double* theta;  // [W][re|im][2][nmax][ldN]
  long rows;            // (K + 1) S
  int cols;             // Wc 2 n
  int z0, s, n, nmax, ldN, ldL;
  __device__ double2 load_a(int, int r, int k) const {
    if (r >= rows) return make_double2(0.0, 0.0);
    return *reinterpret_cast<const double2*>(lr + (size_t)r * ldL + k);
  }
  __device__ double2 load_b(int, int col, int k) const {
    if (col >= cols) return make_double2(0.0, 0.0);
    const int zl = col / (2 * n), rem = col - zl * 2 * n;
    const int c = rem / n, j = rem - c * n;
    const size_t plane = (size_t)nmax * ldN;
    return *reinterpret_cast<const double2*>(theta + ((size_t)(2 * (z0 + zl) + c) * 2 + s) * plane +
                                             (size_t)j * ldN + k);
  }
};

constexpr int UBM = 128, UBN = 128, UBK = 16, UWM = 4, UWN = 2, UPIPE = 2;

__global__ __launch_bounds__(UWM* UWN * 64) void msd_u_kernel(MsdUProb p, int S, int Smax, int K1,
                                                              double* __restrict__ u) {
  __shared__ __attribute__((aligned(16))) double lds[(UPIPE == 2 ? 2 : 1) * TileLds<double, UBM, UBN, UBK>::ELEMS];
  MF<double>::acc_t acc[UBM / UWM / 16][UBN / UWN / 16];
  const long m0 = (long)blockIdx.x * UBM;
  const int n0 = blockIdx.y * UBN;
  mfma_tile_mainloop<double, UBM, UBN, UBK, UWM, UWN, false, MsdUProb, UPIPE>(p, 0, (int)m0, n0, p.ldL, acc, lds);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / UWN, wn = wid % UWN;
#pragma unroll
  for (int i = 0; i < UBM / UWM / 16; ++i)
#pragma unroll
    for (int j = 0; j < UBN / UWN / 16; ++j) {
      const long rb = m0 + wm * (UBM / UWM) + i * 16 + 4 * (lane >> 4);
      const int col = n0 + wn * (UBN / UWN) + j * 16 + (lane & 15);
      if (col >= p.cols) continue;
      const int zl = col / (2 * p.n), rem = col - zl * 2 * p.n;
      const int c = rem / p.n, jj = rem - c * p.n;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long row = rb + r;
        if (row >= p.rows) continue;
        const long g = row / S, rr = row - g * S;
        u[((((size_t)zl * 2 + p.s) * K1 + g) * 2 + c) * Smax * p.nmax + (size_t)rr * p.nmax + jj] = acc[i][j][r];
      }
    }
}

// ---------------------------------------------------------------------------
// Per (walker, chunk of Cholesky blocks): T, tr T, tr T T, R = Y_Q T - V, the
// active blocks r = R[Q][H] and p = (R T)[Q][H].  r goes to rbuf[z][s][g][d]
// (complex, d fastest: a block's entries are one contiguous run); the
// chunk's partial sums of J_g r_g and of p_g, and tr T, tr T T per block, go
// to their own arrays; block K (h1) fills r1 and tr T1 instead.
// ---------------------------------------------------------------------------
struct MsdRpArgs {
  const double* u;      // [Wc][2][K1][2][Smax][nmax]
  const double* yp;     // planar Y [W][2][2][nmax][ldv]
  const int* hlist;     // [2][Hmax] active holes (occupied index)
  const int* qlist;     // [2][Qmax] active particles (virtual index)
  double2* rbuf;        // [Wc][2][ldG][Dmax]
  double2* jpart;       // [Wc][2][nchunk][Dmax]
  double2* ppart;       // [Wc][2][nchunk][Dmax]
  double2* tt;          // [Wc][2][K1]: tr T_g (g = K: tr T1)
  double2* kt;          // [Wc][2][K]
  double2* r1;          // [Wc][2][Dmax]
  int z0, K, K1, nmax, ldv, Smax, ldG, gchunk, nchunk, Hmax, Qmax, Dmax;
  int n[2], S[2], nh[2], nq[2];
};

__global__ __launch_bounds__(RP_T) void msd_rp_kernel(MsdRpArgs a) {
  extern __shared__ __attribute__((aligned(16))) double rp_lds[];
  const int zl = blockIdx.y, ch = blockIdx.x;
  const int z = a.z0 + zl;
  const int g0 = ch * a.gchunk, g1 = min(g0 + a.gchunk, a.K1);
  const int tid = threadIdx.x;
  // LDS: U block (re, im planes) [2][Smax][nmax], Y_Q [2][nmax][Qmax], R [2][Qmax][nmax], J of the chunk
  double* Ul = rp_lds;
  double* Yl = Ul + 2 * a.Smax * a.nmax;
  double* Rl = Yl + 2 * a.nmax * a.Qmax;
  double2* Jl = reinterpret_cast<double2*>(Rl + 2 * a.Qmax * a.nmax);  // [gchunk]
  __shared__ double2 red[RP_T / 64];

  // tr T of both spins for the chunk's blocks (J_g = sum over spins)
  for (int gi = 0; gi < g1 - g0; ++gi) {
    const int g = g0 + gi;
    double2 jt = make_double2(0.0, 0.0);
    for (int s = 0; s < 2; ++s) {
      const int n = a.n[s];
      double2 v = make_double2(0.0, 0.0);
      const double* ub = a.u + ((((size_t)zl * 2 + s) * a.K1 + g) * 2) * a.Smax * a.nmax;
      for (int i = tid; i < n; i += RP_T)
        v = cadd(v, make_double2(ub[(size_t)i * a.nmax + i], ub[(size_t)a.Smax * a.nmax + (size_t)i * a.nmax + i]));
      v = block_sum2(v, red);
      if (tid == 0) a.tt[((size_t)zl * 2 + s) * a.K1 + g] = v;
      jt = cadd(jt, v);
    }
    if (tid == 0) Jl[gi] = jt;
  }
  __syncthreads();

  for (int s = 0; s < 2; ++s) {
    const int n = a.n[s], S = a.S[s], nh = a.nh[s], nq = a.nq[s], D = nh * nq;
    if (n == 0) continue;  // uniform
    // Y_Q^s of the walker: Yl[c][i][q] = Y[i][Q_q]
    const size_t yplane = (size_t)a.nmax * a.ldv;
    for (int e = tid; e < n * nq; e += RP_T) {
      const int i = e / nq, q = e - i * nq;
      const int av = a.qlist[s * a.Qmax + q];
      Yl[(size_t)i * a.Qmax + q] = a.yp[((size_t)(2 * z + 0) * 2 + s) * yplane + (size_t)i * a.ldv + av];
      Yl[(size_t)a.nmax * a.Qmax + (size_t)i * a.Qmax + q] =
          a.yp[((size_t)(2 * z + 1) * 2 + s) * yplane + (size_t)i * a.ldv + av];
    }
    double2 accj[4], accp[4];  // this thread's active entries d = tid + RP_T m (D <= 4 RP_T)
#pragma unroll
    for (int m = 0; m < 4; ++m) accj[m] = accp[m] = make_double2(0.0, 0.0);
    for (int gi = 0; gi < g1 - g0; ++gi) {
      const int g = g0 + gi;
      __syncthreads();  // the previous block's readers of Ul / Rl (and Yl writers) are done
      const double* ub = a.u + ((((size_t)zl * 2 + s) * a.K1 + g) * 2) * a.Smax * a.nmax;
      for (int e = tid; e < 2 * S * a.nmax; e += RP_T) {
        const int c = e / (S * a.nmax), rem = e - c * S * a.nmax;
        Ul[(size_t)c * a.Smax * a.nmax + rem] = ub[(size_t)c * a.Smax * a.nmax + rem];
      }
      __syncthreads();
      const double* Ur = Ul;
      const double* Ui = Ul + (size_t)a.Smax * a.nmax;
      // tr T T (blocks g < K)
      if (g < a.K) {
        double2 v = make_double2(0.0, 0.0);
        for (int e = tid; e < n * n; e += RP_T) {
          const int i = e / n, j = e - i * n;
          const double2 tij = make_double2(Ur[i * a.nmax + j], Ui[i * a.nmax + j]);
          const double2 tji = make_double2(Ur[j * a.nmax + i], Ui[j * a.nmax + i]);
          v = cadd(v, cmul(tij, tji));
        }
        v = block_sum2(v, red);
        if (tid == 0) a.kt[((size_t)zl * 2 + s) * a.K + g] = v;
      }
      // R[q][j] = sum_i Y[i][Q_q] T[i][j] - V[q][j]
      for (int e = tid; e < nq * n; e += RP_T) {
        const int q = e / n, j = e - q * n;
        double2 acc = make_double2(-Ur[(size_t)(n + q) * a.nmax + j], -Ui[(size_t)(n + q) * a.nmax + j]);
        for (int i = 0; i < n; ++i) {
          const double2 y = make_double2(Yl[(size_t)i * a.Qmax + q], Yl[(size_t)a.nmax * a.Qmax + (size_t)i * a.Qmax + q]);
          acc = cadd(acc, cmul(y, make_double2(Ur[i * a.nmax + j], Ui[i * a.nmax + j])));
        }
        Rl[(size_t)q * a.nmax + j] = acc.x;
        Rl[(size_t)a.Qmax * a.nmax + (size_t)q * a.nmax + j] = acc.y;
      }
      __syncthreads();
      const double2 J = Jl[gi];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int d = tid + RP_T * m;
        if (d >= D) break;
        const int q = d / nh, hh = d - q * nh;
        const int h = a.hlist[s * a.Hmax + hh];
        const double2 r = make_double2(Rl[(size_t)q * a.nmax + h], Rl[(size_t)a.Qmax * a.nmax + (size_t)q * a.nmax + h]);
        if (g == a.K) {
          a.r1[((size_t)zl * 2 + s) * a.Dmax + d] = r;
          continue;
        }
        a.rbuf[(((size_t)zl * 2 + s) * a.ldG + g) * a.Dmax + d] = r;
        accj[m] = cadd(accj[m], cmul(J, r));
        double2 pv = make_double2(0.0, 0.0);
        for (int j = 0; j < n; ++j)
          pv = cadd(pv, cmul(make_double2(Rl[(size_t)q * a.nmax + j], Rl[(size_t)a.Qmax * a.nmax + (size_t)q * a.nmax + j]),
                             make_double2(Ur[j * a.nmax + h], Ui[j * a.nmax + h])));
        accp[m] = cadd(accp[m], pv);
      }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int d = tid + RP_T * m;
      if (d >= D) break;
      const size_t o = (((size_t)zl * 2 + s) * a.nchunk + ch) * a.Dmax + d;
      a.jpart[o] = accj[m];
      a.ppart[o] = accp[m];
    }
  }
}

// ---------------------------------------------------------------------------
// The same on the FP64 matrix cores, one wave per (walker, spin, chunk of
// Cholesky blocks), for windows of at most 16 MT active particles, 16 NTL
// electrons and 16 active holes per spin.  Per block g, with lane l = (lg =
// l / 16, lr = l % 16):
//   R = Y_Q T - V: A = Y_Q^T (particle q x occupied i, loaded once), B = T
//     (i x j), the accumulators start at -V; four real products per k step
//     (Re Re, -Im Im, Re Im, Im Re);
//   r = the hole columns of R, written to rbuf / r1; J_g r summed in the
//     accumulator layout (lane (q = 16 mt + lg + 4 rr, j = 16 nt + lr));
//   p = R T[:, H]: R goes through the wave's LDS block into the A layout,
//     B = T[j][H_hh]; summed over the chunk in the accumulator layout
//     (lane (q, hh = lr)).
// tr T of both spins (for J_g) and tr T T come from direct loads and wave
// sums.  The chunk's partial sums go to jpart / ppart in the layout of the
// workgroup kernel, so that the sums kernel serves both.
// ---------------------------------------------------------------------------
constexpr int RPM_WAVES = 4;

__device__ __forceinline__ double2 wave_sum2_(double2 v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

template <int MT, int NTL>
__global__ __launch_bounds__(RPM_WAVES * 64) void msd_rp_mfma_kernel(MsdRpArgs a) {
  constexpr int KS = 4 * NTL;  // k steps over the electrons (4 per step)
  constexpr int RLD = 16 * NTL + 1;
  __shared__ double rl_lds[RPM_WAVES][2][16 * MT][RLD];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int task = blockIdx.x * RPM_WAVES + wv;  // (spin, chunk)
  const int zl = blockIdx.y, z = a.z0 + zl;
  const int s = task / a.nchunk, ch = task - s * a.nchunk;
  if (s >= 2) return;
  const int n = s ? a.n[1] : a.n[0], nq = s ? a.nq[1] : a.nq[0], nh = s ? a.nh[1] : a.nh[0];
  const int g0 = ch * a.gchunk, g1 = min(g0 + a.gchunk, a.K1);
  if (n == 0) {  // no electrons of this spin: tr T = tr T T = 0
    for (int g = g0 + lane; g < g1; g += 64) {
      a.tt[((size_t)zl * 2 + s) * a.K1 + g] = make_double2(0.0, 0.0);
      if (g < a.K) a.kt[((size_t)zl * 2 + s) * a.K + g] = make_double2(0.0, 0.0);
    }
    return;
  }
  const int lg = lane >> 4, lr = lane & 15;
  const size_t plane = (size_t)a.Smax * a.nmax;
  double (*Rl)[16 * MT][RLD] = rl_lds[wv];

  // A = Y_Q^T: [mt][ks] (re, im)
  double yar[MT][KS], yai[MT][KS];
  {
    const size_t yplane = (size_t)a.nmax * a.ldv;
    const double* yr = a.yp + ((size_t)(2 * z + 0) * 2 + s) * yplane;
    const double* yi = a.yp + ((size_t)(2 * z + 1) * 2 + s) * yplane;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int q = 16 * mt + lr;
      const int av = q < nq ? a.qlist[s * a.Qmax + q] : 0;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int i = 4 * ks + lg;
        const bool ok = q < nq && i < n;
        yar[mt][ks] = ok ? yr[(size_t)i * a.ldv + av] : 0.0;
        yai[mt][ks] = ok ? yi[(size_t)i * a.ldv + av] : 0.0;
      }
    }
  }
  // hole position of this lane's column j in each n tile (-1: not a hole)
  int hpos[NTL];
#pragma unroll
  for (int nt = 0; nt < NTL; ++nt) hpos[nt] = -1;
  for (int hh = 0; hh < nh; ++hh) {
    const int h = a.hlist[s * a.Hmax + hh];
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt)
      if (16 * nt + lr == h) hpos[nt] = hh;
  }
  // this lane's hole column for the p products (B = T[j][H_lr])
  const int hcol = lr < nh ? a.hlist[s * a.Hmax + lr] : 0;

  doublex4 jr[MT][NTL], ji[MT][NTL], pr[MT], pi[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    pr[mt] = pi[mt] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) jr[mt][nt] = ji[mt][nt] = doublex4{0.0, 0.0, 0.0, 0.0};
  }

  for (int g = g0; g < g1; ++g) {
    // tr T of both spins (J_g) and tr T T of this spin
    double2 trs[2];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const int n2 = s2 ? a.n[1] : a.n[0];
      const double* ub = a.u + ((((size_t)zl * 2 + s2) * a.K1 + g) * 2) * plane;
      double2 v = make_double2(0.0, 0.0);
      if (lane < n2) v = make_double2(ub[(size_t)lane * a.nmax + lane], ub[plane + (size_t)lane * a.nmax + lane]);
      trs[s2] = wave_sum2_(v);
    }
    const double2 J = cadd(trs[0], trs[1]);
    if (lane == 0) a.tt[((size_t)zl * 2 + s) * a.K1 + g] = s ? trs[1] : trs[0];
    const double* Ur = a.u + ((((size_t)zl * 2 + s) * a.K1 + g) * 2) * plane;
    const double* Ui = Ur + plane;
    if (g < a.K) {
      double2 v = make_double2(0.0, 0.0);
      for (int e = lane; e < n * n; e += 64) {
        const int i = e / n, j = e - i * n;
        const double2 tij = make_double2(Ur[(size_t)i * a.nmax + j], Ui[(size_t)i * a.nmax + j]);
        const double2 tji = make_double2(Ur[(size_t)j * a.nmax + i], Ui[(size_t)j * a.nmax + i]);
        v = cadd(v, cmul(tij, tji));
      }
      v = wave_sum2_(v);
      if (lane == 0) a.kt[((size_t)zl * 2 + s) * a.K + g] = v;
    }
    // R = Y_Q T - V
    doublex4 rr_[MT][NTL], ri_[MT][NTL];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt) {
        const int j = 16 * nt + lr;
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          const int q = 16 * mt + lg + 4 * r4;
          const bool ok = q < nq && j < n;
          rr_[mt][nt][r4] = ok ? -Ur[(size_t)(n + q) * a.nmax + j] : 0.0;
          ri_[mt][nt][r4] = ok ? -Ui[(size_t)(n + q) * a.nmax + j] : 0.0;
        }
      }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int i = 4 * ks + lg;
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt) {
        const int j = 16 * nt + lr;
        const bool ok = i < n && j < n;
        const double tr = ok ? Ur[(size_t)i * a.nmax + j] : 0.0;
        const double ti = ok ? Ui[(size_t)i * a.nmax + j] : 0.0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          rr_[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(yar[mt][ks], tr, rr_[mt][nt], 0, 0, 0);
          rr_[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-yai[mt][ks], ti, rr_[mt][nt], 0, 0, 0);
          ri_[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(yar[mt][ks], ti, ri_[mt][nt], 0, 0, 0);
          ri_[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(yai[mt][ks], tr, ri_[mt][nt], 0, 0, 0);
        }
      }
    }
    // r (the hole columns) out; J_g r into the chunk sums; R into the LDS block
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt)
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          const int q = 16 * mt + lg + 4 * r4;
          const double2 rv = make_double2(rr_[mt][nt][r4], ri_[mt][nt][r4]);
          Rl[0][q][16 * nt + lr] = rv.x;
          Rl[1][q][16 * nt + lr] = rv.y;
          if (q < nq && hpos[nt] >= 0) {
            const int d = q * nh + hpos[nt];
            if (g == a.K)
              a.r1[((size_t)zl * 2 + s) * a.Dmax + d] = rv;
            else
              a.rbuf[(((size_t)zl * 2 + s) * a.ldG + g) * a.Dmax + d] = rv;
          }
          if (g < a.K) {
            jr[mt][nt][r4] += J.x * rv.x - J.y * rv.y;
            ji[mt][nt][r4] += J.x * rv.y + J.y * rv.x;
          }
        }
    __builtin_amdgcn_wave_barrier();  // the block is written before the wave reads it
    if (g < a.K) {
      // p = R T[:, H]: A = R (q x j) from LDS, B = T[j][H_lr]
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int j = 4 * ks + lg;
        const bool ok = j < n && lr < nh;
        const double br = ok ? Ur[(size_t)j * a.nmax + hcol] : 0.0;
        const double bi = ok ? Ui[(size_t)j * a.nmax + hcol] : 0.0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const double ar = Rl[0][16 * mt + lr][j < 16 * NTL ? j : 0];
          const double ai = Rl[1][16 * mt + lr][j < 16 * NTL ? j : 0];
          pr[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, pr[mt], 0, 0, 0);
          pr[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, pr[mt], 0, 0, 0);
          pi[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, pi[mt], 0, 0, 0);
          pi[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, pi[mt], 0, 0, 0);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();  // the block is read before the next block overwrites it
  }
  // the chunk's partial sums, every active entry written (zero where no block contributed)
  const size_t o = (((size_t)zl * 2 + s) * a.nchunk + ch) * a.Dmax;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) {
      const int q = 16 * mt + lg + 4 * r4;
      if (q >= nq) continue;
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt)
        if (hpos[nt] >= 0) a.jpart[o + q * nh + hpos[nt]] = make_double2(jr[mt][nt][r4], ji[mt][nt][r4]);
      if (lr < nh) a.ppart[o + q * nh + lr] = make_double2(pr[mt][r4], pi[mt][r4]);
    }
}

// ---------------------------------------------------------------------------
// Per walker: vJ = sum of the chunks' J r partials, vP likewise (fixed order),
// and the scalars sum_g J_g^2, sum_g tr T T per spin, tr T1 of both spins.
// sc[zl] = {sum J^2, sum tr TT (alpha), sum tr TT (beta), tr T1 (both)}.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void msd_sums_kernel(int K, int K1, int nchunk, int Dmax, int D0, int D1,
                                                       const double2* __restrict__ jpart,
                                                       const double2* __restrict__ ppart,
                                                       const double2* __restrict__ tt, const double2* __restrict__ kt,
                                                       double2* __restrict__ vj, double2* __restrict__ vp,
                                                       double2* __restrict__ sc) {
  __shared__ double2 red[4];
  const int zl = blockIdx.x, tid = threadIdx.x;
  for (int s = 0; s < 2; ++s) {
    const int D = s ? D1 : D0;
    for (int d = tid; d < D; d += 256) {
      double2 j = make_double2(0.0, 0.0), p = make_double2(0.0, 0.0);
      for (int c = 0; c < nchunk; ++c) {
        const size_t o = (((size_t)zl * 2 + s) * nchunk + c) * Dmax + d;
        j = cadd(j, jpart[o]);
        p = cadd(p, ppart[o]);
      }
      vj[((size_t)zl * 2 + s) * Dmax + d] = j;
      vp[((size_t)zl * 2 + s) * Dmax + d] = p;
    }
  }
  double2 j2 = make_double2(0.0, 0.0), ka = j2, kb = j2;
  for (int g = tid; g < K; g += 256) {
    const double2 J = cadd(tt[((size_t)zl * 2 + 0) * K1 + g], tt[((size_t)zl * 2 + 1) * K1 + g]);
    j2 = cadd(j2, cmul(J, J));
    ka = cadd(ka, kt[((size_t)zl * 2 + 0) * K + g]);
    kb = cadd(kb, kt[((size_t)zl * 2 + 1) * K + g]);
  }
  j2 = block_sum2(j2, red);
  ka = block_sum2(ka, red);
  kb = block_sum2(kb, red);
  if (tid == 0) {
    sc[(size_t)zl * 4 + 0] = j2;
    sc[(size_t)zl * 4 + 1] = ka;
    sc[(size_t)zl * 4 + 2] = kb;
    sc[(size_t)zl * 4 + 3] = cadd(tt[((size_t)zl * 2 + 0) * K1 + K], tt[((size_t)zl * 2 + 1) * K1 + K]);
  }
}

// ---------------------------------------------------------------------------
// Gram matrices G^{ss'}[zl][d][d'] = sum_{g < K} r^s_g[d] r^s'_g[d'] (complex,
// no conjugation) for (s, s') = (a, a), (b, b), (a, b): one real FP64 MFMA
// GEMM per (walker, pair) over k = (g, re | im) interleaved, A row d = r^s[d]
// as stored, B row (d', re) = (Re, -Im) pairs and (d', im) = (Im, Re) pairs
// of r^s'[d'], so that C[d][(d', re|im)] = G[d][d'].
// ---------------------------------------------------------------------------
struct MsdGramProb {
  const double* rbuf;  // [Wc][2][ldG][Dmax] complex as doubles
  int Dmax, ldG, D0, D1;
  __device__ void pair(int b, int& zl, int& s, int& sp) const {
    zl = b / 3;
    const int pr = b - zl * 3;
    s = pr == 1 ? 1 : 0;
    sp = pr == 0 ? 0 : 1;
  }
  __device__ double2 load_a(int b, int d, int k) const {
    int zl, s, sp;
    pair(b, zl, s, sp);
    if (d >= (s ? D1 : D0)) return make_double2(0.0, 0.0);
    return *reinterpret_cast<const double2*>(rbuf + ((((size_t)zl * 2 + s) * ldG + (k >> 1)) * Dmax + d) * 2);
  }
  __device__ double2 load_b(int b, int col, int k) const {
    int zl, s, sp;
    pair(b, zl, s, sp);
    const int d = col >> 1, part = col & 1;
    if (d >= (sp ? D1 : D0)) return make_double2(0.0, 0.0);
    const double2 x = *reinterpret_cast<const double2*>(rbuf + ((((size_t)zl * 2 + sp) * ldG + (k >> 1)) * Dmax + d) * 2);
    return part ? make_double2(x.y, x.x) : make_double2(x.x, -x.y);
  }
};

constexpr int GBM = 128, GBN = 64, GBK = 16, GWM2 = 4, GWN2 = 2, GPIPE = 2;

__global__ __launch_bounds__(GWM2* GWN2 * 64) void msd_gram_kernel(MsdGramProb p, int kdim,
                                                                   double2* __restrict__ G) {
  __shared__ __attribute__((aligned(16))) double lds[(GPIPE == 2 ? 2 : 1) * TileLds<double, GBM, GBN, GBK>::ELEMS];
  MF<double>::acc_t acc[GBM / GWM2 / 16][GBN / GWN2 / 16];
  const int b = blockIdx.z;
  int zl, s, sp;
  p.pair(b, zl, s, sp);
  const int D = s ? p.D1 : p.D0, Dp = sp ? p.D1 : p.D0;
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  if (m0 >= D || n0 >= 2 * Dp) return;  // uniform: tiles past this pair's sizes
  mfma_tile_mainloop<double, GBM, GBN, GBK, GWM2, GWN2, false, MsdGramProb, GPIPE>(p, b, m0, n0, kdim, acc, lds);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wm = wid / GWN2, wn = wid % GWN2;
  double* Gd = reinterpret_cast<double*>(G + (size_t)b * p.Dmax * p.Dmax);
#pragma unroll
  for (int i = 0; i < GBM / GWM2 / 16; ++i)
#pragma unroll
    for (int j = 0; j < GBN / GWN2 / 16; ++j) {
      const int rb = m0 + wm * (GBM / GWM2) + i * 16 + 4 * (lane >> 4);
      const int col = n0 + wn * (GBN / GWN2) + j * 16 + (lane & 15);
      if (col >= 2 * Dp) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int d = rb + r;
        if (d < D) Gd[((size_t)d * p.Dmax + (col >> 1)) * 2 + (col & 1)] = acc[i][j][r];
      }
    }
}

// ---------------------------------------------------------------------------
// The expansion contraction, one workgroup per walker, sums in a fixed order.
// ---------------------------------------------------------------------------
struct MsdContractArgs {
  const int* srank;     // [nstr_tot]
  const int* saoff;     // [nstr_tot]
  const int* spos;      // [nstr_tot][2][KM]: hole slot -> H position, particle slot -> Q position
  const int* xa;        // [ncross] alpha string of a determinant excited in both spins
  const int* xb;        // [ncross] its beta string (concatenated index)
  const double* xc;     // [ncross] its coefficient
  const double2* sdet;  // [W][nstr_tot]
  const double2* sadj;  // [W][nadj_tot]
  const double2* uw;    // [W][nstr_tot]
  const double2* ratio; // [W] s
  const double2* G;     // [Wc][3][Dmax][Dmax]
  const double2* vj;    // [Wc][2][Dmax]
  const double2* vp;    // [Wc][2][Dmax]
  const double2* r1;    // [Wc][2][Dmax]
  const double2* sc;    // [Wc][4]
  const double* yp;     // planar Y [W][2][2][nmax][ldv] (zero-determinant strings)
  const int* hlist;     // [2][Hmax]
  const int* qlist;     // [2][Qmax]
  double2* part;        // [Wc][MSD_CT_SPLITS][3] partial sums of E1, EJ, EK
  double2* e;           // [W][3]
  int z0, nstr0, nstr_tot, nadj_tot, ncross, Dmax, nh[2], nmax, ldv, Hmax, Qmax;
};

__device__ __forceinline__ double2 cdivs(double2 a, double2 b) { return cmul(a, cinv(b)); }

// determinant of the leading n x n block of M (n <= KM; M is overwritten),
// elimination with partial pivoting
__device__ double2 small_det(double2 (&M)[KM][KM], int n) {
  double2 det = make_double2(1.0, 0.0);
  for (int c = 0; c < n; ++c) {
    int p = c;
    double best = cabs2(M[c][c]);
    for (int r = c + 1; r < n; ++r) {
      const double v = cabs2(M[r][c]);
      if (v > best) {
        best = v;
        p = r;
      }
    }
    if (best == 0.0) return make_double2(0.0, 0.0);
    if (p != c) {
      for (int j = 0; j < n; ++j) {
        const double2 t = M[c][j];
        M[c][j] = M[p][j];
        M[p][j] = t;
      }
      det = make_double2(-det.x, -det.y);
    }
    det = cmul(det, M[c][c]);
    const double2 ip = cinv(M[c][c]);
    for (int r = c + 1; r < n; ++r) {
      const double2 f = cmul(M[r][c], ip);
      for (int j = c + 1; j < n; ++j) M[r][j] = csub(M[r][j], cmul(f, M[c][j]));
    }
  }
  return det;
}

// sum_g [t^2] det(A + t R_g) for the string u of spin s (A = its Y block):
// sum over row pairs l1 < l2 and column pairs m1 < m2 of the signed
// complementary minor of A times sum_g det R_g[{l1, l2}][{m1, m2}]
__device__ double2 zero_det_quadratic(const MsdContractArgs& a, int u, int s, int k, int z, const double2* Gs) {
  const int nh = a.nh[s];
  int qo[KM], hp[KM];
  for (int l = 0; l < k; ++l) {
    qo[l] = a.spos[((size_t)u * 2 + 1) * KM + l] * nh;
    hp[l] = a.spos[((size_t)u * 2 + 0) * KM + l];
  }
  double2 A[KM][KM];
  const size_t yplane = (size_t)a.nmax * a.ldv;
  const double* yr = a.yp + ((size_t)(2 * z + 0) * 2 + s) * yplane;
  const double* yi = a.yp + ((size_t)(2 * z + 1) * 2 + s) * yplane;
  for (int l = 0; l < k; ++l) {
    const int av = a.qlist[s * a.Qmax + a.spos[((size_t)u * 2 + 1) * KM + l]];
    for (int m = 0; m < k; ++m) {
      const int h = a.hlist[s * a.Hmax + a.spos[((size_t)u * 2 + 0) * KM + m]];
      A[l][m] = make_double2(yr[(size_t)h * a.ldv + av], yi[(size_t)h * a.ldv + av]);
    }
  }
  double2 q2 = make_double2(0.0, 0.0);
  for (int l1 = 0; l1 < k; ++l1)
    for (int l2 = l1 + 1; l2 < k; ++l2)
      for (int m1 = 0; m1 < k; ++m1)
        for (int m2 = m1 + 1; m2 < k; ++m2) {
          double2 M[KM][KM];
          for (int r = 0, rr = 0; r < k; ++r) {
            if (r == l1 || r == l2) continue;
            for (int c = 0, cc = 0; c < k; ++c) {
              if (c == m1 || c == m2) continue;
              M[rr][cc++] = A[r][c];
            }
            ++rr;
          }
          double2 mn = small_det(M, k - 2);
          if ((l1 + l2 + m1 + m2) & 1) mn = make_double2(-mn.x, -mn.y);
          const double2 g2 = csub(Gs[(size_t)(qo[l1] + hp[m1]) * a.Dmax + qo[l2] + hp[m2]],
                                  Gs[(size_t)(qo[l1] + hp[m2]) * a.Dmax + qo[l2] + hp[m1]]);
          q2 = cadd(q2, cmul(mn, g2));
        }
  return q2;
}

// Workgroup (split, walker): strings u = split, split + MSD_CT_SPLITS, ...
// and the doubly excited determinants likewise; its partial sums of E1, EJ,
// EK (times s) go to part.  Each thread keeps the active-pair offsets of its
// current string in its own LDS column (indexed by slot).
__global__ __launch_bounds__(CT_T) void msd_contract_kernel(MsdContractArgs a) {
  __shared__ double2 red[CT_T / 64];
  __shared__ int otab[2 * KM][CT_T];  // [slot][thread]: particle offsets q nh, then hole positions
  const int sp_ = blockIdx.x, zl = blockIdx.y, z = a.z0 + zl, tid = threadIdx.x;
  const int first = sp_ * CT_T + tid, stride = MSD_CT_SPLITS * CT_T;
  const double2* uz = a.uw + (size_t)z * a.nstr_tot;
  const double2* dz = a.sdet + (size_t)z * a.nstr_tot;
  const double2* az = a.sadj + (size_t)z * a.nadj_tot;
  double2 e1 = make_double2(0.0, 0.0), ej = e1, ek = e1;
  for (int u = first; u < a.nstr_tot; u += stride) {
    const int k = a.srank[u];
    if (k == 0) continue;
    const int s = u >= a.nstr0 ? 1 : 0;
    const int nh = a.nh[s];
    const double2* adj = az + a.saoff[u];
    // d(l, m) = qo[l] + hp[m]: particle slot l, hole slot m
    int* qo = &otab[0][0] + tid;       // qo[l] at qo[l * CT_T]
    int* hp = &otab[KM][0] + tid;
    for (int l = 0; l < k; ++l) {
      qo[l * CT_T] = a.spos[((size_t)u * 2 + 1) * KM + l] * nh;
      hp[l * CT_T] = a.spos[((size_t)u * 2 + 0) * KM + l];
    }
    const double2* r1 = a.r1 + ((size_t)zl * 2 + s) * a.Dmax;
    const double2* vj = a.vj + ((size_t)zl * 2 + s) * a.Dmax;
    const double2* vp = a.vp + ((size_t)zl * 2 + s) * a.Dmax;
    const double2* Gs = a.G + ((size_t)zl * 3 + s) * a.Dmax * a.Dmax;
    double2 l1 = make_double2(0.0, 0.0), lj = l1, lp = l1, qj = l1, qk = l1;
    for (int m = 0; m < k; ++m) {
      const int hm = hp[m * CT_T];
      for (int l = 0; l < k; ++l) {
        const double2 f = adj[m * k + l];  // adj(A)[m][l] at (q_l, h_m)
        const int ql = qo[l * CT_T];
        const int d = ql + hm;
        l1 = cadd(l1, cmul(f, r1[d]));
        lj = cadd(lj, cmul(f, vj[d]));
        lp = cadd(lp, cmul(f, vp[d]));
        const double2* Gd = Gs + (size_t)d * a.Dmax;
        for (int m2 = 0; m2 < k; ++m2) {
          const int hm2 = hp[m2 * CT_T];
          const double2* Gl = Gs + (size_t)(ql + hm2) * a.Dmax + hm;
          const double2* Gdm = Gd + hm2;
          for (int l2 = 0; l2 < k; ++l2) {
            const int ql2 = qo[l2 * CT_T];
            const double2 ff = cmul(f, adj[m2 * k + l2]);
            qj = cadd(qj, cmul(ff, Gdm[ql2]));
            qk = cadd(qk, cmul(ff, Gl[ql2]));
          }
        }
      }
    }
    const double2 w = uz[u];
    e1 = csub(e1, cmul(w, l1));
    ej = csub(ej, cmul(w, lj));
    ek = cadd(ek, cmul(w, lp));
    const double2 dd = dz[u];
    if (dd.x != 0.0 || dd.y != 0.0) {
      const double2 f = cdivs(w, dd);
      ej = cadd(ej, cscale(cmul(f, qj), 0.5));
      ek = csub(ek, cscale(cmul(f, qk), 0.5));
    } else if (k >= 2) {
      ej = cadd(ej, cmul(w, zero_det_quadratic(a, u, s, k, z, Gs)));
    }
  }
  const double2* Gab = a.G + ((size_t)zl * 3 + 2) * a.Dmax * a.Dmax;
  for (int x = first; x < a.ncross; x += stride) {
    const int ua = a.xa[x], ub = a.xb[x];
    const int ka = a.srank[ua], kb = a.srank[ub];
    const double2* adja = az + a.saoff[ua];
    const double2* adjb = az + a.saoff[ub];
    int* qb = &otab[0][0] + tid;  // the beta string's offsets
    int* hb = &otab[KM][0] + tid;
    for (int l = 0; l < kb; ++l) {
      qb[l * CT_T] = a.spos[((size_t)ub * 2 + 1) * KM + l] * a.nh[1];
      hb[l * CT_T] = a.spos[((size_t)ub * 2 + 0) * KM + l];
    }
    double2 cr = make_double2(0.0, 0.0);
    for (int m = 0; m < ka; ++m)
      for (int l = 0; l < ka; ++l) {
        const int d = a.spos[((size_t)ua * 2 + 1) * KM + l] * a.nh[0] + a.spos[((size_t)ua * 2 + 0) * KM + m];
        const double2* Gd = Gab + (size_t)d * a.Dmax;
        double2 inner = make_double2(0.0, 0.0);
        for (int m2 = 0; m2 < kb; ++m2) {
          const double2* Gdm = Gd + hb[m2 * CT_T];
          for (int l2 = 0; l2 < kb; ++l2) inner = cadd(inner, cmul(adjb[m2 * kb + l2], Gdm[qb[l2 * CT_T]]));
        }
        cr = cadd(cr, cmul(adja[m * ka + l], inner));
      }
    ej = cadd(ej, cscale(cr, a.xc[x]));
  }
  e1 = block_sum2(e1, red);
  ej = block_sum2(ej, red);
  ek = block_sum2(ek, red);
  if (tid == 0) {
    double2* o = a.part + ((size_t)zl * MSD_CT_SPLITS + sp_) * 3;
    o[0] = e1;
    o[1] = ej;
    o[2] = ek;
  }
}

// Per walker: the splits' partial sums in a fixed order, the reference's
// terms s sum_g ..., division by s.
__global__ void msd_contract_final_kernel(MsdContractArgs a, int nz) {
  const int zl = blockIdx.x * blockDim.x + threadIdx.x;
  if (zl >= nz) return;
  const int z = a.z0 + zl;
  double2 e1 = make_double2(0.0, 0.0), ej = e1, ek = e1;
  for (int sp = 0; sp < MSD_CT_SPLITS; ++sp) {
    const double2* o = a.part + ((size_t)zl * MSD_CT_SPLITS + sp) * 3;
    e1 = cadd(e1, o[0]);
    ej = cadd(ej, o[1]);
    ek = cadd(ek, o[2]);
  }
  const double2 s = a.ratio[z];
  const double2* sc = a.sc + (size_t)zl * 4;
  e1 = cadd(e1, cmul(s, sc[3]));
  ej = cadd(ej, cscale(cmul(s, sc[0]), 0.5));
  ek = csub(ek, cscale(cmul(s, cadd(sc[1], sc[2])), 0.5));
  const double2 is = cinv(s);
  a.e[(size_t)z * 3 + 0] = cmul(e1, is);
  a.e[(size_t)z * 3 + 1] = cmul(ej, is);
  a.e[(size_t)z * 3 + 2] = cmul(ek, is);
}

// rotated rows: lr[g][r][ldL] from the GEMM output out[(g, p)][r] (K1 N x S)
__global__ void msd_lr_pack_kernel(long total, int N, int S, int ldL, const double* __restrict__ out,
                                   double* __restrict__ lr) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;  // over (g, r, p)
  if (e >= total) return;
  const long gr = e / N;
  const int p = (int)(e - gr * N);
  const long g = gr / S;
  const int r = (int)(gr - g * S);
  lr[gr * ldL + p] = out[(g * N + p) * S + r];
}

}  // namespace

hipError_t msd_energy_set_attributes(size_t rp_lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(msd_rp_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)rp_lds);
}

size_t msd_energy_rp_lds(const MsdEnergyDims& e) {
  return (size_t)(2 * e.Smax * e.nmax + 2 * e.nmax * e.Qmax + 2 * e.Qmax * e.nmax) * sizeof(double) +
         (size_t)e.gchunk * sizeof(double2);
}

hipError_t msd_lr_pack(long rows_gp, int N, int S, int ldL, const double* out, double* lr, hipStream_t s) {
  const long total = rows_gp / N * (long)S * N;  // K1 S N entries
  hipLaunchKernelGGL(msd_lr_pack_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, N, S, ldL,
                     out, lr);
  return hipGetLastError();
}

hipError_t launch_msd_energy_chunk(const MsdDims& m, const MsdEnergyDims& e, const MsdEnergyTables& t, int z0,
                                   int nz, const double* theta, const double* yp, const double2* sdet,
                                   const double2* sadj, const double2* uw, const double2* ratio,
                                   const MsdEnergyWork& w, double2* eout, hipStream_t s) {
  hipError_t err;
  // U per spin
  for (int sp = 0; sp < 2; ++sp) {
    const int n = sp ? m.nb : m.na;
    if (n == 0) continue;
    MsdUProb p{t.lr[sp], theta, (long)(e.K + 1) * e.S[sp], nz * 2 * n, z0, sp, n, m.nmax, m.ldN, e.ldL};
    const dim3 grid((unsigned)((p.rows + UBM - 1) / UBM), (unsigned)ceil_div(p.cols, UBN));
    hipLaunchKernelGGL(msd_u_kernel, grid, dim3(UWM * UWN * 64), 0, s, p, e.S[sp], e.Smax, e.K + 1, w.u);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  // r, p per (walker, chunk)
  {
    MsdRpArgs a{};
    a.u = w.u;
    a.yp = yp;
    a.hlist = t.hlist;
    a.qlist = t.qlist;
    a.rbuf = w.rbuf;
    a.jpart = w.jpart;
    a.ppart = w.ppart;
    a.tt = w.tt;
    a.kt = w.kt;
    a.r1 = w.r1;
    a.z0 = z0;
    a.K = e.K;
    a.K1 = e.K + 1;
    a.nmax = m.nmax;
    a.ldv = m.ldv;
    a.Smax = e.Smax;
    a.ldG = e.ldG;
    a.gchunk = e.gchunk;
    a.nchunk = e.nchunk;
    a.Hmax = e.Hmax;
    a.Qmax = e.Qmax;
    a.Dmax = e.Dmax;
    for (int sp = 0; sp < 2; ++sp) {
      a.n[sp] = sp ? m.nb : m.na;
      a.S[sp] = e.S[sp];
      a.nh[sp] = e.nh[sp];
      a.nq[sp] = e.nq[sp];
    }
    const int nqm = std::max(e.nq[0], e.nq[1]), nhm = std::max(e.nh[0], e.nh[1]);
    const dim3 gm((unsigned)ceil_div(2 * e.nchunk, RPM_WAVES), (unsigned)nz), bm(RPM_WAVES * 64);
    if (nhm <= 16 && nqm <= 32 && m.nmax <= 32) {
      // the matrix-core kernel: windows of <= 32 particles, <= 16 holes, <= 32 electrons
      if (nqm <= 16 && m.nmax <= 16)
        hipLaunchKernelGGL((msd_rp_mfma_kernel<1, 1>), gm, bm, 0, s, a);
      else if (nqm <= 16)
        hipLaunchKernelGGL((msd_rp_mfma_kernel<1, 2>), gm, bm, 0, s, a);
      else if (m.nmax <= 16)
        hipLaunchKernelGGL((msd_rp_mfma_kernel<2, 1>), gm, bm, 0, s, a);
      else
        hipLaunchKernelGGL((msd_rp_mfma_kernel<2, 2>), gm, bm, 0, s, a);
    } else {
      hipLaunchKernelGGL(msd_rp_kernel, dim3(e.nchunk, nz), dim3(RP_T), msd_energy_rp_lds(e), s, a);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  hipLaunchKernelGGL(msd_sums_kernel, dim3(nz), dim3(256), 0, s, e.K, e.K + 1, e.nchunk, e.Dmax, e.D[0], e.D[1], w.jpart,
                     w.ppart, w.tt, w.kt, w.vj, w.vp, w.sc);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if (e.Dmax > 0) {  // no active pairs (a single reference): no Gram matrices
    MsdGramProb p{reinterpret_cast<const double*>(w.rbuf), e.Dmax, e.ldG, e.D[0], e.D[1]};
    const dim3 grid((unsigned)ceil_div(e.Dmax, GBM), (unsigned)ceil_div(2 * e.Dmax, GBN), (unsigned)(3 * nz));
    hipLaunchKernelGGL(msd_gram_kernel, grid, dim3(GWM2 * GWN2 * 64), 0, s, p, 2 * e.K, w.G);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  {
    MsdContractArgs a{};
    a.srank = t.srank;
    a.saoff = t.saoff;
    a.spos = t.spos;
    a.xa = t.xa;
    a.xb = t.xb;
    a.xc = t.xc;
    a.sdet = sdet;
    a.sadj = sadj;
    a.uw = uw;
    a.ratio = ratio;
    a.G = w.G;
    a.vj = w.vj;
    a.vp = w.vp;
    a.r1 = w.r1;
    a.sc = w.sc;
    a.e = eout;
    a.z0 = z0;
    a.nstr0 = m.nstr[0];
    a.nstr_tot = m.nstr_tot;
    a.nadj_tot = m.nadj_tot;
    a.ncross = t.ncross;
    a.Dmax = e.Dmax;
    a.nh[0] = e.nh[0];
    a.nh[1] = e.nh[1];
    a.yp = yp;
    a.hlist = t.hlist;
    a.qlist = t.qlist;
    a.nmax = m.nmax;
    a.ldv = m.ldv;
    a.Hmax = e.Hmax;
    a.Qmax = e.Qmax;
    a.part = w.cpart;
    hipLaunchKernelGGL(msd_contract_kernel, dim3(MSD_CT_SPLITS, nz), dim3(CT_T), 0, s, a);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(msd_contract_final_kernel, dim3((unsigned)ceil_div(nz, 64)), dim3(64), 0, s, a, nz);
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  return hipSuccess;
}
