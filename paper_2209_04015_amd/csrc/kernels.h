// Internal launchers of the walker-step kernels (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "exchange_pair.h"

// Sizes shared by every kernel of one Hamiltonian.
struct StepDims {
  int N;      // spatial orbitals
  int na, nb; // electrons per spin
  int nmax;   // max(na, nb)
  int K;      // Cholesky vectors
  int ldN;    // padded orbital stride of theta / Lh rows (multiple of 16)
  int ldK;    // padded Cholesky stride of xs / LT rows (multiple of 16)
  int ldV;    // padded row stride (in real elements) of VHS rows, >= 2N, multiple of 16
  int ldP;    // padded row stride of P (multiple of 16)
  int ncol;   // 2 (na + nb): real columns of a walker's spin-concatenated orbitals
  int ncolp;  // ncol rounded up to a multiple of 4
  int Npk;    // N (N + 1) / 2 packed (p <= q) pairs
  int ldh;    // padded orbital stride of hi/lo split rows (multiple of 32)
  int ldhK;   // padded Cholesky stride of hi/lo split rows (multiple of 32)
};

// hi/lo split formats of the 16-bit contraction modes
enum { SPLIT_NONE = 0, SPLIT_BF16 = 1, SPLIT_F16 = 2 };

// Exchange tile choice: G Cholesky vectors x Z walkers per workgroup.
struct ExTile {
  int G, Z;
};

// --- Green's function / overlap --------------------------------------------
// theta: working-precision planar [W][2 re/im][2 spin][nmax][ldN] (nullable)
// logdet: [W][2] complex log det(PhiT^T phi) per spin; e1: [W][2] (nullable)
template <typename T>
hipError_t launch_gf(const StepDims& d, int W, const double2* phi_a, const double2* phi_b,
                     const double* phiT, const double* hh, T* theta, double2* logdet,
                     double2* e1, int* status, hipStream_t s);

template <typename T>
hipError_t launch_force_bias(const StepDims& d, int W, const T* Lh, const T* theta,
                             double2* vbias, hipStream_t s);

// x = x_base + (ctr ? ctr[0] * x_step : 0)
template <typename T>
// tmax: tslots running-maximum slots of stride tstride, zeroed per walker
hipError_t launch_shift(const StepDims& d, int W, const double2* vbias, const double* x, const int* ctr,
                        long x_step, T* xs, double2* a, unsigned* tmax, int tslots, int tstride, double sdt,
                        const float* lmax, hipStream_t s);
// m_g = max |L_g| per Cholesky vector (FP32, rounded up): with lmax non-null
// the shift also writes each walker's |VHS| bound into tmax slot 1
hipError_t setup_lmax(int K, int N, const double* L, float* lmax, hipStream_t s);

template <typename T>
hipError_t launch_vhs(const StepDims& d, int W, const T* xs, const T* LT, const int2* pq, T* vhs,
                      double sdt, hipStream_t s);

// out = P in, FP64.  mode 0: in = caller walkers, out -> acc (+ per-walker max |.| into tmax)
//                     mode 1: in = acc, out -> caller walkers
template <typename T>
hipError_t launch_pphi(const StepDims& d, int W, const double* P, const double2* phi_a_in,
                       const double2* phi_b_in, double* acc, double2* phi_a_out,
                       double2* phi_b_out, unsigned* tmax, int mode, hipStream_t s);

// t_out = VHS t_in / k; k == 1 reads t_in from acc (= P phi).  Launch k adds
// term k-1 to acc, the last launch (k == order) also adds term k.
template <typename T>
hipError_t launch_taylor(const StepDims& d, int W, const T* vhs, const T* t_in, T* t_out,
                         double* acc, const unsigned* tmax, int k, int order, hipStream_t s);

hipError_t launch_weight(int W, const double2* logdet, const double* corr, const double2* a,
                         double2* log_ovlp, double* log_w, double cst, int* status,
                         hipStream_t s);

hipError_t launch_overlap_store(int W, const double2* logdet, double2* log_ovlp, hipStream_t s);

template <typename T>
ExTile exchange_tile(int n);
// one spin (sp = 0 alpha, 1 beta) of the exchange energy; part[s][g-tile][z]
// gs: Cholesky tiles per L2 group of the XCD-aware tile order (< 1: default)
template <typename T>
hipError_t launch_exchange(const StepDims& d, int W, const T* Lh, const T* theta, double2* part,
                           int sp, int* ntg_out, hipStream_t s, int gs = 0);

// e = e_out + (ctr ? ctr[0] * e_step : 0)
hipError_t launch_energy(const StepDims& d, int W, const double2* e1, const double2* vbias,
                         const double2* part, int ntg, double2* e_out, const int* ctr, long e_step,
                         hipStream_t s);
// device step counter of captured graphs (a kernel, not a memset node)
hipError_t launch_counter_advance(int* ctr, hipStream_t s);
hipError_t launch_counter_set(int* ctr, int v, hipStream_t s);

// QR of every walker and spin (Cholesky QR, twice); corr[W][2] = sum ln R_ii.
hipError_t launch_qr(const StepDims& d, int W, double2* phi_a, double2* phi_b, double* corr,
                     int* status, hipStream_t s);
hipError_t launch_ortho_update(int W, const double* corr, double2* log_ovlp, double* log_w, hipStream_t s);

hipError_t set_kernel_attributes(const StepDims& d);

// --- hi/lo split contraction (split_kernels.hip) ----------------------------
// rows of an FP32 matrix -> split rows (per block of 32 indices: 32 hi then
// 32 lo 16-bit values, 2 ldh halves per row) plus the inverse power-of-two
// row scales
hipError_t launch_split_rows_mode(int mode, long nrows, int ncols, const float* src, int ld_src,
                                  unsigned short* dst, int ldh, float* unscale, hipStream_t s);
// The FP32 shift (launch_shift<float>: the sums a and the |VHS| bound in
// tmax) with its rows written only as split rows (rows 2 z and 2 z + 1 of
// xs_split, 2 ldhK halves, scales xs_unscale), as launch_split_rows_mode over
// the FP32 shifted fields stores them; for ldhK that shift_split_fits accepts
// (hipErrorInvalidValue otherwise).
bool shift_split_fits(int ldhK);
hipError_t launch_shift_split(int mode, const StepDims& d, int W, const double2* vbias, const double* x,
                              const int* ctr, long x_step, unsigned short* xs_split, float* xs_unscale, double2* a,
                              unsigned* tmax, int tslots, int tstride, double sdt, const float* lmax,
                              hipStream_t s);
ExTile exchange_split_tile(int n);
// Walker-tile shapes of the split VHS and pair-exchange kernels (autotuner
// choices): WIDE 80 walkers per tile, NARROW 32 (more workgroups for systems
// with few walkers).  Every output element sums over the same rows in the
// same order in both shapes, so the choice does not change any result bit.
constexpr int SPLIT_TILE_WIDE = 0, SPLIT_TILE_NARROW = 1;
// FP32 output (split_out false): vhs [W][N][ldV] interleaved complex; vmax
// (optional) per-walker max |VHS| (atomic, bit patterns of floats).
// Split output: the same layout with each entry's 8 bytes holding fp16
// (hi Re, hi Im, lo Re, lo Im) of the entry scaled by
// 2^vhs_split_exp(vmax[z]), where vmax (required, read) holds each walker's
// |VHS| bound.  lt: block-packed L split rows (vhs_split_pairs order), blk:
// the blocks.
hipError_t launch_vhs_split(int mode, const StepDims& d, int W, const unsigned short* xs, const float* xs_unscale,
                            const unsigned short* lt, const float* lt_unscale, const int2* blk, int nblk, float* vhs,
                            unsigned* vmax, bool split_out, double sdt, hipStream_t s, int tile = SPLIT_TILE_WIDE);
// blocks of orbital pairs of the split VHS and the pair of each packed row
std::vector<int2> vhs_split_blocks(int N);
std::vector<int2> vhs_split_pairs(int N, const std::vector<int2>& blk);
// Block split: one power-of-two scale per block of nspl x nsub source rows
// (row s * S1 + b * S2 + i of block b), output rows contiguous per block
hipError_t launch_split_blocks_mode(int mode, int nblocks, int nspl, int nsub, int ncols, const float* src, int ld_src,
                                    long S1, long S2, unsigned short* dst, int ldh, float* unscale, hipStream_t s);
// Block split (one scale per block of rows consecutive source rows) and row
// split (one scale per row) of the same rows in one pass: output row
// b * rows + r of dst_blk and dst_row, scales unscale_blk[b] and
// unscale_row[b * rows + r]; bit for bit what launch_split_blocks_mode
// (nspl 1, nsub rows) and launch_split_rows_mode write.  Only for blocks of
// rows and ldh that split_both_fits accepts (hipErrorInvalidValue otherwise).
bool split_both_fits(int rows, int ldh);
hipError_t launch_split_both_mode(int mode, int nblocks, int rows, int ncols, const float* src, int ld_src,
                                  int ldh, unsigned short* dst_blk, float* unscale_blk, unsigned short* dst_row,
                                  float* unscale_row, hipStream_t s);
// vbias = sum_k theta_k Lh_k on block-split operands, the k range in at most
// FB_SPLIT_CHUNKS chunks (chosen per launch); part: [FB_SPLIT_CHUNKS][2 W][K] floats
constexpr int FB_SPLIT_CHUNKS = 8;
hipError_t launch_force_bias_split(int mode, const StepDims& d, int W, const unsigned short* th, const float* th_unscale,
                                   const unsigned short* lh, const float* lh_unscale, float* part, double2* vbias,
                                   hipStream_t s);
// The packed L transposed for the multi-determinant force bias: one split row
// per Cholesky vector g over the pair index c of the row-major upper triangle
// (pq[c] = (p, q), p <= q), 2 ldh halves, scale per g; L is [K][N][N] FP64.
hipError_t setup_split_lt_transposed(int mode, int K, int N, int npk, int ldh, const int2* pq, const double* L,
                                     unsigned short* dst, float* unscale, hipStream_t s);
// vbias [W][K] complex = sum_c gs[(z, re|im)][c] L_g[c]: gs [2 W][ldh] FP32 rows
// (the first npk meaningful) are split in place into rows of 2 ldh halves
// (scales into gs_unscale [2 W]), then contracted with the transposed split L
// on the split engine; part: [FB_SPLIT_CHUNKS][2 W][K] floats.
hipError_t launch_msd_fb_split(int mode, int W, int K, int npk, int ldh, float* gs, float* gs_unscale,
                               const unsigned short* lts, const float* lts_unscale, float* part, double2* vbias,
                               hipStream_t s);
// Taylor order k on split operands: t_k = VHS t_{k-1} / k (t_0 = acc, FP64)
hipError_t launch_taylor_split(int mode, const StepDims& d, int W, const float* vhs, const float* t_in,
                               float* t_out, const double* acc, unsigned* tmax, int tstride, int k,
                               hipStream_t s);
// acc += t_1 + ... + t_order (terms [order][W][N][ncolp])
hipError_t launch_taylor_split_sum(const StepDims& d, int W, int order, const float* terms, double* acc,
                                   hipStream_t s);
hipError_t launch_exchange_split(int mode, const StepDims& d, int W, const unsigned short* lh,
                                 const float* lh_unscale, const unsigned short* th, const float* th_unscale,
                                 double2* part, int sp, int* ntg_out, hipStream_t s, int gs = 0);
size_t qr_lds_bytes(const StepDims& d);
size_t qr_lds_bytes_for(int N, int n);

// --- ensemble (control_kernels.hip) ------------------------------------------
// out[4] = {Re E, Im E, ln sum w, live walkers} of E = sum w E_L / sum w
hipError_t launch_global_energy(int nw, const double* log_w, const double2* e, double* out, hipStream_t s);
// comb population control in place; parent[nw] out; csum/cnt/src: [nw] scratch
hipError_t launch_comb(const StepDims& d, int nw, double u, double2* phi_a, double2* phi_b, double2* log_ovlp,
                       double* log_w, double* csum, int* cnt, int* src, int* parent, int* status, hipStream_t s);
// The comb on the library's static scratch (no allocation): walkers up to
// COMB_STATIC_MAX_WALKERS.  comb_static_scratch gives the scratch's address on
// the current device (looked up once per device).
constexpr int COMB_STATIC_MAX_WALKERS = 65536;
hipError_t comb_static_scratch(void** ptr);
hipError_t launch_comb_static(void* scratch_ptr, const StepDims& d, int nw, double u, double2* phi_a,
                              double2* phi_b, double2* log_ovlp, double* log_w, int* parent, int* status,
                              hipStream_t s);

// --- fused propagation P T(VHS) P phi on split fp16 operands (prop_kernels.hip) ---
struct PropFusedGeom {
  int RT, QP, QCH, TQS, CT, nkbP;
  size_t lds_bytes, psplit_halves;
  bool ok;  // the shape fits the kernel (N <= 320, n_s <= 32, LDS)
};
PropFusedGeom prop_fused_geom(const StepDims& d);
// P (FP64 [N][ldP]) into its split copy with the power-of-two scale 2^pexp
// (pexp out, host; synchronises s); sets the kernel's LDS attribute.
hipError_t setup_prop_fused(const StepDims& d, const double* P, unsigned short* psplit, unsigned* pmax_scratch,
                            int* pexp_host, hipStream_t s);
// phi <- P T_order(VHS) P phi for W walkers in place; vhs: the split rows
// of launch_vhs_split (split output), vbound [W] the |VHS| bounds they were
// scaled by
hipError_t launch_prop_fused(const StepDims& d, int W, double2* phi_a, double2* phi_b, const float* vhs,
                             const unsigned* vbound, const unsigned short* psplit, int pexp, int order,
                             hipStream_t s);

// --- mixed estimators (estimator_kernels.hip) ---------------------------------
// G [W][2][N][N] complex: G_pq = sum_i PhiT[p][i] theta[q][i] per spin
template <typename T>
hipError_t launch_green_full(const StepDims& d, int W, const T* theta, const double* phiT, double2* G,
                             hipStream_t s);
// s2 [W] complex: nb + Ms (Ms + 1) - tr(G^a G^b)
template <typename T>
hipError_t launch_s2(const StepDims& d, int W, const T* theta, const double* phiT, double2* s2, hipStream_t s);
// out [2 m + 2]: weighted means of the m columns of v [nw][m], ln sum w, live walkers
hipError_t launch_weighted_mean(int nw, int m, const double* log_w, const double2* v, double* out, hipStream_t s);

// --- exchange through pair integrals (exchange_pair.h) -------------------------
struct PairLaunch {
  const PairTab* tab;  // device tables of this spin
  int ntiles;          // row tiles of this spin
  int ntg;             // row tiles of the larger spin (stride of the partials)
  long vrow0;          // first pair-integral row of this spin
};
// rows per tile (the tables are built for it)
int exchange_pair_split_rows();
template <typename T>
int exchange_pair_rows();
// one spin; part[sp][row tile][z] (zeros past this spin's tiles)
hipError_t launch_exchange_pair_split(int mode, const StepDims& d, int W, const PairLaunch& pl,
                                      const unsigned short* v, const float* v_unscale, const unsigned short* th,
                                      const float* th_unscale, const float* theta, double2* part, int sp,
                                      hipStream_t s, int gs = 0, int tile = SPLIT_TILE_WIDE);
template <typename T>
hipError_t launch_exchange_pair(const StepDims& d, int W, const PairLaunch& pl, const T* v, const T* theta,
                                double2* part, int sp, hipStream_t s, int gs = 0);

// --- multi-determinant trial (msd_kernels.hip) ---------------------------------
constexpr int MSD_KMAX = 6;  // excitation rank per spin (AFQMC_MSD_MAX_RANK)

struct MsdDims {
  int N, na, nb, nmax;
  int ldN;       // orbital stride of theta (as StepDims::ldN)
  int nv[2];     // virtual orbitals per spin, N - n_s
  int ldv;       // virtual stride of Y and C_virt (>= max nv, multiple of 4)
  int ldq;       // electron stride of planar Q (nmax rounded up to 2)
  int nstr[2];   // excitation strings per spin (concatenated: alpha, then beta)
  int nstr_tot;
  int nadj_tot;  // adjugate entries of all strings (sum of k^2)
  int big0[2];   // first string of rank > 4 of each spin (concatenated index; strings sorted by rank)
  int nbig[2];   // strings of rank > 4 of each spin
  int ntask;     // expansion-sum tasks (CSR rows cut into pieces of at most MSD_TASK entries)
};
constexpr int MSD_TASK = 16;

// Device tables of one expansion.
struct MsdTables {
  const double* cocc;   // [2][N][nmax]  reference orbitals C_s[:, :n_s]
  const double* cvirt;  // [2][N][ldv]   C_s[:, n_s:], zero-padded
  const double* cfull;  // [2][N][ldN]   C_s, zero-padded
  const int* srank;     // [nstr_tot]    k of each string
  const int* sorb;      // [nstr_tot][2][MSD_KMAX] holes; particles as virtual index q - n_s
  const int* saoff;     // [nstr_tot]    first adjugate entry of the string
  const int* crow;      // [nstr_tot + 1] CSR over strings: determinants with that string
  const double* ccoef;  // [2 ndet]      c_a
  const int* cstr;      // [2 ndet]      the determinant's string of the other spin (concatenated index)
  const int* tbeg;      // [ntask + 1]   first CSR entry of each task (tasks in string order)
  const int* trow;      // [nstr_tot + 1] first task of each string
  const int* erow;      // [na nv_a + nb nv_b + 1] CSR over (spin, hole j, virtual a) entries of M
  const int* estr;      // string of each contribution
  const int* eoff;      // adjugate entry of each contribution
};

// workgroups of the expansion sums per walker (rpart holds W of these partials)
int msd_combine_blocks(const MsdDims& m);
// theta [W][2][2][nmax][ldN] FP64 (launch_gf) -> planar Y yp [W][2][2][nmax][ldv], string dets
// sdet [W][nstr_tot], adjugates sadj [W][nadj_tot], string weights uw [W][nstr_tot],
// task sums tpart [W][ntask], partial sums rpart [W][msd_combine_blocks],
// overlap ratios ratio [W] relative to the reference determinant; the
// adjugates only with want_adj (the overlap alone needs none)
hipError_t launch_msd_ratio(const MsdDims& m, int W, const MsdTables& t, const double* theta, double* yp,
                            double2* sdet, double2* sadj, double2* tpart, double2* uw, double2* rpart,
                            double2* ratio, bool want_adj, hipStream_t s);
// out [W] = logdet[z][0] + logdet[z][1] + log ratio[z]
hipError_t launch_msd_overlap_store(int W, const double2* logdet, const double2* ratio, double2* out, int* status,
                                    hipStream_t s);
// out [W][2] = (log <Psi_T|phi_z>, 0): the per-spin pair layout of the weight update
hipError_t launch_msd_overlap_pairs(int W, const double2* logdet, const double2* ratio, double2* out, int* status,
                                    hipStream_t s);
// after launch_msd_ratio: planar Zt zt [W][2][2][nmax][ldN] (M / s in the
// virtual columns, I - M Y / s in the occupied ones), planar Q qp
// [W][2][2][N][ldq], G [W][2][N][N] complex
hipError_t launch_msd_green(const MsdDims& m, int W, const MsdTables& t, const double* theta, const double* yp,
                            const double2* sadj, const double2* uw, const double2* ratio, double* zt, double* qp,
                            double2* G, hipStream_t s);
// after launch_msd_ratio: M / s and the occupied block into zt, Q into qp
hipError_t launch_msd_q(const MsdDims& m, int W, const MsdTables& t, const double* yp, const double2* sadj,
                        const double2* uw, const double2* ratio, double* zt, double* qp, hipStream_t s);
// pair-range splits of the force-bias GEMM whose scratch (packed G of gs_elem_bytes
// per value, then FP64 partials) fits scratch_bytes (0: does not fit)
int msd_fb_splits(int W, int N, int K, int ldK, int ldpk, size_t gs_elem_bytes, size_t scratch_bytes);
// after launch_msd_q: vbias [W][K] complex = sum_s sum_pq G^s_pq L_g,pq through the packed
// symmetric G (scratch: [W][2][ldpk] values of T, then [nsplit][2 W][ldK] doubles) and the
// packed L lt [N (N + 1) / 2][ldK] of type T (row-major upper triangle)
template <typename T>
hipError_t launch_msd_force_bias(const MsdDims& m, int W, const double* theta, const double* qp, const T* lt, int K,
                                 int ldK, int ldpk, int nsplit, void* scratch, double2* vbias, hipStream_t s);
// after launch_msd_q: only the packed symmetric G, gs [W][2][ldpk] FP32 (entries
// past the triangle are not written)
hipError_t launch_msd_gsym_f32(const MsdDims& m, int W, const double* theta, const double* qp, int ldpk, float* gs,
                               hipStream_t s);

// --- local energy of the multi-determinant trial (msd_energy.hip) --------------
struct MsdEnergyDims {
  int K;               // Cholesky vectors (rotated block K holds h1)
  int S[2], Smax;      // rotated rows per spin: n_s occupied + the active particles
  int nh[2], nq[2];    // active holes / particles per spin
  int Hmax, Qmax;      // their maxima (strides of the lists)
  int D[2], Dmax;      // nq * nh per spin (<= 1024)
  int ldL;             // orbital stride of the rotated rows (= MsdDims::ldN)
  int ldG;             // Cholesky stride of the r rows (>= K)
  int gchunk, nchunk;  // Cholesky blocks per workgroup of the r / p kernel, and their count over K + 1
  int Wc;              // walkers per pass
  int nmax;            // electron stride (MsdDims::nmax)
};
struct MsdEnergyTables {
  const double* lr[2];  // [K + 1][S_s][ldL] rotated rows C_S^T L_g (g < K), C_S^T h1 (g = K)
  const int* hlist;     // [2][Hmax] active holes
  const int* qlist;     // [2][Qmax] active particles (virtual index)
  const int* spos;      // [nstr_tot][2][MSD_KMAX] slot positions in H (holes) and Q (particles)
  const int* srank;
  const int* saoff;
  const int* xa;        // determinants excited in both spins: alpha string,
  const int* xb;        // beta string (concatenated index),
  const double* xc;     // coefficient
  int ncross;
};
struct MsdEnergyWork {
  double* u;       // [Wc][2][K + 1][2][Smax][nmax]
  double2* rbuf;   // [Wc][2][ldG][Dmax]
  double2* jpart;  // [Wc][2][nchunk][Dmax]
  double2* ppart;  // [Wc][2][nchunk][Dmax]
  double2* tt;     // [Wc][2][K + 1]
  double2* kt;     // [Wc][2][K]
  double2* r1;     // [Wc][2][Dmax]
  double2* vj;     // [Wc][2][Dmax]
  double2* vp;     // [Wc][2][Dmax]
  double2* sc;     // [Wc][4]
  double2* G;      // [Wc][3][Dmax][Dmax]
  double2* cpart;  // [Wc][MSD_CT_SPLITS][3] contraction partial sums
};
// workgroups per walker of the expansion contraction
constexpr int MSD_CT_SPLITS = 32;
size_t msd_energy_rp_lds(const MsdEnergyDims& e);
hipError_t msd_energy_set_attributes(size_t rp_lds);
// lr[g][r][ldL] from out[(g, p)][r] (rows_gp = (K + 1) N rows of S)
hipError_t msd_lr_pack(long rows_gp, int N, int S, int ldL, const double* out, double* lr, hipStream_t s);
// local energies e[z][3] of walkers z0 .. z0 + nz - 1 (nz <= Wc) from the
// reference theta, Y, string dets, adjugates, string weights and ratios of
// launch_msd_ratio (want_adj)
hipError_t launch_msd_energy_chunk(const MsdDims& m, const MsdEnergyDims& e, const MsdEnergyTables& t, int z0,
                                   int nz, const double* theta, const double* yp, const double2* sdet,
                                   const double2* sadj, const double2* uw, const double2* ratio,
                                   const MsdEnergyWork& w, double2* eout, hipStream_t s);
