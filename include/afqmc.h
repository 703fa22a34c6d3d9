/*
 * afqmc.h -- C ABI of the MI355X phaseless-AFQMC walker-step library.
 *
 * Method: phaseless auxiliary-field quantum Monte Carlo as described in
 * arXiv 2209.04015 (ipie), Sec. II.B (propagator, importance sampling,
 * phaseless weights) and Sec. III (overlap, Green's function, force bias,
 * local energy) for a single-determinant trial.
 *
 * Conventions used by every call
 *   N        number of spatial orbitals (the paper's M)
 *   na, nb   electrons of spin alpha / beta (the paper's N splits into these)
 *   K        number of Cholesky vectors (the paper's N_aux)
 *   nw       number of walkers in a call, 0 <= nw <= max_walkers
 *   complex  numbers are interleaved (re, im) pairs of double ("double2")
 *   arrays   are dense, row-major, with the shapes given in brackets
 *
 * Memory: arguments named host_* are host pointers.  Every other array
 * argument is a DEVICE pointer on the device that was current when the
 * Hamiltonian was created, and must be 16-byte aligned (any torch
 * allocation is).  The library never frees caller memory and never writes
 * arrays passed as const.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = null stream).
 * afqmc_init_hamiltonian may allocate and synchronise.  All other calls
 * except afqmc_get_status are asynchronous on `stream`, do not allocate and
 * do not synchronise.  One Hamiltonian handle serves one stream at a time:
 * its workspace is shared by all calls on it.
 *
 * Errors: every call returns 0 (AFQMC_OK) or an AFQMC_E* code; the text of
 * the last error of the calling thread is available from afqmc_last_error().
 * Numerical events inside kernels (singular overlap, non-finite values) do
 * not fail a call: they set bits of a device status word (afqmc_get_status)
 * and the affected walker gets log weight -inf, which is how the method
 * discards a walker (Eq. ph: max(0, cos theta) = 0).
 */
#ifndef AFQMC_H
#define AFQMC_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
  AFQMC_OK = 0,
  AFQMC_EINVAL = 1,        /* bad argument or shape */
  AFQMC_ENOMEM = 2,        /* device allocation failed (init, afqmc_msd_create) */
  AFQMC_EHIP = 3,          /* a HIP runtime call failed */
  AFQMC_EUNSUPPORTED = 4   /* shape outside what the kernels support */
};

/* Working precision.  In every mode the walkers stay FP64 in memory, and the
 * overlaps, determinants, Green's functions theta (Gauss-Jordan in FP64),
 * weights, QR and every energy sum are FP64.  The modes differ in the
 * contractions:
 *   AFQMC_FP64    every contraction on the FP64 matrix cores
 *   AFQMC_FP32    force bias, VHS build, Taylor products, exchange and both
 *                 one-body half steps P phi (Eq. Bx, split as in
 *                 afqmc_propagate) on the FP32 matrix cores: operands
 *                 rounded to FP32, FP32 accumulation; the Taylor terms are
 *                 summed in FP64
 *   AFQMC_BF16X3  as AFQMC_FP32, except that the exchange contraction
 *                 (Sec. III.C, the quartic term) splits each FP32 operand
 *                 into bf16 hi + lo and keeps the three leading products on
 *                 the bf16 matrix cores (relative operand error ~2^-16)
 *   AFQMC_FP16X3  as AFQMC_FP32, except that the force bias, the VHS build,
 *                 the Taylor products and the exchange split their FP32
 *                 operands into fp16 hi + lo with power-of-two scales and
 *                 keep the three leading products on the fp16 matrix cores
 *                 (relative operand error ~2^-22, close to FP32).  The
 *                 propagation P T(VHS) P phi (Eq. Bx) runs as one launch per
 *                 step in which both one-body half steps are split fp16
 *                 products too and the series is summed by Horner's rule
 *                 (v = t0 + VHS v / k, k = order .. 1, t0 = P phi) in FP32
 *                 (N <= 320 and na, nb <= 32; larger shapes, and
 *                 AFQMC_FLAG_UNFUSED_PROPAGATION, take the term-by-term
 *                 kernels with FP32 one-body half steps and an FP64 sum)
 * afqmc_params.flags & AFQMC_FLAG_ONE_BODY_FP64 keeps the one-body half steps
 * on the FP64 matrix cores in the FP32, BF16X3 and FP16X3 modes (FP16X3 then
 * takes the term-by-term kernels). */
enum { AFQMC_FP64 = 0, AFQMC_FP32 = 1, AFQMC_BF16X3 = 2, AFQMC_FP16X3 = 3 };

/* Status-word bits (afqmc_get_status). */
enum {
  AFQMC_STATUS_SINGULAR = 1,   /* a walker's overlap matrix PhiT^T phi was singular */
  AFQMC_STATUS_NONFINITE = 2,  /* a NaN appeared in an overlap or a weight */
  AFQMC_STATUS_QR_ZERO = 4,    /* a walker orbital vanished in re-orthogonalisation */
  AFQMC_STATUS_NO_LIVE = 8     /* population control found no walker with a finite weight */
};

typedef struct afqmc_params {
  int N, na, nb, K;     /* sizes; 1 <= na <= 45, 0 <= nb <= 45, na, nb <= N */
  double dt;            /* imaginary time step (Eq. Bx) */
  int taylor_order;     /* terms of the exp(VHS) series beyond 1 (default 6) */
  int precision;        /* AFQMC_FP64, AFQMC_FP32, AFQMC_BF16X3 or AFQMC_FP16X3 */
  int max_walkers;      /* workspace is sized for this many walkers */
  double mu;            /* scalar factored out of the one-body half step; NaN -> tr(h')/N */
  double e_shift;       /* energy shift E_T of the weights; NaN -> E_L(PhiT) computed in FP64 */
  int exchange;         /* AFQMC_EXCHANGE_*: algorithm of the exchange energy (0 = automatic) */
  int flags;            /* AFQMC_FLAG_* bits (0 = defaults) */
} afqmc_params;

/* afqmc_params.flags */
enum { AFQMC_FLAG_ONE_BODY_FP64 = 1, AFQMC_FLAG_UNFUSED_PROPAGATION = 2 };

/* Algorithms of the exchange energy E_K = -1/2 sum_s sum_g sum_ij T_ij T_ji
 * (Sec. III.C).  Both give the same sum up to rounding.
 *   AFQMC_EXCHANGE_DIRECT  the direct algorithm of the paper: T_g = Lh_g theta
 *                          formed tile by tile and paired in the tile
 *                          (K n^2 N products per walker and spin)
 *   AFQMC_EXCHANGE_PAIR    the same sum with the Cholesky index summed first:
 *                          pair integrals V_ij[p][q] = sum_g Lh_g[i][p] Lh_g[j][q]
 *                          (i <= j) built at init, E_K from
 *                          sum_ij Theta_j V_ij Theta_i^T (n (n + 1) / 2 N^2
 *                          products; n (n + 1) / 2 N^2 stored values per spin,
 *                          shared by the spins when their trial orbitals are
 *                          equal)
 *   AFQMC_EXCHANGE_AUTO    PAIR when it needs at least 1.5x fewer products
 *                          (2 K n / ((n + 1) N) > 1.5) and its arrays fit in
 *                          48 GB, else DIRECT
 * afqmc_get_exchange_algorithm reports the choice. */
enum { AFQMC_EXCHANGE_AUTO = 0, AFQMC_EXCHANGE_DIRECT = 1, AFQMC_EXCHANGE_PAIR = 2 };

/* Walker ensemble (Eq. stat_wfs), caller-owned device arrays. */
typedef struct afqmc_walkers {
  void* phi_a;      /* complex [nw][N][na]: orbitals of spin alpha        */
  void* phi_b;      /* complex [nw][N][nb]: orbitals of spin beta         */
  void* log_ovlp;   /* complex [nw]: log <Psi_T|phi_z> (log|.| + i arg)   */
  double* log_w;    /* [nw]: log of the walker weight w_z; -inf = discarded */
} afqmc_walkers;

typedef struct afqmc_ham afqmc_ham;

/* Build the step-independent data (run once).
 *   host_h1     [N][N]      one-body integrals h_pq (Eq. Habinitio), real symmetric
 *   host_chol   [K][N][N]   Cholesky vectors L^g_pr, (pr|qs) = sum_g L^g_pr L^g_qs,
 *                           each real symmetric
 *   host_phiT_a [N][na]     trial orbitals of spin alpha (real, Sec. III, N_det = 1)
 *   host_phiT_b [N][nb]     trial orbitals of spin beta (may equal host_phiT_a)
 * Computes h' = h1 - 1/2 sum_g L_g L_g, mu, P = exp(-dt (h' - mu) / 2),
 * the half-rotated vectors Lh^s_g = PhiT_s^T L_g (Sec. III.B), PhiT_s^T h1,
 * the packed L used by the VHS build (FP16X3 also keeps it transposed and
 * split per Cholesky vector, for afqmc_msd_force_bias), and E_T.  Allocates
 * the workspace.
 * On success *out owns device memory until afqmc_destroy. */
int afqmc_init_hamiltonian(const afqmc_params* params, const double* host_h1,
                           const double* host_chol, const double* host_phiT_a,
                           const double* host_phiT_b, void* stream, afqmc_ham** out);

/* log_ovlp[z] = sum_s log det(PhiT_s^T phi_s)  (Sec. III.A, SD overlap). */
int afqmc_overlap(afqmc_ham* ham, const afqmc_walkers* w, int nw, void* stream);

/* vbias[z][g] = sum_pq G^z_pq L^g_pq = sum_s tr(Lh^s_g theta^s_z)  (Eqs. fb, rfb).
 *   vbias  complex [nw][K], written. */
int afqmc_force_bias(afqmc_ham* ham, const afqmc_walkers* w, int nw, void* vbias, void* stream);

/* One importance-sampled phaseless step (Sec. II.B) for every walker:
 *   xbar = -i sqrt(dt) vbias, VHS = i sqrt(dt) sum_g (x_g - xbar_g) L_g,
 *   phi' = P T(VHS) P phi with T the truncated Taylor series of exp,
 *   ln O_z = log<Psi_T|phi'> - log<Psi_T|phi>  (Eq. ovl, e^{-dt mu/2} factors removed),
 *   log w += Re ln O_z + Re(x.xbar - xbar.xbar/2) - dt (mu (na+nb) - E_T)
 *            + ln max(0, cos Im ln O_z)  (Eqs. import, ph, theta).
 *   fields  [nw][K] auxiliary fields x ~ N(0,1), read.
 * phi_a, phi_b, log_ovlp and log_w are updated in place. */
int afqmc_propagate(afqmc_ham* ham, afqmc_walkers* w, int nw, const double* fields,
                    void* stream);

/* Local energy split (Sec. III.C):
 *   e[z][0] = E1 = sum_pq h_pq G_pq,  e[z][1] = EJ = 1/2 sum_g vbias_g^2,
 *   e[z][2] = EK = -1/2 sum_s sum_g sum_ij T_ij T_ji,  T^s_g = Lh^s_g theta^s.
 *   e  complex [nw][3], written.  E_L = e0 + e1 + e2 (complex). */
int afqmc_local_energy(afqmc_ham* ham, const afqmc_walkers* w, int nw, void* e, void* stream);

/* Re-orthogonalise every walker and spin (R9): phi = Q R with R upper
 * triangular with a positive real diagonal (the unique such factors, i.e.
 * Householder QR followed by the phases diag(R_ii/|R_ii|)); phi <- Q,
 * log_ovlp -= sum ln R_ii.  Computed as Cholesky QR applied twice.  E_L and
 * theta are unchanged by this, up to rounding.  A rank-deficient walker sets
 * AFQMC_STATUS_QR_ZERO, keeps its orbitals and is discarded: log_ovlp ->
 * +inf and log_w -> -inf (weight 0, as the step's weight update does). */
int afqmc_orthogonalise(afqmc_ham* ham, afqmc_walkers* w, int nw, void* stream);

/* One full step: afqmc_propagate, then afqmc_orthogonalise if do_qr, then
 * (if e != NULL) afqmc_local_energy of the new walkers into e [nw][3].
 * The Green's function and force bias of the new walkers are kept in the
 * workspace; with flags & AFQMC_STEP_REUSE the next afqmc_step on the same
 * walker arrays and nw starts from them instead of recomputing them.  Only
 * pass AFQMC_STEP_REUSE if the walkers were not changed in between by
 * anything but afqmc_step on this handle.
 * When do_qr is set the overlap and Green's function are taken on the
 * re-orthogonalised walker, and ln O_z adds back sum ln |R_ii|. */
enum { AFQMC_STEP_REUSE = 1 };
int afqmc_step(afqmc_ham* ham, afqmc_walkers* w, int nw, const double* fields, int do_qr,
               void* e, int flags, void* stream);

/* ---- ensemble: global energy, population control, block ----
 * Weights are w_z = exp(log_w[z]); a walker whose log_w is not finite (-inf
 * for a discarded walker, or NaN) has weight 0.  Both reductions run in a
 * fixed order (deterministic), in FP64 in every precision mode. */

/* Walker-averaged energy E = sum_z w_z E_L^z / sum_z w_z (Sec. III.C, the
 * global energy estimate), E_L^z = e[z][0] + e[z][1] + e[z][2] (complex).
 *   e    complex [nw][3] local energy parts as written by afqmc_local_energy
 *        (may be NULL when nw = 0), read
 *   out  device double [4], written: Re E, Im E, ln sum_z w_z, number of
 *        walkers with w_z > 0.  With no such walker: NaN, NaN, -inf, 0. */
int afqmc_global_energy(afqmc_ham* ham, const afqmc_walkers* w, int nw, const void* e, double* out,
                        void* stream);

/* Population control by a comb (named in Sec. I; the paper gives no
 * algorithm, the comb is this library's choice).  With W = sum_z w_z, the nw
 * teeth t_k = (k + u) W / nw, k = 0 .. nw-1, each select the first walker z
 * whose cumulative weight w_0 + ... + w_z exceeds t_k (rounding past the
 * total selects the last walker with w_z > 0).  A walker selected c >= 1
 * times keeps its slot and its c - 1 extra copies fill, in walker order, the
 * slots of the unselected walkers, in slot order.  phi_a, phi_b and log_ovlp
 * are copied accordingly and every log_w becomes ln(W / nw) (the total
 * weight is kept).  Each walker gets floor or ceil of nw w_z / W copies, and
 * the expected number over u is nw w_z / W.
 *   u       comb offset, 0 <= u < 1 (a uniform random number drawn by the
 *           caller; otherwise AFQMC_EINVAL)
 *   parent  device int [nw], written (may be NULL): slot k now holds a copy
 *           of old walker parent[k] (parent[k] = k for survivors)
 * With no walker of finite weight nothing changes, parent[k] = k and
 * AFQMC_STATUS_NO_LIVE is set.  The next afqmc_step recomputes the Green's
 * function (its flags' AFQMC_STEP_REUSE is ignored once). */
int afqmc_population_control(afqmc_ham* ham, afqmc_walkers* w, int nw, double u, int* parent,
                             void* stream);

/* The comb of afqmc_population_control without a Hamiltonian handle and
 * without any allocation, for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same selection, copies, weights and parent map as
 * afqmc_population_control, bit for bit.  Its scratch (cumulative weights,
 * tooth counts, copy sources, 1.25 MB) is a static device array that each
 * GPU holds until the process ends; every call on a GPU shares that GPU's
 * copy, so calls that overlap on one GPU (other streams, other threads)
 * race: serialise them.  Nothing in the scratch is read before the call
 * writes it.
 *   N, na, nb  orbitals and electrons per spin of the walkers
 *   nw         0 <= nw <= 65536 (the scratch's size; larger: AFQMC_EINVAL)
 *   u          comb offset, 0 <= u < 1
 *   parent     device int [nw], written (may be NULL)
 *   status     device int, AFQMC_STATUS_NO_LIVE or-ed in when no walker has a
 *              finite weight (may be NULL)
 * The walkers are on the current device; the call runs on `stream`. */
int afqmc_population_control_noalloc(int N, int na, int nb, afqmc_walkers* w, int nw, double u, int* parent,
                                     int* status, void* stream);

/* One block (Sec. IV.A and IV.C: a number of propagation steps, then one
 * energy evaluation and one re-orthogonalisation):
 *   nsteps afqmc_step calls, re-orthogonalisation and the local energy on
 *   the last; the global energy of the block into out[4]
 *   (afqmc_global_energy); then, if u >= 0, afqmc_population_control(u).
 *   fields  device [nsteps][nw][K] auxiliary fields, read
 *   e       device complex [nw][3]: local energies of the walkers before
 *           population control, written
 *   out     device double [4] (afqmc_global_energy), written
 *   u       comb offset in [0, 1), or negative for no population control
 *   parent  as in afqmc_population_control (may be NULL)
 *   flags   AFQMC_STEP_REUSE applies to the first step */
int afqmc_block(afqmc_ham* ham, afqmc_walkers* w, int nw, const double* fields, int nsteps, double u,
                void* e, double* out, int* parent, int flags, void* stream);

/* ---- mixed estimators (Sec. IV.B) ----
 * These calls recompute theta of the walkers they are given (in the working
 * precision: FP32 in the mixed modes, with FP64 products and sums); a
 * following afqmc_step with AFQMC_STEP_REUSE on the same walkers stays
 * valid. */

/* Full one-body Green's functions of every walker and spin (Eqs. gf,
 * halfgf):  G[z][s][p][q] = <Psi_T|a+_{p s} a_{q s}|phi_z> / <Psi_T|phi_z>
 *                         = sum_i PhiT_s[p][i] theta^s_z[q][i],
 * theta = phi (PhiT^T phi)^-1.  G: complex [nw][2][N][N], written (the beta
 * block is zero when nb = 0).  This is the input of custom one-body mixed
 * estimators: a caller's kernel forms per-walker values from G and
 * afqmc_weighted_mean averages them over the ensemble. */
int afqmc_green_function(afqmc_ham* ham, const afqmc_walkers* w, int nw, void* G, void* stream);

/* Mixed estimator of S^2 for a single-determinant trial (Sec. IV.B):
 *   s2[z] = nb + Ms (Ms + 1) - sum_pq G^a_pq G^b_qp,  Ms = (na - nb) / 2,
 * the trace of the product G^a G^b as Wick's theorem gives for S_- S_+
 * (formed as sum_ij X_ij Y_ji with X = theta_b^T PhiT_a, Y = theta_a^T PhiT_b,
 * without the N x N matrices).  s2: complex [nw], written. */
int afqmc_s2_mixed(afqmc_ham* ham, const afqmc_walkers* w, int nw, void* s2, void* stream);

/* Weighted ensemble average of m per-walker values (the reduction of the
 * global energy, Sec. III.C, for any mixed estimator):
 *   out[2k], out[2k+1] = Re, Im of sum_z w_z v[z][k] / sum_z w_z, k < m;
 *   out[2m] = ln sum_z w_z;  out[2m+1] = walkers with w_z > 0.
 * v: complex [nw][m], read (NULL allowed when nw = 0); out: device double
 * [2m + 2], written; 1 <= m <= 2^24.  With no live walker the means are NaN,
 * out[2m] = -inf and out[2m+1] = 0. */
int afqmc_weighted_mean(afqmc_ham* ham, const afqmc_walkers* w, int nw, const void* v, int m,
                        double* out, void* stream);

/* Synchronise `stream`, return the accumulated status bits in *out and clear them. */
int afqmc_get_status(afqmc_ham* ham, void* stream, int* out);

/* The exchange algorithm in use (AFQMC_EXCHANGE_DIRECT or _PAIR) into *out. */
int afqmc_get_exchange_algorithm(afqmc_ham* ham, int* out);

/* Setup results for inspection: host_P [N][N] (may be NULL), *mu, *e_shift
 * (either may be NULL).  Synchronises the device. */
int afqmc_get_setup(afqmc_ham* ham, double* host_P, double* mu, double* e_shift);

/* Kernel-phase timing.  afqmc_profile_enable(ham, n) creates 2 n HIP events
 * (n = 0 turns timing off); afterwards every kernel phase of every call on
 * `ham` is bracketed by two events recorded on the call's stream, up to n
 * phases.  afqmc_profile_read synchronises on the recorded events, writes
 * the summed milliseconds and the number of recorded launches of each phase
 * into ms[AFQMC_NPHASE] and launches[AFQMC_NPHASE] (host arrays), and starts
 * a new recording.  Enabling synchronises the device and may allocate. */
enum {
  AFQMC_PH_GREEN = 0,    /* overlap, Green's function theta, one-body energy */
  AFQMC_PH_FORCE_BIAS,   /* vbias = Lh . theta */
  AFQMC_PH_SHIFT,        /* xbar, x - xbar, importance exponent (in
                            AFQMC_FP16X3 also the split of x - xbar) */
  AFQMC_PH_VHS,          /* VHS = i sqrt(dt) sum_g (x - xbar)_g L_g */
  AFQMC_PH_ONE_BODY,     /* P phi (one launch per half step) */
  AFQMC_PH_TAYLOR,       /* one launch per Taylor term */
  AFQMC_PH_QR,           /* re-orthogonalisation */
  AFQMC_PH_WEIGHT,       /* overlap ratio, phase, log weight */
  AFQMC_PH_EXCHANGE,     /* one launch per spin */
  AFQMC_PH_ENERGY,       /* assembly of E1, EJ, EK */
  AFQMC_PH_SPLIT,        /* hi/lo splits of theta (16-bit split modes;
                            with the energy in AFQMC_FP16X3 both in one
                            launch), and of the shifted fields where the
                            shift does not split them */
  AFQMC_PH_CONTROL,      /* global energy and population control */
  AFQMC_PH_ESTIMATOR,    /* mixed estimators: full Green's function, S^2, weighted means */
  AFQMC_PH_PROPAGATE,    /* P T(VHS) P phi in one launch (AFQMC_FP16X3) */
  AFQMC_NPHASE
};
int afqmc_profile_enable(afqmc_ham* ham, int max_records);
int afqmc_profile_read(afqmc_ham* ham, double* ms, int* launches);
/* Restricts the timing to the phases whose bit (1 << AFQMC_PH_*) is set in
 * `mask` (initially all): the events of the other phases are not recorded,
 * so one phase can be timed with no events between the kernels of the rest
 * of the step.  Takes effect for the calls that follow; no device work. */
int afqmc_profile_phases(afqmc_ham* ham, unsigned mask);

/* ---- uneven multi-system batch (several Hamiltonians, one graph launch) ----
 *
 * A batch owns one HIP stream per system and advances every system by one
 * full walker step (afqmc_step semantics, with AFQMC_STEP_REUSE) per step.
 * With use_graph the kernel sequences of all systems are captured once into
 * one hipGraph whose branches (one per system) run concurrently, and each
 * step is one hipGraphLaunch; a device step counter inside the graph selects
 * the step's fields and energy slots.  The graph is recaptured when the
 * field / energy arrays, do_qr or a tuning choice change.
 *   hams[i]  Hamiltonians (same device; sizes may differ)
 *   ws[i]    their walker arrays (caller-owned, kept alive while the batch is)
 *   nw[i]    walkers per system, 1 <= nw[i] <= max_walkers of hams[i]
 * The batch does not own the Hamiltonians. */
typedef struct afqmc_batch afqmc_batch;
typedef struct afqmc_batch_opts {
  int use_graph;    /* 1: capture + replay a hipGraph; 0: eager launches on the system streams */
  int reserved[7];
} afqmc_batch_opts;

int afqmc_batch_create(afqmc_ham* const* hams, const afqmc_walkers* ws, const int* nw, int nsys,
                       const afqmc_batch_opts* opts, afqmc_batch** out);

/* Advance all systems by nsteps steps on `stream`.
 *   fields[i]  device [nsteps][nw[i]][K_i] auxiliary fields of system i
 *   e[i]       device complex [nsteps][nw[i]][3] local energies, or NULL (no
 *              energy for system i); e itself may be NULL
 *   do_qr      re-orthogonalise every step (1) or never (0)
 * Asynchronous; the first call (and any call that recaptures) allocates the
 * graph and synchronises. */
int afqmc_batch_step(afqmc_batch* b, const double* const* fields, void* const* e, int nsteps,
                     int do_qr, void* stream);

/* Kernel tiling of one Hamiltonian (no result depends
 * on it; every output element sums over the same terms in the same order).
 *   ex_tile_m x ex_tile_n    output tile of the exchange kernels: rows of
 *                            the Cholesky or pair-integral operand by
 *                            (walker, re|im) columns
 *   ex_group                 tile-order group size of the exchange launch
 *                            (0: the kernel's default)
 *   vhs_tile_m x vhs_tile_n  output tile of the VHS build: (walker, re|im)
 *                            rows by orbital-pair columns
 * Offered shapes: the split pair exchange (BF16X3, FP16X3 with pair
 * integrals) 128 x 128 or 128 x 64; the split VHS build (FP16X3) 128 x 128
 * or 64 x 128; every other kernel one shape (split direct exchange
 * 160 x 160, FP32 / FP64 exchange 192 x 160, FP32 / FP64 VHS 64 x 64). */
typedef struct afqmc_tuning {
  int ex_tile_m, ex_tile_n;
  int ex_group;
  int vhs_tile_m, vhs_tile_n;
} afqmc_tuning;

/* The handle's current choices into *out. */
int afqmc_get_tuning(const afqmc_ham* ham, afqmc_tuning* out);

/* Set the choices (a shape the handle does not offer: AFQMC_EUNSUPPORTED;
 * ex_group outside [0, 1024]: AFQMC_EINVAL).  Applies to the next call; a
 * batch whose graph holds the old choices recaptures it at its next step.
 * Must not overlap a call on the handle. */
int afqmc_set_tuning(afqmc_ham* ham, const afqmc_tuning* t);

/* Choose per system, by timing the candidates on the current walkers, the
 * exchange tile shape and tile-order group size (every offered shape x
 * groups 1, 2, 4, 8, 16, 32) and the VHS tile shape (afqmc_tuning); or read
 * them from cache_path, a text file of lines
 *   <key> ex=<m>x<n>/<group> vhs=<m>x<n>
 * when it holds the system's key (device, N, na, nb, K, walkers, precision,
 * exchange algorithm).  New results are appended to cache_path (NULL: no
 * cache).  Synchronises. */
int afqmc_autotune(afqmc_batch* b, const char* cache_path);

void afqmc_batch_destroy(afqmc_batch* b);

/* ---------------------------------------------------------------------------
 * Multi-determinant trial (Sec. III.A, Eq. msdovlp; the MSD numerator of
 * Eq. gf through the generalised Wick's theorem, Eq. msdgf0).
 *
 *   |Psi_T> = sum_a c_a t_a |psi_0>,  psi_0 = columns 0 .. n_s - 1 of C_s,
 *   t_a = prod_s prod_m a+_{s, q_m} a_{s, h_m}  (orbitals of C_s),
 * i.e. determinant a is psi_0 with column h_m replaced, in place, by column
 * q_m of C_s (hole m paired with particle m).  The excitation format:
 *   coeff  host double [ndet]             c_a (real)
 *   rank   host int [ndet][2]             k_{a,s} in [0, AFQMC_MSD_MAX_RANK]
 *   orbs   host int [ndet][2][2][AFQMC_MSD_MAX_RANK]
 *          orbs[a][s][0][m] = h_m in [0, n_s), distinct;
 *          orbs[a][s][1][m] = q_m in [n_s, N), distinct; slots m >= k unread.
 *   C_a, C_b  host double [N][N], orthogonal (C^T C = I; not checked).
 * afqmc_msd_create copies everything (the caller keeps its arrays), groups
 * the determinants by their per-spin excitation strings and allocates a
 * workspace for max_walkers walkers; it synchronises `stream`.  Limits:
 * 1 <= na <= 45, 0 <= nb <= 45, ndet >= 1.  Errors: AFQMC_EINVAL for bad
 * sizes or an invalid excitation (message names the determinant),
 * AFQMC_ENOMEM when the workspace does not fit.
 * ------------------------------------------------------------------------- */
#define AFQMC_MSD_MAX_RANK 6
typedef struct afqmc_msd afqmc_msd;

int afqmc_msd_create(int N, int na, int nb, const double* host_C_a, const double* host_C_b, int ndet,
                     const double* host_coeff, const int* host_rank, const int* host_orbs,
                     int max_walkers, void* stream, afqmc_msd** out);

/* log <Psi_T|phi_z> = log det(C_a,occ^T phi_a) + log det(C_b,occ^T phi_b)
 *                   + log sum_a c_a det A^a_a det A^b_a     (Eq. msdovlp)
 * with A^s_a[l][m] = Y^s[q_l][h_m], Y^s = C_s,virt^T phi_s (C_s,occ^T phi_s)^-1.
 * w->phi_a, w->phi_b are read (log_ovlp and log_w are not used);
 * log_ovlp: device complex [nw], written.  A walker with a singular
 * reference overlap or a zero sum gets -inf and sets AFQMC_STATUS_SINGULAR
 * (read with afqmc_msd_get_status).  Asynchronous on `stream`; nw <= max_walkers. */
int afqmc_msd_overlap(afqmc_msd* t, const afqmc_walkers* w, int nw, void* log_ovlp, void* stream);

/* G[z][s][p][q] = <Psi_T|a+_{p s} a_{q s}|phi_z> / <Psi_T|phi_z> for the
 * multi-determinant trial (the numerator of Eq. gf through the generalised
 * Wick's theorem, Sec. III.B).  G: device complex [nw][2][N][N], written
 * (beta block zero when nb = 0).  Same inputs and status as afqmc_msd_overlap. */
int afqmc_msd_green_function(afqmc_msd* t, const afqmc_walkers* w, int nw, void* G, void* stream);

/* Force bias of the multi-determinant trial (Eq. fb with the G above):
 *   vbias[z][g] = sum_s sum_pq G^s_pq L_g,pq,
 * formed from the packed symmetric sum_s (G^s + G^s^T) and the packed L of
 * `ham` without storing G.  ham: a Hamiltonian of any precision with the
 * same N: FP64 contracts with its FP64 packed L; FP32 and BF16X3 round the
 * packed G to FP32 and contract with the FP32 packed L on the FP32 matrix
 * cores; FP16X3 splits the packed G (one power-of-two scale per walker and
 * component) and contracts it with the packed L transposed, kept split per
 * Cholesky vector since init, on the fp16 matrix cores (three products,
 * FP32 accumulation).  A Hamiltonian of another N, or nw above either
 * handle's max_walkers: AFQMC_EINVAL.  vbias: device complex [nw][K],
 * written.  The call uses ham's VHS workspace (and, in FP16X3, its
 * force-bias partial sums) as scratch: it must not overlap a call on the
 * same Hamiltonian (the next afqmc_step recomputes both).  Asynchronous on
 * `stream`. */
int afqmc_msd_force_bias(afqmc_msd* t, afqmc_ham* ham, const afqmc_walkers* w, int nw, void* vbias, void* stream);

/* One phaseless step under the multi-determinant trial (Sec. II.B with the
 * force bias above and the expansion's overlap ratio): the same propagator
 * as afqmc_propagate (P, VHS, Taylor series of `ham`), with
 *   vbias = the multi-determinant force bias, and
 *   ln O_z = log <Psi_T|phi'_z> - w->log_ovlp[z] from the expansion.
 * w->phi_a, w->phi_b, w->log_ovlp (must hold log <Psi_T|phi> of the
 * expansion, e.g. from afqmc_msd_overlap) and w->log_w are updated in place.
 * fields: device [nw][K].  ham: any precision (its working precision for
 * the force bias, VHS and propagation), with the trial's N, na and nb (its own
 * trial orbitals are not used here except through its energy shift, a
 * constant per step); ham's VHS and force-bias workspaces are used, so the
 * call must not overlap another call on ham.  afqmc_orthogonalise(ham, ...)
 * may follow: it rescales every determinant's overlap alike.  A walker with
 * a singular reference overlap or a zero expansion sum is discarded
 * (log_w = -inf) and sets AFQMC_STATUS_SINGULAR in the trial's status. */
int afqmc_msd_propagate(afqmc_msd* t, afqmc_ham* ham, afqmc_walkers* w, int nw, const double* fields,
                        void* stream);

/* Attach the Hamiltonian whose local energy afqmc_msd_local_energy takes:
 *   K          number of Cholesky vectors
 *   host_h1    host [N][N] one-body integrals (the energy uses h1, Sec. III.C)
 *   host_chol  host [K][N][N] real symmetric Cholesky vectors
 * Builds, in FP64, the rotated rows C_S^T L_g and C_S^T h1 of each spin,
 * where S = the reference's occupied orbitals and the active particles
 * (the virtual orbitals some determinant excites into), and a workspace for
 * passes over a few walkers at a time.  Allocates and synchronises `stream`;
 * once per trial (AFQMC_EINVAL otherwise).  The number of (active particle,
 * active hole) pairs of a spin must not exceed 1024: expansions within an
 * active space, as selected-CI trials are (AFQMC_EUNSUPPORTED otherwise). */
int afqmc_msd_set_hamiltonian(afqmc_msd* t, int K, const double* host_h1, const double* host_chol,
                              void* stream);

/* Local energy of every walker against the multi-determinant trial
 * (Sec. III.C: the one-body part through the expansion's Green's function,
 * the two-body numerator through the generalised Wick's theorem):
 *   E_L = sum_a c_a <D_a|phi> E_L(D_a, phi) / sum_a c_a <D_a|phi>,
 * split like afqmc_local_energy: e[z] = (E1, EJ, EK), device complex
 * [nw][3], written.  The Cholesky sum is taken once per walker through the
 * Gram matrices of the active blocks (FP64 matrix cores); the expansion
 * enters through per-string and per-determinant contractions with them.
 * A determinant whose overlap with a walker is exactly zero contributes only
 * its linear terms (its own local energy is undefined).  Requires
 * afqmc_msd_set_hamiltonian.  Asynchronous on `stream`; nw <= max_walkers. */
int afqmc_msd_local_energy(afqmc_msd* t, const afqmc_walkers* w, int nw, void* e, void* stream);

/* Excitation strings per spin after grouping (for sizing and reports). */
int afqmc_msd_get_strings(afqmc_msd* t, int* nstr_a, int* nstr_b);
/* Synchronise `stream`, return the accumulated status bits in *out and clear them. */
int afqmc_msd_get_status(afqmc_msd* t, void* stream, int* out);
void afqmc_msd_destroy(afqmc_msd* t);

void afqmc_destroy(afqmc_ham* ham);
const char* afqmc_last_error(void);
int afqmc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AFQMC_H */
