// C ABI of the walker-step library: argument checking, workspace ownership
// and the kernel sequence of each call.  No arithmetic of the method runs on
// the host; every step is a kernel from the *_kernels.hip sources.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/afqmc.h"
#include "common.h"
#include "kernels.h"
#include "setup.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? AFQMC_ENOMEM : AFQMC_EHIP,                \
                  "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),               \
                  __FILE__, __LINE__);                                                 \
  } while (0)

// Device temporaries of one setup routine, freed on every return path (after
// the device has finished with them).
class TempAllocs {
 public:
  TempAllocs() = default;
  TempAllocs(const TempAllocs&) = delete;
  TempAllocs& operator=(const TempAllocs&) = delete;
  ~TempAllocs() {
    if (p_.empty()) return;
    (void)hipDeviceSynchronize();
    for (void* q : p_) (void)hipFree(q);
  }
  template <typename T>
  hipError_t get(T** out, size_t bytes) {
    *out = nullptr;
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
    if (e != hipSuccess) return e;
    p_.push_back(q);
    *out = static_cast<T*>(q);
    return hipSuccess;
  }

 private:
  std::vector<void*> p_;
};

}  // namespace

struct afqmc_ham {
  afqmc_params prm{};
  StepDims d{};
  int device = 0;
  int prec = AFQMC_FP64;
  double mu = 0.0, e_shift = 0.0, cst = 0.0, sdt = 0.0;
  size_t tsize = 8;  // bytes of the working precision
  // Hamiltonian data
  double* P = nullptr;      // [N][ldP]
  void* Lh = nullptr;       // T [2][K][nmax][ldN]
  void* LT = nullptr;       // T [Npk][ldK]
  int2* pq = nullptr;       // [Npk]
  double* phiT = nullptr;   // [2][N][nmax]
  double* hh = nullptr;     // [2][nmax][N]
  // hi/lo split operands of the 16-bit exchange (AFQMC_BF16X3 / AFQMC_FP16X3)
  int split = SPLIT_NONE;
  unsigned short* lh_split = nullptr;  // [2][K][nmax][2 ldh] split rows
  float* lh_unscale = nullptr;           // [2][K][nmax]
  unsigned short* th_split = nullptr;  // [W][2][2][nmax][2 ldh]
  unsigned short* lt_split = nullptr;  // [nvblk * 160][2 ldhK] split L in VHS block order
  float* lt_unscale = nullptr;         // [nvblk * 160]
  unsigned short* lt_t_split = nullptr;  // [K][2 ldhp] packed L transposed, split (multi-determinant force bias)
  float* lt_t_unscale = nullptr;         // [K]
  int ldhp = 0;                          // pair-index row length: round_up(N (N + 1) / 2, 32)
  int2* vblk = nullptr;                // [nvblk] VHS blocks (P, Q)
  int nvblk = 0;
  unsigned short* xs_split = nullptr;  // [W][2][2 ldhK]
  float* xs_unscale = nullptr;         // [W][2]
  float* tk = nullptr;                 // [taylor_order][W][N][ncolp] Taylor terms (split path)
  unsigned short* fb_lh = nullptr;     // [K][2][nmax][2 ldh] Lh split per Cholesky vector (force bias)
  float* fb_lh_unscale = nullptr;      // [K]
  unsigned short* fb_th = nullptr;     // [W][2][2][nmax][2 ldh] theta split per (walker, re|im)
  float* fb_th_unscale = nullptr;      // [W][2]
  float* fb_part = nullptr;            // [FB_SPLIT_CHUNKS][2 W][K] split-K partial sums
  // fused propagation (FP16X3)
  bool prop_fused = false;
  unsigned short* psplit = nullptr;    // P split into fp16 hi/lo, scaled by 2^pexp
  int pexp = 0;
  float* lmax = nullptr;               // [K] max |L_g|: each walker's |VHS| bound, the scale of its split VHS
  float* th_unscale = nullptr;           // [W][2][2][nmax]
  // workspace (sized for max_walkers)
  void* theta = nullptr;    // T [W][2][2][nmax][ldN]
  double2* logdet = nullptr;  // [W][2]
  double2* e1 = nullptr;      // [W][2]
  double2* vbias = nullptr;   // [W][K]
  void* xs = nullptr;         // T [W][2][ldK]
  double2* a = nullptr;       // [W]
  void* vhs = nullptr;        // T [W][N][ldV]
  double* acc = nullptr;      // [W][N][ncolp]
  void* t0 = nullptr;         // T [W][N][ncolp]
  void* t1 = nullptr;
  unsigned* tmax = nullptr;   // [taylor_order + 2][W] running maxima
  double2* part = nullptr;    // [2][ntg][W]
  double* corr = nullptr;     // [W][2]
  int* status = nullptr;
  // population control (comb): cumulative weights, tooth counts, extra-copy
  // sources, parents
  double* pc_csum = nullptr;  // [W]
  int* pc_cnt = nullptr;      // [W]
  int* pc_src = nullptr;      // [W]
  int* pc_parent = nullptr;   // [W]
  int ntg = 0;
  // exchange through pair integrals (AFQMC_EXCHANGE_PAIR)
  int ex_algo = AFQMC_EXCHANGE_DIRECT;
  void* vpair = nullptr;                 // T [rows][ldN] (FP32 / FP64)
  unsigned short* vpair_split = nullptr; // [rows][2 ldh] (16-bit split modes)
  float* vpair_unscale = nullptr;        // [rows]
  PairTab* pair_tab = nullptr;           // device [2]
  int pair_ntiles[2] = {0, 0};
  int pair_ntg = 0;
  long pair_vrow0[2] = {0, 0};
  int ex_gs = 0;         // exchange tile-order group size (0: built-in default; set by the autotuner)
  int ex_tile = SPLIT_TILE_WIDE;   // split pair-exchange walker tile (autotuner choice)
  int vhs_tile = SPLIT_TILE_WIDE;  // split VHS walker tile (autotuner choice)
  int tune_gen = 0;                // bumped by every change of the three choices above
  bool capturing = false;  // inside a graph capture: no phase-timing events
  std::vector<void*> allocs;
  // phase timing (afqmc_profile_enable)
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  unsigned prof_mask = ~0u;  // phases that are timed (bit p: phase p)
  struct Rec { int phase, e0, e1; };
  std::vector<Rec> recs;
  // afqmc_step cache
  const void* c_phi_a = nullptr;
  const void* c_phi_b = nullptr;
  int c_nw = -1;
  bool c_valid = false;
};

namespace {

template <class H>
int dalloc(H* h, void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return fail(AFQMC_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  h->allocs.push_back(*p);
  e = hipMemset(*p, 0, bytes);
  if (e != hipSuccess) return fail(AFQMC_EHIP, "hipMemset failed: %s", hipGetErrorString(e));
  return AFQMC_OK;
}

template <typename T, class H>
int dalloc_t(H* h, T** p, size_t count) {
  return dalloc(h, reinterpret_cast<void**>(p), count * sizeof(T));
}

void free_all(afqmc_ham* h) {
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
}

int check_walkers(const afqmc_ham* h, const afqmc_walkers* w, int nw) {
  if (!h) return fail(AFQMC_EINVAL, "null Hamiltonian handle");
  if (nw < 0 || nw > h->prm.max_walkers)
    return fail(AFQMC_EINVAL, "nw = %d outside [0, max_walkers = %d]", nw, h->prm.max_walkers);
  if (nw == 0) return AFQMC_OK;
  if (!w) return fail(AFQMC_EINVAL, "null walkers");
  if (!w->phi_a || (h->d.nb > 0 && !w->phi_b) || !w->log_ovlp || !w->log_w)
    return fail(AFQMC_EINVAL, "null walker array");
  return AFQMC_OK;
}

int set_device(const afqmc_ham* h) {
  HIP_TRY(hipSetDevice(h->device));
  return AFQMC_OK;
}

// Phase timing: an event before and after each selected kernel phase, on the
// call's stream.
int prof_mark(afqmc_ham* h, int phase, hipStream_t s) {
  if (h->capturing || h->ev.empty() || h->ev_used + 2 > (int)h->ev.size()) return -1;
  if (!((h->prof_mask >> phase) & 1u)) return -1;
  if (hipEventRecord(h->ev[h->ev_used], s) != hipSuccess) return -1;
  return h->ev_used++;
}
void prof_close(afqmc_ham* h, int phase, int e0, hipStream_t s) {
  if (e0 < 0) return;
  if (hipEventRecord(h->ev[h->ev_used], s) != hipSuccess) return;
  h->recs.push_back({phase, e0, h->ev_used++});
}

#define PHASE(h, ph, s, expr)            \
  do {                                   \
    const int e0__ = prof_mark((h), (ph), (s)); \
    HIP_TRY(expr);                       \
    prof_close((h), (ph), e0__, (s));    \
  } while (0)

// ---------------------------------------------------------------------------
// step sequences, per working precision
// ---------------------------------------------------------------------------

template <typename T>
int seq_theta(afqmc_ham* h, const afqmc_walkers* w, int nw, bool want_e1, hipStream_t s) {
  PHASE(h, AFQMC_PH_GREEN, s,
        (launch_gf<T>(h->d, nw, (const double2*)w->phi_a, (const double2*)w->phi_b, h->phiT, h->hh,
                      (T*)h->theta, h->logdet, want_e1 ? h->e1 : nullptr, h->status, s)));
  return AFQMC_OK;
}

// The force bias, VHS build and Taylor products run on split operands only
// in AFQMC_FP16X3, whose 22-bit operands match FP32; bf16 operands (16 bits)
// would carry ~1e-5 relative errors into every propagated walker, so
// AFQMC_BF16X3 splits the exchange only.
static bool vhs_split(const afqmc_ham* h) { return h->split == SPLIT_F16; }

// Whether the force bias can leave the exchange's split rows of theta beside
// its own (one pass over theta for both, when the exchange follows).
static bool split_theta_both(const afqmc_ham* h) {
  return vhs_split(h) && split_both_fits(2 * h->d.nmax, h->d.ldh);
}

// rows_too: also write the exchange's split rows of theta (only when
// split_theta_both holds).
template <typename T>
int seq_force_bias(afqmc_ham* h, int nw, double2* vbias, hipStream_t s, bool rows_too = false) {
  if (vhs_split(h)) {
    const StepDims& d = h->d;
    if (rows_too)
      PHASE(h, AFQMC_PH_SPLIT, s,
            launch_split_both_mode(h->split, nw * 2, 2 * d.nmax, d.N, (const float*)h->theta, d.ldN, d.ldh,
                                   h->fb_th, h->fb_th_unscale, h->th_split, h->th_unscale, s));
    else
      PHASE(h, AFQMC_PH_SPLIT, s,
            launch_split_blocks_mode(h->split, nw * 2, 2, d.nmax, d.N, (const float*)h->theta, d.ldN, d.nmax,
                                     2L * d.nmax, h->fb_th, d.ldh, h->fb_th_unscale, s));
    PHASE(h, AFQMC_PH_FORCE_BIAS, s,
          launch_force_bias_split(h->split, d, nw, h->fb_th, h->fb_th_unscale, h->fb_lh, h->fb_lh_unscale,
                                  h->fb_part, vbias, s));
    return AFQMC_OK;
  }
  PHASE(h, AFQMC_PH_FORCE_BIAS, s,
        (launch_force_bias<T>(h->d, nw, (const T*)h->Lh, (const T*)h->theta, vbias, s)));
  return AFQMC_OK;
}

// Per-step inputs and outputs: fields = fields_base + ctr[0] * fstep and
// e = e_base + ctr[0] * estep when ctr (device) is set, else the bases.
struct StepIO {
  const double* fields = nullptr;
  double2* e = nullptr;
  const int* ctr = nullptr;
  long fstep = 0, estep = 0;
};

// Exchange partials of one spin into h->part with the handle's algorithm and
// precision (theta, and its split rows in the split modes, already built).
hipError_t launch_exchange_spin(afqmc_ham* h, int nw, int sp, int* ntg, hipStream_t s, int gs, int tile) {
  const StepDims& d = h->d;
  if (h->ex_algo == AFQMC_EXCHANGE_PAIR) {
    const PairLaunch pl{h->pair_tab + sp, h->pair_ntiles[sp], h->pair_ntg, h->pair_vrow0[sp]};
    *ntg = h->pair_ntg;
    if (h->split != SPLIT_NONE)
      return launch_exchange_pair_split(h->split, d, nw, pl, h->vpair_split, h->vpair_unscale, h->th_split,
                                        h->th_unscale, (const float*)h->theta, h->part, sp, s, gs, tile);
    if (h->prec != AFQMC_FP64)
      return launch_exchange_pair<float>(d, nw, pl, (const float*)h->vpair, (const float*)h->theta, h->part, sp,
                                         s, gs);
    return launch_exchange_pair<double>(d, nw, pl, (const double*)h->vpair, (const double*)h->theta, h->part,
                                        sp, s, gs);
  }
  if (h->split != SPLIT_NONE)
    return launch_exchange_split(h->split, d, nw, h->lh_split, h->lh_unscale, h->th_split, h->th_unscale,
                                 h->part, sp, ntg, s, gs);
  if (h->prec != AFQMC_FP64)
    return launch_exchange<float>(d, nw, (const float*)h->Lh, (const float*)h->theta, h->part, sp, ntg, s, gs);
  return launch_exchange<double>(d, nw, (const double*)h->Lh, (const double*)h->theta, h->part, sp, ntg, s, gs);
}

// rows_ready: the split rows of theta are already built (by the force bias).
template <typename T>
int seq_energy_from_theta(afqmc_ham* h, int nw, double2* e_out, hipStream_t s,
                          const int* ctr = nullptr, long estep = 0, bool rows_ready = false) {
  int ntg = 0;
  if (h->split != SPLIT_NONE && !rows_ready) {
    const StepDims& d = h->d;
    PHASE(h, AFQMC_PH_SPLIT, s,
          launch_split_rows_mode(h->split, (long)nw * 4 * d.nmax, d.N, (const float*)h->theta, d.ldN,
                                 h->th_split, d.ldh, h->th_unscale, s));
  }
  for (int sp = 0; sp < 2; ++sp)
    PHASE(h, AFQMC_PH_EXCHANGE, s, launch_exchange_spin(h, nw, sp, &ntg, s, h->ex_gs, h->ex_tile));
  PHASE(h, AFQMC_PH_ENERGY, s,
        launch_energy(h->d, nw, h->e1, h->vbias, h->part, ntg, e_out, ctr, estep, s));
  return AFQMC_OK;
}


// phi' = P T(VHS) P phi with vbias (of phi) already in h->vbias.
template <typename T>
int seq_propagate_core(afqmc_ham* h, afqmc_walkers* w, int nw, const StepIO& io, hipStream_t s) {
  const StepDims& d = h->d;
  // the split VHS build reads only the split rows of the shifted fields: the
  // shift writes them itself when a walker's row fits its registers
  const bool shift_split = std::is_same<T, float>::value && vhs_split(h) && shift_split_fits(d.ldhK);
  if (shift_split)
    PHASE(h, AFQMC_PH_SHIFT, s,
          launch_shift_split(h->split, d, nw, h->vbias, io.fields, io.ctr, io.fstep, h->xs_split, h->xs_unscale,
                             h->a, h->tmax, h->prm.taylor_order + 2, h->prm.max_walkers, h->sdt, h->lmax, s));
  else
    PHASE(h, AFQMC_PH_SHIFT, s,
          (launch_shift<T>(d, nw, h->vbias, io.fields, io.ctr, io.fstep, (T*)h->xs, h->a, h->tmax,
                           h->prm.taylor_order + 2, h->prm.max_walkers, h->sdt, h->lmax, s)));
  if (vhs_split(h)) {
    if (!shift_split)
      PHASE(h, AFQMC_PH_SPLIT, s,
            launch_split_rows_mode(h->split, (long)nw * 2, d.K, (const float*)h->xs, d.ldK, h->xs_split, d.ldhK,
                                   h->xs_unscale, s));
    PHASE(h, AFQMC_PH_VHS, s,
          launch_vhs_split(h->split, d, nw, h->xs_split, h->xs_unscale, h->lt_split, h->lt_unscale, h->vblk,
                           h->nvblk, (float*)h->vhs, h->tmax + h->prm.max_walkers, h->prop_fused, h->sdt, s,
                           h->vhs_tile));
  } else {
    PHASE(h, AFQMC_PH_VHS, s,
          (launch_vhs<T>(d, nw, (const T*)h->xs, (const T*)h->LT, h->pq, (T*)h->vhs, h->sdt, s)));
  }
  if (h->prop_fused) {
    PHASE(h, AFQMC_PH_PROPAGATE, s,
          launch_prop_fused(d, nw, (double2*)w->phi_a, (double2*)w->phi_b, (const float*)h->vhs,
                            h->tmax + h->prm.max_walkers, h->psplit, h->pexp, h->prm.taylor_order, s));
    return AFQMC_OK;
  }
  const bool pphi64 = sizeof(T) == 8 || (h->prm.flags & AFQMC_FLAG_ONE_BODY_FP64);
  PHASE(h, AFQMC_PH_ONE_BODY, s,
        pphi64 ? launch_pphi<double>(d, nw, h->P, (const double2*)w->phi_a, (const double2*)w->phi_b, h->acc,
                                     nullptr, nullptr, h->tmax, 0, s)
               : launch_pphi<float>(d, nw, h->P, (const double2*)w->phi_a, (const double2*)w->phi_b, h->acc,
                                    nullptr, nullptr, h->tmax, 0, s));
  const int order = h->prm.taylor_order;
  if (vhs_split(h)) {
    // every term kept (tk[k - 1]), summed into acc once at the end
    const size_t tsz = (size_t)nw * d.N * d.ncolp;
    float* tk = h->tk;
    for (int k = 1; k <= order; ++k)
      PHASE(h, AFQMC_PH_TAYLOR, s,
            launch_taylor_split(h->split, d, nw, (const float*)h->vhs, k == 1 ? nullptr : tk + (k - 2) * tsz,
                                tk + (k - 1) * tsz, h->acc, h->tmax, h->prm.max_walkers, k, s));
    PHASE(h, AFQMC_PH_TAYLOR, s, launch_taylor_split_sum(d, nw, order, tk, h->acc, s));
  } else {
    T* bufs[2] = {(T*)h->t0, (T*)h->t1};
    for (int k = 1; k <= order; ++k) {
      const T* tin = k == 1 ? nullptr : bufs[(k - 2) & 1];
      T* tout = bufs[(k - 1) & 1];
      PHASE(h, AFQMC_PH_TAYLOR, s,
            (launch_taylor<T>(d, nw, (const T*)h->vhs, tin, tout, h->acc, h->tmax, k, order, s)));
    }
  }
  PHASE(h, AFQMC_PH_ONE_BODY, s,
        pphi64 ? launch_pphi<double>(d, nw, h->P, nullptr, nullptr, h->acc, (double2*)w->phi_a,
                                     (double2*)w->phi_b, nullptr, 1, s)
               : launch_pphi<float>(d, nw, h->P, nullptr, nullptr, h->acc, (double2*)w->phi_a,
                                    (double2*)w->phi_b, nullptr, 1, s));
  return AFQMC_OK;
}

template <typename T>
int seq_propagate(afqmc_ham* h, afqmc_walkers* w, int nw, const double* fields, hipStream_t s) {
  int rc;
  if ((rc = seq_theta<T>(h, w, nw, false, s))) return rc;
  if ((rc = seq_force_bias<T>(h, nw, h->vbias, s))) return rc;
  StepIO io;
  io.fields = fields;
  if ((rc = seq_propagate_core<T>(h, w, nw, io, s))) return rc;
  if ((rc = seq_theta<T>(h, w, nw, false, s))) return rc;
  PHASE(h, AFQMC_PH_WEIGHT, s,
        launch_weight(nw, h->logdet, nullptr, h->a, (double2*)w->log_ovlp, w->log_w, h->cst,
                      h->status, s));
  h->c_valid = false;
  return AFQMC_OK;
}

template <typename T>
int seq_local_energy(afqmc_ham* h, const afqmc_walkers* w, int nw, double2* e, hipStream_t s) {
  int rc;
  const bool both = split_theta_both(h);
  if ((rc = seq_theta<T>(h, w, nw, true, s))) return rc;
  if ((rc = seq_force_bias<T>(h, nw, h->vbias, s, both))) return rc;
  if ((rc = seq_energy_from_theta<T>(h, nw, e, s, nullptr, 0, both))) return rc;
  h->c_valid = false;
  return AFQMC_OK;
}

template <typename T>
int seq_step(afqmc_ham* h, afqmc_walkers* w, int nw, const StepIO& io, int do_qr, int flags,
             hipStream_t s) {
  int rc;
  const bool reuse = (flags & AFQMC_STEP_REUSE) && h->c_valid && h->c_phi_a == w->phi_a &&
                     h->c_phi_b == w->phi_b && h->c_nw == nw;
  if (!reuse) {
    if ((rc = seq_theta<T>(h, w, nw, false, s))) return rc;
    if ((rc = seq_force_bias<T>(h, nw, h->vbias, s))) return rc;
  }
  if ((rc = seq_propagate_core<T>(h, w, nw, io, s))) return rc;
  if (do_qr)
    PHASE(h, AFQMC_PH_QR, s,
          launch_qr(h->d, nw, (double2*)w->phi_a, (double2*)w->phi_b, h->corr, h->status, s));
  if ((rc = seq_theta<T>(h, w, nw, io.e != nullptr, s))) return rc;
  PHASE(h, AFQMC_PH_WEIGHT, s,
        launch_weight(nw, h->logdet, do_qr ? h->corr : nullptr, h->a, (double2*)w->log_ovlp,
                      w->log_w, h->cst, h->status, s));
  const bool both = io.e && split_theta_both(h);
  if ((rc = seq_force_bias<T>(h, nw, h->vbias, s, both))) return rc;
  if (io.e) {
    if ((rc = seq_energy_from_theta<T>(h, nw, io.e, s, io.ctr, io.estep, both))) return rc;
  }
  h->c_valid = true;
  h->c_phi_a = w->phi_a;
  h->c_phi_b = w->phi_b;
  h->c_nw = nw;
  return AFQMC_OK;
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------

template <typename T>
int build_working_arrays(afqmc_ham* h, const double* dL, const double* Y_a, const double* Y_b,
                         hipStream_t s) {
  const StepDims& d = h->d;
  int rc;
  if ((rc = dalloc(h, &h->Lh, (size_t)2 * d.K * d.nmax * d.ldN * sizeof(T)))) return rc;
  HIP_TRY((setup_pack_lh<T>(d.K, d.N, d.na, d.nmax, d.ldN, Y_a, (T*)h->Lh, s)));
  if (d.nb > 0)
    HIP_TRY((setup_pack_lh<T>(d.K, d.N, d.nb, d.nmax, d.ldN, Y_b,
                              (T*)h->Lh + (size_t)d.K * d.nmax * d.ldN, s)));
  if (!vhs_split(h)) {
    if ((rc = dalloc(h, &h->LT, (size_t)d.Npk * d.ldK * sizeof(T)))) return rc;
    HIP_TRY((setup_pack_lt<T>(d.K, d.N, d.Npk, d.ldK, h->pq, dL, (T*)h->LT, s)));
    return AFQMC_OK;
  }
  // the split VHS keeps only the split L in block order: the FP32 one is a temporary
  const std::vector<int2> blk = vhs_split_blocks(d.N);
  const std::vector<int2> pqb = vhs_split_pairs(d.N, blk);
  const long nrow = (long)pqb.size();
  h->nvblk = (int)blk.size();
  int2* pqb_dev = nullptr;
  if ((rc = dalloc_t(h, &h->vblk, blk.size()))) return rc;
  HIP_TRY(hipMemcpy(h->vblk, blk.data(), blk.size() * sizeof(int2), hipMemcpyHostToDevice));
  if ((rc = dalloc_t(h, &h->lt_split, (size_t)nrow * 2 * d.ldhK))) return rc;
  if ((rc = dalloc_t(h, &h->lt_unscale, (size_t)nrow))) return rc;
  float* lt32 = nullptr;
  TempAllocs tmp;
  HIP_TRY(tmp.get(&lt32, (size_t)nrow * d.ldK * sizeof(float)));
  HIP_TRY(tmp.get(&pqb_dev, (size_t)nrow * sizeof(int2)));
  HIP_TRY(hipMemcpy(pqb_dev, pqb.data(), (size_t)nrow * sizeof(int2), hipMemcpyHostToDevice));
  HIP_TRY(setup_pack_lt<float>(d.K, d.N, (int)nrow, d.ldK, pqb_dev, dL, lt32, s));
  HIP_TRY(launch_split_rows_mode(h->split, nrow, d.K, lt32, d.ldK, h->lt_split, d.ldhK, h->lt_unscale, s));
  HIP_TRY(hipStreamSynchronize(s));
  // force bias: Lh split with one scale per Cholesky vector (rows (spin, i))
  if ((rc = dalloc_t(h, &h->fb_lh, (size_t)d.K * 2 * d.nmax * 2 * d.ldh))) return rc;
  if ((rc = dalloc_t(h, &h->fb_lh_unscale, (size_t)d.K))) return rc;
  HIP_TRY(launch_split_blocks_mode(h->split, d.K, 2, d.nmax, d.N, (const float*)h->Lh, d.ldN,
                                   (long)d.K * d.nmax, d.nmax, h->fb_lh, d.ldh, h->fb_lh_unscale, s));
  // multi-determinant force bias: the packed L transposed, one split row per g
  h->ldhp = round_up(d.Npk, 32);
  if ((rc = dalloc_t(h, &h->lt_t_split, (size_t)d.K * 2 * h->ldhp))) return rc;
  if ((rc = dalloc_t(h, &h->lt_t_unscale, (size_t)d.K))) return rc;
  HIP_TRY(setup_split_lt_transposed(h->split, d.K, d.N, d.Npk, h->ldhp, h->pq, dL, h->lt_t_split, h->lt_t_unscale, s));
  return AFQMC_OK;
}

// E_T = E_L(PhiT), always evaluated with FP64 contractions.
int trial_energy_fp64(afqmc_ham* h, const double* Y_a, const double* Y_b, hipStream_t s, double* et) {
  const StepDims& d = h->d;
  TempAllocs tmp;
  void* Lh64 = h->Lh;
  void* theta64 = h->theta;
  if (h->prec != AFQMC_FP64) {
    double* tmp_lh = nullptr;
    double* tmp_theta = nullptr;
    HIP_TRY(tmp.get(&tmp_lh, (size_t)2 * d.K * d.nmax * d.ldN * sizeof(double)));
    HIP_TRY(hipMemset(tmp_lh, 0, (size_t)2 * d.K * d.nmax * d.ldN * sizeof(double)));
    HIP_TRY(tmp.get(&tmp_theta, (size_t)4 * d.nmax * d.ldN * sizeof(double)));
    HIP_TRY(hipMemset(tmp_theta, 0, (size_t)4 * d.nmax * d.ldN * sizeof(double)));
    HIP_TRY((setup_pack_lh<double>(d.K, d.N, d.na, d.nmax, d.ldN, Y_a, tmp_lh, s)));
    if (d.nb > 0)
      HIP_TRY((setup_pack_lh<double>(d.K, d.N, d.nb, d.nmax, d.ldN, Y_b,
                                     tmp_lh + (size_t)d.K * d.nmax * d.ldN, s)));
    Lh64 = tmp_lh;
    theta64 = tmp_theta;
  }
  double2 *wa = nullptr, *wb = nullptr, *e = nullptr;
  HIP_TRY(tmp.get(&wa, (size_t)d.N * d.nmax * sizeof(double2)));
  HIP_TRY(tmp.get(&wb, (size_t)d.N * d.nmax * sizeof(double2)));
  HIP_TRY(tmp.get(&e, 3 * sizeof(double2)));
  HIP_TRY(setup_trial_walker(d.N, d.na, d.nmax, h->phiT, wa, s));
  HIP_TRY(setup_trial_walker(d.N, d.nb, d.nmax, h->phiT + (size_t)d.N * d.nmax, wb, s));
  HIP_TRY((launch_gf<double>(d, 1, wa, wb, h->phiT, h->hh, (double*)theta64, h->logdet, h->e1,
                             h->status, s)));
  HIP_TRY((launch_force_bias<double>(d, 1, (const double*)Lh64, (const double*)theta64, h->vbias, s)));
  int ntg = 0;
  for (int sp = 0; sp < 2; ++sp)
    HIP_TRY((launch_exchange<double>(d, 1, (const double*)Lh64, (const double*)theta64, h->part, sp,
                                     &ntg, s)));
  HIP_TRY(launch_energy(d, 1, h->e1, h->vbias, h->part, ntg, e, nullptr, 0, s));
  double2 he[3];
  HIP_TRY(hipMemcpyAsync(he, e, sizeof he, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *et = he[0].x + he[1].x + he[2].x;
  return AFQMC_OK;
}

// Bytes of the pair integrals (both spins, or one when they are shared) and
// of the largest temporary of their construction.
void pair_bytes(const afqmc_ham* h, bool shared, double* keep, double* temp) {
  const StepDims& d = h->d;
  const double Np = (d.N + 3) & ~3;
  double rows = 0.0, rmax = 0.0, cmax = 0.0;
  for (int sp = 0; sp < (shared ? 1 : 2); ++sp) {
    const double n = sp ? d.nb : d.na;
    const double r = Np * n * (n + 1) / 2;
    rows += r;
    rmax = r > rmax ? r : rmax;
    const double c = (double)d.N * n * d.N * n * 8.0;
    cmax = c > cmax ? c : cmax;
  }
  const double per = h->split != SPLIT_NONE ? 2.0 * d.ldh * 2 + 4 : (double)d.ldN * h->tsize;
  *keep = rows * per;
  *temp = cmax + (h->split != SPLIT_NONE ? rmax * d.ldN * 4.0 : 0.0);
}

// Pair integrals V_ij = sum_g Lh_g[i] (x) Lh_g[j] of each spin (i <= j,
// rows (i, j, p) over q, i < j blocks doubled), in the working format of the
// exchange kernels, and the row-tile tables of both spins.  Y_s: FP64
// half-rotated vectors [K][N][n_s].  shared: the beta pair integrals are the
// alpha ones (same trial orbitals).
int build_pair_integrals(afqmc_ham* h, const double* Y_a, const double* Y_b, bool shared, hipStream_t s) {
  const StepDims& d = h->d;
  const int N = d.N, Np = (N + 3) & ~3;
  const int BM = h->split != SPLIT_NONE ? exchange_pair_split_rows()
                                        : (h->prec == AFQMC_FP64 ? exchange_pair_rows<double>()
                                                                 : exchange_pair_rows<float>());
  PairTab tabs[2];
  memset(tabs, 0, sizeof tabs);
  long rows[2] = {0, 0};
  for (int sp = 0; sp < 2; ++sp) {
    const int n = sp ? d.nb : d.na;
    int st = 0, vb = 0;
    for (int i = 0; i < n; ++i) {
      tabs[sp].start[i] = st;
      tabs[sp].vbase[i] = vb;
      st += ceil_div((n - i) * Np, BM);
      vb += (n - i) * Np;
    }
    tabs[sp].start[n] = st;
    tabs[sp].vbase[n] = vb;
    h->pair_ntiles[sp] = st;
    rows[sp] = vb;
  }
  h->pair_ntg = h->pair_ntiles[0] > h->pair_ntiles[1] ? h->pair_ntiles[0] : h->pair_ntiles[1];
  h->pair_vrow0[0] = 0;
  h->pair_vrow0[1] = shared ? 0 : rows[0];
  const long total = shared ? rows[0] : rows[0] + rows[1];
  int rc;
  if ((rc = dalloc_t(h, &h->pair_tab, (size_t)2))) return rc;
  HIP_TRY(hipMemcpy(h->pair_tab, tabs, sizeof tabs, hipMemcpyHostToDevice));
  if (h->split != SPLIT_NONE) {
    if ((rc = dalloc_t(h, &h->vpair_split, (size_t)total * 2 * d.ldh))) return rc;
    if ((rc = dalloc_t(h, &h->vpair_unscale, (size_t)total))) return rc;
  } else {
    if ((rc = dalloc(h, &h->vpair, (size_t)total * d.ldN * h->tsize))) return rc;
  }
  double* C = nullptr;
  float* tmp = nullptr;
  TempAllocs temps;
  const int nmx = shared ? d.na : d.nmax;
  HIP_TRY(temps.get(&C, (size_t)N * nmx * N * nmx * sizeof(double)));
  if (h->split != SPLIT_NONE) {
    const long rmax = rows[0] > rows[1] ? rows[0] : rows[1];
    HIP_TRY(temps.get(&tmp, (size_t)rmax * d.ldN * sizeof(float)));
  }
  for (int sp = 0; sp < (shared ? 1 : 2); ++sp) {
    const int n = sp ? d.nb : d.na;
    if (n == 0) continue;
    const double* Y = sp ? Y_b : Y_a;
    const int M = N * n;
    // C[p n + i][q n + j] = sum_g Y[g][p][i] Y[g][q][j]
    HIP_TRY(setup_gemm(M, M, d.K, 1, Y, M, Y, M, C, M, nullptr, 1, s));
    const long r0 = h->pair_vrow0[sp];
    if (h->split != SPLIT_NONE) {
      HIP_TRY(setup_pack_vpair<float>(N, n, Np, d.ldN, rows[sp], C, tmp, s));
      HIP_TRY(launch_split_rows_mode(h->split, rows[sp], N, tmp, d.ldN, h->vpair_split + (size_t)r0 * 2 * d.ldh,
                                     d.ldh, h->vpair_unscale + r0, s));
    } else if (h->prec != AFQMC_FP64) {
      HIP_TRY(setup_pack_vpair<float>(N, n, Np, d.ldN, rows[sp], C, (float*)h->vpair + (size_t)r0 * d.ldN, s));
    } else {
      HIP_TRY(setup_pack_vpair<double>(N, n, Np, d.ldN, rows[sp], C, (double*)h->vpair + (size_t)r0 * d.ldN, s));
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  return AFQMC_OK;
}

int init_impl(afqmc_ham* h, const double* host_h1, const double* host_chol, const double* host_pa,
              const double* host_pb, hipStream_t s) {
  const afqmc_params& p = h->prm;
  StepDims& d = h->d;
  int rc;
  HIP_TRY(hipGetDevice(&h->device));
  d.N = p.N;
  d.na = p.na;
  d.nb = p.nb;
  d.nmax = p.na > p.nb ? p.na : p.nb;
  d.K = p.K;
  d.ldN = round_up(p.N, 16);
  d.ldK = round_up(p.K, 16);
  d.ldV = round_up(2 * p.N, 32);  // whole 32-float k blocks per VHS row (zero padded)
  d.ldP = round_up(p.N, 16);
  d.ncol = 2 * (p.na + p.nb);
  d.ncolp = round_up(d.ncol, 4);
  d.Npk = p.N * (p.N + 1) / 2;
  d.ldh = round_up(p.N, 32);
  d.ldhK = round_up(p.K, 32);
  h->prec = p.precision;
  h->tsize = p.precision == AFQMC_FP64 ? sizeof(double) : sizeof(float);
  h->split = p.precision == AFQMC_BF16X3 ? SPLIT_BF16 : (p.precision == AFQMC_FP16X3 ? SPLIT_F16 : SPLIT_NONE);
  h->sdt = sqrt(p.dt);
  HIP_TRY(set_kernel_attributes(d));

  const int N = d.N, K = d.K, nmax = d.nmax;
  const size_t NN = (size_t)N * N;
  // ---- inputs ----
  TempAllocs tmp;  // setup temporaries (L alone is K N^2 doubles), freed on every exit
  double *dh1 = nullptr, *dL = nullptr;
  HIP_TRY(tmp.get(&dh1, NN * sizeof(double)));
  HIP_TRY(hipMemcpy(dh1, host_h1, NN * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(tmp.get(&dL, (size_t)K * NN * sizeof(double)));
  HIP_TRY(hipMemcpy(dL, host_chol, (size_t)K * NN * sizeof(double), hipMemcpyHostToDevice));
  if ((rc = dalloc_t(h, &h->phiT, (size_t)2 * N * nmax))) return rc;
  {
    // index packing only: [N][ns] -> [2][N][nmax]
    std::vector<double> pk((size_t)2 * N * nmax, 0.0);
    for (int q = 0; q < N; ++q) {
      for (int j = 0; j < d.na; ++j) pk[(size_t)q * nmax + j] = host_pa[(size_t)q * d.na + j];
      for (int j = 0; j < d.nb; ++j) pk[(size_t)N * nmax + (size_t)q * nmax + j] = host_pb[(size_t)q * d.nb + j];
    }
    HIP_TRY(hipMemcpy(h->phiT, pk.data(), pk.size() * sizeof(double), hipMemcpyHostToDevice));
    std::vector<int2> tab(d.Npk);
    size_t c = 0;
    for (int a = 0; a < N; ++a)
      for (int b = a; b < N; ++b) tab[c++] = make_int2(a, b);
    if ((rc = dalloc_t(h, &h->pq, (size_t)d.Npk))) return rc;
    HIP_TRY(hipMemcpy(h->pq, tab.data(), tab.size() * sizeof(int2), hipMemcpyHostToDevice));
  }

  // ---- h' = h1 - 1/2 sum_g L_g L_g, mu ----
  double *LL = nullptr, *hp = nullptr, *scal = nullptr, *scratch = nullptr;
  HIP_TRY(tmp.get(&LL, NN * sizeof(double)));
  HIP_TRY(tmp.get(&hp, NN * sizeof(double)));
  HIP_TRY(tmp.get(&scal, 4 * sizeof(double)));
  const int nchunk = 64;
  HIP_TRY(tmp.get(&scratch, (size_t)nchunk * NN * sizeof(double)));
  HIP_TRY(setup_gemm(N, N, K * N, 2, dL, N, dL, N, LL, N, scratch, nchunk, s));
  HIP_TRY(setup_hprime(N, dh1, LL, hp, scal, s));
  double tr = 0.0;
  HIP_TRY(hipMemcpyAsync(&tr, scal, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  h->mu = isnan(p.mu) ? tr / N : p.mu;

  // ---- P = exp(-dt/2 (h' - mu)) ----
  double *A = LL, *R = nullptr, *T = scratch;
  HIP_TRY(setup_expm_arg(N, hp, h->mu, -0.5 * p.dt, A, scal + 1, s));
  double nrm = 0.0;
  HIP_TRY(hipMemcpyAsync(&nrm, scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int sq = 0;
  while (nrm > 0.5 && sq < 60) {
    nrm *= 0.5;
    ++sq;
  }
  HIP_TRY(tmp.get(&R, NN * sizeof(double)));
  HIP_TRY(setup_expm(N, A, sq, 18, R, T, s));
  if ((rc = dalloc_t(h, &h->P, (size_t)N * d.ldP))) return rc;
  HIP_TRY(setup_copy_pad(N, N, R, N, h->P, d.ldP, s));

  // ---- half-rotated vectors: Y_s = [K N][N] x PhiT_s -> Lh ----
  double *Y_a = nullptr, *Y_b = nullptr, *pa_dense = nullptr, *pb_dense = nullptr;
  HIP_TRY(tmp.get(&Y_a, (size_t)K * N * (d.na > 0 ? d.na : 1) * sizeof(double)));
  HIP_TRY(tmp.get(&Y_b, (size_t)K * N * (d.nb > 0 ? d.nb : 1) * sizeof(double)));
  HIP_TRY(tmp.get(&pa_dense, (size_t)N * (d.na > 0 ? d.na : 1) * sizeof(double)));
  HIP_TRY(tmp.get(&pb_dense, (size_t)N * (d.nb > 0 ? d.nb : 1) * sizeof(double)));
  HIP_TRY(hipMemcpy(pa_dense, host_pa, (size_t)N * d.na * sizeof(double), hipMemcpyHostToDevice));
  if (d.nb > 0) HIP_TRY(hipMemcpy(pb_dense, host_pb, (size_t)N * d.nb * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(setup_gemm(K * N, d.na, N, 0, dL, N, pa_dense, d.na, Y_a, d.na, nullptr, 1, s));
  if (d.nb > 0) HIP_TRY(setup_gemm(K * N, d.nb, N, 0, dL, N, pb_dense, d.nb, Y_b, d.nb, nullptr, 1, s));
  if ((rc = dalloc_t(h, &h->hh, (size_t)2 * nmax * N))) return rc;
  HIP_TRY(setup_hh(N, d.na, nmax, h->phiT, dh1, h->hh, s));
  HIP_TRY(setup_hh(N, d.nb, nmax, h->phiT + (size_t)N * nmax, dh1, h->hh + (size_t)nmax * N, s));
  if (h->prec != AFQMC_FP64)
    rc = build_working_arrays<float>(h, dL, Y_a, Y_b, s);
  else
    rc = build_working_arrays<double>(h, dL, Y_a, Y_b, s);
  if (rc) return rc;
  if (h->split != SPLIT_NONE) {
    const size_t rows = (size_t)2 * K * nmax;
    if ((rc = dalloc_t(h, &h->lh_split, rows * 2 * d.ldh))) return rc;
    if ((rc = dalloc_t(h, &h->lh_unscale, rows))) return rc;
    HIP_TRY(launch_split_rows_mode(h->split, (long)rows, N, (const float*)h->Lh, d.ldN, h->lh_split,
                                   d.ldh, h->lh_unscale, s));
  }

  // ---- exchange algorithm: pair integrals when they pay and fit ----
  {
    bool shared = d.na == d.nb;
    for (size_t e = 0; shared && e < (size_t)N * d.na; ++e) shared = host_pa[e] == host_pb[e];
    double keep = 0.0, temp = 0.0;
    pair_bytes(h, shared, &keep, &temp);
    const bool fits = keep + temp <= 48.0 * (1 << 30);
    // direct: K n^2 N products per walker and spin; pair: n (n + 1) / 2 N^2
    const double gain = 2.0 * K * nmax / ((nmax + 1.0) * N);
    int algo = p.exchange;
    if (algo == AFQMC_EXCHANGE_AUTO) algo = (gain > 1.5 && fits) ? AFQMC_EXCHANGE_PAIR : AFQMC_EXCHANGE_DIRECT;
    if (algo == AFQMC_EXCHANGE_PAIR && !fits)
      return fail(AFQMC_ENOMEM, "pair integrals need %.1f GB (+%.1f GB during setup)", keep / 1e9, temp / 1e9);
    h->ex_algo = algo;
    if (algo == AFQMC_EXCHANGE_PAIR && (rc = build_pair_integrals(h, Y_a, Y_b, shared, s))) return rc;
  }

  // ---- workspace ----
  const size_t W = (size_t)p.max_walkers;
  // the FP64 trial-energy pass may use the FP64 tile even in the mixed path
  const ExTile t32 = exchange_tile<float>(nmax), t64 = exchange_tile<double>(nmax);
  const ExTile tsp = exchange_split_tile(nmax);
  int gmin = t32.G < t64.G ? t32.G : t64.G;
  if (tsp.G < gmin) gmin = tsp.G;
  h->ntg = ceil_div(K, gmin);
  if (h->pair_ntg > h->ntg) h->ntg = h->pair_ntg;
  const size_t ts = h->tsize;
  const size_t wtheta = (W > 1 ? W : 1);
  if ((rc = dalloc(h, &h->theta, wtheta * 4 * nmax * d.ldN * ts))) return rc;
  if ((rc = dalloc_t(h, &h->logdet, wtheta * 2))) return rc;
  if ((rc = dalloc_t(h, &h->e1, wtheta * 2))) return rc;
  if ((rc = dalloc_t(h, &h->vbias, wtheta * K))) return rc;
  if ((rc = dalloc(h, &h->xs, W * 2 * d.ldK * ts))) return rc;
  if ((rc = dalloc_t(h, &h->a, W))) return rc;
  if ((rc = dalloc(h, &h->vhs, W * N * d.ldV * ts))) return rc;
  if ((rc = dalloc_t(h, &h->acc, W * N * d.ncolp))) return rc;
  if (!vhs_split(h)) {  // Taylor ping-pong terms (the split path keeps every term in tk)
    if ((rc = dalloc(h, &h->t0, W * N * d.ncolp * ts))) return rc;
    if ((rc = dalloc(h, &h->t1, W * N * d.ncolp * ts))) return rc;
  }
  // running maxima: slot 0 max |P phi|, 1 max |VHS| (fused propagation: a
  // bound on |VHS|, written by the shift), 1 + k max |t_k|
  if ((rc = dalloc_t(h, &h->tmax, W * (size_t)(p.taylor_order + 2)))) return rc;
  if ((rc = dalloc_t(h, &h->part, (size_t)2 * h->ntg * wtheta))) return rc;
  if ((rc = dalloc_t(h, &h->corr, W * 2))) return rc;
  if ((rc = dalloc_t(h, &h->status, (size_t)1))) return rc;
  if ((rc = dalloc_t(h, &h->pc_csum, W))) return rc;
  if ((rc = dalloc_t(h, &h->pc_cnt, W))) return rc;
  if ((rc = dalloc_t(h, &h->pc_src, W))) return rc;
  if ((rc = dalloc_t(h, &h->pc_parent, W))) return rc;
  if (h->split != SPLIT_NONE) {
    const size_t rows = wtheta * 4 * nmax;
    if ((rc = dalloc_t(h, &h->th_split, rows * 2 * d.ldh))) return rc;
    if ((rc = dalloc_t(h, &h->th_unscale, rows))) return rc;
  }
  if (vhs_split(h)) {
    if ((rc = dalloc_t(h, &h->xs_split, W * 2 * 2 * d.ldhK))) return rc;
    if ((rc = dalloc_t(h, &h->xs_unscale, W * 2))) return rc;
    const PropFusedGeom pg = prop_fused_geom(d);
    h->prop_fused = pg.ok && !(p.flags & (AFQMC_FLAG_ONE_BODY_FP64 | AFQMC_FLAG_UNFUSED_PROPAGATION));
    if (h->prop_fused) {
      if ((rc = dalloc_t(h, &h->psplit, pg.psplit_halves))) return rc;
      unsigned* pmax = nullptr;
      HIP_TRY(tmp.get(&pmax, sizeof(unsigned)));
      HIP_TRY(setup_prop_fused(d, h->P, h->psplit, pmax, &h->pexp, s));
      if ((rc = dalloc_t(h, &h->lmax, (size_t)K))) return rc;
      HIP_TRY(setup_lmax(K, N, dL, h->lmax, s));
    } else {
      if ((rc = dalloc_t(h, &h->tk, (size_t)p.taylor_order * W * N * d.ncolp))) return rc;
    }
    if ((rc = dalloc_t(h, &h->fb_th, W * 2 * 2 * nmax * 2 * d.ldh))) return rc;
    if ((rc = dalloc_t(h, &h->fb_th_unscale, W * 2))) return rc;
    if ((rc = dalloc_t(h, &h->fb_part, (size_t)FB_SPLIT_CHUNKS * 2 * W * K))) return rc;
  }

  // ---- E_T ----
  if (isnan(p.e_shift)) {
    double et = 0.0;
    if ((rc = trial_energy_fp64(h, Y_a, Y_b, s, &et))) return rc;
    h->e_shift = et;
  } else {
    h->e_shift = p.e_shift;
  }
  h->cst = -p.dt * (h->mu * (d.na + d.nb) - h->e_shift);
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemset(h->status, 0, sizeof(int)));
  return AFQMC_OK;
}

}  // namespace

// ===========================================================================
// exported entry points
// ===========================================================================

namespace {

// theta of the given walkers into the workspace; the step cache survives only
// if these are the cached walkers (theta is then recomputed bit for bit).
template <typename T>
int seq_theta_keep_cache(afqmc_ham* h, const afqmc_walkers* w, int nw, hipStream_t s) {
  const bool same = h->c_valid && h->c_phi_a == w->phi_a && h->c_phi_b == w->phi_b && h->c_nw == nw;
  int rc = seq_theta<T>(h, w, nw, false, s);
  if (!same) h->c_valid = false;
  return rc;
}

}  // namespace

extern "C" {

int afqmc_version(void) { return 1; }

const char* afqmc_last_error(void) { return g_last_error.c_str(); }

int afqmc_init_hamiltonian(const afqmc_params* params, const double* host_h1,
                           const double* host_chol, const double* host_phiT_a,
                           const double* host_phiT_b, void* stream, afqmc_ham** out) {
  if (!out) return fail(AFQMC_EINVAL, "null output handle pointer");
  *out = nullptr;
  if (!params || !host_h1 || !host_chol || !host_phiT_a)
    return fail(AFQMC_EINVAL, "null input pointer");
  const afqmc_params& p = *params;
  if (p.N < 1 || p.K < 1 || p.na < 1 || p.nb < 0 || p.na > p.N || p.nb > p.N)
    return fail(AFQMC_EINVAL, "bad sizes N=%d na=%d nb=%d K=%d", p.N, p.na, p.nb, p.K);
  if (p.nb > 0 && !host_phiT_b) return fail(AFQMC_EINVAL, "null host_phiT_b with nb > 0");
  if (p.na > 45 || p.nb > 45)
    return fail(AFQMC_EUNSUPPORTED, "at most 45 electrons per spin are supported (got %d, %d)", p.na, p.nb);
  if (!(p.dt > 0.0)) return fail(AFQMC_EINVAL, "dt must be positive");
  if (p.taylor_order < 1 || p.taylor_order > 30) return fail(AFQMC_EINVAL, "taylor_order must be in [1, 30]");
  if (p.precision < AFQMC_FP64 || p.precision > AFQMC_FP16X3)
    return fail(AFQMC_EINVAL, "unknown precision %d", p.precision);
  if (p.max_walkers < 1) return fail(AFQMC_EINVAL, "max_walkers must be >= 1");
  if (p.exchange < AFQMC_EXCHANGE_AUTO || p.exchange > AFQMC_EXCHANGE_PAIR)
    return fail(AFQMC_EINVAL, "unknown exchange algorithm %d", p.exchange);
  if (p.flags & ~(AFQMC_FLAG_ONE_BODY_FP64 | AFQMC_FLAG_UNFUSED_PROPAGATION))
    return fail(AFQMC_EINVAL, "unknown flags 0x%x", p.flags);
  const int nmax = p.na > p.nb ? p.na : p.nb;
  if (qr_lds_bytes_for(p.N, nmax) > 160 * 1024)
    return fail(AFQMC_EUNSUPPORTED, "N * max(na, nb) too large for the in-LDS QR (N=%d, n=%d)", p.N, nmax);
  {
    const ExTile t = p.precision == AFQMC_FP64 ? exchange_tile<double>(nmax) : exchange_tile<float>(nmax);
    if (t.G < 1 || t.Z < 1) return fail(AFQMC_EUNSUPPORTED, "electron count %d too large for the exchange tile", nmax);
  }
  afqmc_ham* h = new afqmc_ham();
  h->prm = p;
  const int rc = init_impl(h, host_h1, host_chol, host_phiT_a, p.nb > 0 ? host_phiT_b : host_phiT_a,
                           (hipStream_t)stream);
  if (rc) {
    free_all(h);
    delete h;
    return rc;
  }
  *out = h;
  return AFQMC_OK;
}

int afqmc_overlap(afqmc_ham* h, const afqmc_walkers* w, int nw, void* stream) {
  int rc = check_walkers(h, w, nw);
  if (rc || nw == 0) return rc;
  if ((rc = set_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY((launch_gf<double>(h->d, nw, (const double2*)w->phi_a, (const double2*)w->phi_b, h->phiT,
                             h->hh, nullptr, h->logdet, nullptr, h->status, s)));
  HIP_TRY(launch_overlap_store(nw, h->logdet, (double2*)w->log_ovlp, s));
  return AFQMC_OK;
}

int afqmc_force_bias(afqmc_ham* h, const afqmc_walkers* w, int nw, void* vbias, void* stream) {
  int rc = check_walkers(h, w, nw);
  if (rc || nw == 0) return rc;
  if (!vbias) return fail(AFQMC_EINVAL, "null vbias");
  if ((rc = set_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (h->prec != AFQMC_FP64) {
    if ((rc = seq_theta<float>(h, w, nw, false, s))) return rc;
    rc = seq_force_bias<float>(h, nw, (double2*)vbias, s);
  } else {
    if ((rc = seq_theta<double>(h, w, nw, false, s))) return rc;
    rc = seq_force_bias<double>(h, nw, (double2*)vbias, s);
  }
  h->c_valid = false;
  return rc;
}

int afqmc_propagate(afqmc_ham* h, afqmc_walkers* w, int nw, const double* fields, void* stream) {
  int rc = check_walkers(h, w, nw);
  if (rc || nw == 0) return rc;
  if (!fields) return fail(AFQMC_EINVAL, "null fields");
  if ((rc = set_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  return h->prec != AFQMC_FP64 ? seq_propagate<float>(h, w, nw, fields, s)
                               : seq_propagate<double>(h, w, nw, fields, s);
}

int afqmc_local_energy(afqmc_ham* h, const afqmc_walkers* w, int nw, void* e, void* stream) {
  int rc = check_walkers(h, w, nw);
  if (rc || nw == 0) return rc;
  if (!e) return fail(AFQMC_EINVAL, "null energy output");
  if ((rc = set_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  return h->prec != AFQMC_FP64 ? seq_local_energy<float>(h, w, nw, (double2*)e, s)
                               : seq_local_energy<double>(h, w, nw, (double2*)e, s);
}

int afqmc_orthogonalise(afqmc_ham* h, afqmc_walkers* w, int nw, void* stream) {
  int rc = check_walkers(h, w, nw);
  if (rc || nw == 0) return rc;
  if ((rc = set_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  PHASE(h, AFQMC_PH_QR, s,
        launch_qr(h->d, nw, (double2*)w->phi_a, (double2*)w->phi_b, h->corr, h->status, s));
  HIP_TRY(launch_ortho_update(nw, h->corr, (double2*)w->log_ovlp, w->log_w, s));
  // theta is invariant under re-orthogonalisation; the cached force bias stays valid.
  return AFQMC_OK;
}

int afqmc_step(afqmc_ham* h, afqmc_walkers* w, int nw, const double* fields, int do_qr, void* e,
               int flags, void* stream) {
  int rc = check_walkers(h, w, nw);
  if (rc || nw == 0) return rc;
  if (!fields) return fail(AFQMC_EINVAL, "null fields");
  if ((rc = set_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  StepIO io;
  io.fields = fields;
  io.e = (double2*)e;
  return h->prec != AFQMC_FP64 ? seq_step<float>(h, w, nw, io, do_qr, flags, s)
                               : seq_step<double>(h, w, nw, io, do_qr, flags, s);
}

int afqmc_global_energy(afqmc_ham* h, const afqmc_walkers* w, int nw, const void* e, double* out,
                        void* stream) {
  int rc = check_walkers(h, w, nw);
  if (rc) return rc;
  if (!out || (nw > 0 && !e)) return fail(AFQMC_EINVAL, "null energy or output array");
  if ((rc = set_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  PHASE(h, AFQMC_PH_CONTROL, s,
        launch_global_energy(nw, nw ? w->log_w : nullptr, (const double2*)e, out, s));
  return AFQMC_OK;
}

namespace {

int seq_comb(afqmc_ham* h, afqmc_walkers* w, int nw, double u, int* parent, hipStream_t s) {
  PHASE(h, AFQMC_PH_CONTROL, s,
        launch_comb(h->d, nw, u, (double2*)w->phi_a, (double2*)w->phi_b, (double2*)w->log_ovlp, w->log_w,
                    h->pc_csum, h->pc_cnt, h->pc_src, parent ? parent : h->pc_parent, h->status, s));
  h->c_valid = false;  // walkers moved: the cached Green's function no longer matches
  return AFQMC_OK;
}

}  // namespace

int afqmc_population_control(afqmc_ham* h, afqmc_walkers* w, int nw, double u, int* parent, void* stream) {
  int rc = check_walkers(h, w, nw);
  if (rc || nw == 0) return rc;
  if (!(u >= 0.0 && u < 1.0)) return fail(AFQMC_EINVAL, "comb offset u = %g outside [0, 1)", u);
  if ((rc = set_device(h))) return rc;
  return seq_comb(h, w, nw, u, parent, (hipStream_t)stream);
}

int afqmc_population_control_noalloc(int N, int na, int nb, afqmc_walkers* w, int nw, double u, int* parent,
                                     int* status, void* stream) {
  if (N < 1 || na < 0 || nb < 0 || na > N || nb > N)
    return fail(AFQMC_EINVAL, "bad sizes N = %d, na = %d, nb = %d", N, na, nb);
  if (nw < 0 || nw > COMB_STATIC_MAX_WALKERS)
    return fail(AFQMC_EINVAL, "nw = %d outside [0, %d] (the static scratch's limit)", nw, COMB_STATIC_MAX_WALKERS);
  if (nw == 0) return AFQMC_OK;
  if (!w || (na > 0 && !w->phi_a) || (nb > 0 && !w->phi_b) || !w->log_ovlp || !w->log_w)
    return fail(AFQMC_EINVAL, "null walker array");
  if (!(u >= 0.0 && u < 1.0)) return fail(AFQMC_EINVAL, "comb offset u = %g outside [0, 1)", u);
  void* sp = nullptr;
  HIP_TRY(comb_static_scratch(&sp));
  StepDims d{};
  d.N = N;
  d.na = na;
  d.nb = nb;
  HIP_TRY(launch_comb_static(sp, d, nw, u, (double2*)w->phi_a, (double2*)w->phi_b, (double2*)w->log_ovlp, w->log_w,
                             parent, status, (hipStream_t)stream));
  return AFQMC_OK;
}

int afqmc_block(afqmc_ham* h, afqmc_walkers* w, int nw, const double* fields, int nsteps, double u, void* e,
                double* out, int* parent, int flags, void* stream) {
  int rc = check_walkers(h, w, nw);
  if (rc) return rc;
  if (nsteps < 1) return fail(AFQMC_EINVAL, "nsteps = %d must be >= 1", nsteps);
  if (!out || (nw > 0 && (!fields || !e))) return fail(AFQMC_EINVAL, "null fields, energy or output array");
  if (!(u < 1.0)) return fail(AFQMC_EINVAL, "comb offset u = %g must be < 1 (negative: no comb)", u);
  if ((rc = set_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (nw == 0) {
    HIP_TRY(launch_global_energy(0, nullptr, nullptr, out, s));
    return AFQMC_OK;
  }
  for (int st = 0; st < nsteps; ++st) {
    const bool last = st == nsteps - 1;
    StepIO io;
    io.fields = fields + (size_t)st * nw * h->d.K;
    io.e = last ? (double2*)e : nullptr;
    const int f = st ? AFQMC_STEP_REUSE : flags;
    rc = h->prec != AFQMC_FP64 ? seq_step<float>(h, w, nw, io, last, f, s)
                               : seq_step<double>(h, w, nw, io, last, f, s);
    if (rc) return rc;
  }
  PHASE(h, AFQMC_PH_CONTROL, s, launch_global_energy(nw, w->log_w, (const double2*)e, out, s));
  if (u >= 0.0) return seq_comb(h, w, nw, u, parent, s);
  return AFQMC_OK;
}

int afqmc_green_function(afqmc_ham* h, const afqmc_walkers* w, int nw, void* G, void* stream) {
  int rc = check_walkers(h, w, nw);
  if (rc || nw == 0) return rc;
  if (!G) return fail(AFQMC_EINVAL, "null G");
  if ((rc = set_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (h->prec != AFQMC_FP64) {
    if ((rc = seq_theta_keep_cache<float>(h, w, nw, s))) return rc;
    PHASE(h, AFQMC_PH_ESTIMATOR, s, launch_green_full<float>(h->d, nw, (const float*)h->theta, h->phiT, (double2*)G, s));
  } else {
    if ((rc = seq_theta_keep_cache<double>(h, w, nw, s))) return rc;
    PHASE(h, AFQMC_PH_ESTIMATOR, s, launch_green_full<double>(h->d, nw, (const double*)h->theta, h->phiT, (double2*)G, s));
  }
  return AFQMC_OK;
}

int afqmc_s2_mixed(afqmc_ham* h, const afqmc_walkers* w, int nw, void* s2, void* stream) {
  int rc = check_walkers(h, w, nw);
  if (rc || nw == 0) return rc;
  if (!s2) return fail(AFQMC_EINVAL, "null s2");
  if ((rc = set_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (h->prec != AFQMC_FP64) {
    if ((rc = seq_theta_keep_cache<float>(h, w, nw, s))) return rc;
    PHASE(h, AFQMC_PH_ESTIMATOR, s, launch_s2<float>(h->d, nw, (const float*)h->theta, h->phiT, (double2*)s2, s));
  } else {
    if ((rc = seq_theta_keep_cache<double>(h, w, nw, s))) return rc;
    PHASE(h, AFQMC_PH_ESTIMATOR, s, launch_s2<double>(h->d, nw, (const double*)h->theta, h->phiT, (double2*)s2, s));
  }
  return AFQMC_OK;
}

int afqmc_weighted_mean(afqmc_ham* h, const afqmc_walkers* w, int nw, const void* v, int m, double* out,
                        void* stream) {
  int rc = check_walkers(h, w, nw);
  if (rc) return rc;
  if (m < 1 || m > (1 << 24)) return fail(AFQMC_EINVAL, "m = %d outside [1, 2^24]", m);
  if (!out || (nw > 0 && !v)) return fail(AFQMC_EINVAL, "null value or output array");
  if ((rc = set_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  PHASE(h, AFQMC_PH_ESTIMATOR, s,
        launch_weighted_mean(nw, m, nw ? w->log_w : nullptr, (const double2*)v, out, s));
  return AFQMC_OK;
}

int afqmc_get_status(afqmc_ham* h, void* stream, int* out) {
  if (!h || !out) return fail(AFQMC_EINVAL, "null argument");
  int rc;
  if ((rc = set_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  int v = 0;
  HIP_TRY(hipMemcpyAsync(&v, h->status, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int zero = 0;
  HIP_TRY(hipMemcpyAsync(h->status, &zero, sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = v;
  return AFQMC_OK;
}

int afqmc_get_exchange_algorithm(afqmc_ham* h, int* out) {
  if (!h || !out) return fail(AFQMC_EINVAL, "null argument");
  *out = h->ex_algo;
  return AFQMC_OK;
}

int afqmc_get_setup(afqmc_ham* h, double* host_P, double* mu, double* e_shift) {
  if (!h) return fail(AFQMC_EINVAL, "null Hamiltonian handle");
  int rc;
  if ((rc = set_device(h))) return rc;
  HIP_TRY(hipDeviceSynchronize());
  if (host_P) {
    std::vector<double> tmp((size_t)h->d.N * h->d.ldP);
    HIP_TRY(hipMemcpy(tmp.data(), h->P, tmp.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int r = 0; r < h->d.N; ++r)
      memcpy(host_P + (size_t)r * h->d.N, tmp.data() + (size_t)r * h->d.ldP, h->d.N * sizeof(double));
  }
  if (mu) *mu = h->mu;
  if (e_shift) *e_shift = h->e_shift;
  return AFQMC_OK;
}

int afqmc_profile_enable(afqmc_ham* h, int max_records) {
  if (!h) return fail(AFQMC_EINVAL, "null Hamiltonian handle");
  if (max_records < 0) return fail(AFQMC_EINVAL, "max_records must be >= 0");
  int rc;
  if ((rc = set_device(h))) return rc;
  HIP_TRY(hipDeviceSynchronize());
  for (hipEvent_t e : h->ev) HIP_TRY(hipEventDestroy(e));
  h->ev.clear();
  h->recs.clear();
  h->ev_used = 0;
  for (int i = 0; i < 2 * max_records; ++i) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    h->ev.push_back(e);
  }
  h->recs.reserve(max_records);
  return AFQMC_OK;
}

int afqmc_profile_phases(afqmc_ham* h, unsigned mask) {
  if (!h) return fail(AFQMC_EINVAL, "null Hamiltonian handle");
  h->prof_mask = mask;
  return AFQMC_OK;
}

int afqmc_profile_read(afqmc_ham* h, double* ms, int* launches) {
  if (!h || !ms || !launches) return fail(AFQMC_EINVAL, "null argument");
  int rc;
  if ((rc = set_device(h))) return rc;
  for (int p = 0; p < AFQMC_NPHASE; ++p) {
    ms[p] = 0.0;
    launches[p] = 0;
  }
  for (const auto& r : h->recs) {
    HIP_TRY(hipEventSynchronize(h->ev[r.e1]));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, h->ev[r.e0], h->ev[r.e1]));
    ms[r.phase] += t;
    launches[r.phase] += 1;
  }
  h->recs.clear();
  h->ev_used = 0;
  return AFQMC_OK;
}

void afqmc_destroy(afqmc_ham* h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  free_all(h);
  delete h;
}

}  // extern "C"

// ===========================================================================
// multi-determinant trial (Sec. III.A, III.B; kernels in msd_kernels.hip)
// ===========================================================================

struct afqmc_msd {
  int device = 0;
  int max_walkers = 0;
  int ndet = 0;
  MsdDims m{};
  StepDims d{};  // the sizes launch_gf reads (N, na, nb, nmax, ldN)
  MsdTables t{};
  double* hh0 = nullptr;  // zero one-body matrix: launch_gf's energy input, unused here
  double* theta = nullptr;
  double2* logdet = nullptr;
  double* yp = nullptr;  // planar Y [W][2][2][nmax][ldv]
  double2* sdet = nullptr;
  double2* sadj = nullptr;
  double2* tpart = nullptr;
  double2* uw = nullptr;
  double2* rpart = nullptr;
  double2* ratio = nullptr;
  double2* lpair = nullptr;  // [W][2] (log overlap, 0) for the weight update
  double* zt = nullptr;  // planar Zt [W][2][2][nmax][ldN]
  double* qp = nullptr;  // planar Q [W][2][2][N][ldq]
  int* status = nullptr;
  std::vector<void*> allocs;
  // local energy (afqmc_msd_set_hamiltonian): host copies of the orbitals,
  // the active sets, the tables and workspace of msd_energy.hip
  std::vector<double> C_host[2];
  std::vector<int> hl[2], ql[2];
  MsdEnergyDims ed{};
  MsdEnergyTables et{};
  MsdEnergyWork ew{};
  bool has_ham = false;
};

namespace {

void msd_free(afqmc_msd* t) {
  for (void* p : t->allocs) (void)hipFree(p);
  t->allocs.clear();
}

template <typename T>
int msd_upload(afqmc_msd* t, const T** dst, const std::vector<T>& v) {
  T* p = nullptr;
  int rc = dalloc_t(t, &p, v.size());
  if (rc) return rc;
  if (!v.empty()) HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *dst = p;
  return AFQMC_OK;
}

// Host-only check of the excitation format (before any device call).
int msd_validate(int N, int na, int nb, int ndet, const int* rank, const int* orbs) {
  const int nel[2] = {na, nb};
  std::vector<char> used(N);
  for (int a = 0; a < ndet; ++a) {
    for (int s = 0; s < 2; ++s) {
      const int k = rank[a * 2 + s];
      const int n = nel[s];
      if (k < 0 || k > MSD_KMAX || k > n || k > N - n)
        return fail(AFQMC_EINVAL, "determinant %d spin %d: rank %d outside [0, min(%d, n, N - n)]", a, s, k,
                    MSD_KMAX);
      std::fill(used.begin(), used.end(), 0);
      for (int x = 0; x < k; ++x) {
        const int h = orbs[((a * 2 + s) * 2 + 0) * MSD_KMAX + x];
        const int q = orbs[((a * 2 + s) * 2 + 1) * MSD_KMAX + x];
        if (h < 0 || h >= n || q < n || q >= N || used[h] || used[q])
          return fail(AFQMC_EINVAL, "determinant %d spin %d: invalid or repeated hole %d / particle %d", a, s,
                      h, q);
        used[h] = used[q] = 1;
      }
    }
  }
  return AFQMC_OK;
}

// Groups the determinants by per-spin excitation string and builds the
// device tables (layouts in kernels.h).
int msd_build(afqmc_msd* t, const double* C[2], const double* coeff, const int* rank, const int* orbs) {
  MsdDims& m = t->m;
  const int N = m.N, ndet = t->ndet;
  const int nel[2] = {m.na, m.nb};
  std::map<std::vector<int>, int> sid[2];
  std::vector<std::vector<int>> strs[2];
  std::vector<int> dstr[2] = {std::vector<int>(ndet), std::vector<int>(ndet)};
  for (int a = 0; a < ndet; ++a) {
    for (int s = 0; s < 2; ++s) {
      const int k = rank[a * 2 + s];  // validated by msd_validate
      std::vector<int> key(1 + 2 * k);
      key[0] = k;
      for (int x = 0; x < k; ++x) {
        key[1 + x] = orbs[((a * 2 + s) * 2 + 0) * MSD_KMAX + x];
        key[1 + k + x] = orbs[((a * 2 + s) * 2 + 1) * MSD_KMAX + x];
      }
      auto it = sid[s].find(key);
      if (it == sid[s].end()) {
        it = sid[s].emplace(key, (int)strs[s].size()).first;
        strs[s].push_back(key);
      }
      dstr[s][a] = it->second;
    }
  }
  // sort each spin's strings by rank (stable): the waves of the string
  // kernel then take one branch, and ranks above 4 form a tail
  for (int s = 0; s < 2; ++s) {
    std::vector<int> order(strs[s].size());
    for (size_t u = 0; u < order.size(); ++u) order[u] = (int)u;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return strs[s][x][0] < strs[s][y][0]; });
    std::vector<int> pos(order.size());
    std::vector<std::vector<int>> sorted(order.size());
    for (size_t u = 0; u < order.size(); ++u) {
      pos[order[u]] = (int)u;
      sorted[u] = strs[s][order[u]];
    }
    strs[s].swap(sorted);
    for (int a = 0; a < ndet; ++a) dstr[s][a] = pos[dstr[s][a]];
  }
  m.nstr[0] = (int)strs[0].size();
  m.nstr[1] = (int)strs[1].size();
  m.nstr_tot = m.nstr[0] + m.nstr[1];
  for (int s = 0; s < 2; ++s) {
    int first = m.nstr[s];
    for (int u = 0; u < m.nstr[s]; ++u)
      if (strs[s][u][0] > 4) {
        first = u;
        break;
      }
    m.big0[s] = (s ? m.nstr[0] : 0) + first;
    m.nbig[s] = m.nstr[s] - first;
  }
  // strings: rank, orbitals, adjugate offsets
  std::vector<int> srank(m.nstr_tot), sorb((size_t)m.nstr_tot * 2 * MSD_KMAX, -1), saoff(m.nstr_tot);
  long nadj = 0;
  for (int s = 0, u = 0; s < 2; ++s) {
    for (const auto& key : strs[s]) {
      const int k = key[0];
      srank[u] = k;
      saoff[u] = (int)nadj;
      for (int x = 0; x < k; ++x) {
        sorb[((size_t)u * 2 + 0) * MSD_KMAX + x] = key[1 + x];
        sorb[((size_t)u * 2 + 1) * MSD_KMAX + x] = key[1 + k + x] - nel[s];
      }
      nadj += (long)k * k;
      ++u;
    }
  }
  if (nadj > (1L << 30)) return fail(AFQMC_EUNSUPPORTED, "expansion too large (%ld adjugate entries)", nadj);
  m.nadj_tot = (int)nadj;
  // CSR over strings: the determinants of each string, in increasing a
  std::vector<int> crow(m.nstr_tot + 1, 0), cstr(2 * (size_t)ndet);
  std::vector<double> ccoef(2 * (size_t)ndet);
  for (int a = 0; a < ndet; ++a) {
    ++crow[dstr[0][a] + 1];
    ++crow[m.nstr[0] + dstr[1][a] + 1];
  }
  for (int u = 0; u < m.nstr_tot; ++u) crow[u + 1] += crow[u];
  {
    std::vector<int> fill(crow.begin(), crow.end() - 1);
    for (int a = 0; a < ndet; ++a) {
      const int ua = dstr[0][a], ub = m.nstr[0] + dstr[1][a];
      ccoef[fill[ua]] = coeff[a];
      cstr[fill[ua]++] = ub;
      ccoef[fill[ub]] = coeff[a];
      cstr[fill[ub]++] = ua;
    }
  }
  // tasks: each string's CSR row cut into pieces of at most MSD_TASK entries
  std::vector<int> tbeg, trow(m.nstr_tot + 1);
  for (int u = 0; u < m.nstr_tot; ++u) {
    trow[u] = (int)tbeg.size();
    for (int e = crow[u]; e < crow[u + 1]; e += MSD_TASK) tbeg.push_back(e);
  }
  trow[m.nstr_tot] = (int)tbeg.size();
  m.ntask = (int)tbeg.size();
  tbeg.push_back(crow[m.nstr_tot]);  // every row is non-empty: task t ends at tbeg[t + 1]
  // CSR over the (spin, hole j, virtual a) entries of M: contributions in
  // increasing string, then (m, l) order
  const int nent0 = m.na * m.nv[0], nent = nent0 + m.nb * m.nv[1];
  std::vector<std::vector<std::pair<int, int>>> ent(nent);
  for (int u = 0; u < m.nstr_tot; ++u) {
    const int s = u >= m.nstr[0] ? 1 : 0;
    const int k = srank[u];
    for (int x = 0; x < k; ++x)      // hole slot m
      for (int l = 0; l < k; ++l) {  // particle slot l
        const int j = sorb[((size_t)u * 2 + 0) * MSD_KMAX + x];
        const int av = sorb[((size_t)u * 2 + 1) * MSD_KMAX + l];
        ent[(s ? nent0 : 0) + j * m.nv[s] + av].push_back({u, saoff[u] + x * k + l});
      }
  }
  std::vector<int> erow(nent + 1, 0), estr, eoff;
  for (int e = 0; e < nent; ++e) {
    erow[e + 1] = erow[e] + (int)ent[e].size();
    for (const auto& pr : ent[e]) {
      estr.push_back(pr.first);
      eoff.push_back(pr.second);
    }
  }
  // local energy: the active holes and particles of each spin (those that
  // some string excites), every string slot's position among them, and the
  // determinants excited in both spins
  {
    std::vector<int> hpos[2], qpos[2];
    for (int s = 0; s < 2; ++s) {
      std::vector<char> hu(nel[s], 0), qu(m.nv[s], 0);
      for (const auto& key : strs[s])
        for (int x = 0; x < key[0]; ++x) {
          hu[key[1 + x]] = 1;
          qu[key[1 + key[0] + x] - nel[s]] = 1;
        }
      hpos[s].assign(nel[s], -1);
      qpos[s].assign(m.nv[s], -1);
      t->hl[s].clear();
      t->ql[s].clear();
      for (int i = 0; i < nel[s]; ++i)
        if (hu[i]) {
          hpos[s][i] = (int)t->hl[s].size();
          t->hl[s].push_back(i);
        }
      for (int a = 0; a < m.nv[s]; ++a)
        if (qu[a]) {
          qpos[s][a] = (int)t->ql[s].size();
          t->ql[s].push_back(a);
        }
    }
    const int hmax = std::max<int>(1, std::max(t->hl[0].size(), t->hl[1].size()));
    const int qmax = std::max<int>(1, std::max(t->ql[0].size(), t->ql[1].size()));
    std::vector<int> hlist((size_t)2 * hmax, 0), qlist((size_t)2 * qmax, 0);
    for (int s = 0; s < 2; ++s) {
      for (size_t x = 0; x < t->hl[s].size(); ++x) hlist[(size_t)s * hmax + x] = t->hl[s][x];
      for (size_t x = 0; x < t->ql[s].size(); ++x) qlist[(size_t)s * qmax + x] = t->ql[s][x];
    }
    std::vector<int> spos((size_t)m.nstr_tot * 2 * MSD_KMAX, 0);
    for (int u = 0; u < m.nstr_tot; ++u) {
      const int s = u >= m.nstr[0] ? 1 : 0;
      for (int x = 0; x < srank[u]; ++x) {
        spos[((size_t)u * 2 + 0) * MSD_KMAX + x] = hpos[s][sorb[((size_t)u * 2 + 0) * MSD_KMAX + x]];
        spos[((size_t)u * 2 + 1) * MSD_KMAX + x] = qpos[s][sorb[((size_t)u * 2 + 1) * MSD_KMAX + x]];
      }
    }
    std::vector<int> xa, xb;
    std::vector<double> xc;
    for (int a = 0; a < ndet; ++a) {
      const int ua = dstr[0][a], ub = m.nstr[0] + dstr[1][a];
      if (srank[ua] > 0 && srank[ub] > 0) {
        xa.push_back(ua);
        xb.push_back(ub);
        xc.push_back(coeff[a]);
      }
    }
    MsdEnergyDims& e = t->ed;
    e.Hmax = hmax;
    e.Qmax = qmax;
    for (int s = 0; s < 2; ++s) {
      e.nh[s] = (int)t->hl[s].size();
      e.nq[s] = (int)t->ql[s].size();
      e.D[s] = e.nh[s] * e.nq[s];
      e.S[s] = nel[s] + e.nq[s];
    }
    e.Dmax = std::max(1, std::max(e.D[0], e.D[1]));
    e.Smax = std::max(e.S[0], e.S[1]);
    e.nmax = m.nmax;
    int rc2;
    MsdEnergyTables& et = t->et;
    et.ncross = (int)xa.size();
    if (xa.empty()) {  // keep valid device pointers
      xa.push_back(0);
      xb.push_back(0);
      xc.push_back(0.0);
    }
    if ((rc2 = msd_upload(t, &et.hlist, hlist)) || (rc2 = msd_upload(t, &et.qlist, qlist)) ||
        (rc2 = msd_upload(t, &et.spos, spos)) || (rc2 = msd_upload(t, &et.xa, xa)) ||
        (rc2 = msd_upload(t, &et.xb, xb)) || (rc2 = msd_upload(t, &et.xc, xc)))
      return rc2;
  }
  // orbitals
  std::vector<double> cocc((size_t)2 * N * m.nmax, 0.0), cvirt((size_t)2 * N * m.ldv, 0.0);
  std::vector<double> cfull((size_t)2 * N * m.ldN, 0.0);
  for (int s = 0; s < 2; ++s)
    for (int p = 0; p < N; ++p) {
      for (int x = 0; x < N; ++x) cfull[((size_t)s * N + p) * m.ldN + x] = C[s][(size_t)p * N + x];
      for (int i = 0; i < nel[s]; ++i) cocc[((size_t)s * N + p) * m.nmax + i] = C[s][(size_t)p * N + i];
      for (int a = 0; a < m.nv[s]; ++a) cvirt[((size_t)s * N + p) * m.ldv + a] = C[s][(size_t)p * N + nel[s] + a];
    }
  int rc;
  MsdTables& tb = t->t;
  if ((rc = msd_upload(t, &tb.cocc, cocc)) || (rc = msd_upload(t, &tb.cvirt, cvirt)) ||
      (rc = msd_upload(t, &tb.cfull, cfull)) ||
      (rc = msd_upload(t, &tb.srank, srank)) || (rc = msd_upload(t, &tb.sorb, sorb)) ||
      (rc = msd_upload(t, &tb.saoff, saoff)) || (rc = msd_upload(t, &tb.crow, crow)) ||
      (rc = msd_upload(t, &tb.ccoef, ccoef)) || (rc = msd_upload(t, &tb.cstr, cstr)) ||
      (rc = msd_upload(t, &tb.tbeg, tbeg)) || (rc = msd_upload(t, &tb.trow, trow)) ||
      (rc = msd_upload(t, &tb.erow, erow)) || (rc = msd_upload(t, &tb.estr, estr)) ||
      (rc = msd_upload(t, &tb.eoff, eoff)))
    return rc;
  t->et.srank = tb.srank;
  t->et.saoff = tb.saoff;
  for (int s = 0; s < 2; ++s) t->C_host[s].assign(C[s], C[s] + (size_t)N * N);
  return AFQMC_OK;
}

int msd_workspace(afqmc_msd* t) {
  const MsdDims& m = t->m;
  const size_t W = (size_t)t->max_walkers;
  int rc;
  if ((rc = dalloc_t(t, &t->hh0, (size_t)2 * m.nmax * m.N))) return rc;
  if ((rc = dalloc_t(t, &t->theta, W * 4 * m.nmax * m.ldN))) return rc;
  if ((rc = dalloc_t(t, &t->logdet, W * 2))) return rc;
  if ((rc = dalloc_t(t, &t->yp, W * 4 * m.nmax * m.ldv))) return rc;
  if ((rc = dalloc_t(t, &t->sdet, W * m.nstr_tot))) return rc;
  if ((rc = dalloc_t(t, &t->sadj, W * m.nadj_tot))) return rc;
  if ((rc = dalloc_t(t, &t->tpart, W * m.ntask))) return rc;
  if ((rc = dalloc_t(t, &t->uw, W * m.nstr_tot))) return rc;
  if ((rc = dalloc_t(t, &t->rpart, W * msd_combine_blocks(m)))) return rc;
  if ((rc = dalloc_t(t, &t->ratio, W))) return rc;
  if ((rc = dalloc_t(t, &t->lpair, W * 2))) return rc;
  if ((rc = dalloc_t(t, &t->zt, W * 4 * m.nmax * m.ldN))) return rc;
  if ((rc = dalloc_t(t, &t->qp, W * 4 * m.N * m.ldq))) return rc;
  if ((rc = dalloc_t(t, &t->status, (size_t)1))) return rc;
  return AFQMC_OK;
}

int msd_check(const afqmc_msd* t, const afqmc_walkers* w, int nw) {
  if (!t) return fail(AFQMC_EINVAL, "null multi-determinant trial handle");
  if (nw < 0 || nw > t->max_walkers)
    return fail(AFQMC_EINVAL, "nw = %d outside [0, max_walkers = %d]", nw, t->max_walkers);
  if (nw == 0) return AFQMC_OK;
  if (!w) return fail(AFQMC_EINVAL, "null walkers");
  if (!w->phi_a || (t->m.nb > 0 && !w->phi_b)) return fail(AFQMC_EINVAL, "null walker array");
  return AFQMC_OK;
}

// reference theta and log det, then the string determinants and the overlap ratio
int msd_ratio(afqmc_msd* t, const afqmc_walkers* w, int nw, bool want_adj, hipStream_t s) {
  HIP_TRY(hipSetDevice(t->device));
  const double2* pb = (const double2*)(t->m.nb > 0 ? w->phi_b : w->phi_a);  // not read when nb = 0
  HIP_TRY((launch_gf<double>(t->d, nw, (const double2*)w->phi_a, pb, t->t.cocc, t->hh0, t->theta, t->logdet,
                             nullptr, t->status, s)));
  HIP_TRY(launch_msd_ratio(t->m, nw, t->t, t->theta, t->yp, t->sdet, t->sadj, t->tpart, t->uw, t->rpart,
                           t->ratio, want_adj, s));
  return AFQMC_OK;
}

// checks shared by the calls that combine the trial with a Hamiltonian
int msd_check_ham(const afqmc_msd* t, const afqmc_ham* h, int nw, int* nsplit, int* ldpk) {
  if (!h) return fail(AFQMC_EINVAL, "null Hamiltonian handle");
  if (h->d.N != t->m.N) return fail(AFQMC_EINVAL, "orbital counts differ (%d, %d)", h->d.N, t->m.N);
  if (nw > h->prm.max_walkers)
    return fail(AFQMC_EINVAL, "nw = %d above the Hamiltonian's max_walkers = %d", nw, h->prm.max_walkers);
  const int npk = t->m.N * (t->m.N + 1) / 2;
  // scratch: the Hamiltonian's VHS workspace, idle outside its own steps
  const size_t cap = (size_t)h->prm.max_walkers * h->d.N * h->d.ldV * h->tsize;
  if (h->prec == AFQMC_FP16X3) {
    // packed symmetric G in FP32 rows of ldhp (split in place), then one scale per row
    *ldpk = h->ldhp;
    *nsplit = 1;
    if (!h->lt_t_split || (size_t)2 * h->prm.max_walkers * (h->ldhp + 1) * sizeof(float) > cap)
      return fail(AFQMC_EUNSUPPORTED, "force-bias scratch does not fit the Hamiltonian's workspace");
    return AFQMC_OK;
  }
  *ldpk = (npk + 15) / 16 * 16;
  *nsplit = msd_fb_splits(nw > 0 ? nw : 1, t->m.N, h->d.K, h->d.ldK, *ldpk, h->tsize, cap);
  if (*nsplit < 1) return fail(AFQMC_EUNSUPPORTED, "force-bias scratch does not fit the Hamiltonian's workspace");
  return AFQMC_OK;
}

// vbias of the walkers w for the trial t into `vbias` (scratch: h's VHS workspace)
int msd_vbias(afqmc_msd* t, afqmc_ham* h, const afqmc_walkers* w, int nw, int nsplit, int ldpk, double2* vbias,
              hipStream_t s) {
  int rc;
  if ((rc = msd_ratio(t, w, nw, true, s))) return rc;
  HIP_TRY(launch_msd_q(t->m, nw, t->t, t->yp, t->sadj, t->uw, t->ratio, t->zt, t->qp, s));
  if (h->prec == AFQMC_FP64) {
    HIP_TRY(launch_msd_force_bias<double>(t->m, nw, t->theta, t->qp, (const double*)h->LT, h->d.K, h->d.ldK, ldpk,
                                          nsplit, h->vhs, vbias, s));
  } else if (h->prec == AFQMC_FP16X3) {
    float* gs = (float*)h->vhs;                        // [nw][2][ldhp]
    float* gs_unscale = gs + (size_t)2 * nw * h->ldhp;  // [2 nw]
    HIP_TRY(launch_msd_gsym_f32(t->m, nw, t->theta, t->qp, h->ldhp, gs, s));
    HIP_TRY(launch_msd_fb_split(h->split, nw, h->d.K, h->d.Npk, h->ldhp, gs, gs_unscale, h->lt_t_split,
                                h->lt_t_unscale, h->fb_part, vbias, s));
  } else {
    HIP_TRY(launch_msd_force_bias<float>(t->m, nw, t->theta, t->qp, (const float*)h->LT, h->d.K, h->d.ldK, ldpk,
                                         nsplit, h->vhs, vbias, s));
  }
  return AFQMC_OK;
}

}  // namespace

extern "C" {

int afqmc_msd_create(int N, int na, int nb, const double* host_C_a, const double* host_C_b, int ndet,
                     const double* host_coeff, const int* host_rank, const int* host_orbs, int max_walkers,
                     void* stream, afqmc_msd** out) {
  if (!out) return fail(AFQMC_EINVAL, "null output handle pointer");
  *out = nullptr;
  if (N < 1 || na < 1 || nb < 0 || na > N || nb > N)
    return fail(AFQMC_EINVAL, "bad sizes N=%d na=%d nb=%d", N, na, nb);
  if (na > 45 || nb > 45)
    return fail(AFQMC_EUNSUPPORTED, "at most 45 electrons per spin are supported (got %d, %d)", na, nb);
  if (ndet < 1 || ndet > (1 << 28)) return fail(AFQMC_EINVAL, "ndet = %d outside [1, 2^28]", ndet);
  if (max_walkers < 1) return fail(AFQMC_EINVAL, "max_walkers must be >= 1");
  if (!host_C_a || (nb > 0 && !host_C_b) || !host_coeff || !host_rank || !host_orbs)
    return fail(AFQMC_EINVAL, "null input pointer");
  {
    const int rv = msd_validate(N, na, nb, ndet, host_rank, host_orbs);
    if (rv) return rv;
  }
  afqmc_msd* t = new afqmc_msd();
  int rc = AFQMC_OK;
  if (hipGetDevice(&t->device) != hipSuccess) rc = fail(AFQMC_EHIP, "hipGetDevice failed");
  t->max_walkers = max_walkers;
  t->ndet = ndet;
  MsdDims& m = t->m;
  m.N = N;
  m.na = na;
  m.nb = nb;
  m.nmax = na > nb ? na : nb;
  m.ldN = (N + 15) / 16 * 16;
  m.nv[0] = N - na;
  m.nv[1] = N - nb;
  m.ldv = ((m.nv[0] > m.nv[1] ? m.nv[0] : m.nv[1]) + 3) / 4 * 4;
  if (m.ldv == 0) m.ldv = 4;
  m.ldq = (m.nmax + 1) / 2 * 2;
  t->d.N = N;
  t->d.na = na;
  t->d.nb = nb;
  t->d.nmax = m.nmax;
  t->d.ldN = m.ldN;
  const double* C[2] = {host_C_a, nb > 0 ? host_C_b : host_C_a};
  if (!rc && set_kernel_attributes(t->d) != hipSuccess) rc = fail(AFQMC_EHIP, "kernel attribute setup failed");
  if (!rc) rc = msd_build(t, C, host_coeff, host_rank, host_orbs);
  if (!rc) rc = msd_workspace(t);
  if (!rc && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) rc = fail(AFQMC_EHIP, "stream sync failed");
  if (rc) {
    msd_free(t);
    delete t;
    return rc;
  }
  *out = t;
  return AFQMC_OK;
}

int afqmc_msd_overlap(afqmc_msd* t, const afqmc_walkers* w, int nw, void* log_ovlp, void* stream) {
  int rc = msd_check(t, w, nw);
  if (rc || nw == 0) return rc;
  if (!log_ovlp) return fail(AFQMC_EINVAL, "null log_ovlp");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = msd_ratio(t, w, nw, false, s))) return rc;
  HIP_TRY(launch_msd_overlap_store(nw, t->logdet, t->ratio, (double2*)log_ovlp, t->status, s));
  return AFQMC_OK;
}

int afqmc_msd_green_function(afqmc_msd* t, const afqmc_walkers* w, int nw, void* G, void* stream) {
  int rc = msd_check(t, w, nw);
  if (rc || nw == 0) return rc;
  if (!G) return fail(AFQMC_EINVAL, "null G");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = msd_ratio(t, w, nw, true, s))) return rc;
  HIP_TRY(launch_msd_green(t->m, nw, t->t, t->theta, t->yp, t->sadj, t->uw, t->ratio, t->zt, t->qp, (double2*)G,
                           s));
  return AFQMC_OK;
}

int afqmc_msd_force_bias(afqmc_msd* t, afqmc_ham* h, const afqmc_walkers* w, int nw, void* vbias, void* stream) {
  int rc = msd_check(t, w, nw);
  if (rc) return rc;
  int nsplit, ldpk;
  if ((rc = msd_check_ham(t, h, nw, &nsplit, &ldpk))) return rc;
  if (nw == 0) return AFQMC_OK;
  if (!vbias) return fail(AFQMC_EINVAL, "null vbias");
  return msd_vbias(t, h, w, nw, nsplit, ldpk, (double2*)vbias, (hipStream_t)stream);
}

int afqmc_msd_propagate(afqmc_msd* t, afqmc_ham* h, afqmc_walkers* w, int nw, const double* fields, void* stream) {
  int rc = msd_check(t, w, nw);
  if (rc) return rc;
  int nsplit, ldpk;
  if ((rc = msd_check_ham(t, h, nw, &nsplit, &ldpk))) return rc;
  if (h->d.na != t->m.na || h->d.nb != t->m.nb)
    return fail(AFQMC_EINVAL, "electron counts differ (%d, %d) vs (%d, %d)", h->d.na, h->d.nb, t->m.na, t->m.nb);
  if (nw == 0) return AFQMC_OK;
  if (!fields) return fail(AFQMC_EINVAL, "null fields");
  if (!w->log_ovlp || !w->log_w) return fail(AFQMC_EINVAL, "null walker array");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = msd_vbias(t, h, w, nw, nsplit, ldpk, h->vbias, s))) return rc;
  StepIO io;
  io.fields = fields;
  if (h->prec == AFQMC_FP64)
    rc = seq_propagate_core<double>(h, w, nw, io, s);
  else
    rc = seq_propagate_core<float>(h, w, nw, io, s);
  if (rc) return rc;
  if ((rc = msd_ratio(t, w, nw, false, s))) return rc;
  HIP_TRY(launch_msd_overlap_pairs(nw, t->logdet, t->ratio, t->lpair, t->status, s));
  HIP_TRY(launch_weight(nw, t->lpair, nullptr, h->a, (double2*)w->log_ovlp, w->log_w, h->cst, h->status, s));
  h->c_valid = false;
  return AFQMC_OK;
}


int afqmc_msd_set_hamiltonian(afqmc_msd* t, int K, const double* host_h1, const double* host_chol, void* stream) {
  if (!t) return fail(AFQMC_EINVAL, "null trial handle");
  if (K < 1) return fail(AFQMC_EINVAL, "K = %d must be >= 1", K);
  if (!host_h1 || !host_chol) return fail(AFQMC_EINVAL, "null h1 or Cholesky vectors");
  if (t->has_ham) return fail(AFQMC_EINVAL, "the trial already has a Hamiltonian");
  MsdEnergyDims& e = t->ed;
  const MsdDims& m = t->m;
  if (e.Dmax > 1024)
    return fail(AFQMC_EUNSUPPORTED,
                "the local energy needs at most 1024 (active particle, active hole) pairs per spin; the expansion "
                "excites %d x %d (alpha) and %d x %d (beta)",
                e.nq[0], e.nh[0], e.nq[1], e.nh[1]);
  e.K = K;
  e.ldL = m.ldN;
  e.ldG = round_up(K, 8);
  e.gchunk = 8;
  e.nchunk = ceil_div(K + 1, e.gchunk);
  const size_t lds = msd_energy_rp_lds(e);
  if (lds > 160 * 1024)
    return fail(AFQMC_EUNSUPPORTED, "the active space is too large for the local energy (%zu bytes of LDS)", lds);
  // walkers per pass: the workspace of one walker, within about 16 GB (64 walkers at most:
  // 209 -> 196 ms per call at 10^4 determinants for 512 walkers of 290 orbitals against 32)
  const size_t K1 = (size_t)K + 1;
  const size_t per = 2 * K1 * 2 * e.Smax * m.nmax * sizeof(double) + 2 * (size_t)e.Dmax * e.ldG * 16 +
                     4 * (size_t)e.nchunk * e.Dmax * 16 + 3 * (size_t)e.Dmax * e.Dmax * 16 + 8 * K1 * 16;
  e.Wc = (int)std::max<size_t>(1, std::min<size_t>({(size_t)64, (size_t)t->max_walkers, (size_t(16) << 30) / per}));
  int rc;
  HIP_TRY(hipSetDevice(t->device));
  HIP_TRY(msd_energy_set_attributes(lds));
  hipStream_t s = (hipStream_t)stream;
  const int N = m.N;
  const size_t NN = (size_t)N * N;
  {
    // rotated rows C_S^T L_g (and C_S^T h1 as block K), C_S = [C_occ | C_virt[:, Q]]
    TempAllocs tmp;
    double *dL = nullptr, *cs = nullptr, *out = nullptr;
    HIP_TRY(tmp.get(&dL, K1 * NN * sizeof(double)));
    HIP_TRY(hipMemcpy(dL, host_chol, (size_t)K * NN * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dL + (size_t)K * NN, host_h1, NN * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(tmp.get(&cs, NN * sizeof(double)));
    HIP_TRY(tmp.get(&out, K1 * N * e.Smax * sizeof(double)));
    const int nel[2] = {m.na, m.nb};
    for (int sp = 0; sp < 2; ++sp) {
      const int S = e.S[sp];
      double* lr = nullptr;
      if ((rc = dalloc_t(t, &lr, K1 * (size_t)std::max(S, 1) * e.ldL))) return rc;
      t->et.lr[sp] = lr;
      if (nel[sp] == 0) continue;
      std::vector<double> h((size_t)N * S);
      for (int p = 0; p < N; ++p) {
        for (int i = 0; i < nel[sp]; ++i) h[(size_t)p * S + i] = t->C_host[sp][(size_t)p * N + i];
        for (int q = 0; q < e.nq[sp]; ++q)
          h[(size_t)p * S + nel[sp] + q] = t->C_host[sp][(size_t)p * N + nel[sp] + t->ql[sp][q]];
      }
      HIP_TRY(hipMemcpy(cs, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
      // out[(g, p)][r] = sum_q L_g[p][q] C_S[q][r] = (C_S^T L_g)[r][p] (L_g symmetric)
      HIP_TRY(setup_gemm((int)(K1 * N), S, N, 0, dL, N, cs, S, out, S, nullptr, 1, s));
      HIP_TRY(msd_lr_pack((long)K1 * N, N, S, e.ldL, out, lr, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
  }
  // workspace for Wc walkers
  const size_t Wc = (size_t)e.Wc;
  MsdEnergyWork& w = t->ew;
  if ((rc = dalloc_t(t, &w.u, Wc * 2 * K1 * 2 * e.Smax * m.nmax)) || (rc = dalloc_t(t, &w.rbuf, Wc * 2 * e.Dmax * e.ldG)) ||
      (rc = dalloc_t(t, &w.jpart, Wc * 2 * e.nchunk * e.Dmax)) ||
      (rc = dalloc_t(t, &w.ppart, Wc * 2 * e.nchunk * e.Dmax)) || (rc = dalloc_t(t, &w.tt, Wc * 2 * K1)) ||
      (rc = dalloc_t(t, &w.kt, Wc * 2 * (size_t)K)) || (rc = dalloc_t(t, &w.r1, Wc * 2 * e.Dmax)) ||
      (rc = dalloc_t(t, &w.vj, Wc * 2 * e.Dmax)) || (rc = dalloc_t(t, &w.vp, Wc * 2 * e.Dmax)) ||
      (rc = dalloc_t(t, &w.sc, Wc * 4)) || (rc = dalloc_t(t, &w.G, Wc * 3 * e.Dmax * e.Dmax)) ||
      (rc = dalloc_t(t, &w.cpart, Wc * MSD_CT_SPLITS * 3)))
    return rc;
  t->has_ham = true;
  return AFQMC_OK;
}

int afqmc_msd_local_energy(afqmc_msd* t, const afqmc_walkers* w, int nw, void* e, void* stream) {
  int rc;
  if ((rc = msd_check(t, w, nw)) || nw == 0) return rc;
  if (!e) return fail(AFQMC_EINVAL, "null energy output");
  if (!t->has_ham) return fail(AFQMC_EINVAL, "the trial has no Hamiltonian (afqmc_msd_set_hamiltonian)");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = msd_ratio(t, w, nw, true, s))) return rc;
  for (int z0 = 0; z0 < nw; z0 += t->ed.Wc) {
    const int nz = std::min(t->ed.Wc, nw - z0);
    HIP_TRY(launch_msd_energy_chunk(t->m, t->ed, t->et, z0, nz, t->theta, t->yp, t->sdet, t->sadj, t->uw, t->ratio,
                                    t->ew, (double2*)e, s));
  }
  return AFQMC_OK;
}

int afqmc_msd_get_strings(afqmc_msd* t, int* nstr_a, int* nstr_b) {
  if (!t) return fail(AFQMC_EINVAL, "null multi-determinant trial handle");
  if (nstr_a) *nstr_a = t->m.nstr[0];
  if (nstr_b) *nstr_b = t->m.nstr[1];
  return AFQMC_OK;
}

int afqmc_msd_get_status(afqmc_msd* t, void* stream, int* out) {
  if (!t || !out) return fail(AFQMC_EINVAL, "null argument");
  HIP_TRY(hipSetDevice(t->device));
  hipStream_t s = (hipStream_t)stream;
  int v = 0;
  HIP_TRY(hipMemcpyAsync(&v, t->status, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int zero = 0;
  HIP_TRY(hipMemcpyAsync(t->status, &zero, sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  *out = v;
  return AFQMC_OK;
}

void afqmc_msd_destroy(afqmc_msd* t) {
  if (!t) return;
  (void)hipSetDevice(t->device);
  (void)hipDeviceSynchronize();
  msd_free(t);
  delete t;
}

}  // extern "C"

// ===========================================================================
// uneven multi-system batch
// ===========================================================================

struct afqmc_batch {
  std::vector<afqmc_ham*> hams;
  std::vector<afqmc_walkers> ws;
  std::vector<int> nw;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
  hipStream_t origin = nullptr;
  int* ctr = nullptr;
  int use_graph = 1;
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // what the current graph was captured for
  std::vector<const double*> g_fields;
  std::vector<void*> g_e;
  std::vector<int> g_tune;  // tune_gen of each Hamiltonian
  int g_qr = -1;
};

namespace {

void batch_drop_graph(afqmc_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->g_qr = -1;
}

int batch_step_one(afqmc_batch* b, size_t i, const StepIO& io, int do_qr, hipStream_t s) {
  afqmc_ham* h = b->hams[i];
  afqmc_walkers* w = &b->ws[i];
  return h->prec != AFQMC_FP64 ? seq_step<float>(h, w, b->nw[i], io, do_qr, AFQMC_STEP_REUSE, s)
                               : seq_step<double>(h, w, b->nw[i], io, do_qr, AFQMC_STEP_REUSE, s);
}

// theta and vbias of the current walkers of every system (the captured
// step starts from them)
int batch_prime(afqmc_batch* b, hipStream_t s) {
  int rc;
  for (size_t i = 0; i < b->hams.size(); ++i) {
    afqmc_ham* h = b->hams[i];
    afqmc_walkers* w = &b->ws[i];
    if (h->prec != AFQMC_FP64) {
      if ((rc = seq_theta<float>(h, w, b->nw[i], false, s))) return rc;
      if ((rc = seq_force_bias<float>(h, b->nw[i], h->vbias, s))) return rc;
    } else {
      if ((rc = seq_theta<double>(h, w, b->nw[i], false, s))) return rc;
      if ((rc = seq_force_bias<double>(h, b->nw[i], h->vbias, s))) return rc;
    }
    h->c_valid = true;
    h->c_phi_a = w->phi_a;
    h->c_phi_b = w->phi_b;
    h->c_nw = b->nw[i];
  }
  return AFQMC_OK;
}

StepIO batch_io(const afqmc_batch* b, size_t i, const double* const* fields, void* const* e,
                const int* ctr, int step) {
  const afqmc_ham* h = b->hams[i];
  StepIO io;
  const long fstep = (long)b->nw[i] * h->d.K, estep = (long)b->nw[i] * 3;
  io.ctr = ctr;
  io.fstep = fstep;
  io.estep = estep;
  io.fields = fields[i] + (ctr ? 0 : (size_t)step * fstep);
  double2* eb = (e && e[i]) ? (double2*)e[i] : nullptr;
  io.e = eb ? eb + (ctr ? 0 : (size_t)step * estep) : nullptr;
  return io;
}

int batch_capture(afqmc_batch* b, const double* const* fields, void* const* e, int do_qr) {
  batch_drop_graph(b);
  HIP_TRY(hipStreamBeginCapture(b->origin, hipStreamCaptureModeThreadLocal));
  int rc = AFQMC_OK;
  hipError_t he = hipEventRecord(b->fork, b->origin);
  for (size_t i = 0; i < b->hams.size() && he == hipSuccess && rc == AFQMC_OK; ++i) {
    he = hipStreamWaitEvent(b->streams[i], b->fork, 0);
    if (he != hipSuccess) break;
    b->hams[i]->capturing = true;
    rc = batch_step_one(b, i, batch_io(b, i, fields, e, b->ctr, 0), do_qr, b->streams[i]);
    b->hams[i]->capturing = false;
    if (rc) break;
    he = hipEventRecord(b->joins[i], b->streams[i]);
    if (he == hipSuccess) he = hipStreamWaitEvent(b->origin, b->joins[i], 0);
  }
  if (he == hipSuccess && rc == AFQMC_OK) he = launch_counter_advance(b->ctr, b->origin);
  hipGraph_t g = nullptr;
  const hipError_t he2 = hipStreamEndCapture(b->origin, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (he != hipSuccess || he2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(AFQMC_EHIP, "graph capture failed: %s",
                hipGetErrorString(he != hipSuccess ? he : he2));
  }
  b->graph = g;
  HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->g_fields.assign(fields, fields + b->hams.size());
  b->g_e.assign(b->hams.size(), nullptr);
  if (e)
    for (size_t i = 0; i < b->hams.size(); ++i) b->g_e[i] = e[i];
  b->g_qr = do_qr;
  b->g_tune.resize(b->hams.size());
  for (size_t i = 0; i < b->hams.size(); ++i) b->g_tune[i] = b->hams[i]->tune_gen;
  return AFQMC_OK;
}

std::string tune_key(const afqmc_ham* h, int nw) {
  hipDeviceProp_t prop;
  std::string dev = "gfx";
  if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) dev = prop.gcnArchName;
  std::ostringstream k;
  k << "tiles:" << dev << ":N" << h->d.N << ":na" << h->d.na << ":nb" << h->d.nb << ":K" << h->d.K << ":W" << nw
    << ":p" << h->prec << ":x" << h->ex_algo;
  return k.str();
}

// Tile shapes the handle's kernels offer: the split pair exchange and the
// split VHS build come in a wide and a narrow walker tile; every other
// exchange and VHS kernel has one shape.
bool ex_tiles_offered(const afqmc_ham* h) { return h->split != SPLIT_NONE && h->ex_algo == AFQMC_EXCHANGE_PAIR; }
bool vhs_tiles_offered(const afqmc_ham* h) { return vhs_split(h); }

void tile_shapes(const afqmc_ham* h, int ex_tile, int vhs_tile, afqmc_tuning* t) {
  if (ex_tiles_offered(h)) {  // the split pair exchange
    t->ex_tile_m = 128;
    t->ex_tile_n = ex_tile == SPLIT_TILE_NARROW ? 64 : 128;
  } else if (h->split != SPLIT_NONE) {  // the split direct exchange
    t->ex_tile_m = 160;
    t->ex_tile_n = 160;
  } else {
    t->ex_tile_m = 192;
    t->ex_tile_n = 160;
  }
  if (vhs_split(h)) {
    t->vhs_tile_m = vhs_tile == SPLIT_TILE_NARROW ? 64 : 128;
    t->vhs_tile_n = 128;
  } else {
    t->vhs_tile_m = 64;
    t->vhs_tile_n = 64;
  }
}

// the tile choices of a shape, or false if the handle does not offer it
bool tiles_of_shapes(const afqmc_ham* h, const afqmc_tuning& want, int* ex_tile, int* vhs_tile) {
  for (int et = 0; et < 2; ++et)
    for (int vt = 0; vt < 2; ++vt) {
      if ((et && !ex_tiles_offered(h)) || (vt && !vhs_tiles_offered(h))) continue;
      afqmc_tuning t;
      tile_shapes(h, et, vt, &t);
      if (t.ex_tile_m == want.ex_tile_m && t.ex_tile_n == want.ex_tile_n && t.vhs_tile_m == want.vhs_tile_m &&
          t.vhs_tile_n == want.vhs_tile_n) {
        *ex_tile = et;
        *vhs_tile = vt;
        return true;
      }
    }
  return false;
}

// one cache line: "<key> ex=<m>x<n>/<group> vhs=<m>x<n>"
std::string tune_line(const afqmc_ham* h) {
  afqmc_tuning t;
  tile_shapes(h, h->ex_tile, h->vhs_tile, &t);
  std::ostringstream o;
  o << "ex=" << t.ex_tile_m << "x" << t.ex_tile_n << "/" << h->ex_gs << " vhs=" << t.vhs_tile_m << "x"
    << t.vhs_tile_n;
  return o.str();
}

bool tune_parse(const afqmc_ham* h, const std::string& v, int* ex_tile, int* ex_gs, int* vhs_tile) {
  afqmc_tuning t;
  int g = 0;
  if (std::sscanf(v.c_str(), "ex=%dx%d/%d vhs=%dx%d", &t.ex_tile_m, &t.ex_tile_n, &g, &t.vhs_tile_m,
                  &t.vhs_tile_n) != 5 ||
      g < 0)
    return false;
  if (!tiles_of_shapes(h, t, ex_tile, vhs_tile)) return false;
  *ex_gs = g;
  return true;
}

}  // namespace

extern "C" {

int afqmc_batch_create(afqmc_ham* const* hams, const afqmc_walkers* ws, const int* nw, int nsys,
                       const afqmc_batch_opts* opts, afqmc_batch** out) {
  if (!out) return fail(AFQMC_EINVAL, "null output batch pointer");
  *out = nullptr;
  if (!hams || !ws || !nw || nsys < 1) return fail(AFQMC_EINVAL, "empty or null batch description");
  for (int i = 0; i < nsys; ++i) {
    if (!hams[i]) return fail(AFQMC_EINVAL, "null Hamiltonian %d", i);
    if (hams[i]->device != hams[0]->device) return fail(AFQMC_EINVAL, "systems on different devices");
    if (nw[i] < 1) return fail(AFQMC_EINVAL, "system %d: nw must be >= 1", i);
    int rc = check_walkers(hams[i], &ws[i], nw[i]);
    if (rc) return rc;
    for (int j = 0; j < i; ++j)
      if (hams[j] == hams[i]) return fail(AFQMC_EINVAL, "Hamiltonian %d appears twice (its workspace is per handle)", i);
  }
  afqmc_batch* b = new afqmc_batch();
  b->device = hams[0]->device;
  b->use_graph = opts ? opts->use_graph : 1;
  b->hams.assign(hams, hams + nsys);
  b->ws.assign(ws, ws + nsys);
  b->nw.assign(nw, nw + nsys);
  auto cleanup = [b]() { afqmc_batch_destroy(b); };
  if (hipSetDevice(b->device) != hipSuccess) { cleanup(); return fail(AFQMC_EHIP, "hipSetDevice failed"); }
  hipError_t e = hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int i = 0; i < nsys && e == hipSuccess; ++i) {
    hipStream_t s;
    hipEvent_t ev;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) break;
    b->streams.push_back(s);
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) break;
    b->joins.push_back(ev);
  }
  if (e == hipSuccess) e = hipMalloc(&b->ctr, sizeof(int));
  if (e == hipSuccess) e = hipMemset(b->ctr, 0, sizeof(int));
  if (e != hipSuccess) {
    cleanup();
    return fail(AFQMC_EHIP, "batch setup failed: %s", hipGetErrorString(e));
  }
  *out = b;
  return AFQMC_OK;
}

int afqmc_batch_step(afqmc_batch* b, const double* const* fields, void* const* e, int nsteps,
                     int do_qr, void* stream) {
  if (!b) return fail(AFQMC_EINVAL, "null batch");
  if (nsteps < 0) return fail(AFQMC_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return AFQMC_OK;
  if (!fields) return fail(AFQMC_EINVAL, "null fields array");
  for (size_t i = 0; i < b->hams.size(); ++i)
    if (!fields[i]) return fail(AFQMC_EINVAL, "null fields of system %zu", i);
  HIP_TRY(hipSetDevice(b->device));
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if ((rc = batch_prime(b, s))) return rc;
  if (!b->use_graph) {
    // eager: each step forks the systems onto their streams and joins them
    for (int k = 0; k < nsteps; ++k) {
      HIP_TRY(hipEventRecord(b->fork, s));
      for (size_t i = 0; i < b->hams.size(); ++i) {
        HIP_TRY(hipStreamWaitEvent(b->streams[i], b->fork, 0));
        if ((rc = batch_step_one(b, i, batch_io(b, i, fields, e, nullptr, k), do_qr, b->streams[i])))
          return rc;
        HIP_TRY(hipEventRecord(b->joins[i], b->streams[i]));
        HIP_TRY(hipStreamWaitEvent(s, b->joins[i], 0));
      }
    }
    return AFQMC_OK;
  }
  bool same = b->exec && b->g_qr == do_qr;
  for (size_t i = 0; same && i < b->hams.size(); ++i) {
    void* ei = (e && e[i]) ? e[i] : nullptr;
    same = b->g_fields[i] == fields[i] && b->g_e[i] == ei && b->g_tune[i] == b->hams[i]->tune_gen;
  }
  if (!same) {
    HIP_TRY(hipStreamSynchronize(s));
    if ((rc = batch_capture(b, fields, e, do_qr))) return rc;
  }
  HIP_TRY(launch_counter_set(b->ctr, 0, s));
  for (int k = 0; k < nsteps; ++k) HIP_TRY(hipGraphLaunch(b->exec, s));
  return AFQMC_OK;
}

int afqmc_autotune(afqmc_batch* b, const char* cache_path) {
  if (!b) return fail(AFQMC_EINVAL, "null batch");
  HIP_TRY(hipSetDevice(b->device));
  std::map<std::string, std::string> cache;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      const size_t sp = line.find(' ');
      if (sp != std::string::npos) cache[line.substr(0, sp)] = line.substr(sp + 1);
    }
  }
  static const int cand[] = {1, 2, 4, 8, 16, 32};
  hipEvent_t t0, t1;
  HIP_TRY(hipEventCreate(&t0));
  HIP_TRY(hipEventCreate(&t1));
  std::vector<std::pair<std::string, std::string>> fresh;
  int rc = AFQMC_OK;
  // mean of launches 2 and 3 of f (the first warms up), in ms
  auto time3 = [&](hipStream_t s, auto&& f, float* out) -> int {
    float tot = 0.f;
    for (int rep = 0; rep < 3; ++rep) {
      HIP_TRY(hipEventRecord(t0, s));
      HIP_TRY(f());
      HIP_TRY(hipEventRecord(t1, s));
      HIP_TRY(hipEventSynchronize(t1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
      if (rep > 0) tot += ms;
    }
    *out = tot / 2;
    return AFQMC_OK;
  };
  for (size_t i = 0; i < b->hams.size() && rc == AFQMC_OK; ++i) {
    afqmc_ham* h = b->hams[i];
    const int nw = b->nw[i];
    const std::string key = tune_key(h, nw);
    auto it = cache.find(key);
    if (it != cache.end() && tune_parse(h, it->second, &h->ex_tile, &h->ex_gs, &h->vhs_tile)) {
      ++h->tune_gen;
      continue;
    }
    hipStream_t s = b->streams[i];
    // theta of the current walkers, then the exchange alone per candidate
    rc = h->prec != AFQMC_FP64 ? seq_theta<float>(h, &b->ws[i], nw, false, s)
                               : seq_theta<double>(h, &b->ws[i], nw, false, s);
    if (rc) break;
    const StepDims& d = h->d;
    if (h->split != SPLIT_NONE)
      HIP_TRY(launch_split_rows_mode(h->split, (long)nw * 4 * d.nmax, d.N, (const float*)h->theta, d.ldN,
                                     h->th_split, d.ldh, h->th_unscale, s));
    float best = 1e30f;
    int best_gs = 0, best_tile = SPLIT_TILE_WIDE;
    for (int tile = 0; tile < (ex_tiles_offered(h) ? 2 : 1) && !rc; ++tile)
      for (int gs : cand) {
        float ms = 0.f;
        rc = time3(s, [&]() -> hipError_t {
          int ntg = 0;
          for (int sp = 0; sp < 2; ++sp) {
            const hipError_t e = launch_exchange_spin(h, nw, sp, &ntg, s, gs, tile);
            if (e != hipSuccess) return e;
          }
          return hipSuccess;
        }, &ms);
        if (rc) break;
        if (ms < best) {
          best = ms;
          best_gs = gs;
          best_tile = tile;
        }
      }
    if (rc) break;
    h->ex_gs = best_gs;
    h->ex_tile = best_tile;
    // the VHS build alone per walker tile, on the current shifted fields
    // (their values do not change the time; the next step rebuilds VHS)
    h->vhs_tile = SPLIT_TILE_WIDE;
    if (vhs_tiles_offered(h)) {
      best = 1e30f;
      for (int tile = 0; tile < 2 && !rc; ++tile) {
        float ms = 0.f;
        rc = time3(s, [&]() -> hipError_t {
          return launch_vhs_split(h->split, d, nw, h->xs_split, h->xs_unscale, h->lt_split, h->lt_unscale, h->vblk,
                                  h->nvblk, (float*)h->vhs, h->tmax + h->prm.max_walkers, h->prop_fused, h->sdt, s,
                                  tile);
        }, &ms);
        if (!rc && ms < best) {
          best = ms;
          h->vhs_tile = tile;
        }
      }
      if (rc) break;
    }
    ++h->tune_gen;
    fresh.emplace_back(key, tune_line(h));
    h->c_valid = false;  // theta was recomputed outside a step
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (rc) return rc;
  if (cache_path && !fresh.empty()) {
    std::ofstream outf(cache_path, std::ios::app);
    for (auto& kv : fresh) outf << kv.first << " " << kv.second << "\n";
  }
  batch_drop_graph(b);  // tile choices are baked into a captured graph
  return AFQMC_OK;
}

int afqmc_get_tuning(const afqmc_ham* h, afqmc_tuning* out) {
  if (!h || !out) return fail(AFQMC_EINVAL, "null argument");
  tile_shapes(h, h->ex_tile, h->vhs_tile, out);
  out->ex_group = h->ex_gs;
  return AFQMC_OK;
}

int afqmc_set_tuning(afqmc_ham* h, const afqmc_tuning* t) {
  if (!h || !t) return fail(AFQMC_EINVAL, "null argument");
  if (t->ex_group < 0 || t->ex_group > 1024) return fail(AFQMC_EINVAL, "ex_group = %d outside [0, 1024]", t->ex_group);
  int et = 0, vt = 0;
  if (!tiles_of_shapes(h, *t, &et, &vt))
    return fail(AFQMC_EUNSUPPORTED, "tile shapes exchange %dx%d, VHS %dx%d are not offered by this Hamiltonian",
                t->ex_tile_m, t->ex_tile_n, t->vhs_tile_m, t->vhs_tile_n);
  h->ex_tile = et;
  h->vhs_tile = vt;
  h->ex_gs = t->ex_group;
  ++h->tune_gen;  // a batch that captured the old choices recaptures
  return AFQMC_OK;
}

void afqmc_batch_destroy(afqmc_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  batch_drop_graph(b);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->joins) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->origin) (void)hipStreamDestroy(b->origin);
  if (b->ctr) (void)hipFree(b->ctr);
  delete b;
}

}  // extern "C"
