"""Plain FP64 CPU oracle of the phaseless-AFQMC walker step.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The product
path (the HIP library and its binding) never calls it, and it shares no
code with that path.

What it computes follows arXiv 2209.04015 (ipie):

* Hamiltonian and its Cholesky form: Sec. II.B, Eq. (Habinitio) and the
  factorisation (pr|qs) = sum_a L^a_pr L^a_qs written under it.
* Propagator, importance function, overlap ratio, optimal force bias,
  phaseless projection and weight update: Sec. II.B, Eqs. (Bx), (import),
  (ovl), the force-bias definition, (ph), (theta) and the two update
  equations that close the section.
* Overlap: Sec. III.A, the single-determinant overlap det(C_psi0^dagger C_phi).
* Green's function, half-rotated Cholesky vectors and force bias:
  Sec. III.B, Eqs. (fb), (gf), (halfgf), (rfb).
* Local energy (one-body, Coulomb, exchange): Sec. III.C, the E_L
  definition, the exchange formula and the T intermediate.
* Multi-determinant trial: Sec. III.A (the expansion and Eq. msdovlp) and
  the MSD Green's function of Sec. III.B, each taken by its definition, a
  sum over determinants (R23, R24); the generalised Wick's theorem that the
  paper uses to evaluate them is not used here.  The phaseless step under
  that trial (Sec. II.B) takes its force bias and overlap from them.

Readings where the paper is silent:

* R1  The one-body operator inside B(x): H is rewritten as
      sum h'_pq a+_p a_q + 1/2 sum_g v_g^2 with v_g = sum L_g,pq a+_p a_q and
      h' = h1 - 1/2 sum_g L_g L_g (exact for real symmetric L_g).
* R2  Symmetric Trotter split B = e^{-dt h'/2} e^{VHS} e^{-dt h'/2}, with the
      scalar e^{-dt mu/2} factored out of each half step: P = e^{-dt (h'-mu)/2}.
* R3  Weights are kept as log w.  The per-step constant
      -dt (mu (n_a + n_b) - E_T) (mu factored out of P, E_T the energy
      shift) is added to every walker.
* R4  v' = i v (Hubbard-Stratonovich of e^{-dt v^2/2}); vbias = sum G L (Eq. fb);
      xbar = -i sqrt(dt) vbias; VHS = i sqrt(dt) sum_g (x_g - xbar_g) L_g.
* R5  No cap on the force bias.
* R6  exp(VHS) is the Taylor series truncated after the order-6 term.
* R7  Determinants through LU with partial pivoting, kept as complex logs.
* R8  The phase is theta = arg(O_z) of the overlap ratio alone.
* R9  QR re-orthogonalisation: phi = Q R, phi <- Q D with D = diag(R_ii/|R_ii|);
      log overlap -= sum ln |R_ii|.
* R10 E1 = sum_s tr(hh^s theta^s); EJ = 1/2 sum_g (sum_s tr T^s_g)^2;
      EK = -1/2 sum_s sum_g tr(T^s_g T^s_g); no nuclear term.
* R11 G_pq = <a+_p a_q> = (phi S^-1 PhiT^T)_qp with S = PhiT^T phi.
* R17 Population control (named in Sec. I, no algorithm given) is a comb:
      with weights w_z = exp(log w_z) (0 for a non-finite log w), inclusive
      cumulative sums C_z and total W_tot, the nw teeth sit at
      t_k = (k + u) W_tot / nw for a given u in [0, 1); tooth k selects the
      first walker z with C_z > t_k (a tooth past the last sum, possible
      only through rounding, selects the last live walker).  Afterwards
      every walker has weight W_tot / nw (the total is kept).  Slots: a
      walker with at least one copy keeps its slot; the extra copies, in
      increasing walker order, fill the slots of the walkers with no copy,
      in increasing slot order.  With no live walker nothing changes.
* R18 Global energy (Sec. III.C): E = sum_z w_z E_L^z / sum_z w_z with the
      complex E_L = E1 + EJ + EK and w_z as in R17.
* R20 Mixed S^2 (Sec. IV.B): <Psi_T|S^2|phi>/<Psi_T|phi> =
      nb + Ms (Ms + 1) - sum_pq G^a_pq G^b_qp, Ms = (na - nb)/2.  The sum is
      the trace of the product G^a G^b, as Wick's theorem gives for S_- S_+
      and as the paper's code listing computes; the printed equation's index
      order (no transpose) differs from it when G is not symmetric.
* R21 Weighted walker mean of any per-walker value v_z (the reduction of
      the global energy, R18, and of the mixed estimators of Sec. IV.B):
      sum_z w_z v_z / sum_z w_z.
* R23 Multi-determinant trial (Sec. III.A): |Psi_T> = sum_a c_a t_a |psi_0>
      with real c_a, psi_0 the first n_s columns of an orthogonal orbital
      matrix C^s per spin, and t_a = prod_s prod_m a+_{s,q_m} a_{s,h_m} in
      those orbitals (hole h_m paired with particle q_m).  t_a |psi_0> is the
      determinant D_a whose orbital matrix is psi_0's with column h_m
      replaced in place by column q_m of C^s, so
      <Psi_T|phi> = sum_a c_a det(D_a^aT phi^a) det(D_a^bT phi^b).
* R24 Its Green's function (Eq. gf with the MSD numerator of Sec. III.B):
      G^s = sum_a c_a O_a G^s_a / sum_a c_a O_a, O_a = <D_a|phi> and G^s_a
      the single-determinant Green's function of D_a^s (R11).  The force bias
      of an MSD trial is Eq. (fb) with this G.
* R25 Local energy of a multi-determinant trial (Sec. III.C with the
      expansion of R23): E_L = <Psi_T|H|phi>/<Psi_T|phi>
      = sum_a c_a O_a E_L^a / sum_a c_a O_a, O_a = <D_a|phi> and E_L^a the
      single-determinant local energy of phi with trial D_a (R10).  Each part
      (E1, EJ, EK) is reported with the same weights; E1 so equals
      sum_s tr(h G^s) with the Green's function of R24.
* R19 Block (Sec. IV.A and IV.C): nsteps propagation steps, the last one
      followed by re-orthogonalisation and the local energy, then the global
      energy of the block, then the comb.

Array conventions: walkers phi are [W, N, n] complex128 per spin; the trial
PhiT is [N, n] float64 per spin; theta = phi S^-1 is [W, N, n];
Lh^s[g, i, p] = sum_q PhiT^s[q, i] L[g, q, p].
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "OracleHamiltonian",
    "setup",
    "log_det",
    "theta_and_logdet",
    "overlap",
    "full_green",
    "force_bias",
    "shift",
    "vhs",
    "taylor_apply",
    "propagate",
    "local_energy",
    "orthogonalise",
    "step",
    "global_energy",
    "comb",
    "block",
    "s2_mixed",
    "weighted_mean",
    "OracleMSD",
    "msd_setup",
    "msd_determinant",
    "msd_overlap",
    "msd_green",
    "msd_force_bias",
    "msd_propagate",
    "msd_local_energy",
]


@dataclasses.dataclass
class OracleHamiltonian:
    h1: np.ndarray          # [N, N] one-body integrals (used by the energy)
    L: np.ndarray           # [K, N, N] Cholesky vectors
    phiT_a: np.ndarray      # [N, na]
    phiT_b: np.ndarray      # [N, nb]
    dt: float
    taylor_order: int
    hprime: np.ndarray      # [N, N] h' of R1
    mu: float               # scalar factored out of the one-body half step (R2)
    P: np.ndarray           # [N, N] exp(-dt/2 (h' - mu))
    Lh_a: np.ndarray        # [K, na, N] half-rotated Cholesky vectors (Sec. III.B)
    Lh_b: np.ndarray        # [K, nb, N]
    hh_a: np.ndarray        # [na, N] PhiT_a^T h1
    hh_b: np.ndarray        # [nb, N]
    e_shift: float          # E_T of R3

    @property
    def N(self):
        return self.h1.shape[0]

    @property
    def K(self):
        return self.L.shape[0]

    @property
    def nelec(self):
        return self.phiT_a.shape[1] + self.phiT_b.shape[1]


def setup(h1, L, phiT_a, phiT_b=None, dt=0.005, taylor_order=6, mu=None, e_shift=None):
    """Precompute the step-independent arrays (run once).

    h' follows R1; P follows R2 with mu = tr(h')/N unless given; the
    half-rotated vectors follow Sec. III.B; E_T defaults to the local
    energy of the trial itself.
    """
    h1 = np.asarray(h1, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    phiT_a = np.asarray(phiT_a, dtype=np.float64)
    phiT_b = phiT_a if phiT_b is None else np.asarray(phiT_b, dtype=np.float64)
    K, N, _ = L.shape
    # sum_g L_g L_g as one matrix product: [N, (g, r)] x [(g, r), N]
    LL = L.transpose(1, 0, 2).reshape(N, K * N) @ L.reshape(K * N, N)
    hprime = h1 - 0.5 * LL
    if mu is None:
        mu = float(np.trace(hprime)) / N
    evals, evecs = np.linalg.eigh(hprime)
    P = (evecs * np.exp(-0.5 * dt * (evals - mu))) @ evecs.T
    Lh_a = np.matmul(phiT_a.T[None, :, :], L)
    Lh_b = np.matmul(phiT_b.T[None, :, :], L)
    ham = OracleHamiltonian(
        h1=h1, L=L, phiT_a=phiT_a, phiT_b=phiT_b, dt=float(dt),
        taylor_order=int(taylor_order), hprime=hprime, mu=float(mu), P=P,
        Lh_a=Lh_a, Lh_b=Lh_b, hh_a=phiT_a.T @ h1, hh_b=phiT_b.T @ h1,
        e_shift=0.0,
    )
    if e_shift is None:
        e = local_energy(ham, phiT_a[None].astype(np.complex128),
                         phiT_b[None].astype(np.complex128))
        e_shift = float(np.real(e[0].sum()))
    ham.e_shift = float(e_shift)
    return ham


# ---------------------------------------------------------------------------
# Overlap and Green's function (Sec. III.A, III.B)
# ---------------------------------------------------------------------------

def log_det(S):
    """Complex log det of a stack of square matrices via LU with partial pivoting (R7).

    Returns log|det| + i arg(det); the phase is defined modulo 2 pi.
    """
    sign, logabs = np.linalg.slogdet(S)
    return logabs + 1j * np.angle(sign)


def theta_and_logdet(phiT, phi):
    """theta = phi (PhiT^T phi)^{-1} and log det(PhiT^T phi) for each walker.

    theta[z, p, j] is the paper's theta^z_jp (Eq. halfgf), stored N x n.
    """
    S = np.einsum("pi,zpj->zij", phiT, phi)          # S = PhiT^T phi  [W, n, n]
    ld = log_det(S)
    # theta S = phi  <=>  S^T theta^T = phi^T
    theta = np.linalg.solve(np.swapaxes(S, 1, 2), np.swapaxes(phi, 1, 2))
    return np.swapaxes(theta, 1, 2), ld


def overlap(ham, phi_a, phi_b):
    """log <Psi_T|phi_z> = sum over spins of log det(PhiT^T phi) (Sec. III.A)."""
    _, la = theta_and_logdet(ham.phiT_a, phi_a)
    _, lb = theta_and_logdet(ham.phiT_b, phi_b)
    return la + lb


def full_green(phiT, phi):
    """G[z, p, q] = <Psi_T|a+_p a_q|phi_z>/<Psi_T|phi_z> = (phi S^-1 PhiT^T)_qp (Eq. halfgf, R11)."""
    theta, _ = theta_and_logdet(phiT, phi)
    Gcal = theta @ phiT.T                            # phi S^-1 PhiT^T
    return np.swapaxes(Gcal, 1, 2)


def force_bias(ham, phi_a, phi_b):
    """vbias[z, g] = sum_s sum_{i,p} Lh^s[g, i, p] theta^s_z[p, i] (Eq. rfb; = sum_pq G_pq L^g_pq, Eq. fb)."""
    ta, _ = theta_and_logdet(ham.phiT_a, phi_a)
    tb, _ = theta_and_logdet(ham.phiT_b, phi_b)
    K = ham.K
    W = phi_a.shape[0]
    # [K, (i,p)] x [(i,p), W] with theta transposed to (i, p) order
    va = ham.Lh_a.reshape(K, -1) @ np.swapaxes(ta, 1, 2).reshape(W, -1).T
    vb = ham.Lh_b.reshape(K, -1) @ np.swapaxes(tb, 1, 2).reshape(W, -1).T
    return (va + vb).T


# ---------------------------------------------------------------------------
# Propagation and weights (Sec. II.B)
# ---------------------------------------------------------------------------

def shift(ham, vbias, x):
    """xbar = -i sqrt(dt) vbias (R4); xs = x - xbar; a_z = sum_g (x xbar - xbar^2 / 2) (Eq. import)."""
    sdt = math.sqrt(ham.dt)
    xbar = -1j * sdt * vbias
    xs = x - xbar
    a = np.sum(x * xbar - 0.5 * xbar * xbar, axis=1)
    return xs, a


def vhs(ham, xs):
    """VHS_z = i sqrt(dt) sum_g xs_zg L_g, an N x N complex symmetric matrix per walker (R4)."""
    K, N, _ = ham.L.shape
    Lf = ham.L.reshape(K, N * N)
    v = (xs.real @ Lf) + 1j * (xs.imag @ Lf)
    return 1j * math.sqrt(ham.dt) * v.reshape(-1, N, N)


def taylor_apply(A, phi, order):
    """sum_{k=0}^{order} A^k phi / k!, formed as t_0 = phi, t_k = A t_{k-1} / k (R6)."""
    t = phi
    acc = phi.copy()
    for k in range(1, order + 1):
        t = np.matmul(A, t) / k
        acc = acc + t
    return acc


def _b_apply(ham, V, phi):
    """B(x - xbar) phi with the scalar e^{-dt mu/2} of each half step removed (R2)."""
    t = np.matmul(ham.P[None], phi)
    t = taylor_apply(V, t, ham.taylor_order)
    return np.matmul(ham.P[None], t)


def propagate(ham, phi_a, phi_b, log_ovlp, log_w, x):
    """One importance-sampled phaseless step for every walker (Sec. II.B).

    Returns new (phi_a, phi_b, log_ovlp, log_w).  x is [W, K] real.
    Order: theta -> vbias -> xbar, xs, a -> VHS -> phi' = B phi ->
    ln O_z = log<Psi_T|phi'> - log<Psi_T|phi> -> phase -> log w.
    """
    return _propagate(ham, lambda a, b: force_bias(ham, a, b), lambda a, b: overlap(ham, a, b),
                      phi_a, phi_b, log_ovlp, log_w, x)


def _propagate(ham, vbias_of, overlap_of, phi_a, phi_b, log_ovlp, log_w, x):
    """The step of `propagate` with the trial entering only through the
    force bias and the overlap (a single determinant, or R23's expansion)."""
    vb = vbias_of(phi_a, phi_b)
    xs, a = shift(ham, vb, x)
    V = vhs(ham, xs)
    na = _b_apply(ham, V, phi_a)
    nb = _b_apply(ham, V, phi_b)
    new_lo = overlap_of(na, nb)
    ln_o = new_lo - log_ovlp
    theta_ph = np.imag(ln_o)                       # arg O_z (Eq. theta, R8)
    cos_t = np.cos(theta_ph)
    const = -ham.dt * (ham.mu * ham.nelec - ham.e_shift)      # R3
    with np.errstate(divide="ignore"):
        log_cos = np.where(cos_t > 0.0, np.log(np.where(cos_t > 0.0, cos_t, 1.0)), -np.inf)
    new_lw = log_w + np.real(ln_o) + np.real(a) + const + log_cos     # Eqs. (import), (ph)
    return na, nb, new_lo, new_lw


# ---------------------------------------------------------------------------
# Local energy (Sec. III.C)
# ---------------------------------------------------------------------------

def _energy_spin(Lh, hh, theta):
    """(E1, sum_g tr T_g, EK) for one spin and one walker; T_g = Lh_g theta (n x n)."""
    e1 = np.sum(hh * theta.T)                      # tr(hh theta)
    T = np.matmul(Lh, theta[None])                 # [K, n, n], T_ij = sum_p Lh_ip theta_pj
    tr = np.trace(T, axis1=1, axis2=2)             # [K]
    ek = -0.5 * np.sum(T * np.swapaxes(T, 1, 2))   # -1/2 sum_g sum_ij T_ij T_ji
    return e1, tr, ek


def local_energy(ham, phi_a, phi_b):
    """E_L split as [W, 3] complex: (E1, EJ, EK) (Sec. III.C, R10)."""
    ta, _ = theta_and_logdet(ham.phiT_a, phi_a)
    tb, _ = theta_and_logdet(ham.phiT_b, phi_b)
    W = phi_a.shape[0]
    out = np.zeros((W, 3), dtype=np.complex128)
    for z in range(W):                             # direct algorithm: T per walker, consumed at once
        e1a, tra, eka = _energy_spin(ham.Lh_a, ham.hh_a, ta[z])
        e1b, trb, ekb = _energy_spin(ham.Lh_b, ham.hh_b, tb[z])
        out[z, 0] = e1a + e1b
        out[z, 1] = 0.5 * np.sum((tra + trb) ** 2)
        out[z, 2] = eka + ekb
    return out


# ---------------------------------------------------------------------------
# Re-orthogonalisation
# ---------------------------------------------------------------------------

def orthogonalise(phi_a, phi_b, log_ovlp):
    """QR of every walker and spin (R9); returns new (phi_a, phi_b, log_ovlp)."""
    out = []
    corr = np.zeros(phi_a.shape[0])
    for phi in (phi_a, phi_b):
        q, r = np.linalg.qr(phi)                   # Householder (LAPACK geqrf/ungqr)
        d = np.diagonal(r, axis1=1, axis2=2)
        ad = np.abs(d)
        out.append(q * (d / ad)[:, None, :])
        corr += np.sum(np.log(ad), axis=1)
    return out[0], out[1], log_ovlp - corr


def step(ham, phi_a, phi_b, log_ovlp, log_w, x, do_qr):
    """One full step in the order of the method: propagate, optional QR, local energy."""
    phi_a, phi_b, log_ovlp, log_w = propagate(ham, phi_a, phi_b, log_ovlp, log_w, x)
    if do_qr:
        phi_a, phi_b, log_ovlp = orthogonalise(phi_a, phi_b, log_ovlp)
    e = local_energy(ham, phi_a, phi_b)
    return phi_a, phi_b, log_ovlp, log_w, e


# ---------------------------------------------------------------------------
# Global energy, population control, block (R17-R19)
# ---------------------------------------------------------------------------

def _linear_weights(log_w):
    """w_z / max_z w_z and ln max_z w_z; non-finite log w counts as weight 0."""
    log_w = np.asarray(log_w, dtype=np.float64)
    live = np.isfinite(log_w)
    if not live.any():
        return np.zeros_like(log_w), -np.inf
    m = float(np.max(log_w[live]))
    w = np.zeros_like(log_w)
    w[live] = np.exp(log_w[live] - m)
    return w, m


def global_energy(log_w, e):
    """(E, ln sum_z w_z, live walkers): E = sum_z w_z E_L^z / sum_z w_z (R18).

    e is [W, 3] complex (E1, EJ, EK).  With no live walker E is NaN.
    """
    w, m = _linear_weights(log_w)
    den = float(np.sum(w))
    live = int(np.count_nonzero(w))
    if live == 0:
        return complex(np.nan, np.nan), -np.inf, 0
    el = np.asarray(e).sum(axis=1)
    return complex(np.sum(w * el) / den), m + math.log(den), live


def comb(log_w, u):
    """Comb population control (R17).

    Returns (parent, new_log_w): the new walker in slot k is a copy of the
    old walker parent[k]; every new log weight is new_log_w.  With no live
    walker, parent = identity and new_log_w = None (weights unchanged).
    """
    nw = len(log_w)
    w, m = _linear_weights(log_w)
    C = np.cumsum(w)                               # inclusive, left to right
    wtot = float(C[-1]) if nw else 0.0
    if not (wtot > 0.0) or not math.isfinite(wtot):
        return np.arange(nw), None
    teeth = (np.arange(nw) + u) * wtot / nw
    pick = np.searchsorted(C, teeth, side="right")     # first z with C_z > t_k
    last_live = int(np.nonzero(w)[0][-1])
    pick = np.where(pick >= nw, last_live, pick)
    copies = np.bincount(pick, minlength=nw)
    extra_src = []
    for z in range(nw):                            # extra copies in walker order
        extra_src.extend([z] * max(int(copies[z]) - 1, 0))
    parent = np.arange(nw)
    empty = np.nonzero(copies == 0)[0]             # slots freed, in slot order
    parent[empty] = extra_src
    return parent, m + math.log(wtot / nw)


def block(ham, phi_a, phi_b, log_ovlp, log_w, x, u):
    """One block (R19): len(x) steps, QR and energy at the last, global energy, comb.

    x is [nsteps, W, K].  Returns (phi_a, phi_b, log_ovlp, log_w, e, E, parent)
    where e [W, 3] are the local energies before the comb and E the global
    energy.  u = None skips the comb.
    """
    nsteps = len(x)
    for s in range(nsteps):
        last = s == nsteps - 1
        phi_a, phi_b, log_ovlp, log_w = propagate(ham, phi_a, phi_b, log_ovlp, log_w, x[s])
        if last:
            phi_a, phi_b, log_ovlp = orthogonalise(phi_a, phi_b, log_ovlp)
    e = local_energy(ham, phi_a, phi_b)
    E, _, _ = global_energy(log_w, e)
    if u is None:                                  # no population control
        return phi_a, phi_b, log_ovlp, log_w, e, E, np.arange(len(log_w))
    parent, lw = comb(log_w, u)
    if lw is not None:
        phi_a, phi_b, log_ovlp = phi_a[parent], phi_b[parent], log_ovlp[parent]
        log_w = np.full_like(log_w, lw)
    return phi_a, phi_b, log_ovlp, log_w, e, E, parent


# ---------------------------------------------------------------------------
# Mixed estimators (Sec. IV.B; R20, R21)
# ---------------------------------------------------------------------------

def s2_mixed(ham, phi_a, phi_b):
    """<Psi_T|S^2|phi_z>/<Psi_T|phi_z> for each walker (R20), complex [W]."""
    na, nb = ham.phiT_a.shape[1], ham.phiT_b.shape[1]
    ms = 0.5 * (na - nb)
    out = np.full(phi_a.shape[0], nb + ms * (ms + 1.0), dtype=np.complex128)
    if na == 0 or nb == 0:
        return out
    Ga = full_green(ham.phiT_a, phi_a)
    Gb = full_green(ham.phiT_b, phi_b)
    return out - np.einsum("zpq,zqp->z", Ga, Gb)


def weighted_mean(log_w, v):
    """(sum_z w_z v_z / sum_z w_z for every column of v [W, m], ln sum w, live walkers) (R21).

    Weights as in R17; with no live walker the means are NaN.
    """
    w, m = _linear_weights(log_w)
    v = np.asarray(v).reshape(len(w), -1)
    live = int(np.count_nonzero(w))
    if live == 0:
        return np.full(v.shape[1], complex(np.nan, np.nan)), -np.inf, 0
    den = float(np.sum(w))
    return (w @ v) / den, m + math.log(den), live


# ---------------------------------------------------------------------------
# Multi-determinant trial (Sec. III.A, III.B; R23, R24)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class OracleMSD:
    C: tuple                # (C_a, C_b), each [N, N] orthogonal float64
    nel: tuple              # (na, nb)
    coeff: np.ndarray       # [ndet] float64
    exc: list               # per determinant: ((holes_a, parts_a), (holes_b, parts_b))


def msd_setup(C_a, C_b, na, nb, coeff, rank, orbs):
    """Expansion from the array form: rank [ndet, 2]; orbs [ndet, 2, 2, kmax]
    (spin, holes | particles, slot), hole m paired with particle m."""
    exc = []
    for a in range(len(coeff)):
        exc.append(tuple((tuple(int(v) for v in orbs[a, s, 0, :rank[a, s]]),
                          tuple(int(v) for v in orbs[a, s, 1, :rank[a, s]])) for s in range(2)))
    return OracleMSD((np.asarray(C_a, np.float64), np.asarray(C_b, np.float64)), (na, nb),
                     np.asarray(coeff, np.float64), exc)


def msd_determinant(C, n, holes, parts):
    """Orbital matrix of t_a psi_0: psi_0 = C[:, :n] with column h_m replaced by C[:, q_m] (R23)."""
    D = np.array(C[:, :n], copy=True)
    for h, q in zip(holes, parts):
        D[:, h] = C[:, q]
    return D


def _msd_log_terms(msd, phi_a, phi_b):
    """[ndet, W]: complex log of c_a <D_a|phi_z> = c_a det(D_a^aT phi^a) det(D_a^bT phi^b)."""
    logs = []
    for ca, spins in zip(msd.coeff, msd.exc):
        la = np.full(phi_a.shape[0], np.log(complex(ca)))
        for s, phi in enumerate((phi_a, phi_b)):
            D = msd_determinant(msd.C[s], msd.nel[s], *spins[s])
            if D.shape[1]:
                la = la + log_det(D.T @ phi)   # det(D^T phi), Sec. III.A
        logs.append(la)
    return np.array(logs)


def msd_overlap(msd, phi_a, phi_b):
    """log <Psi_T|phi_z> = log sum_a c_a det(D_a^aT phi^a) det(D_a^bT phi^b) (R23), complex [W].

    The sum is taken relative to its largest |term| (exact up to rounding).
    """
    logs = _msd_log_terms(msd, phi_a, phi_b)
    m = np.max(logs.real, axis=0)
    return m + np.log(np.sum(np.exp(logs - m), axis=0))


def msd_green(msd, phi_a, phi_b):
    """G[z, s, p, q] = <Psi_T|a+_ps a_qs|phi_z>/<Psi_T|phi_z> (R24), complex [W, 2, N, N]."""
    logs = _msd_log_terms(msd, phi_a, phi_b)
    m = np.max(logs.real, axis=0)
    w = np.exp(logs - m)                      # c_a O_a / e^m, [ndet, W]
    N = phi_a.shape[1]
    G = np.zeros((phi_a.shape[0], 2, N, N), complex)
    for a, spins in enumerate(msd.exc):
        for s, phi in enumerate((phi_a, phi_b)):
            D = msd_determinant(msd.C[s], msd.nel[s], *spins[s])
            if D.shape[1]:
                G[:, s] += w[a][:, None, None] * full_green(D, phi)
    return G / np.sum(w, axis=0)[:, None, None, None]


def msd_force_bias(msd, L, phi_a, phi_b):
    """vbias[z, g] = sum_s sum_pq G^s_pq L_g,pq with the MSD Green's function (Eq. fb, R24)."""
    G = msd_green(msd, phi_a, phi_b)
    return np.einsum("zspq,gpq->zg", G, L)


def msd_propagate(ham, msd, phi_a, phi_b, log_ovlp, log_w, x):
    """One phaseless step under the multi-determinant trial (Sec. II.B with
    R23, R24): the force bias is Eq. fb with the MSD Green's function and the
    overlap ratio of the importance function is that of the expansion; the
    propagator is the Hamiltonian's (P, VHS, Taylor series).  log_ovlp holds
    log <Psi_T|phi> of the expansion.  Returns new (phi_a, phi_b, log_ovlp, log_w).
    """
    return _propagate(ham, lambda a, b: msd_force_bias(msd, ham.L, a, b), lambda a, b: msd_overlap(msd, a, b),
                      phi_a, phi_b, log_ovlp, log_w, x)


def _sd_local_energy(h1, L, D_a, D_b, phi_a, phi_b):
    """Single-determinant local energy parts [W, 3] of phi with trial orbitals
    (D_a, D_b) (Sec. III.C, R10): the half-rotated vectors D^T L_g and
    D^T h1 of this trial, then the same sums as local_energy."""
    Lh_a = np.matmul(D_a.T[None, :, :], L)
    Lh_b = np.matmul(D_b.T[None, :, :], L)
    ta, _ = theta_and_logdet(D_a, phi_a)
    tb, _ = theta_and_logdet(D_b, phi_b)
    W = phi_a.shape[0]
    out = np.zeros((W, 3), dtype=np.complex128)
    for z in range(W):
        e1a, tra, eka = _energy_spin(Lh_a, D_a.T @ h1, ta[z])
        if D_b.shape[1]:
            e1b, trb, ekb = _energy_spin(Lh_b, D_b.T @ h1, tb[z])
        else:
            e1b, trb, ekb = 0.0, 0.0, 0.0
        out[z, 0] = e1a + e1b
        out[z, 1] = 0.5 * np.sum((tra + trb) ** 2)
        out[z, 2] = eka + ekb
    return out


def msd_local_energy(msd, h1, L, phi_a, phi_b):
    """E_L split [W, 3] complex (E1, EJ, EK) for the multi-determinant trial
    (R25): sum_a c_a O_a E_L^a / sum_a c_a O_a, one determinant at a time."""
    logs = _msd_log_terms(msd, phi_a, phi_b)
    m = np.max(logs.real, axis=0)
    w = np.exp(logs - m)                      # c_a O_a / e^m, [ndet, W]
    out = np.zeros((phi_a.shape[0], 3), dtype=np.complex128)
    for a, spins in enumerate(msd.exc):
        D_a = msd_determinant(msd.C[0], msd.nel[0], *spins[0])
        D_b = msd_determinant(msd.C[1], msd.nel[1], *spins[1])
        out += w[a][:, None] * _sd_local_energy(h1, L, D_a, D_b, phi_a, phi_b)
    return out / np.sum(w, axis=0)[:, None]
