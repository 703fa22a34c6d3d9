"""Seeded synthetic inputs for the phaseless-AFQMC walker step.

The paper measures on real molecules (acenes, Cu2O2) whose integrals and
trial wavefunctions are not available; these generators stand in for them
with the same array shapes and structure:

* ``h1``: real symmetric N x N one-body matrix, off-diagonal and diagonal
  entries ~ N(0, 0.1) (the upper triangle is drawn and mirrored) plus
  ``diag(linspace(-2, 0, N))``.
* ``L``: K real symmetric N x N Cholesky-like vectors, each the mirror of an
  N(0, 1) draw scaled by ``exp(-gamma / decay)``, so that sum_g L_g (x) L_g is
  positive semidefinite, as a factorised two-electron tensor is
  (Sec. II.B, the Cholesky factorisation below the ab initio Hamiltonian).
* ``phiT``: the n lowest eigenvectors of ``h1`` (a restricted, single
  determinant trial as in Sec. III), each column's sign fixed so that its
  largest-magnitude entry is positive.
* ``fields``: auxiliary fields ~ N(0, 1), shape (steps, W, K) (Eq. Bx).
* ``orbitals`` / ``msd_expansion``: a multi-determinant trial (Sec. III.A)
  as excitations of the reference determinant within the full eigenvector
  basis of h1, with decaying, sorted coefficients.  The paper's expansions
  come from selected CI on real molecules; these stand in for them with the
  same structure (reference first, mostly low-rank excitations of both
  spins, no duplicates).

Seeding: ``SeedSequence(seed).spawn(3)`` gives independent streams for the
Hamiltonian, the fields and auxiliary draws (walker perturbations).  All
streams are numpy PCG64 ``default_rng``.

This module holds none of the method's arithmetic: it only draws and shapes
inputs.  Both the oracle tests and the GPU tests take their inputs from it.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Config",
    "CONFIGS",
    "hamiltonian",
    "trial",
    "fields",
    "walkers_at_trial",
    "walkers_perturbed",
    "uneven_batch",
    "MSD_MAX_RANK",
    "orbitals",
    "msd_expansion",
]


@dataclasses.dataclass(frozen=True)
class Config:
    """One synthetic workload: sizes, time step and schedule."""

    name: str
    N: int          # spatial orbitals
    n: int          # electrons per spin (n_alpha = n_beta)
    K: int          # Cholesky vectors (N_aux in the paper)
    decay: float    # L_gamma scale exp(-gamma / decay)
    W: int          # walkers
    steps: int
    qr_interval: int
    dt: float = 0.005
    taylor_order: int = 6


CONFIGS = {
    # CPU-oracle size: every array is < 0.2 MB.
    "n20": Config("n20", N=20, n=5, K=60, decay=15.0, W=16, steps=10, qr_interval=5),
    # FP64 GPU baseline; 640 walkers and dt = 0.005 as in the Cu2O2 runs (Sec. IV).
    "n100": Config("n100", N=100, n=20, K=400, decay=80.0, W=640, steps=200, qr_interval=5),
    # Mixed-precision size.
    "n200": Config("n200", N=200, n=32, K=1000, decay=200.0, W=1000, steps=100, qr_interval=1),
    # The (52e, 290o) shape of the largest Cu2O2 active space (Tables III-IV).
    "n290": Config("n290", N=290, n=26, K=2900, decay=580.0, W=512, steps=50, qr_interval=1),
}


def _streams(seed: int):
    ham_ss, field_ss, aux_ss = np.random.SeedSequence(seed).spawn(3)
    return ham_ss, field_ss, aux_ss


def _mirror(a: np.ndarray) -> np.ndarray:
    return np.triu(a) + np.triu(a, 1).T


def hamiltonian(N: int, K: int, decay: float, seed: int = 0):
    """Return ``(h1 [N,N], L [K,N,N])`` as float64, drawn from the Hamiltonian stream."""
    ham_ss, _, _ = _streams(seed)
    rng = np.random.default_rng(ham_ss)
    h1 = _mirror(rng.normal(0.0, 0.1, size=(N, N))) + np.diag(np.linspace(-2.0, 0.0, N))
    L = np.empty((K, N, N), dtype=np.float64)
    for g in range(K):
        L[g] = _mirror(rng.standard_normal((N, N))) * np.exp(-g / decay)
    return h1, L


def trial(h1: np.ndarray, n: int) -> np.ndarray:
    """The n lowest eigenvectors of h1 as an [N, n] float64 array (sign-fixed)."""
    _, vecs = np.linalg.eigh(h1)
    phi = np.array(vecs[:, :n], dtype=np.float64, copy=True)
    for j in range(n):
        k = int(np.argmax(np.abs(phi[:, j])))
        if phi[k, j] < 0:
            phi[:, j] = -phi[:, j]
    return phi


def fields(W: int, K: int, steps: int, seed: int = 0) -> np.ndarray:
    """Auxiliary fields x ~ N(0, 1), shape (steps, W, K), float64."""
    _, field_ss, _ = _streams(seed)
    rng = np.random.default_rng(field_ss)
    return rng.standard_normal((steps, W, K))


def walkers_at_trial(phiT: np.ndarray, W: int) -> np.ndarray:
    """W walkers equal to the trial determinant, [W, N, n] complex128."""
    return np.repeat(phiT[None, :, :].astype(np.complex128), W, axis=0)


def walkers_perturbed(phiT: np.ndarray, W: int, scale: float, seed: int = 0,
                      stream: int = 0, complex_noise: bool = True) -> np.ndarray:
    """Walkers ``phiT + scale * R`` with R drawn from the auxiliary stream.

    ``stream`` selects an independent child of the auxiliary stream so that
    several perturbed sets (e.g. alpha and beta) can be drawn from one seed.
    With ``complex_noise`` R = (R1 + i R2) / sqrt(2), else R real.
    """
    _, _, aux_ss = _streams(seed)
    child = aux_ss.spawn(stream + 1)[stream]
    rng = np.random.default_rng(child)
    N, n = phiT.shape
    if complex_noise:
        r = (rng.standard_normal((W, N, n)) + 1j * rng.standard_normal((W, N, n))) / np.sqrt(2.0)
    else:
        r = rng.standard_normal((W, N, n)).astype(np.complex128)
    return phiT[None, :, :] + scale * r


def uneven_batch(seed: int = 0):
    """The uneven multi-system workload: 8 systems with N in {40, 60, ..., 160, 200},
    n = N / 5 electrons per spin, K = 4 N, decay = K / 5; walkers per system
    drawn from {64, ..., 512} with the auxiliary stream of `seed`.  System s
    draws its Hamiltonian and fields with seed s.  Returns a list of
    (N, n, K, decay, walkers, seed)."""
    _, _, aux_ss = _streams(seed)
    rng = np.random.default_rng(aux_ss)
    sizes = [40, 60, 80, 100, 120, 140, 160, 200]
    walkers = rng.integers(64, 513, size=len(sizes))
    return [(N, N // 5, 4 * N, 4 * N / 5.0, int(w), s) for s, (N, w) in enumerate(zip(sizes, walkers))]


MSD_MAX_RANK = 6  # excitation rank per spin supported by the expansion format


def orbitals(h1: np.ndarray) -> np.ndarray:
    """All eigenvectors of h1, ascending, as an [N, N] float64 orthogonal matrix.

    Column signs follow ``trial``: ``orbitals(h1)[:, :n] == trial(h1, n)``.
    """
    return trial(h1, h1.shape[0])


# From this many determinants on, an expansion in an active window is drawn in
# vectorised batches (same distribution, another sequence of draws).
MSD_FAST_DETS = 20000


def _msd_draw_window(rng, ndet, nel, hole_lo, nocc_act, nvirt, kmax, prob):
    """Distinct excitations in an active window, drawn in batches: per spin a
    rank from prob, a random k-subset of the window's holes (the first k of a
    random order of the window, sorted) and of its particles (the first k of
    another random order, kept in that order: the pairing), the reference
    pair (0, 0) excluded; duplicates (same hole and particle sets) are
    dropped in draw order."""
    exc = [((), (), (), ())]
    seen = set()
    while len(exc) < ndet:
        B = int(1.3 * (ndet - len(exc))) + 1024
        ks = [rng.choice(len(pr), size=B, p=pr) for pr in prob]
        keep = (ks[0] + ks[1]) > 0
        cols = []
        for s in range(2):
            horder = np.argsort(rng.random((B, nocc_act[s])), axis=1)[:, :max(kmax[s], 1)]
            porder = np.argsort(rng.random((B, nvirt[s])), axis=1)[:, :max(kmax[s], 1)]
            cols.append((horder, porder))
        for b in np.nonzero(keep)[0]:
            key, ident = [], []
            for s in range(2):
                k = int(ks[s][b])
                horder, porder = cols[s]
                holes = tuple(sorted(hole_lo[s] + int(h) for h in horder[b, :k]))
                parts = tuple(nel[s] + int(q) for q in porder[b, :k])
                key += [holes, parts]
                ident += [holes, tuple(sorted(parts))]
            ident = tuple(ident)
            if ident in seen:
                continue
            seen.add(ident)
            exc.append(tuple(key))
            if len(exc) == ndet:
                break
    return exc


def msd_expansion(N: int, na: int, nb: int, ndet: int, max_rank: int = 4, seed: int = 0,
                  stream: int = 0, active=None):
    """A synthetic multi-determinant expansion of ``ndet`` distinct determinants.

    Returns ``(coeff [ndet] float64, rank [ndet, 2] int32,
    orbs [ndet, 2, 2, MSD_MAX_RANK] int32)``.  Determinant a excites, in spin
    s, ``rank[a, s]`` electrons: holes ``orbs[a, s, 0, :rank]`` (ascending,
    in [0, n_s)) to particles ``orbs[a, s, 1, :rank]`` (in [n_s, N), in a
    random order: hole m is paired with particle m); unused slots hold -1.
    Determinant 0 is the reference with coefficient 1.  Per-spin ranks are
    drawn with probability proportional to 0.45^k (k <= max_rank and the
    available holes and particles), the pair (0, 0) excluded after the
    reference; coefficients are +-0.2 exp(-3 a / ndet) (1 - u / 2), u ~ U(0, 1),
    sorted by decreasing magnitude after the reference.

    ``active = (n_ao, n_av)`` confines the excitations to an active space, as
    selected-CI trials are: holes among the n_ao highest occupied orbitals
    [n_s - n_ao, n_s), particles among the n_av lowest virtual ones
    [n_s, n_s + n_av) (None: every orbital).
    """
    if not 0 <= max_rank <= MSD_MAX_RANK:
        raise ValueError("max_rank out of range")
    _, _, aux_ss = _streams(seed)
    rng = np.random.default_rng(aux_ss.spawn(stream + 1)[stream])
    nel = (na, nb)
    if active is None:
        hole_lo = [0, 0]
        nvirt = [N - na, N - nb]
    else:
        n_ao, n_av = active
        hole_lo = [max(0, n - n_ao) for n in nel]
        nvirt = [min(n_av, N - n) for n in nel]
    nocc_act = [nel[s] - hole_lo[s] for s in range(2)]
    kmax = [min(max_rank, nocc_act[s], nvirt[s]) for s in range(2)]
    seen = {((), (), (), ())}
    exc = [((), (), (), ())]
    limit = 1
    for k_a in range(kmax[0] + 1):
        for k_b in range(kmax[1] + 1):
            limit += (math.comb(nocc_act[0], k_a) * math.comb(nvirt[0], k_a)
                      * math.comb(nocc_act[1], k_b) * math.comb(nvirt[1], k_b))
    if ndet > limit - 1:
        raise ValueError("more determinants requested than the excitation space holds")
    prob = [np.array([0.45 ** k for k in range(km + 1)]) for km in kmax]
    prob = [pr / pr.sum() for pr in prob]
    if active is not None and ndet >= MSD_FAST_DETS and max(nocc_act) <= 64 and max(nvirt) <= 64:
        exc = _msd_draw_window(rng, ndet, nel, hole_lo, nocc_act, nvirt, kmax, prob)
    while len(exc) < ndet:
        ks = [int(rng.choice(len(pr), p=pr)) for pr in prob]
        if ks == [0, 0]:
            continue
        key, ident = [], []
        for s in range(2):
            if active is None:
                holes = tuple(sorted(int(h) for h in rng.choice(nel[s], ks[s], replace=False)))
                parts = tuple(int(q) for q in rng.permutation(rng.choice(np.arange(nel[s], N), ks[s],
                                                                         replace=False)))
            else:
                holes = tuple(sorted(hole_lo[s] + int(h) for h in rng.choice(nocc_act[s], ks[s], replace=False)))
                parts = tuple(int(q) for q in rng.permutation(
                    rng.choice(np.arange(nel[s], nel[s] + nvirt[s]), ks[s], replace=False)))
            key += [holes, parts]
            ident += [holes, tuple(sorted(parts))]   # the determinant, whatever the pairing
        if tuple(ident) in seen:
            continue
        seen.add(tuple(ident))
        exc.append(tuple(key))
    mag = 0.2 * np.exp(-3.0 * np.arange(1, ndet) / ndet) * (1.0 - 0.5 * rng.random(ndet - 1))
    sign = np.where(rng.random(ndet - 1) < 0.5, -1.0, 1.0)
    order = np.argsort(-mag, kind="stable")
    coeff = np.concatenate([[1.0], (sign * mag)[order]])
    exc = [exc[0]] + [exc[1 + i] for i in order]
    rank = np.zeros((ndet, 2), dtype=np.int32)
    orbs = np.full((ndet, 2, 2, MSD_MAX_RANK), -1, dtype=np.int32)
    for a, (ha, pa, hb, pb) in enumerate(exc):
        for s, (h, q) in enumerate(((ha, pa), (hb, pb))):
            rank[a, s] = len(h)
            orbs[a, s, 0, :len(h)] = h
            orbs[a, s, 1, :len(q)] = q
    return coeff, rank, orbs
