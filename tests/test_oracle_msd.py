"""Pins of the oracle's multi-determinant trial (Sec. III.A, III.B).

The oracle takes the plain definition: the trial's overlap is the
c_a-weighted sum of determinant overlaps, and its Green's function is the
c_a O_a-weighted sum of single-determinant ones.  The pins check it
against things other than itself:
* the Fock-space brute force, with the trial built from the excitation
  operators acting on the reference, which pins how an excitation maps to
  a determinant (hole/particle pairing and signs);
* Cauchy-Binet: the complete expansion of one determinant psi in an
  orthogonal basis has the overlap and Green's function of psi itself;
* the single-reference limit and the trace of G;
* the force bias as the derivative of the log overlap (Eq. fb).
"""

import itertools

import numpy as np
import pytest
import scipy.linalg

from oracle import afqmc_oracle as orc
from paper_2209_04015_amd import inputs
from fock import FockSpace, excitation_trial


def _orbitals(N, K=4, seed=3):
    h1, L = inputs.hamiltonian(N, K, decay=3.0, seed=seed)
    C_a = inputs.orbitals(h1)
    C_b = inputs.orbitals(h1 + np.diag(np.linspace(0.0, 0.6, N)))
    return h1, L, C_a, C_b


def _walkers(C, n, W, seed, stream, scale=0.5):
    return inputs.walkers_perturbed(C[:, :n], W, scale, seed=seed, stream=stream)


def _fock_trial(fs, msd):
    return excitation_trial(fs, msd.C, msd.nel, msd.coeff, msd.exc)


@pytest.mark.parametrize("na,nb,ndet,seed", [(2, 1, 9, 1), (2, 2, 12, 2), (1, 3, 7, 3)])
def test_msd_overlap_and_green_match_fock_space(na, nb, ndet, seed):
    N = 4
    _, _, C_a, C_b = _orbitals(N, seed=seed)
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, ndet, max_rank=2, seed=seed)
    msd = orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs)
    pa = _walkers(C_a, na, 2, seed, 0)
    pb = _walkers(C_b, nb, 2, seed, 1)
    fs = FockSpace(N)
    psiT = _fock_trial(fs, msd)
    lo = orc.msd_overlap(msd, pa, pb)
    G = orc.msd_green(msd, pa, pb)
    for z in range(2):
        v = fs.determinant(pa[z], pb[z])
        ovl = np.vdot(psiT, v)
        assert np.exp(lo[z]) == pytest.approx(ovl, rel=1e-12)
        for p in range(N):
            for q in range(N):
                for s in range(2):
                    ref = np.vdot(psiT, fs.cre(s * N + p, fs.ann(s * N + q, v))) / ovl
                    assert G[z, s, p, q] == pytest.approx(ref, abs=1e-11)


def test_excitation_operators_replace_columns_in_place():
    """t_a |psi_0> equals the determinant of R23's column-replaced orbitals (pairing order kept)."""
    N, na, nb = 5, 2, 2
    _, _, C_a, C_b = _orbitals(N, seed=4)
    fs = FockSpace(N)
    for holes, parts in [((0,), (3,)), ((0, 1), (4, 2)), ((0, 1), (2, 4)), ((1,), (2,))]:
        msd = orc.OracleMSD((C_a, C_b), (na, nb), np.array([1.0]), [((holes, parts), ((), ()))])
        D = orc.msd_determinant(C_a, na, holes, parts)
        ref = fs.determinant(D, C_b[:, :nb])
        assert np.allclose(_fock_trial(fs, msd), ref, atol=1e-13)


def _complete_expansion(C, n, psi):
    """Every determinant of n orbitals of C as an excitation of C[:, :n], c = det(D^T psi)."""
    N = C.shape[0]
    ref = set(range(n))
    out = []
    for occ in itertools.combinations(range(N), n):
        holes = tuple(sorted(ref - set(occ)))
        parts = tuple(sorted(set(occ) - ref))
        D = orc.msd_determinant(C, n, holes, parts)
        out.append((holes, parts, np.linalg.det(D.T @ psi)))
    return out


def test_msd_complete_expansion_is_cauchy_binet():
    """sum over all determinants S of det(C_S^T psi) det(C_S^T phi) = det(psi^T phi) (C orthogonal)."""
    N, na, nb = 6, 3, 2
    rng = np.random.default_rng(11)
    _, _, C_a, C_b = _orbitals(N, seed=5)
    psi_a = rng.normal(size=(N, na))
    psi_b = rng.normal(size=(N, nb))
    ea = _complete_expansion(C_a, na, psi_a)
    eb = _complete_expansion(C_b, nb, psi_b)
    exc, coeff = [], []
    for (ha, qa, ca), (hb, qb, cb) in itertools.product(ea, eb):
        exc.append(((ha, qa), (hb, qb)))
        coeff.append(ca * cb)
    msd = orc.OracleMSD((C_a, C_b), (na, nb), np.array(coeff), exc)
    pa = _walkers(C_a, na, 3, 7, 0)
    pb = _walkers(C_b, nb, 3, 7, 1)
    ref = orc.log_det(np.einsum("pi,zpj->zij", psi_a, pa)) + orc.log_det(np.einsum("pi,zpj->zij", psi_b, pb))
    assert np.allclose(np.exp(orc.msd_overlap(msd, pa, pb)), np.exp(ref), rtol=1e-11)
    G = orc.msd_green(msd, pa, pb)
    assert np.allclose(G[:, 0], orc.full_green(psi_a, pa), atol=1e-11)
    assert np.allclose(G[:, 1], orc.full_green(psi_b, pb), atol=1e-11)


def test_msd_single_reference_is_the_single_determinant_trial():
    N, na, nb = 9, 3, 2
    _, _, C_a, C_b = _orbitals(N, seed=6)
    msd = orc.OracleMSD((C_a, C_b), (na, nb), np.array([0.7]), [(((), ()), ((), ()))])
    pa = _walkers(C_a, na, 4, 8, 0)
    pb = _walkers(C_b, nb, 4, 8, 1)
    _, la = orc.theta_and_logdet(C_a[:, :na], pa)
    _, lb = orc.theta_and_logdet(C_b[:, :nb], pb)
    assert np.allclose(np.exp(orc.msd_overlap(msd, pa, pb)), 0.7 * np.exp(la + lb), rtol=1e-12)
    G = orc.msd_green(msd, pa, pb)
    assert np.allclose(G[:, 0], orc.full_green(C_a[:, :na], pa), atol=1e-12)
    assert np.allclose(G[:, 1], orc.full_green(C_b[:, :nb], pb), atol=1e-12)


def test_msd_green_trace_is_the_electron_count():
    N, na, nb = 12, 4, 3
    _, _, C_a, C_b = _orbitals(N, seed=7)
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, 60, max_rank=3, seed=9)
    msd = orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs)
    G = orc.msd_green(msd, _walkers(C_a, na, 3, 9, 0), _walkers(C_b, nb, 3, 9, 1))
    tr = np.trace(G, axis1=2, axis2=3)
    assert np.allclose(tr[:, 0], na, atol=1e-11) and np.allclose(tr[:, 1], nb, atol=1e-11)


def test_msd_force_bias_is_derivative_of_log_overlap():
    """vbias_g = d/dl log <Psi_T| e^{l v_g} |phi> at l = 0 (Eq. fb; Thouless: e^{l v}|phi> = |e^{l L} phi>)."""
    N, na, nb, K = 8, 3, 2, 3
    h1, L, C_a, C_b = _orbitals(N, K=K, seed=8)
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, 25, max_rank=3, seed=10)
    msd = orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs)
    pa = _walkers(C_a, na, 2, 10, 0)
    pb = _walkers(C_b, nb, 2, 10, 1)
    vb = orc.msd_force_bias(msd, L, pa, pb)
    h = 1e-4
    for g in range(K):
        Ep = scipy.linalg.expm(h * L[g])
        Em = scipy.linalg.expm(-h * L[g])
        fd = (orc.msd_overlap(msd, Ep @ pa, Ep @ pb) - orc.msd_overlap(msd, Em @ pa, Em @ pb)) / (2 * h)
        assert np.allclose(fd, vb[:, g], rtol=1e-7, atol=1e-7)


def test_msd_expansion_format():
    """Generator output: reference first, distinct determinants, valid and paired slots."""
    N, na, nb = 10, 4, 3
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, 200, max_rank=4, seed=12)
    assert coeff[0] == 1.0 and np.all(rank[0] == 0)
    assert np.all(np.diff(np.abs(coeff[1:])) <= 0)
    keys = set()
    for a in range(len(coeff)):
        key = []
        for s, n in enumerate((na, nb)):
            k = rank[a, s]
            h, q = orbs[a, s, 0, :k], orbs[a, s, 1, :k]
            assert np.all(orbs[a, s, :, k:] == -1)
            assert np.all((h >= 0) & (h < n)) and np.all((q >= n) & (q < N))
            assert len(set(h)) == k and len(set(q)) == k and np.all(np.diff(h) > 0)
            key.append((tuple(h), tuple(sorted(q))))
        keys.add(tuple(key))
    assert len(keys) == len(coeff)


# ---------------------------------------------------------------------------
# Phaseless step under the multi-determinant trial (Sec. II.B with R23, R24)
# ---------------------------------------------------------------------------

def test_msd_propagate_with_one_reference_is_the_single_determinant_step():
    N, na, nb, K, W = 10, 3, 2, 6, 3
    h1, L, C_a, C_b = _orbitals(N, K=K, seed=15)
    ham = orc.setup(h1, L, C_a[:, :na], C_b[:, :nb], dt=0.01)
    msd = orc.OracleMSD((C_a, C_b), (na, nb), np.array([1.0]), [(((), ()), ((), ()))])
    pa = _walkers(C_a, na, W, 15, 0, scale=0.3)
    pb = _walkers(C_b, nb, W, 15, 1, scale=0.3)
    lo = orc.overlap(ham, pa, pb)
    lw = np.zeros(W)
    x = inputs.fields(W, K, 1, seed=15)[0]
    ref = orc.propagate(ham, pa, pb, lo, lw, x)
    got = orc.msd_propagate(ham, msd, pa, pb, orc.msd_overlap(msd, pa, pb), lw, x)
    for r, g in zip(ref, got):
        assert np.allclose(g, r, rtol=1e-11, atol=1e-11)


def test_msd_optimal_force_bias_cancels_first_order_field_dependence():
    """With the MSD force bias, d ln I / dx = O(dt), not O(sqrt(dt)), where the
    importance function carries the expansion's overlap (Eq. import, force bias)."""
    N, na, nb, K = 8, 2, 2, 3
    h1, L, C_a, C_b = _orbitals(N, K=K, seed=16)
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, 12, max_rank=2, seed=16)
    coeff = coeff * np.where(np.arange(len(coeff)) == 0, 1.0, 3.0)   # far from one determinant
    msd = orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs)
    pa = _walkers(C_a, na, 1, 16, 0, scale=0.3)
    pb = _walkers(C_b, nb, 1, 16, 1, scale=0.3)

    def ln_i(ham, x):
        vb = orc.msd_force_bias(msd, ham.L, pa, pb)
        xs, a = orc.shift(ham, vb, x)
        V = orc.vhs(ham, xs)
        qa = orc._b_apply(ham, V, pa)
        qb = orc._b_apply(ham, V, pb)
        return orc.msd_overlap(msd, qa, qb) - orc.msd_overlap(msd, pa, pb) + a

    grads = []
    for dt in (1e-3, 1e-5):
        ham = orc.setup(h1, L, C_a[:, :na], C_b[:, :nb], dt=dt, taylor_order=12)
        g = []
        for k in range(K):
            e = np.zeros((1, K))
            e[0, k] = 1e-3
            g.append((ln_i(ham, e) - ln_i(ham, -e))[0] / 2e-3)
        grads.append(np.linalg.norm(g))
    assert grads[0] / grads[1] > 50.0        # O(dt); O(sqrt dt) would give ~10


def test_msd_propagate_overlap_bookkeeping():
    """The returned log overlap is the expansion's overlap of the new walkers,
    and without the two-body part (L = 0) the weight follows in closed form."""
    N, na, nb, K, W = 9, 3, 2, 2, 4
    h1, _, C_a, C_b = _orbitals(N, K=K, seed=17)
    L = np.zeros((K, N, N))
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, 20, max_rank=2, seed=17)
    msd = orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs)
    ham = orc.setup(h1, L, C_a[:, :na], C_b[:, :nb], dt=0.02)
    pa = _walkers(C_a, na, W, 17, 0, scale=0.3)
    pb = _walkers(C_b, nb, W, 17, 1, scale=0.3)
    lo = orc.msd_overlap(msd, pa, pb)
    lw = np.linspace(-0.3, 0.2, W)
    na_, nb_, lo2, lw2 = orc.msd_propagate(ham, msd, pa, pb, lo, lw, np.zeros((W, K)))
    # L = 0: B = P^2 (h' = h1), a = 0, and the new walkers are P^2 phi exactly
    P2 = scipy.linalg.expm(-ham.dt * (h1 - ham.mu * np.eye(N)))
    assert np.allclose(na_, P2 @ pa, atol=1e-12) and np.allclose(nb_, P2 @ pb, atol=1e-12)
    assert np.allclose(lo2, orc.msd_overlap(msd, na_, nb_), atol=1e-12)
    d = lo2 - lo
    cos_t = np.cos(d.imag)
    expect = lw + d.real - ham.dt * (ham.mu * (na + nb) - ham.e_shift) + np.log(np.where(cos_t > 0, cos_t, np.nan))
    ok = cos_t > 0
    assert np.allclose(lw2[ok], expect[ok], atol=1e-12) and np.all(lw2[~ok] == -np.inf)


# ---------------------------------------------------------------------------
# Local energy of the multi-determinant trial (Sec. III.C with R23; R25)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("na,nb,ndet,seed", [(2, 1, 9, 21), (2, 2, 12, 22), (1, 2, 6, 23)])
def test_msd_local_energy_matches_fock_space(na, nb, ndet, seed):
    """<Psi_T|H|phi> / <Psi_T|phi> with H of Eq. Habinitio written literally in
    Fock space and the trial built from the excitation operators."""
    N, K = 4, 3
    h1, L, C_a, C_b = _orbitals(N, K=K, seed=seed)
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, ndet, max_rank=2, seed=seed)
    msd = orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs)
    pa = _walkers(C_a, na, 2, seed, 0)
    pb = _walkers(C_b, nb, 2, seed, 1)
    fs = FockSpace(N)
    psiT = _fock_trial(fs, msd)
    e = orc.msd_local_energy(msd, h1, L, pa, pb)
    for z in range(2):
        v = fs.determinant(pa[z], pb[z])
        ref = np.vdot(psiT, fs.hamiltonian(h1, L, v)) / np.vdot(psiT, v)
        assert e[z].sum() == pytest.approx(ref, rel=1e-11, abs=1e-11)
        # the one-body part alone: the same Fock-space ratio with h1 only
        ref1 = np.vdot(psiT, fs.one_body(h1, v)) / np.vdot(psiT, v)
        assert e[z, 0] == pytest.approx(ref1, rel=1e-11, abs=1e-11)


def test_msd_local_energy_single_reference_is_the_single_determinant_energy():
    N, na, nb, K = 9, 3, 2, 5
    h1, L, C_a, C_b = _orbitals(N, K=K, seed=24)
    msd = orc.OracleMSD((C_a, C_b), (na, nb), np.array([-1.3]), [(((), ()), ((), ()))])
    ham = orc.setup(h1, L, C_a[:, :na], C_b[:, :nb], dt=0.01)
    pa = _walkers(C_a, na, 3, 24, 0)
    pb = _walkers(C_b, nb, 3, 24, 1)
    assert np.allclose(orc.msd_local_energy(msd, h1, L, pa, pb), orc.local_energy(ham, pa, pb),
                       rtol=1e-12, atol=1e-12)


def test_msd_local_energy_complete_expansion_is_the_determinant_energy():
    """The complete expansion of one determinant psi (c = det(D^T psi), Cauchy-Binet)
    has the local energy of psi itself as a single-determinant trial."""
    N, na, nb, K = 6, 3, 2, 4
    rng = np.random.default_rng(25)
    h1, L, C_a, C_b = _orbitals(N, K=K, seed=25)
    psi_a = rng.normal(size=(N, na))
    psi_b = rng.normal(size=(N, nb))
    ea = _complete_expansion(C_a, na, psi_a)
    eb = _complete_expansion(C_b, nb, psi_b)
    exc, coeff = [], []
    for (ha, qa, ca), (hb, qb, cb) in itertools.product(ea, eb):
        exc.append(((ha, qa), (hb, qb)))
        coeff.append(ca * cb)
    msd = orc.OracleMSD((C_a, C_b), (na, nb), np.array(coeff), exc)
    pa = _walkers(C_a, na, 3, 25, 0)
    pb = _walkers(C_b, nb, 3, 25, 1)
    ham = orc.setup(h1, L, psi_a, psi_b, dt=0.01)
    got = orc.msd_local_energy(msd, h1, L, pa, pb)
    ref = orc.local_energy(ham, pa, pb)
    # the total and the one-body part are trial-expansion invariants; the
    # split of the two-body part between EJ and EK is per determinant
    assert np.allclose(got.sum(axis=1), ref.sum(axis=1), rtol=1e-10, atol=1e-10)
    assert np.allclose(got[:, 0], ref[:, 0], rtol=1e-10, atol=1e-10)
