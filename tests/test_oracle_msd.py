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
from fock import FockSpace


def _orbitals(N, K=4, seed=3):
    h1, L = inputs.hamiltonian(N, K, decay=3.0, seed=seed)
    C_a = inputs.orbitals(h1)
    C_b = inputs.orbitals(h1 + np.diag(np.linspace(0.0, 0.6, N)))
    return h1, L, C_a, C_b


def _walkers(C, n, W, seed, stream, scale=0.5):
    return inputs.walkers_perturbed(C[:, :n], W, scale, seed=seed, stream=stream)


def _mo_cre(fs, C, off, x, v):
    """a+ of orbital x (column x of C) on the Fock vector v."""
    out = np.zeros_like(v)
    for p in range(C.shape[0]):
        if C[p, x] != 0:
            out = out + C[p, x] * fs.cre(off + p, v)
    return out


def _mo_ann(fs, C, off, x, v):
    out = np.zeros_like(v)
    for p in range(C.shape[0]):
        if C[p, x] != 0:
            out = out + C[p, x] * fs.ann(off + p, v)
    return out


def _fock_trial(fs, msd):
    """sum_a c_a t_a |psi_0>, t_a = prod_s prod_m a+_{s,q_m} a_{s,h_m} applied in Fock space."""
    N = fs.N
    psi0 = fs.determinant(msd.C[0][:, :msd.nel[0]], msd.C[1][:, :msd.nel[1]])
    out = np.zeros_like(psi0)
    for ca, spins in zip(msd.coeff, msd.exc):
        v = psi0
        for s, (holes, parts) in enumerate(spins):
            for h, q in zip(holes, parts):
                v = _mo_cre(fs, msd.C[s], s * N, q, _mo_ann(fs, msd.C[s], s * N, h, v))
        out = out + ca * v
    return out


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
