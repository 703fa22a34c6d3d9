"""Parity of the multi-determinant trial calls (afqmc_msd_overlap,
afqmc_msd_green_function) with the FP64 oracle, through the C ABI.

The oracle sums the expansion determinant by determinant (the definition);
the library goes through the generalised Wick's theorem (reference theta,
Y = C_virt^T theta, per-string determinants and adjugates).  Both are FP64.

Bar.  The two routes differ by rounding only.  The reference overlap matrix
S_0 = C_occ^T phi is inverted on both sides, so theta_0 and Y carry a
relative error of about u cond(S_0) (u = 2^-53); a string determinant of
rank k (k <= 6) and its adjugate add at most a few k^2 u on top, and the
expansion sums add one u per term relative to the sum of |terms|.  With
cond(S_0) < 1e3 for these walkers (perturbations of 0.3 around psi_0) and
u = 1.1e-16 the relative error stays below 1e-13 times a small factor; the
tests use 1e-12 of max |G| and 1e-12 relative on <Psi_T|phi>, times the
cancellation of the expansion sum_a |c_a O_a| / |sum_a c_a O_a| (computed
from the oracle's terms).  Measured on the MI355X: at most 7e-15 (overlap)
and 1e-14 (G) with cancellations up to 71.
"""

import numpy as np
import pytest

from oracle import afqmc_oracle as orc
from paper_2209_04015_amd import inputs

pytestmark = pytest.mark.gpu


def _problem(N, na, nb, ndet, max_rank, W, seed=0, uhf=True, scale=0.3):
    h1, _ = inputs.hamiltonian(N, 4, 3.0, seed=seed)
    C_a = inputs.orbitals(h1)
    C_b = inputs.orbitals(h1 + np.diag(np.linspace(0.0, 0.5, N))) if uhf else C_a
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, ndet, max_rank=max_rank, seed=seed + 1)
    pa = inputs.walkers_perturbed(C_a[:, :na], W, scale, seed=seed + 2, stream=0)
    pb = inputs.walkers_perturbed(C_b[:, :nb], W, scale, seed=seed + 2, stream=1)
    return C_a, C_b, coeff, rank, orbs, pa, pb


def _run(C_a, C_b, na, nb, coeff, rank, orbs, pa, pb, max_walkers=None):
    from paper_2209_04015_amd import afqmc

    W = pa.shape[0]
    t = afqmc.MSDTrial(C_a, C_b, na, nb, coeff, rank, orbs, max_walkers=max_walkers or W)
    w = afqmc.Walkers.from_numpy(pa, pb, device="cuda")
    lo = t.overlap(w).cpu().numpy()
    G = t.green_function(w).cpu().numpy()
    st = t.status()
    return t, lo, G, st


def _cancellation(msd, pa, pb):
    """sum_a |c_a O_a| / |sum_a c_a O_a| per walker (1 without cancellation)."""
    logs = orc._msd_log_terms(msd, pa, pb)
    terms = np.exp(logs - logs.real.max(axis=0))
    return np.abs(terms).sum(axis=0) / np.abs(terms.sum(axis=0))


def _compare(msd, lo, G, pa, pb, rtol=1e-12):
    ref_lo = orc.msd_overlap(msd, pa, pb)
    ref_G = orc.msd_green(msd, pa, pb)
    canc = _cancellation(msd, pa, pb)
    d = np.exp(lo - ref_lo) - 1.0            # relative overlap error (phase mod 2 pi)
    scale = np.abs(ref_G).max(axis=(1, 2, 3))
    err = np.abs(G - ref_G).max(axis=(1, 2, 3))
    print(f"[gpu] msd errors: overlap {np.abs(d).max():.2e}, G {(err / scale).max():.2e} of max|G|, "
          f"cancellation {canc.max():.2f}", flush=True)
    assert np.all(np.abs(d) <= rtol * canc), (np.abs(d).max(), canc.max())
    assert np.all(err <= rtol * canc * scale), (err / scale).max()


CASES = [
    # N, na, nb, ndet, max_rank, W, uhf
    (12, 4, 3, 40, 3, 5, True),
    (37, 9, 6, 300, 6, 37, True),       # ragged sizes, every rank up to 6
    (20, 5, 5, 120, 4, 16, False),      # one orbital set for both spins
    (64, 13, 11, 800, 4, 70, True),     # several workgroups of strings and walkers
]


@pytest.mark.parametrize("N,na,nb,ndet,max_rank,W,uhf", CASES)
def test_msd_overlap_and_green_match_oracle(N, na, nb, ndet, max_rank, W, uhf):
    print(f"[gpu] msd N={N} na={na} nb={nb} ndet={ndet} rank<={max_rank} W={W}", flush=True)
    C_a, C_b, coeff, rank, orbs, pa, pb = _problem(N, na, nb, ndet, max_rank, W, uhf=uhf)
    t, lo, G, st = _run(C_a, C_b, na, nb, coeff, rank, orbs, pa, pb)
    assert st == 0
    msd = orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs)
    _compare(msd, lo, G, pa, pb)
    t.close()


def test_msd_without_beta_electrons():
    N, na, nb = 15, 4, 0
    C_a, C_b, coeff, rank, orbs, pa, pb = _problem(N, na, nb, 30, 3, 6)
    print("[gpu] msd nb=0", flush=True)
    t, lo, G, st = _run(C_a, C_b, na, nb, coeff, rank, orbs, pa, pb)
    assert st == 0 and np.all(G[:, 1] == 0)
    _compare(orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs), lo, G, pa, pb)
    t.close()


def test_msd_single_reference_is_the_single_determinant_trial():
    N, na, nb, W = 30, 7, 5, 9
    C_a, C_b, _, _, _, pa, pb = _problem(N, na, nb, 2, 1, W)
    rank = np.zeros((1, 2), np.int32)
    orbs = np.full((1, 2, 2, inputs.MSD_MAX_RANK), -1, np.int32)
    print("[gpu] msd single reference", flush=True)
    t, lo, G, st = _run(C_a, C_b, na, nb, np.array([1.0]), rank, orbs, pa, pb)
    _, la = orc.theta_and_logdet(C_a[:, :na], pa)
    _, lb = orc.theta_and_logdet(C_b[:, :nb], pb)
    assert np.all(np.abs(np.exp(lo - la - lb) - 1) <= 1e-12)
    for s, (C, n, phi) in enumerate(((C_a, na, pa), (C_b, nb, pb))):
        ref = orc.full_green(C[:, :n], phi)
        assert np.abs(G[:, s] - ref).max() <= 1e-12 * np.abs(ref).max()
    t.close()


def test_msd_results_are_deterministic_and_nw_prefix_matches():
    C_a, C_b, coeff, rank, orbs, pa, pb = _problem(40, 8, 7, 400, 4, 33)
    from paper_2209_04015_amd import afqmc

    print("[gpu] msd determinism", flush=True)
    t = afqmc.MSDTrial(C_a, C_b, 8, 7, coeff, rank, orbs, max_walkers=33)
    w = afqmc.Walkers.from_numpy(pa, pb, device="cuda")
    G1 = t.green_function(w).cpu().numpy()
    l1 = t.overlap(w).cpu().numpy()
    G2 = t.green_function(w).cpu().numpy()
    l2 = t.overlap(w).cpu().numpy()
    assert np.array_equal(G1, G2) and np.array_equal(l1, l2)
    G3 = t.green_function(w, nw=10).cpu().numpy()       # smaller call on the same workspace
    assert np.array_equal(G3, G1[:10])
    t.close()


def test_msd_singular_reference_sets_status():
    """A walker with a zero orbital has a singular reference overlap matrix and a
    zero overlap with every determinant: log overlap -inf, status bit set."""
    from paper_2209_04015_amd import afqmc

    N, na, nb = 14, 3, 3
    C_a, C_b, coeff, rank, orbs, pa, pb = _problem(N, na, nb, 20, 2, 3)
    pa = pa.copy()
    pa[1, :, 0] = 0.0                               # exactly singular C_occ^T phi
    print("[gpu] msd singular reference", flush=True)
    t = afqmc.MSDTrial(C_a, C_b, na, nb, coeff, rank, orbs, max_walkers=3)
    w = afqmc.Walkers.from_numpy(pa, pb, device="cuda")
    lo = t.overlap(w).cpu().numpy()
    assert t.status() & afqmc.STATUS_SINGULAR
    assert lo[1].real == -np.inf and np.all(np.isfinite(lo[[0, 2]]))
    assert t.status() == 0                          # cleared by the read
    t.close()


def test_msd_rejects_invalid_expansions():
    from paper_2209_04015_amd import afqmc

    N, na, nb = 10, 3, 2
    C = inputs.orbitals(inputs.hamiltonian(N, 2, 3.0, seed=1)[0])
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, 10, 2, seed=3)
    bad = []
    o = orbs.copy(); r = rank.copy(); r[4, 0] = 2; o[4, 0, 0, :2] = [1, 1]; o[4, 0, 1, :2] = [5, 6]
    bad.append((r, o))                                   # repeated hole
    o = orbs.copy(); r = rank.copy(); r[5, 1] = 1; o[5, 1, 0, 0] = 0; o[5, 1, 1, 0] = 1
    bad.append((r, o))                                   # particle inside the reference
    o = orbs.copy(); r = rank.copy(); r[2, 0] = 7
    bad.append((r, o))                                   # rank above the maximum
    o = orbs.copy(); r = rank.copy(); r[3, 1] = 1; o[3, 1, 0, 0] = 0; o[3, 1, 1, 0] = N
    bad.append((r, o))                                   # particle outside the basis
    for r, o in bad:
        with pytest.raises(afqmc.AfqmcError) as e:
            afqmc.MSDTrial(C, C, na, nb, coeff, r, o, max_walkers=2)
        assert e.value.code == 1 and "determinant" in str(e.value)


def test_msd_at_n290_shape_sampled():
    """The 290-orbital, 26 + 26 electron shape with 512 walkers and 1000
    determinants, all walkers in one launch; the oracle checks a sample."""
    from paper_2209_04015_amd import afqmc
    import torch

    N, n, W, ndet = 290, 26, 512, 1000
    h1, _ = inputs.hamiltonian(N, 4, 3.0, seed=4)
    C = inputs.orbitals(h1)
    coeff, rank, orbs = inputs.msd_expansion(N, n, n, ndet, max_rank=4, seed=5)
    pa = inputs.walkers_perturbed(C[:, :n], W, 0.1, seed=6, stream=0)
    pb = inputs.walkers_perturbed(C[:, :n], W, 0.1, seed=6, stream=1)
    print("[gpu] msd n290 W=512 ndet=1000", flush=True)
    t = afqmc.MSDTrial(C, C, n, n, coeff, rank, orbs, max_walkers=W)
    w = afqmc.Walkers.from_numpy(pa, pb, device="cuda")
    lo = t.overlap(w).cpu().numpy()
    G = t.green_function(w)
    torch.cuda.synchronize()
    assert t.status() == 0
    sample = [0, 511]
    Gs = G[sample].cpu().numpy()
    del G
    msd = orc.msd_setup(C, C, n, n, coeff, rank, orbs)
    _compare(msd, lo[sample], Gs, pa[sample], pb[sample])
    t.close()


# ---------------------------------------------------------------------------
# Force bias of the multi-determinant trial (Eq. fb with the MSD G)
# ---------------------------------------------------------------------------
# Bar: vbias_g = sum_pq G_pq L_g,pq in FP64 on both sides; the GPU forms the
# packed symmetric G from theta_0 and Q (each ~1e-14 relative, as above) and
# contracts it with L.  Per (walker, g) the bar is 1e-12 times the
# cancellation of the expansion times sum_s sum_pq |G^s_pq| |L_g,pq|.

FB_CASES = [
    # N, na, nb, K, ndet, max_rank, W
    (12, 4, 3, 10, 40, 3, 5),
    (37, 9, 6, 50, 300, 6, 37),
    (64, 13, 11, 120, 500, 4, 70),
]


def _fb_problem(N, na, nb, K, ndet, max_rank, W, seed=0, precision="fp64"):
    from paper_2209_04015_amd import afqmc

    h1, L = inputs.hamiltonian(N, K, K / 5.0, seed=seed)
    C_a = inputs.orbitals(h1)
    C_b = inputs.orbitals(h1 + np.diag(np.linspace(0.0, 0.5, N)))
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, ndet, max_rank=max_rank, seed=seed + 1)
    pa = inputs.walkers_perturbed(C_a[:, :na], W, 0.3, seed=seed + 2, stream=0)
    pb = inputs.walkers_perturbed(C_b[:, :nb], W, 0.3, seed=seed + 2, stream=1)
    ham = afqmc.Hamiltonian(h1, L, C_a[:, :na], C_b[:, :nb], dt=0.005, max_walkers=W, precision=precision)
    t = afqmc.MSDTrial(C_a, C_b, na, nb, coeff, rank, orbs, max_walkers=W)
    return h1, L, C_a, C_b, coeff, rank, orbs, pa, pb, ham, t


def _fb_compare(msd, L, vb, pa, pb, rtol=1e-12):
    ref = orc.msd_force_bias(msd, L, pa, pb)
    G = orc.msd_green(msd, pa, pb)
    scale = np.einsum("zspq,gpq->zg", np.abs(G), np.abs(L))
    canc = _cancellation(msd, pa, pb)
    err = np.abs(vb - ref)
    print(f"[gpu] msd force bias error {(err / scale).max():.2e} of sum |G||L|", flush=True)
    assert np.all(err <= rtol * canc[:, None] * scale)


@pytest.mark.parametrize("N,na,nb,K,ndet,max_rank,W", FB_CASES)
def test_msd_force_bias_matches_oracle(N, na, nb, K, ndet, max_rank, W):
    from paper_2209_04015_amd import afqmc

    print(f"[gpu] msd force bias N={N} na={na} nb={nb} K={K} ndet={ndet} W={W}", flush=True)
    h1, L, C_a, C_b, coeff, rank, orbs, pa, pb, ham, t = _fb_problem(N, na, nb, K, ndet, max_rank, W)
    w = afqmc.Walkers.from_numpy(pa, pb, device="cuda")
    vb = t.force_bias(ham, w).cpu().numpy()
    assert t.status() == 0
    _fb_compare(orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs), L, vb, pa, pb)
    t.close()
    ham.close()


@pytest.mark.parametrize("precision", ["fp64", "fp16x3"])
def test_msd_force_bias_leaves_the_hamiltonian_step_unchanged(precision):
    """The call borrows the Hamiltonian's VHS workspace (and, in FP16X3, its
    split force-bias partials); a step after it equals one without it."""
    import torch
    from paper_2209_04015_amd import afqmc

    N, na, nb, K, W = 20, 5, 4, 30, 8
    h1, L, C_a, C_b, coeff, rank, orbs, pa, pb, ham, t = _fb_problem(N, na, nb, K, 60, 3, W, seed=3,
                                                                     precision=precision)
    x = torch.as_tensor(inputs.fields(W, K, 1, seed=2)[0], device="cuda")
    print(f"[gpu] msd force bias then step ({precision})", flush=True)

    def run(between):
        w = afqmc.Walkers.from_numpy(pa, pb, device="cuda")
        ham.overlap(w)
        between(w)
        ham.step(w, x, reuse=False)
        torch.cuda.synchronize()
        return w.phi_a.cpu().numpy(), w.log_w.cpu().numpy()

    a0, l0 = run(lambda w: None)
    a1, l1 = run(lambda w: t.force_bias(ham, w))
    assert np.array_equal(a0, a1) and np.array_equal(l0, l1)
    t.close()
    ham.close()


@pytest.mark.parametrize("precision", ["fp64", "fp16x3"])
def test_msd_force_bias_checks_the_hamiltonian(precision):
    """A Hamiltonian of another orbital count, or fewer walkers than asked
    for, is refused with AFQMC_EINVAL before any work."""
    from paper_2209_04015_amd import afqmc

    N, na, nb, K = 12, 3, 3, 8
    h1, L = inputs.hamiltonian(N, K, 2.0, seed=1)
    C = inputs.orbitals(h1)
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, 10, 2, seed=2)
    h1b, Lb = inputs.hamiltonian(N + 1, K, 2.0, seed=1)
    Cb = inputs.orbitals(h1b)
    other = afqmc.Hamiltonian(h1b, Lb, Cb[:, :na], Cb[:, :nb], dt=0.005, max_walkers=4, precision=precision)
    small = afqmc.Hamiltonian(h1, L, C[:, :na], C[:, :nb], dt=0.005, max_walkers=1, precision=precision)
    t = afqmc.MSDTrial(C, C, na, nb, coeff, rank, orbs, max_walkers=2)
    w = afqmc.Walkers.from_numpy(inputs.walkers_perturbed(C[:, :na], 2, 0.2, seed=1),
                                 inputs.walkers_perturbed(C[:, :nb], 2, 0.2, seed=1, stream=1), device="cuda")
    for ham in (other, small):
        with pytest.raises(afqmc.AfqmcError) as e:
            t.force_bias(ham, w)
        assert e.value.code == 1
    t.close()
    other.close()
    small.close()


@pytest.mark.parametrize("precision", ["fp64", "fp16x3"])
def test_msd_force_bias_at_n290_shape_sampled(precision):
    """290 orbitals, 26 + 26 electrons, K = 2900, 512 walkers and 300
    determinants in one call; the oracle checks two walkers."""
    from paper_2209_04015_amd import afqmc

    cfg = inputs.CONFIGS["n290"]
    N, n, W, ndet = cfg.N, cfg.n, cfg.W, 300
    h1, L = inputs.hamiltonian(N, cfg.K, cfg.decay, seed=0)
    C = inputs.orbitals(h1)
    coeff, rank, orbs = inputs.msd_expansion(N, n, n, ndet, max_rank=4, seed=5)
    pa = inputs.walkers_perturbed(C[:, :n], W, 0.1, seed=6, stream=0)
    pb = inputs.walkers_perturbed(C[:, :n], W, 0.1, seed=6, stream=1)
    print(f"[gpu] msd force bias n290 W=512 ndet=300 {precision}", flush=True)
    ham = afqmc.Hamiltonian(h1, L, C[:, :n], C[:, :n], dt=cfg.dt, max_walkers=W, precision=precision)
    t = afqmc.MSDTrial(C, C, n, n, coeff, rank, orbs, max_walkers=W)
    w = afqmc.Walkers.from_numpy(pa, pb, device="cuda")
    vb = t.force_bias(ham, w).cpu().numpy()
    assert t.status() == 0
    sample = [0, 511]
    msd = orc.msd_setup(C, C, n, n, coeff, rank, orbs)
    rtol = 1e-12 if precision == "fp64" else 4 * 2.0 ** -24 * np.sqrt(N * (N + 1) // 2)
    _fb_compare(msd, L, vb[sample], pa[sample], pb[sample], rtol=rtol)
    t.close()
    ham.close()


# ---------------------------------------------------------------------------
# Phaseless step under the multi-determinant trial (Sec. II.B)
# ---------------------------------------------------------------------------
# Bars as for the single-determinant step in FP64 (the same propagator
# kernels; the force bias and overlap add errors of ~1e-15 relative):
# orbitals 1e-11 of max|phi|, log overlap and log weight 1e-10 absolute.

def _assert_step(w, ref, tol_phi=1e-11, tol_log=1e-10):
    na, nb, lo, lw = ref
    for g, r in ((w.phi_a.cpu().numpy(), na), (w.phi_b.cpu().numpy(), nb)):
        scale = np.abs(r).reshape(r.shape[0], -1).max(axis=1)
        err = np.abs(g - r).reshape(r.shape[0], -1).max(axis=1)
        print(f"[gpu] msd step: max rel phi err {(err / scale).max():.3e}", flush=True)
        assert np.all(err <= tol_phi * scale)
    glo, glw = w.log_ovlp.cpu().numpy(), w.log_w.cpu().numpy()
    assert np.abs(glo.real - lo.real).max() < tol_log
    assert np.abs(np.exp(1j * (glo.imag - lo.imag)) - 1).max() < tol_log
    live = np.isfinite(lw)
    assert np.array_equal(np.isfinite(glw), live)
    assert np.abs(glw[live] - lw[live]).max(initial=0.0) < tol_log


@pytest.mark.parametrize("N,na,nb,K,ndet,max_rank,W", FB_CASES[:2])
def test_msd_propagate_matches_oracle(N, na, nb, K, ndet, max_rank, W):
    import torch
    from paper_2209_04015_amd import afqmc

    print(f"[gpu] msd step N={N} na={na} nb={nb} K={K} ndet={ndet} W={W}", flush=True)
    h1, L, C_a, C_b, coeff, rank, orbs, pa, pb, ham, t = _fb_problem(N, na, nb, K, ndet, max_rank, W)
    msd = orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs)
    oh = orc.setup(h1, L, C_a[:, :na], C_b[:, :nb], dt=0.005)
    x = inputs.fields(W, K, 2, seed=4)
    lw0 = np.linspace(-0.5, 0.5, W)
    w = afqmc.Walkers.from_numpy(pa, pb, None, lw0, device="cuda")
    t.overlap(w, out=w.log_ovlp)
    t.propagate(ham, w, torch.as_tensor(x[0], device="cuda"))
    ref = orc.msd_propagate(oh, msd, pa, pb, orc.msd_overlap(msd, pa, pb), lw0, x[0])
    _assert_step(w, ref)
    # re-orthogonalise, then a second step from the oracle's own first step
    ham.orthogonalise(w)
    qa, qb, lo = orc.orthogonalise(ref[0], ref[1], ref[2])
    t.propagate(ham, w, torch.as_tensor(x[1], device="cuda"))
    ref2 = orc.msd_propagate(oh, msd, qa, qb, lo, ref[3], x[1])
    _assert_step(w, ref2, tol_phi=1e-10, tol_log=1e-9)
    assert t.status() == 0
    t.close()
    ham.close()


def test_msd_propagate_with_one_reference_equals_the_single_determinant_step():
    """An expansion of the reference alone (c = 1) gives the Hamiltonian's own
    step when the Hamiltonian's trial is that reference."""
    import torch
    from paper_2209_04015_amd import afqmc

    N, na, nb, K, W = 30, 7, 6, 40, 16
    h1, L = inputs.hamiltonian(N, K, K / 5.0, seed=9)
    C = inputs.orbitals(h1)
    pa = inputs.walkers_perturbed(C[:, :na], W, 0.3, seed=9, stream=0)
    pb = inputs.walkers_perturbed(C[:, :nb], W, 0.3, seed=9, stream=1)
    ham = afqmc.Hamiltonian(h1, L, C[:, :na], C[:, :nb], dt=0.005, max_walkers=W, precision="fp64")
    t = afqmc.MSDTrial(C, C, na, nb, np.array([1.0]), np.zeros((1, 2), np.int32),
                       np.full((1, 2, 2, inputs.MSD_MAX_RANK), -1, np.int32), max_walkers=W)
    x = torch.as_tensor(inputs.fields(W, K, 1, seed=9)[0], device="cuda")
    print("[gpu] msd step with one reference", flush=True)
    w1 = afqmc.Walkers.from_numpy(pa, pb, device="cuda")
    ham.overlap(w1)
    ham.propagate(w1, x)
    w2 = afqmc.Walkers.from_numpy(pa, pb, device="cuda")
    t.overlap(w2, out=w2.log_ovlp)
    t.propagate(ham, w2, x)
    for a, b in ((w1.phi_a, w2.phi_a), (w1.phi_b, w2.phi_b)):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.abs(a - b).max() <= 1e-11 * np.abs(a).max()
    l1, l2 = w1.log_w.cpu().numpy(), w2.log_w.cpu().numpy()
    live = np.isfinite(l1)                          # the phaseless projection discards the same walkers
    assert np.array_equal(live, np.isfinite(l2)) and live.any()
    assert np.abs(l1[live] - l2[live]).max() < 1e-10
    d = w1.log_ovlp.cpu().numpy() - w2.log_ovlp.cpu().numpy()
    assert np.abs(d.real).max() < 1e-10 and np.abs(np.exp(1j * d.imag) - 1).max() < 1e-10
    t.close()
    ham.close()


# Mixed paths (FP32 packed L): the packed symmetric G is rounded to FP32
# (u = 2^-24) and the contraction over the c = N (N + 1) / 2 pairs accumulates
# in FP32 on the matrix cores, so the bar is 4 u sqrt(c) times the
# magnitude scale sum |G| |L| (the single-determinant FP32 force bias uses
# 4 u sqrt(c) with its own contraction length).  FP16X3 splits G (per walker
# row) and L (per Cholesky vector) into fp16 hi + lo, 22 significant bits
# down to 2^-16 of each row's maximum, every hi x hi, hi x lo, lo x hi
# product exact in FP32, the dropped lo x lo below 2^-22 of |G||L|: the same
# FP32 accumulation bar.  The step takes the FP32 single-determinant bars:
# orbitals 1e-4 of max|phi|, logs 1e-3.

@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3"])
def test_msd_force_bias_on_the_fp32_packed_l(precision):
    from paper_2209_04015_amd import afqmc

    N, na, nb, K, ndet, max_rank, W = FB_CASES[1]
    print(f"[gpu] msd force bias {precision} N={N} K={K}", flush=True)
    h1, L, C_a, C_b, coeff, rank, orbs, pa, pb, ham, t = _fb_problem(N, na, nb, K, ndet, max_rank, W,
                                                                     precision=precision)
    w = afqmc.Walkers.from_numpy(pa, pb, device="cuda")
    vb = t.force_bias(ham, w).cpu().numpy()
    c = N * (N + 1) // 2
    _fb_compare(orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs), L, vb, pa, pb,
                rtol=4 * 2.0 ** -24 * np.sqrt(c))
    t.close()
    ham.close()


@pytest.mark.parametrize("precision", ["fp32", "fp16x3"])
def test_msd_propagate_on_the_mixed_paths(precision):
    import torch
    from paper_2209_04015_amd import afqmc

    N, na, nb, K, ndet, max_rank, W = FB_CASES[1]
    print(f"[gpu] msd step {precision}", flush=True)
    h1, L, C_a, C_b, coeff, rank, orbs, pa, pb, ham, t = _fb_problem(N, na, nb, K, ndet, max_rank, W,
                                                                     precision=precision)
    msd = orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs)
    oh = orc.setup(h1, L, C_a[:, :na], C_b[:, :nb], dt=0.005)
    x = inputs.fields(W, K, 1, seed=4)[0]
    lw0 = np.zeros(W)
    w = afqmc.Walkers.from_numpy(pa, pb, None, lw0, device="cuda")
    t.overlap(w, out=w.log_ovlp)
    t.propagate(ham, w, torch.as_tensor(x, device="cuda"))
    ref = orc.msd_propagate(oh, msd, pa, pb, orc.msd_overlap(msd, pa, pb), lw0, x)
    _assert_step(w, ref, tol_phi=1e-4, tol_log=1e-3)
    t.close()
    ham.close()


# ---------------------------------------------------------------------------
# Local energy against the expansion (afqmc_msd_local_energy): the library
# takes the generalised Wick route (Gram matrices of the active blocks over
# the Cholesky index, per-string and per-determinant contractions); the
# oracle evaluates sum_a c_a O_a E_L(D_a) / sum_a c_a O_a determinant by
# determinant.  Both FP64.  Bar: 1e-11 of S = |E1| + |EJ| + |EK| per walker,
# times the expansion's cancellation (the terms are inverted determinants
# and products of Cholesky contractions: a few hundred roundings of
# relative size u = 1.1e-16, amplified by cond(S_0) and by the cancellation
# of sum_a c_a O_a).  Measured on the MI355X: at most 1.3e-13 of S
# (cancellation 77); 2e-15 at the n290 shape.
# ---------------------------------------------------------------------------
ENERGY_CASES = [
    # N, na, nb, K, ndet, max_rank, W, uhf, active
    (12, 4, 3, 10, 40, 3, 5, True, None),
    (20, 5, 5, 30, 120, 4, 16, False, None),
    (37, 9, 6, 25, 200, 4, 11, True, (6, 8)),        # ragged, an active space
    (52, 11, 11, 70, 300, 4, 37, False, (8, 10)),     # several Cholesky chunks and Gram tiles
    (60, 10, 9, 40, 200, 4, 9, True, (8, 24)),        # more than 16 active particles
    (80, 20, 18, 30, 200, 3, 7, False, (10, 20)),     # more than 16 electrons and 16 particles
    (50, 20, 19, 20, 150, 3, 6, True, (18, 6)),       # more than 16 active holes (workgroup kernel)
]


def _energy_problem(N, na, nb, K, ndet, max_rank, W, uhf, active, seed=3):
    h1, L = inputs.hamiltonian(N, K, max(2.0, K / 5), seed=seed)
    C_a = inputs.orbitals(h1)
    C_b = inputs.orbitals(h1 + np.diag(np.linspace(0.0, 0.5, N))) if uhf else C_a
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, ndet, max_rank=max_rank, seed=seed + 1, active=active)
    pa = inputs.walkers_perturbed(C_a[:, :na], W, 0.3, seed=seed + 2, stream=0)
    pb = inputs.walkers_perturbed(C_b[:, :nb], W, 0.3, seed=seed + 2, stream=1)
    return h1, L, C_a, C_b, coeff, rank, orbs, pa, pb


def _energy_compare(e, ref, canc, rtol=1e-11):
    S = np.abs(ref).sum(axis=1)
    err = np.abs(e - ref).max(axis=1)
    print(f"[gpu] msd local energy: max |dE| {err.max():.3e} Ha = {(err / S).max():.2e} of S "
          f"(S up to {S.max():.3e} Ha), cancellation {canc.max():.2f}", flush=True)
    assert np.all(err <= rtol * canc * S), (err / S / canc).max()


@pytest.mark.parametrize("N,na,nb,K,ndet,max_rank,W,uhf,active", ENERGY_CASES)
def test_msd_local_energy_matches_oracle(N, na, nb, K, ndet, max_rank, W, uhf, active):
    from paper_2209_04015_amd import afqmc

    print(f"[gpu] msd local energy N={N} na={na} nb={nb} K={K} ndet={ndet} W={W} active={active}", flush=True)
    h1, L, C_a, C_b, coeff, rank, orbs, pa, pb = _energy_problem(N, na, nb, K, ndet, max_rank, W, uhf, active)
    t = afqmc.MSDTrial(C_a, C_b, na, nb, coeff, rank, orbs, max_walkers=W)
    t.set_hamiltonian(h1, L)
    w = afqmc.Walkers.from_numpy(pa, pb, device="cuda")
    e = t.local_energy(w).cpu().numpy()
    assert t.status() == 0
    msd = orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs)
    ref = orc.msd_local_energy(msd, h1, L, pa, pb)
    _energy_compare(e, ref, _cancellation(msd, pa, pb))
    # a prefix of the walkers gives the same values (passes of a few walkers)
    e5 = t.local_energy(w, nw=min(5, W)).cpu().numpy()
    assert np.array_equal(e5, e[:min(5, W)])
    t.close()


def test_msd_local_energy_without_beta_electrons():
    from paper_2209_04015_amd import afqmc

    N, na, nb, K, W = 15, 4, 0, 8, 6
    h1, L, C_a, C_b, coeff, rank, orbs, pa, pb = _energy_problem(N, na, nb, K, 30, 3, W, True, None)
    print("[gpu] msd local energy nb=0", flush=True)
    t = afqmc.MSDTrial(C_a, C_b, na, nb, coeff, rank, orbs, max_walkers=W)
    t.set_hamiltonian(h1, L)
    e = t.local_energy(afqmc.Walkers.from_numpy(pa, pb, device="cuda")).cpu().numpy()
    msd = orc.msd_setup(C_a, C_b, na, nb, coeff, rank, orbs)
    _energy_compare(e, orc.msd_local_energy(msd, h1, L, pa, pb), _cancellation(msd, pa, pb))
    t.close()


def test_msd_local_energy_single_reference_is_the_single_determinant_energy():
    from paper_2209_04015_amd import afqmc

    N, na, nb, K, W = 24, 6, 5, 20, 9
    h1, L, C_a, C_b, _, _, _, pa, pb = _energy_problem(N, na, nb, K, 2, 1, W, True, None)
    rank = np.zeros((1, 2), np.int32)
    orbs = np.full((1, 2, 2, inputs.MSD_MAX_RANK), -1, np.int32)
    print("[gpu] msd local energy, single reference", flush=True)
    t = afqmc.MSDTrial(C_a, C_b, na, nb, np.array([1.0]), rank, orbs, max_walkers=W)
    t.set_hamiltonian(h1, L)
    e = t.local_energy(afqmc.Walkers.from_numpy(pa, pb, device="cuda")).cpu().numpy()
    oh = orc.setup(h1, L, C_a[:, :na], C_b[:, :nb])
    ref = orc.local_energy(oh, pa, pb)
    _energy_compare(e, ref, np.ones(W))
    t.close()


def test_msd_local_energy_refuses_a_large_excitation_space():
    from paper_2209_04015_amd import afqmc

    N, na, nb = 120, 30, 30
    h1, L = inputs.hamiltonian(N, 4, 3.0, seed=0)
    C = inputs.orbitals(h1)
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, 3000, max_rank=3, seed=2)
    t = afqmc.MSDTrial(C, C, na, nb, coeff, rank, orbs, max_walkers=2)
    with pytest.raises(afqmc.AfqmcError, match="1024"):
        t.set_hamiltonian(h1, L)
    w = afqmc.Walkers.from_numpy(C[None, :, :na].astype(complex), C[None, :, :nb].astype(complex), device="cuda")
    with pytest.raises(afqmc.AfqmcError, match="no Hamiltonian"):
        t.local_energy(w)
    t.close()


def test_msd_local_energy_at_n290_sampled():
    """The n290 shape (N = 290, 26 + 26 electrons, K = 2900) with an expansion
    in a (32e, 32o) active space, 512 walkers in one call, two of them
    against the oracle (whose cost is one full half-rotation of L per
    determinant, so the expansion is kept to 12 determinants here)."""
    from paper_2209_04015_amd import afqmc

    cfg = inputs.CONFIGS["n290"]
    h1, L = inputs.hamiltonian(cfg.N, cfg.K, cfg.decay, seed=0)
    C = inputs.orbitals(h1)
    coeff, rank, orbs = inputs.msd_expansion(cfg.N, cfg.n, cfg.n, 12, max_rank=3, seed=5, active=(16, 16))
    pa = inputs.walkers_perturbed(C[:, :cfg.n], cfg.W, 0.2, seed=6, stream=0)
    pb = inputs.walkers_perturbed(C[:, :cfg.n], cfg.W, 0.2, seed=6, stream=1)
    print("[gpu] msd local energy n290 (512 walkers, 12 determinants)", flush=True)
    t = afqmc.MSDTrial(C, C, cfg.n, cfg.n, coeff, rank, orbs, max_walkers=cfg.W)
    t.set_hamiltonian(h1, L)
    e = t.local_energy(afqmc.Walkers.from_numpy(pa, pb, device="cuda")).cpu().numpy()
    assert t.status() == 0
    s = np.array([0, 511])
    msd = orc.msd_setup(C, C, cfg.n, cfg.n, coeff, rank, orbs)
    ref = orc.msd_local_energy(msd, h1, L, pa[s], pb[s])
    _energy_compare(e[s], ref, _cancellation(msd, pa[s], pb[s]))
    t.close()


@pytest.mark.parametrize("N,na,nb,ndet,max_rank", [(6, 3, 2, 24, 3), (8, 4, 3, 40, 4)])
def test_msd_local_energy_with_walkers_at_the_reference(N, na, nb, ndet, max_rank):
    """Walkers whose virtual rows are exactly zero in the orbital basis (C = I,
    phi = psi_0 R): Y = 0, so every excited string's determinant is exactly
    zero and the doubles enter only through the zero-determinant form of the
    quadratic terms.  Compared with <Psi_T|H|phi> / <Psi_T|phi> in Fock space
    (H written literally, the trial built from the excitation operators), the
    total and the one-body part; EJ and EK are not separately defined there."""
    from fock import FockSpace, excitation_trial

    from paper_2209_04015_amd import afqmc

    K = 4
    h1, L = inputs.hamiltonian(N, K, 3.0, seed=31)
    C = np.eye(N)
    coeff, rank, orbs = inputs.msd_expansion(N, na, nb, ndet, max_rank=max_rank, seed=32)
    assert rank.max() == max_rank
    msd = orc.msd_setup(C, C, na, nb, coeff, rank, orbs)
    rng = np.random.default_rng(33)
    pert_a = inputs.walkers_perturbed(C[:, :na], 1, 0.3, seed=34, stream=0)[0]
    pert_b = inputs.walkers_perturbed(C[:, :nb], 1, 0.3, seed=34, stream=1)[0]
    ref_a, ref_b = C[:, :na].astype(complex), C[:, :nb].astype(complex)
    mix_a = ref_a @ (rng.normal(size=(na, na)) + 1j * rng.normal(size=(na, na)) + 3 * np.eye(na))
    mix_b = ref_b @ (rng.normal(size=(nb, nb)) + 1j * rng.normal(size=(nb, nb)) + 3 * np.eye(nb))
    pa = np.stack([ref_a, ref_a, pert_a, mix_a, pert_a])
    pb = np.stack([ref_b, pert_b, ref_b, mix_b, pert_b])
    print(f"[gpu] msd local energy at the reference N={N} na={na} nb={nb} ranks<={max_rank}", flush=True)
    t = afqmc.MSDTrial(C, C, na, nb, coeff, rank, orbs, max_walkers=pa.shape[0])
    t.set_hamiltonian(h1, L)
    e = t.local_energy(afqmc.Walkers.from_numpy(pa, pb, device="cuda")).cpu().numpy()
    assert t.status() == 0
    fs = FockSpace(N)
    psiT = excitation_trial(fs, msd.C, msd.nel, msd.coeff, msd.exc)
    for z in range(pa.shape[0]):
        v = fs.determinant(pa[z], pb[z])
        ov = np.vdot(psiT, v)
        ref = np.vdot(psiT, fs.hamiltonian(h1, L, v)) / ov
        ref1 = np.vdot(psiT, fs.one_body(h1, v)) / ov
        S = np.abs(e[z]).sum() + abs(ref)
        print(f"[gpu]   walker {z}: |dE| {abs(e[z].sum() - ref):.2e}, |dE1| {abs(e[z, 0] - ref1):.2e} (S {S:.2e})",
              flush=True)
        assert abs(e[z].sum() - ref) <= 1e-12 * S
        assert abs(e[z, 0] - ref1) <= 1e-12 * S
    # the generic walker also matches the oracle part by part
    ref = orc.msd_local_energy(msd, h1, L, pa[4:], pb[4:])
    _energy_compare(e[4:], ref, _cancellation(msd, pa[4:], pb[4:]))
    t.close()
