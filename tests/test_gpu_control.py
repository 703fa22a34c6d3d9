"""Parity of the ensemble calls (global energy, comb population control, block)
with the FP64 oracle, through the C ABI.

Bars: parent maps, walker copies and live counts bit-exact (integer and copy
work); the comb decisions are FP64 on both sides, so every case first checks
that no tooth lies within 1e-12 of the total weight of a cumulative-weight
boundary (except in exact-arithmetic cases: equal weights), where the two
summation orders could disagree.  Global energy and log weights: 1e-13
relative (a few roundings of FP64 sums of at most a few thousand terms).
"""

import numpy as np
import pytest

from oracle import afqmc_oracle as orc
from paper_2209_04015_amd import inputs

pytestmark = pytest.mark.gpu

_SMALL = {}


def _small(max_walkers=3000):
    """A tiny Hamiltonian whose handle serves the ensemble calls (walker state only)."""
    from paper_2209_04015_amd import afqmc

    if "ham" not in _SMALL:
        h1, L = inputs.hamiltonian(8, 10, 3.0, seed=1)
        phiT = inputs.trial(h1, 2)
        _SMALL["ham"] = afqmc.Hamiltonian(h1, L, phiT, phiT, dt=0.01, max_walkers=max_walkers,
                                          precision="fp64")
        _SMALL["phiT"] = phiT
    return _SMALL["ham"], _SMALL["phiT"]


def _log_weights(nw, seed, dead=0.1, nan=0.02, spread=2.0, offset=0.0):
    rng = np.random.default_rng(seed)
    lw = rng.normal(offset, spread, nw)
    lw[rng.random(nw) < dead] = -np.inf
    lw[rng.random(nw) < nan] = np.nan
    if not np.isfinite(lw).any():
        lw[0] = offset
    return lw


def _min_gap(lw, u):
    live = np.isfinite(lw)
    w = np.where(live, np.exp(np.where(live, lw, 0.0) - np.max(lw[live])), 0.0)
    C = np.cumsum(w)
    t = (np.arange(len(lw)) + u) * C[-1] / len(lw)
    return np.min(np.abs(t[:, None] - C[None, :])) / C[-1]


def _walker_state(nw, seed):
    torch = pytest.importorskip("torch")
    from paper_2209_04015_amd import afqmc

    ham, phiT = _small()
    rng = np.random.default_rng(seed)
    pa = rng.normal(size=(nw, 8, 2)) + 1j * rng.normal(size=(nw, 8, 2))
    pb = rng.normal(size=(nw, 8, 2)) + 1j * rng.normal(size=(nw, 8, 2))
    lo = rng.normal(size=nw) + 1j * rng.normal(size=nw)
    return ham, pa, pb, lo, torch, afqmc


@pytest.mark.parametrize("nw", [1, 37, 1000, 1024, 2500])
def test_global_energy_matches_oracle(nw):
    torch = pytest.importorskip("torch")
    ham, _ = _small()
    from paper_2209_04015_amd import afqmc

    lw = _log_weights(nw, seed=nw, offset=30.0)
    rng = np.random.default_rng(nw + 1)
    e = rng.normal(size=(nw, 3)) + 1j * rng.normal(size=(nw, 3))
    w = afqmc.Walkers.from_numpy(np.zeros((nw, 8, 2), complex), np.zeros((nw, 8, 2), complex),
                                 np.zeros(nw, complex), lw, device="cuda")
    print(f"[gpu] global energy nw={nw}", flush=True)
    out = ham.global_energy(w, torch.as_tensor(e, device="cuda")).cpu().numpy()
    E, lsw, live = orc.global_energy(lw, e)
    assert out[3] == live
    assert abs(complex(out[0], out[1]) - E) <= 1e-13 * np.abs(e.sum(axis=1)).max()
    assert abs(out[2] - lsw) <= 1e-13 * abs(lsw)


def test_global_energy_without_live_walkers():
    torch = pytest.importorskip("torch")
    ham, _ = _small()
    from paper_2209_04015_amd import afqmc

    nw = 5
    lw = np.array([-np.inf, np.nan, -np.inf, -np.inf, np.nan])
    w = afqmc.Walkers.from_numpy(np.zeros((nw, 8, 2), complex), np.zeros((nw, 8, 2), complex),
                                 np.zeros(nw, complex), lw, device="cuda")
    out = ham.global_energy(w, torch.ones((nw, 3), dtype=torch.complex128, device="cuda")).cpu().numpy()
    assert np.isnan(out[0]) and np.isnan(out[1]) and out[2] == -np.inf and out[3] == 0


def _run_comb(nw, lw, u, seed):
    ham, pa, pb, lo, torch, afqmc = _walker_state(nw, seed)
    w = afqmc.Walkers.from_numpy(pa, pb, lo, lw, device="cuda")
    print(f"[gpu] comb nw={nw} u={u!r}", flush=True)
    parent = ham.population_control(w, u).cpu().numpy()
    torch.cuda.synchronize()
    return parent, w, pa, pb, lo


@pytest.mark.parametrize("nw,seed", [(1, 0), (2, 1), (37, 2), (1024, 3), (1500, 4), (2500, 5)])
def test_comb_matches_oracle(nw, seed):
    lw = _log_weights(nw, seed, offset=-50.0)
    u = float(np.random.default_rng(seed + 100).random())
    assert _min_gap(lw, u) > 1e-12 or nw == 1
    parent, w, pa, pb, lo = _run_comb(nw, lw, u, seed)
    ref, nlw = orc.comb(lw, u)
    assert np.array_equal(parent, ref)
    # copies are exact
    assert np.array_equal(w.phi_a.cpu().numpy(), pa[ref])
    assert np.array_equal(w.phi_b.cpu().numpy(), pb[ref])
    assert np.array_equal(w.log_ovlp.cpu().numpy(), lo[ref])
    got_lw = w.log_w.cpu().numpy()
    assert np.all(np.abs(got_lw - nlw) <= 1e-13 * abs(nlw))


def test_comb_equal_weights_and_boundary_ties_are_identity():
    for nw, u in [(7, 0.0), (64, 0.0), (1100, 0.999)]:
        parent, w, pa, *_ = _run_comb(nw, np.full(nw, 2.5), u, seed=nw)
        assert np.array_equal(parent, np.arange(nw))
        assert np.array_equal(w.phi_a.cpu().numpy(), pa)


def test_comb_rounding_past_the_total_selects_last_live_walker():
    lw = np.array([-0.13, 0.64, 0.10, -0.54, 0.36, -np.inf])
    u = 1.0 - 2.0 ** -53
    parent, *_ = _run_comb(len(lw), lw, u, seed=3)
    ref, _ = orc.comb(lw, u)
    assert np.array_equal(parent, ref)
    assert np.bincount(parent, minlength=6)[5] == 0


def test_comb_without_live_walkers_changes_nothing():
    from paper_2209_04015_amd import afqmc

    nw = 9
    lw = np.full(nw, -np.inf)
    lw[4] = np.nan
    ham, _ = _small()
    ham.status()
    parent, w, pa, pb, lo = _run_comb(nw, lw, 0.5, seed=7)
    assert np.array_equal(parent, np.arange(nw))
    assert np.array_equal(w.phi_a.cpu().numpy(), pa)
    assert ham.status() & afqmc.STATUS_NO_LIVE


def test_comb_rejects_bad_offset():
    from paper_2209_04015_amd import afqmc

    ham, pa, pb, lo, torch, _ = _walker_state(4, 0)
    w = afqmc.Walkers.from_numpy(pa, pb, lo, np.zeros(4), device="cuda")
    for u in (1.0, -0.1, float("nan")):
        with pytest.raises(afqmc.AfqmcError):
            ham.population_control(w, u)


@pytest.mark.parametrize("precision", ["fp64", "fp16x3"])
def test_block_matches_oracle(precision):
    """n20 walkers, 4 steps (QR and energy at the last), global energy, comb.
    dt = 0.001 keeps every walker of this synthetic system alive over the block."""
    torch = pytest.importorskip("torch")
    from paper_2209_04015_amd import afqmc

    cfg = inputs.CONFIGS["n20"]
    h1, L = inputs.hamiltonian(cfg.N, cfg.K, cfg.decay, seed=0)
    phiT = inputs.trial(h1, cfg.n)
    dt = 0.001
    oh = orc.setup(h1, L, phiT, phiT, dt=dt)
    ham = afqmc.Hamiltonian(h1, L, phiT, phiT, dt=dt, max_walkers=cfg.W, precision=precision)
    W, nsteps = cfg.W, 4
    pa = inputs.walkers_perturbed(phiT, W, 0.01, seed=2, stream=0)
    pb = inputs.walkers_perturbed(phiT, W, 0.01, seed=2, stream=1)
    lo = orc.overlap(oh, pa, pb)
    lw = np.random.default_rng(3).normal(0.0, 0.5, W)
    x = inputs.fields(W, cfg.K, nsteps, seed=4)
    u = 0.3141
    ra, rb, rlo, rlw, re, rE, rpar = orc.block(oh, pa, pb, lo, lw, x, u)
    # the GPU's own pre-comb log weights: the same block without the comb (u < 0)
    # from the same start; the block is deterministic, so these are the weights
    # the comb below acts on
    w0 = afqmc.Walkers.from_numpy(pa, pb, lo, lw, device="cuda")
    print(f"[gpu] block {precision} (no comb)", flush=True)
    ham.block(w0, torch.as_tensor(x, device="cuda"), -1.0)
    lw_gpu = w0.log_w.cpu().numpy()
    w = afqmc.Walkers.from_numpy(pa, pb, lo, lw, device="cuda")
    print(f"[gpu] block {precision}", flush=True)
    e, out, parent = ham.block(w, torch.as_tensor(x, device="cuda"), u)
    e = e.cpu().numpy()
    out = out.cpu().numpy()
    parent = parent.cpu().numpy()
    S = np.abs(re).sum(axis=1)
    tol_e = 1e-11 if precision == "fp64" else 1e-4
    assert np.all(np.abs(e.sum(axis=1) - re.sum(axis=1)) <= tol_e * S)
    assert abs(complex(out[0], out[1]) - rE) <= tol_e * S.max()
    assert out[3] == W == np.count_nonzero(np.isfinite(orc.block(oh, pa, pb, lo, lw, x, None)[3]))
    # the comb decision: the same walkers selected when no tooth is near a
    # boundary of the (pre-comb) cumulative weights
    lw_steps = orc.block(oh, pa, pb, lo, lw, x, None)[3]
    gap = _min_gap(lw_steps, u)
    if gap > (1e-9 if precision == "fp64" else 1e-3):
        assert np.array_equal(parent, rpar)
        tol_phi = 1e-10 if precision == "fp64" else 1e-4
        ga = w.phi_a.cpu().numpy()
        assert np.abs(ga - ra).max() <= tol_phi * np.abs(ra).max()
        assert np.abs(w.log_w.cpu().numpy() - rlw).max() <= (1e-10 if precision == "fp64" else 1e-3)
    # whatever the gap to the oracle's weights, the GPU's parent map is the
    # comb (R17) of the GPU's own pre-comb weights, decided in FP64 on both
    # sides: exact unless a tooth lies within rounding of a boundary of those
    # weights
    assert _min_gap(lw_gpu, u) > 1e-12
    gref, glw = orc.comb(lw_gpu, u)
    assert np.array_equal(parent, gref)
    assert np.all(np.abs(w.log_w.cpu().numpy() - glw) <= 1e-13 * max(1.0, abs(glw)))
    ham.close()
