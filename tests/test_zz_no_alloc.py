"""The allocation-free comb (afqmc_population_control_noalloc, static device
scratch, no handle) against the comb of afqmc_population_control on the same
walkers, through the C ABI: two calls in a row, the second with fewer
walkers, so the second call runs on scratch the first one left behind.

Bar: bit-exact parent maps, walker copies and log weights (the two calls run
the same kernels on the same inputs; only where the scratch lives differs),
and both agree with the oracle's comb.
"""

import numpy as np
import pytest

from oracle import afqmc_oracle as orc
from paper_2209_04015_amd import inputs

pytestmark = pytest.mark.gpu

N, NA, NB = 9, 3, 2


def _state(nw, seed):
    rng = np.random.default_rng(seed)
    pa = rng.normal(size=(nw, N, NA)) + 1j * rng.normal(size=(nw, N, NA))
    pb = rng.normal(size=(nw, N, NB)) + 1j * rng.normal(size=(nw, N, NB))
    lo = rng.normal(size=nw) + 1j * rng.normal(size=nw)
    lw = rng.normal(-20.0, 2.0, nw)
    lw[rng.random(nw) < 0.1] = -np.inf
    lw[rng.random(nw) < 0.02] = np.nan
    lw[0] = -20.0
    return pa, pb, lo, lw


def _handle():
    from paper_2209_04015_amd import afqmc

    h1, L = inputs.hamiltonian(N, 6, 3.0, seed=3)
    phiT = inputs.trial(h1, NA)
    phiTb = inputs.trial(h1, NB)
    return afqmc.Hamiltonian(h1, L, phiT, phiTb, dt=0.01, max_walkers=4000, precision="fp64")


def test_noalloc_comb_equals_the_handle_comb_twice():
    torch = pytest.importorskip("torch")
    from paper_2209_04015_amd import afqmc

    ham = _handle()
    try:
        for nw, seed in ((3001, 11), (517, 12)):
            pa, pb, lo, lw = _state(nw, seed)
            u = float(np.random.default_rng(seed + 7).random())
            print(f"[gpu] noalloc comb nw={nw} u={u!r}", flush=True)
            w_ref = afqmc.Walkers.from_numpy(pa, pb, lo, lw, device="cuda")
            w_new = afqmc.Walkers.from_numpy(pa, pb, lo, lw, device="cuda")
            p_ref = ham.population_control(w_ref, u)
            p_new = torch.full((nw,), -7, dtype=torch.int32, device="cuda")
            status = torch.zeros(1, dtype=torch.int32, device="cuda")
            afqmc.population_control_noalloc(w_new, u, parent=p_new, status=status)
            torch.cuda.synchronize()
            ref, nlw = orc.comb(lw, u)
            assert np.array_equal(p_ref.cpu().numpy(), ref)
            assert np.array_equal(p_new.cpu().numpy(), p_ref.cpu().numpy())
            for a, b in ((w_new.phi_a, w_ref.phi_a), (w_new.phi_b, w_ref.phi_b),
                         (w_new.log_ovlp, w_ref.log_ovlp), (w_new.log_w, w_ref.log_w)):
                assert torch.equal(a, b)
            assert int(status.item()) == 0
    finally:
        ham.close()


def test_noalloc_comb_without_parent_and_without_live_walkers():
    torch = pytest.importorskip("torch")
    from paper_2209_04015_amd import afqmc

    nw = 40
    pa, pb, lo, lw = _state(nw, 21)
    u = 0.25
    ref, _ = orc.comb(lw, u)
    w = afqmc.Walkers.from_numpy(pa, pb, lo, lw, device="cuda")
    afqmc.population_control_noalloc(w, u)          # parent kept in the scratch only
    torch.cuda.synchronize()
    assert np.array_equal(w.phi_a.cpu().numpy(), pa[ref])
    dead = np.full(nw, -np.inf)
    w = afqmc.Walkers.from_numpy(pa, pb, lo, dead, device="cuda")
    parent = torch.full((nw,), -1, dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    afqmc.population_control_noalloc(w, u, parent=parent, status=status)
    torch.cuda.synchronize()
    assert np.array_equal(parent.cpu().numpy(), np.arange(nw))
    assert int(status.item()) == afqmc.STATUS_NO_LIVE
    assert np.array_equal(w.phi_a.cpu().numpy(), pa)


def test_noalloc_comb_rejects_sizes_beyond_the_scratch():
    torch = pytest.importorskip("torch")
    from paper_2209_04015_amd import afqmc

    nw = 65537
    z = torch.zeros((nw, 1, 1), dtype=torch.complex128, device="cuda")
    w = afqmc.Walkers(z, z.clone(), torch.zeros(nw, dtype=torch.complex128, device="cuda"),
                      torch.zeros(nw, dtype=torch.float64, device="cuda"))
    with pytest.raises(afqmc.AfqmcError, match="65536"):
        afqmc.population_control_noalloc(w, 0.5)
    with pytest.raises(afqmc.AfqmcError, match="offset"):
        afqmc.population_control_noalloc(w, 1.0, nw=10)
