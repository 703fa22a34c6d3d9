"""Parity of the mixed-estimator calls (full Green's function, S^2, weighted
mean) with the FP64 oracle, through the C ABI.

Bars.  FP64: 1e-12 of the scale of each quantity (sums of at most N n
products).  Mixed modes (theta rounded to FP32, unit roundoff u = 2^-24,
products and sums in FP64): G_pq = sum_i PhiT_pi theta_qi is off by at most
u sum_i |PhiT_pi| |theta_qi| per element, and S^2 = ... - sum_ij X_ij Y_ji by
at most 2 u sum_ij Xt_ij Yt_ji with Xt = |theta_b|^T |PhiT_a|, Yt =
|theta_a|^T |PhiT_b|; the tests use twice these bounds, computed from the
oracle's theta.
"""

import numpy as np
import pytest

from oracle import afqmc_oracle as orc
from paper_2209_04015_amd import inputs

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
RAGGED = inputs.Config("ragged", N=52, n=11, K=150, decay=40.0, W=37, steps=3, qr_interval=1)


def _setup(name, precision, uhf):
    import torch
    from paper_2209_04015_amd import afqmc

    cfg = RAGGED if name == "ragged" else inputs.CONFIGS[name]
    h1, L = inputs.hamiltonian(cfg.N, cfg.K, cfg.decay, seed=0)
    pT_a = inputs.trial(h1, cfg.n)
    pT_b = inputs.trial(h1 + np.diag(np.linspace(0.0, 0.4, cfg.N)), max(cfg.n - 3, 1)) if uhf else pT_a
    oh = orc.setup(h1, L, pT_a, pT_b, dt=cfg.dt)
    ham = afqmc.Hamiltonian(h1, L, pT_a, pT_b, dt=cfg.dt, max_walkers=cfg.W, precision=precision)
    pa = inputs.walkers_perturbed(pT_a, cfg.W, 0.3, seed=5, stream=0)
    pb = inputs.walkers_perturbed(pT_b, cfg.W, 0.3, seed=5, stream=1)
    lo = orc.overlap(oh, pa, pb)
    w = afqmc.Walkers.from_numpy(pa, pb, lo, np.zeros(cfg.W), device="cuda")
    return cfg, oh, ham, w, pa, pb, torch


CASES = [("n20", "fp64", False), ("ragged", "fp64", True), ("ragged", "fp32", False),
         ("ragged", "fp16x3", True), ("ragged", "bf16x3", True)]


@pytest.mark.parametrize("name,precision,uhf", CASES)
def test_green_function_matches_oracle(name, precision, uhf):
    cfg, oh, ham, w, pa, pb, torch = _setup(name, precision, uhf)
    print(f"[gpu] green function {name} {precision} uhf={uhf}", flush=True)
    G = ham.green_function(w).cpu().numpy()
    for s, (pT, phi) in enumerate(((oh.phiT_a, pa), (oh.phiT_b, pb))):
        ref = orc.full_green(pT, phi)
        if precision == "fp64":
            bar = 1e-12 * np.abs(ref).max()
        else:
            th, _ = orc.theta_and_logdet(pT, phi)
            # per element: u sum_i |PhiT_pi| |theta_qi| (real and imaginary parts)
            bar = 2 * U32 * np.einsum("pi,zqi->zpq", np.abs(pT), np.abs(th.real) + np.abs(th.imag))
        assert np.all(np.abs(G[:, s] - ref) <= bar)
    ham.close()


def test_green_function_beta_block_is_zero_without_beta_electrons():
    import torch
    from paper_2209_04015_amd import afqmc

    h1, L = inputs.hamiltonian(10, 20, 5.0, seed=2)
    pT = inputs.trial(h1, 3)
    ham = afqmc.Hamiltonian(h1, L, pT, pT[:, :0], dt=0.005, max_walkers=4, precision="fp64")
    pa = inputs.walkers_perturbed(pT, 4, 0.3, seed=1, stream=0)
    w = afqmc.Walkers.from_numpy(pa, np.zeros((4, 10, 0), complex), np.zeros(4, complex), np.zeros(4),
                                 device="cuda")
    G = ham.green_function(w).cpu().numpy()
    assert np.all(G[:, 1] == 0)
    assert np.abs(G[:, 0] - orc.full_green(pT, pa)).max() < 1e-12
    s2 = ham.s2_mixed(w).cpu().numpy()
    assert np.allclose(s2, 1.5 * 2.5, atol=0)            # Ms = 3/2, nothing to subtract
    ham.close()


@pytest.mark.parametrize("name,precision,uhf", CASES)
def test_s2_matches_oracle(name, precision, uhf):
    cfg, oh, ham, w, pa, pb, torch = _setup(name, precision, uhf)
    print(f"[gpu] s2 {name} {precision} uhf={uhf}", flush=True)
    got = ham.s2_mixed(w).cpu().numpy()
    ref = orc.s2_mixed(oh, pa, pb)
    ta, _ = orc.theta_and_logdet(oh.phiT_a, pa)
    tb, _ = orc.theta_and_logdet(oh.phiT_b, pb)
    absc = lambda a: np.abs(a.real) + np.abs(a.imag)
    Xt = np.einsum("zpi,pj->zij", absc(tb), np.abs(oh.phiT_a))
    Yt = np.einsum("zpj,pi->zji", absc(ta), np.abs(oh.phiT_b))
    scale = np.einsum("zij,zji->z", Xt, Yt)
    bar = (1e-12 if precision == "fp64" else 4 * U32) * scale + 1e-13
    assert np.all(np.abs(got - ref) <= bar)
    ham.close()


def test_s2_of_trial_is_exact():
    from paper_2209_04015_amd import afqmc

    cfg = inputs.CONFIGS["n20"]
    h1, L = inputs.hamiltonian(cfg.N, cfg.K, cfg.decay, seed=0)
    pT = inputs.trial(h1, cfg.n)
    ham = afqmc.Hamiltonian(h1, L, pT, pT, dt=cfg.dt, max_walkers=3, precision="fp64")
    pa = np.repeat(pT[None].astype(np.complex128), 3, axis=0)
    w = afqmc.Walkers.from_numpy(pa, pa.copy(), np.zeros(3, complex), np.zeros(3), device="cuda")
    assert np.abs(ham.s2_mixed(w).cpu().numpy()).max() < 1e-12      # closed-shell singlet
    ham.close()


@pytest.mark.parametrize("nw,m", [(1, 1), (37, 3), (1000, 7), (2500, 2)])
def test_weighted_mean_matches_oracle(nw, m):
    import torch
    from paper_2209_04015_amd import afqmc

    h1, L = inputs.hamiltonian(8, 10, 3.0, seed=1)
    pT = inputs.trial(h1, 2)
    ham = afqmc.Hamiltonian(h1, L, pT, pT, dt=0.01, max_walkers=nw, precision="fp64")
    rng = np.random.default_rng(nw)
    lw = rng.normal(10.0, 2.0, nw)
    lw[rng.random(nw) < 0.1] = -np.inf
    if not np.isfinite(lw).any():
        lw[0] = 1.0
    v = rng.normal(size=(nw, m)) + 1j * rng.normal(size=(nw, m))
    w = afqmc.Walkers.from_numpy(np.zeros((nw, 8, 2), complex), np.zeros((nw, 8, 2), complex),
                                 np.zeros(nw, complex), lw, device="cuda")
    out = ham.weighted_mean(w, torch.as_tensor(v, device="cuda")).cpu().numpy()
    mean, lsw, live = orc.weighted_mean(lw, v)
    got = out[0:2 * m:2] + 1j * out[1:2 * m:2]
    assert np.all(np.abs(got - mean) <= 1e-13 * np.abs(v).max())
    assert abs(out[2 * m] - lsw) <= 1e-13 * abs(lsw) and out[2 * m + 1] == live
    ham.close()


@pytest.mark.parametrize("precision", ["fp64", "fp16x3"])
def test_estimators_keep_the_step_cache_valid(precision):
    """A step that reuses the cached Green's function after an estimator call on
    the same walkers equals one after no estimator call (bit for bit), and an
    estimator call on other walkers makes the next step recompute it."""
    import torch
    from paper_2209_04015_amd import afqmc

    cfg = inputs.CONFIGS["n20"]
    h1, L = inputs.hamiltonian(cfg.N, cfg.K, cfg.decay, seed=0)
    pT = inputs.trial(h1, cfg.n)
    ham = afqmc.Hamiltonian(h1, L, pT, pT, dt=0.001, max_walkers=cfg.W, precision=precision)
    pa = inputs.walkers_perturbed(pT, cfg.W, 0.05, seed=3, stream=0)
    x = torch.as_tensor(inputs.fields(cfg.W, cfg.K, 2, seed=1), device="cuda")

    def run(between):
        w = afqmc.Walkers.from_numpy(pa, pa.copy(), np.zeros(cfg.W, complex), np.zeros(cfg.W), device="cuda")
        ham.overlap(w)
        ham.step(w, x[0], reuse=False)
        between(w)
        ham.step(w, x[1], reuse=True)
        torch.cuda.synchronize()
        return w.phi_a.cpu().numpy(), w.log_w.cpu().numpy()

    a0, l0 = run(lambda w: None)
    a1, l1 = run(lambda w: ham.s2_mixed(w))
    other = afqmc.Walkers.from_numpy(pa[::-1].copy(), pa[::-1].copy(), np.zeros(cfg.W, complex),
                                     np.zeros(cfg.W), device="cuda")
    a2, l2 = run(lambda w: ham.green_function(other))
    assert np.array_equal(a0, a1) and np.array_equal(l0, l1)
    assert np.array_equal(a0, a2) and np.array_equal(l0, l2)
    ham.close()
