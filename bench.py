"""Throughput of the phaseless-AFQMC walker step on one MI355X.

One step = one full walker step for every walker: Green's function, force
bias, VHS, propagation (two one-body half steps around a 6-term Taylor
series), overlap ratio and phaseless weight, QR re-orthogonalisation on the
workload's schedule, and the local energy (E1, EJ, EK) of every walker.

The headline is the FP16X3 path (16-bit hi/lo split force bias, VHS and
exchange contractions on the matrix cores, and the propagation P T6(VHS) P as
one launch of split products per (walker, spin); FP64 walkers, overlaps,
solves, QR, weights and energy sums); the FP64, FP32 and
BF16X3 paths run on the same seeded inputs and are reported beside it.  The
headline pass runs without events inside the step; a second pass of the same
steps brackets every kernel phase with HIP events and gives the phase
breakdown and the rooflines (algorithmic work per phase against the peak of
the matrix-core dtype, or of HBM).  Also on the line: the oracle's CPU rate
(median of several steps), the per-walker energy error against the oracle,
the paper's direct exchange algorithm, the propagation-only and 25-step block
rates, the n100 and n200 workloads at their own sizes, the multi-determinant
trial's calls, and the uneven multi-system batch with its per-system energy
error.  Inputs are synthetic (seeded generators), resident in HBM before
timing starts.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "walker-steps/s at N=290 mixed vs FP64 on 1 GPU; energy err vs FP64 oracle"
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0, "fp16": 2500.0}   # MI355X dense matrix peaks
HBM_GBS = 8000.0                                                             # MI355X HBM3E peak
MODES = ("fp64", "fp32", "fp16x3", "bf16x3")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def exchange_flops_per_launch(cfg, W, algo):
    """Algorithmic flops of one exchange launch (one spin) for the algorithm in use."""
    N, n, K = cfg.N, cfg.n, cfg.K
    if algo == "pair":
        # pair integrals: U = V_ij Theta_i for i <= j, n (n + 1) / 2 N^2 real x complex
        # multiply-adds per walker (4 flops), then U . Theta_j: n (n + 1) / 2 N complex
        # multiply-adds (8 flops)
        P = n * (n + 1) / 2.0
        return W * (4.0 * P * N * N + 8.0 * P * N)
    # direct: T = Lh_g theta_z for every (g, z): K n^2 N real x complex multiply-adds
    # (4 flops each); the T_ij T_ji pairing adds 8 K n^2 flops per walker.
    return W * (4.0 * K * n * n * N + 8.0 * K * n * n)


def vhs_flops_per_launch(cfg, W):
    # VHS_z = i sqrt(dt) sum_g xs_zg L_g on the N (N + 1) / 2 packed pairs: complex x real
    return W * 2.0 * cfg.K * cfg.N * (cfg.N + 1)


def step_flops(cfg, algo="direct"):
    """Algorithmic flops of one walker-step (both spins), by part."""
    N, n, K = cfg.N, cfg.n, cfg.K
    return {
        "green": 2 * (8 * N * n * n + 5.3 * n ** 3 + 8 * N * n * n),
        "force_bias": 8.0 * K * N * n,
        "vhs": 2.0 * K * N * (N + 1),
        "one_body": 16.0 * N * N * n,
        "taylor": 96.0 * N * N * n,
        "exchange": 2.0 * exchange_flops_per_launch(cfg, 1, algo),
    }


BLOCK_STEPS = 25   # propagation steps per block (the paper's timing convention)


def run_gpu(cfg, h1, L, phiT, precision, steps, warmup, fields_dev, block_fields_dev, device,
            exchange="auto", sample=1, secondary=True, profile=True):
    """Times `steps` full steps (propagate, QR on the workload's schedule,
    local energy) of the workload with no events inside the step (the
    headline), then the same number of steps again with HIP events around
    every kernel phase (phase breakdown and the per-kernel launch times of the
    rooflines).  Returns the handle, walkers, energies, headline ms, phases,
    status, secondary rates and the sampled state for the oracle check."""
    import torch

    from paper_2209_04015_amd import afqmc

    W = cfg.W
    t = time.time()
    ham = afqmc.Hamiltonian(h1, L, phiT, phiT, dt=cfg.dt, max_walkers=W, precision=precision, exchange=exchange,
                            taylor_order=cfg.taylor_order)
    log(f"{cfg.name} {precision}: init {time.time() - t:.1f} s, exchange algorithm {ham.exchange}")
    pa = torch.as_tensor(np.repeat(phiT[None].astype(np.complex128), W, axis=0), device=device)
    w = afqmc.Walkers(pa, pa.clone())
    ham.overlap(w)
    e = torch.empty((W, 3), dtype=torch.complex128, device=device)
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        ham.step(w, fields_dev[i], do_qr=((i + 1) % cfg.qr_interval == 0), energy_out=e, reuse=(i > 0))
    torch.cuda.synchronize()
    log(f"{cfg.name} {precision}: warmup done")
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)

    def timed_steps(first):
        torch.cuda.synchronize()
        start.record(stream)
        for i in range(first, first + steps):
            ham.step(w, fields_dev[i], do_qr=((i + 1) % cfg.qr_interval == 0), energy_out=e, reuse=True)
        stop.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop)

    ms = timed_steps(warmup)
    status = ham.status()
    log(f"{cfg.name} {precision}: {steps} steps in {ms:.1f} ms ({ms / steps:.3f} ms/step), status {status}")
    # the oracle comparison uses the walkers and energies of the last timed step
    # (before the runs below move them)
    sample_state = (w.phi_a[:sample].cpu().numpy(), w.phi_b[:sample].cpu().numpy(), e[:sample].cpu().numpy())
    phases, ms_prof = None, None
    if profile:
        ham.profile_enable(steps * 40)
        ms_prof = timed_steps(warmup)
        phases = ham.profile_read()
        # each roofline kernel again in a pass of its own in which only its
        # phase is bracketed by events (none between the other kernels)
        iso = {}
        for ph in ROOFLINE_PHASES:
            if phases[ph][1] == 0:
                continue
            ham.profile_phases([ph])
            timed_steps(warmup)
            iso[ph] = ham.profile_read()[ph]
        ham.profile_phases(None)
        ham.profile_enable(0)
        phases["_isolated"] = iso
        log(f"{cfg.name} {precision}: profiled pass {ms_prof / steps:.3f} ms/step")
    extra = {"exchange_algorithm": ham.exchange}
    if profile:
        extra["profiled_pass_ms_per_step"] = round(ms_prof / steps, 4)
    if secondary:
        # secondary figures on the same walkers: propagation only (no QR, no
        # energy), and one block in the paper's convention (BLOCK_STEPS steps,
        # QR and energy at the last, global energy, comb)
        torch.cuda.synchronize()
        start.record(stream)
        for i in range(steps):
            ham.step(w, fields_dev[i], do_qr=False, energy_out=None, reuse=True)
        stop.record(stream)
        torch.cuda.synchronize()
        ms_prop = start.elapsed_time(stop)
        start.record(stream)
        ham.block(w, block_fields_dev, 0.5, energy_out=e, reuse=True)
        stop.record(stream)
        torch.cuda.synchronize()
        ms_block = start.elapsed_time(stop)
        log(f"{cfg.name} {precision}: propagation only {ms_prop / steps:.2f} ms/step; block of {BLOCK_STEPS} "
            f"steps {ms_block:.1f} ms")
        extra.update({
            "propagation_only": {"value": round(W * steps / (ms_prop * 1e-3), 2), "unit": "walker-steps/s",
                                 "ms_per_step": round(ms_prop / steps, 4)},
            "block": {"value": round(W * BLOCK_STEPS / (ms_block * 1e-3), 2), "unit": "walker-steps/s",
                      "ms_per_block": round(ms_block, 3),
                      "definition": f"{BLOCK_STEPS} steps, QR and local energy at the last, "
                                    "global energy, comb population control"}})
    return ham, w, e, ms, phases, status, extra, sample_state


MSD_DETS = 10000


def msd_flops_per_walker(N, n):
    """Algorithmic FP64 flops per walker of the Green's function call beyond
    the determinant sums: Y = C_virt^T theta (4 N nv n), M Y (8 n^2 nv),
    Q (4 N n (n + nv)) and G = theta Q^T (8 N^2 n), per spin."""
    nv = N - n
    return 2 * (4 * N * nv * n + 8 * n * n * nv + 4 * N * n * (n + nv) + 8 * N * N * n)


MSD_ACTIVE = (16, 16)   # holes, particles per spin: the (32e, 32o) active space of the Cu2O2 trials (Sec. IV)
MSD_BLOCK_STEPS = 25    # propagation steps per energy evaluation in the paper's block timings (Sec. IV)


def msd_energy_flops_per_walker(N, n, K, S, D):
    """Algorithmic FP64 flops per walker of the expansion's local energy on
    the matrix cores: the rotated vectors against theta_0 (S rows of each of
    K + 1 blocks by 2n real columns over N, per spin) and the three Gram
    matrices (D x D over the 2K real Cholesky components)."""
    return 2 * (2 * (K + 1) * S * 2 * n * N) + 3 * 8 * D * D * K


def run_msd(cfg, h1, L, device, steps, ndet=MSD_DETS):
    """Multi-determinant trial (Sec. III.A): overlap, Green's function and
    force bias of every walker against a synthetic ndet-determinant expansion
    in a (16 holes, 16 particles per spin) active window of the eigenvector
    basis of the workload's h1, timed over `steps` calls each on the current
    stream; the expansion's local energy (Sec. III.C), and one block of 25
    steps with the energy at its end.  The force bias contracts with the
    packed L of an FP64 Hamiltonian of the same workload."""
    import torch

    from paper_2209_04015_amd import afqmc, inputs

    N, n, W, K = cfg.N, cfg.n, cfg.W, cfg.K
    t = time.time()
    C = inputs.orbitals(h1)
    coeff, rank, orbs = inputs.msd_expansion(N, n, n, ndet, max_rank=4, seed=5, active=MSD_ACTIVE)
    pa = inputs.walkers_perturbed(C[:, :n], W, 0.1, seed=6, stream=0)
    pb = inputs.walkers_perturbed(C[:, :n], W, 0.1, seed=6, stream=1)
    trial = afqmc.MSDTrial(C, C, n, n, coeff, rank, orbs, max_walkers=W)
    ham = afqmc.Hamiltonian(h1, L, C[:, :n], C[:, :n], dt=cfg.dt, max_walkers=W, precision="fp64")
    w = afqmc.Walkers.from_numpy(pa, pb, device=device)
    lo = torch.empty(W, dtype=torch.complex128, device=device)
    G = torch.empty((W, 2, N, N), dtype=torch.complex128, device=device)
    vb = torch.empty((W, K), dtype=torch.complex128, device=device)
    log(f"msd: {ndet} determinants, strings {trial.strings}, set up in {time.time() - t:.1f} s")
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)

    def timed(f):
        f()
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(steps):
            f()
        stop.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / steps

    ms_o = timed(lambda: trial.overlap(w, out=lo))
    ms_g = timed(lambda: trial.green_function(w, out=G))
    del G
    torch.cuda.empty_cache()
    ms_f = timed(lambda: trial.force_bias(ham, w, out=vb))
    # phaseless steps under the trial, re-orthogonalised every step (the
    # workload's schedule), from the expansion's overlap of these walkers
    x = torch.as_tensor(inputs.fields(W, K, 1, seed=7)[0], device=device)
    trial.overlap(w, out=w.log_ovlp)

    def step():
        trial.propagate(ham, w, x)
        ham.orthogonalise(w)

    ms_s = timed(step)
    status = trial.status() | ham.status()
    ham.close()
    # the same step on the FP32 path (FP32 packed L, FP32 VHS and Taylor products)
    ham32 = afqmc.Hamiltonian(h1, L, C[:, :n], C[:, :n], dt=cfg.dt, max_walkers=W, precision="fp32")
    trial.overlap(w, out=w.log_ovlp)

    def step32():
        trial.propagate(ham32, w, x)
        ham32.orthogonalise(w)

    ms_s32 = timed(step32)
    status |= trial.status() | ham32.status()
    ham32.close()
    torch.cuda.empty_cache()
    # the FP16X3 path (split force bias against the transposed split L, split
    # VHS build, the fused propagation)
    ham16 = afqmc.Hamiltonian(h1, L, C[:, :n], C[:, :n], dt=cfg.dt, max_walkers=W, precision="fp16x3")
    ms_f16 = timed(lambda: trial.force_bias(ham16, w, out=vb))
    trial.overlap(w, out=w.log_ovlp)

    def step16():
        trial.propagate(ham16, w, x)
        ham16.orthogonalise(w)

    ms_s16 = timed(step16)
    # the expansion's local energy (FP64), then one block: 25 steps on the
    # FP16X3 path and the energy at its end
    t = time.time()
    trial.set_hamiltonian(h1, L)
    log(f"msd: local energy set up in {time.time() - t:.1f} s")
    E = torch.empty((W, 3), dtype=torch.complex128, device=device)
    esteps = max(1, min(steps, 5))
    trial.local_energy(w, out=E)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(esteps):
        trial.local_energy(w, out=E)
    stop.record(stream)
    torch.cuda.synchronize()
    ms_e = start.elapsed_time(stop) / esteps
    e_finite = bool(torch.isfinite(torch.view_as_real(E)).all())
    start.record(stream)
    for _ in range(MSD_BLOCK_STEPS):
        step16()
    trial.local_energy(w, out=E)
    stop.record(stream)
    torch.cuda.synchronize()
    ms_block = start.elapsed_time(stop)
    status |= trial.status() | ham16.status()
    ham16.close()
    trial.close()
    del E
    torch.cuda.empty_cache()
    S = n + MSD_ACTIVE[1]
    D = MSD_ACTIVE[0] * MSD_ACTIVE[1]
    e_gflop = W * msd_energy_flops_per_walker(N, n, K, S, D) / 1e9
    log(f"msd: overlap {ms_o:.3f} ms, Green's function {ms_g:.3f} ms, force bias {ms_f:.3f} ms per call, "
        f"step {ms_s:.3f} ms (FP32 path {ms_s32:.3f} ms; FP16X3 force bias {ms_f16:.3f} ms, step {ms_s16:.3f} ms), "
        f"local energy {ms_e:.3f} ms "
        f"({e_gflop / ms_e:.1f} TFLOP/s on the dense parts), block of {MSD_BLOCK_STEPS} steps + energy "
        f"{ms_block:.1f} ms, status {status}")
    gbytes = W * 2 * N * N * 16
    npk = N * (N + 1) // 2
    return {"workload": f"multi-determinant trial: {ndet} determinants (ranks <= 4 per spin) in a "
                        f"({2 * MSD_ACTIVE[0]}e, {MSD_ACTIVE[0] + MSD_ACTIVE[1]}o) active space "
                        f"({MSD_ACTIVE[0]} holes, {MSD_ACTIVE[1]} particles per spin) of the eigenvector "
                        f"basis of the {cfg.name} h1, {N} orbitals, na=nb={n}, {W} walkers, K={K}, FP64",
            "determinants": ndet, "strings_per_spin": list(trial.strings), "walkers": W,
            "overlap": {"value": round(W * ndet / (ms_o * 1e-3), 1), "unit": "walker-determinants/s",
                        "ms_per_call": round(ms_o, 4)},
            "green_function": {"value": round(W * ndet / (ms_g * 1e-3), 1), "unit": "walker-determinants/s",
                               "ms_per_call": round(ms_g, 4),
                               "G_written_GB": round(gbytes / 1e9, 3),
                               "G_write_bound_ms": round(gbytes / 8e12 * 1e3, 4),
                               "dense_fp64_gflop": round(W * msd_flops_per_walker(N, n) / 1e9, 2)},
            "force_bias": {"value": round(W / (ms_f * 1e-3), 1), "unit": "walkers/s",
                           "ms_per_call": round(ms_f, 4),
                           "contraction_fp64_gflop": round(2 * 2 * W * npk * K / 1e9, 1)},
            "step": {"value": round(W / (ms_s * 1e-3), 1), "unit": "walker-steps/s",
                     "ms_per_step": round(ms_s, 4),
                     "definition": "afqmc_msd_propagate (force bias, VHS, P T6(VHS) P, the expansion's overlap "
                                   "ratio, weights) + QR; no local energy; FP64 path"},
            "step_fp32": {"value": round(W / (ms_s32 * 1e-3), 1), "unit": "walker-steps/s",
                          "ms_per_step": round(ms_s32, 4),
                          "definition": "the same on the FP32 path (FP32 packed L, VHS and Taylor products)"},
            "force_bias_fp16x3": {"value": round(W / (ms_f16 * 1e-3), 1), "unit": "walkers/s",
                                  "ms_per_call": round(ms_f16, 4),
                                  "split_tflops": round(2 * 2 * W * npk * K / 1e9 / ms_f16, 1)},
            "step_fp16x3": {"value": round(W / (ms_s16 * 1e-3), 1), "unit": "walker-steps/s",
                            "ms_per_step": round(ms_s16, 4),
                            "definition": "the same on the FP16X3 path (split force bias against the transposed "
                                          "split L, split VHS build, fused propagation)"},
            "local_energy": {"value": round(W / (ms_e * 1e-3), 1), "unit": "walkers/s",
                             "ms_per_call": round(ms_e, 3), "finite": e_finite,
                             "dense_fp64_gflop": round(e_gflop, 1),
                             "dense_fp64_tflops": round(e_gflop / ms_e, 2),
                             "definition": "afqmc_msd_local_energy: E1, EJ, EK of every walker against the "
                                           "whole expansion (generalised Wick, Gram matrices over the "
                                           "Cholesky index), FP64"},
            "block": {"ms_per_block": round(ms_block, 2),
                      "value": round(W * MSD_BLOCK_STEPS / (ms_block * 1e-3), 1), "unit": "walker-steps/s",
                      "definition": f"{MSD_BLOCK_STEPS} steps on the FP16X3 path (afqmc_msd_propagate + QR) and "
                                    "the expansion's local energy at the end"},
            "status": status}


def run_batch(device, steps, precision="fp16x3"):
    """The uneven multi-system workload (8 systems, N = 40 .. 200) advanced
    together by one hipGraph launch per step (autotuned exchange and VHS tile
    shapes and exchange tile order; the same graph with the default tiles for
    comparison),
    QR and local energy every step; and the same steps taken system after
    system with afqmc_step on one stream, for comparison."""
    import torch

    from paper_2209_04015_amd import afqmc, inputs

    from oracle import afqmc_oracle as orc

    t = time.time()
    systems = inputs.uneven_batch()
    hams, ws, fs, es, starts, defs = [], [], [], [], [], []
    for (N, n, K, decay, W, seed) in systems:
        h1, L = inputs.hamiltonian(N, K, decay, seed=seed)
        phiT = inputs.trial(h1, n)
        defs.append((h1, L, phiT))
        ham = afqmc.Hamiltonian(h1, L, phiT, phiT, dt=0.005, max_walkers=W, precision=precision)
        pa = np.repeat(phiT[None].astype(np.complex128), W, axis=0)
        w = afqmc.Walkers.from_numpy(pa, pa.copy(), device=device)
        ham.overlap(w)
        hams.append(ham)
        ws.append(w)
        starts.append((w.phi_a.clone(), w.phi_b.clone(), w.log_ovlp.clone(), w.log_w.clone()))
        fs.append(torch.as_tensor(inputs.fields(W, K, steps, seed=seed), device=device))
        es.append(torch.empty((steps, W, 3), dtype=torch.complex128, device=device))
    wtot = sum(s[4] for s in systems)
    log(f"batch: {len(systems)} systems, {wtot} walkers, set up in {time.time() - t:.1f} s")
    b = afqmc.Batch(hams, ws, use_graph=True)
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)

    def graph_ms():
        for w, (a0, b0, l0, lw0) in zip(ws, starts):
            w.phi_a.copy_(a0)
            w.phi_b.copy_(b0)
            w.log_ovlp.copy_(l0)
            w.log_w.copy_(lw0)
        b.step(fs, es, do_qr=True)          # capture + first replays (untimed)
        torch.cuda.synchronize()
        start.record(stream)
        b.step(fs, es, do_qr=True)
        stop.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop)

    ms_default = graph_ms()             # built-in tiles (80 walkers per exchange and VHS tile)
    b.autotune()
    tunings = [h.tuning() for h in hams]
    ms_b = graph_ms()
    st_b = sum(h.status() for h in hams)
    b.close()
    # per-system energy error: the last step's local energies of sampled
    # walkers against the oracle's local energy of the same walkers
    per_sys = []
    for (N, n, K, decay, W, seed), (h1, L, phiT), w, e in zip(systems, defs, ws, es):
        k = min(4, W)
        oh = orc.setup(h1, L, phiT, phiT, dt=0.005)
        v = energy_errors(oh, {"s": (w.phi_a[:k].cpu().numpy(), w.phi_b[:k].cpu().numpy(),
                                     e[-1, :k].cpu().numpy())})["s"]
        per_sys.append({"N": N, "walkers": W, **v})
    log("batch energy errors (of S): " + ", ".join(f"N{p['N']} {p['max_rel_to_S']:.1e}" for p in per_sys))
    # the same steps system after system (eager, one stream), from the same start
    for w, (a0, b0, l0, lw0) in zip(ws, starts):
        w.phi_a.copy_(a0)
        w.phi_b.copy_(b0)
        w.log_ovlp.copy_(l0)
        w.log_w.copy_(lw0)

    def seq():
        for ham, w, f, e in zip(hams, ws, fs, es):
            for k in range(steps):
                ham.step(w, f[k], do_qr=True, energy_out=e[k], reuse=k > 0)

    seq()
    torch.cuda.synchronize()
    start.record(stream)
    seq()
    stop.record(stream)
    torch.cuda.synchronize()
    ms_s = start.elapsed_time(stop)
    for h in hams:
        h.close()
    torch.cuda.empty_cache()
    log(f"batch: {steps} steps in {ms_b:.1f} ms (graph, autotuned tiles; {ms_default:.1f} ms with the default "
        f"tiles) vs {ms_s:.1f} ms (systems in turn)")
    return {"workload": "uneven multi-system batch: 8 systems, N = 40, 60, ..., 160, 200, n = N/5, K = 4N, "
                        f"walkers {[s[4] for s in systems]}, {precision}, QR and local energy every step, "
                        "one hipGraph launch per step, autotuned exchange and VHS tile shapes and exchange "
                        "tile order",
            "value": round(wtot * steps / (ms_b * 1e-3), 1), "unit": "walker-steps/s",
            "ms_per_step": round(ms_b / steps, 4), "status": st_b,
            "energy_error_vs_fp64_oracle": per_sys,
            "tuning": [{"N": sy[0], "exchange_tile": list(t["exchange_tile"]), "exchange_group": t["exchange_group"],
                        "vhs_tile": list(t["vhs_tile"])} for sy, t in zip(systems, tunings)],
            "default_tiles": {"value": round(wtot * steps / (ms_default * 1e-3), 1), "unit": "walker-steps/s",
                              "ms_per_step": round(ms_default / steps, 4)},
            "systems_in_turn": {"value": round(wtot * steps / (ms_s * 1e-3), 1), "unit": "walker-steps/s",
                                "ms_per_step": round(ms_s / steps, 4)}}


# Sources that define each roofline kernel: its HBM traffic figure (from the
# rocprofv3 counter summaries under profiles/) is used only while these are
# unchanged since the counters were taken.
KERNEL_SOURCES = {
    "exchange_split_kernel": ["split_kernels.hip", "split_tile.h", "exchange_tri.h", "tile_order.h", "common.h"],
    "exchange_kernel": ["step_kernels.hip", "mfma_tile.h", "exchange_epilogue.h", "tile_order.h", "common.h"],
    "exchange_pair_split_kernel": ["split_kernels.hip", "split_tile.h", "exchange_pair.h", "tile_order.h",
                                   "common.h"],
    "exchange_pair_kernel": ["step_kernels.hip", "mfma_tile.h", "exchange_pair.h", "tile_order.h", "common.h"],
    "vhs_split_kernel": ["split_kernels.hip", "split_tile.h", "tile_order.h", "common.h"],
    "vhs_kernel": ["step_kernels.hip", "mfma_tile.h", "tile_order.h", "common.h"],
    "prop_fused_kernel": ["prop_kernels.hip", "split_tile.h", "common.h"],
}


def kernel_sources_sha256(kernel):
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2209_04015_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def hbm_traffic(kernel, instance, workload):
    """HBM bytes per launch of `instance` on `workload` from the committed counter
    summaries (lines 'hbm-traffic <instance> <workload> bytes_per_launch=...
    sources_sha256=...'), or None if absent or the kernel changed since."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    sha = kernel_sources_sha256(kernel)
    for name in sorted(os.listdir(pdir)):
        if not name.endswith("_hbm.md"):
            continue
        with open(os.path.join(pdir, name)) as fh:
            for line in fh:
                f = line.strip().strip("`").split()
                # instance names are written without spaces
                if len(f) < 4 or f[0] != "hbm-traffic" or f[1] != instance.replace(" ", "") or f[2] != workload:
                    continue
                kv = dict(x.split("=", 1) for x in f[3:] if "=" in x)
                if kv.get("sources_sha256") == sha:
                    return int(kv["bytes_per_launch"])
    return None


def mfma_busy(kernel, instance, workload):
    """MFMA-busy share of a kernel from the committed counter summaries (lines
    'mfma-busy <instance> <workload> frac=... sources_sha256=...'), or None."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    sha = kernel_sources_sha256(kernel)
    for name in sorted(os.listdir(pdir)):
        if not name.endswith("_hbm.md"):
            continue
        with open(os.path.join(pdir, name)) as fh:
            for line in fh:
                f = line.strip().strip("`").split()
                if len(f) < 4 or f[0] != "mfma-busy" or f[1] != instance.replace(" ", "") or f[2] != workload:
                    continue
                kv = dict(x.split("=", 1) for x in f[3:] if "=" in x)
                if kv.get("sources_sha256") == sha:
                    return float(kv["frac"])
    return None


# kernel (and its template instance in the rocprofv3 summaries) per phase,
# precision and exchange algorithm
def _kernel_of(phase, precision, algo):
    split = precision in ("fp16x3", "bf16x3")
    H = {"fp16x3": "HalfF16", "bf16x3": "HalfBF16"}.get(precision)
    T = {"fp32": "float", "fp64": "double", "bf16x3": "float", "fp16x3": "float"}[precision]
    if phase == "exchange":
        base = ("exchange_pair" if algo == "pair" else "exchange") + ("_split_kernel" if split else "_kernel")
        if split and algo == "pair":   # the default (wide) walker tile of the split pair kernel
            return base, f"{base}<{H},SplitCfgT<128,128,3>>"
        return base, f"{base}<{H if split else T}>"
    if phase == "propagate":
        return "prop_fused_kernel", "prop_fused_kernel<4>"
    if phase == "vhs":
        if precision == "fp16x3":   # the VHS runs on split operands only in FP16X3 (default wide tile)
            return "vhs_split_kernel", "vhs_split_kernel<HalfF16,SplitCfgT<128,128,3>>"
        # tile template arguments of the FP32 / FP64 VHS instances (step_kernels.hip)
        return "vhs_kernel", {"double": "vhs_kernel<double, 64, 64, 16, 2, 2>",
                              "float": "vhs_kernel<float, 64, 64, 32, 2, 2>"}[T]
    return None, None


def _mfma_dtype(phase, precision):
    """The type the matrix cores of a phase execute in (whose peak the phase is
    measured against)."""
    if precision == "fp64":
        return "fp64"
    if phase == "exchange" and precision in ("fp16x3", "bf16x3"):
        return precision[:4]
    if phase in ("vhs", "taylor", "force_bias", "propagate") and precision == "fp16x3":
        return "fp16"
    return "fp32"


def phase_work(cfg, phase, precision, algo):
    """Algorithmic work of one step's launches of a phase: (bound, amount, unit).
    Flops: a real x complex multiply-add counts 4, complex x complex 8.  Bytes:
    the arrays the phase must read and write once."""
    N, n, K, W = cfg.N, cfg.n, cfg.K, cfg.W
    ne = 2 * n                                # electrons, both spins
    ts = 8 if precision == "fp64" else 4      # bytes of the working precision
    if phase == "vhs":
        return "mfma", vhs_flops_per_launch(cfg, W), "flop"
    if phase == "exchange":
        return "mfma", 2 * exchange_flops_per_launch(cfg, W, algo), "flop"   # two spins
    if phase == "taylor":
        return "mfma", W * cfg.taylor_order * 8.0 * N * N * n * 2, "flop"
    if phase == "one_body":
        return "mfma", 2 * W * 4.0 * N * N * ne, "flop"                   # two half steps
    if phase == "propagate":   # one launch: both one-body half steps and the Taylor series
        return ("mfma", phase_work(cfg, "one_body", precision, algo)[1]
                + phase_work(cfg, "taylor", precision, algo)[1], "flop")
    if phase == "force_bias":
        return "mfma", W * 4.0 * K * N * ne, "flop"
    if phase == "green":
        return "hbm", W * N * ne * (16 + 2 * ts), "byte"                  # read phi, write theta
    if phase == "qr":
        return "hbm", 2 * W * N * ne * 16, "byte"                         # read and write phi
    return None, None, None


ROOFLINE_PHASES = ("vhs", "exchange", "propagate", "taylor", "one_body", "force_bias", "qr", "green")


def roofline_of(cfg, phases, precision, algo, phase, steps):
    """Roofline entry of one phase: algorithmic work of one step's launches /
    their measured time (from the pass in which only this phase is timed, when
    there is one), against the peak of the unit the phase runs on (matrix
    cores of the MFMA dtype, or HBM)."""
    ms, launches = phases.get("_isolated", {}).get(phase, phases[phase])
    if launches == 0:
        return None
    bound, work, unit = phase_work(cfg, phase, precision, algo)
    if bound is None:
        return None
    ms_step = ms / steps
    per_step_launches = launches / steps
    if bound == "mfma":
        dt = _mfma_dtype(phase, precision)
        peak = PEAK_TFLOPS[dt]
        achieved = work / (ms_step * 1e-3) / 1e12
        out = {"phase": phase, "bound": "mfma", "mfma_dtype": dt, "achieved": round(achieved, 2),
               "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
               "flops_per_step": work}
        if dt in ("fp16", "bf16"):
            # three 16-bit products per algorithmic multiply-add (hi/lo split):
            # the share of the matrix-core pipe the products occupy
            out["mfma_pipe_frac"] = round(3.0 * achieved / peak, 4)
    else:
        achieved = work / (ms_step * 1e-3) / 1e9
        out = {"phase": phase, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_GBS,
               "unit": "GB/s", "frac": round(achieved / HBM_GBS, 4), "bytes_per_step": work}
    kernel, instance = _kernel_of(phase, precision, algo)
    if kernel:
        out["kernel"] = kernel
        out["traffic"] = hbm_traffic(kernel, instance, cfg.name)
        busy = mfma_busy(kernel, instance, cfg.name)
        if busy is not None:
            out["mfma_busy_counter"] = busy
    out["ms_per_step"] = round(ms_step, 4)
    out["launches_per_step"] = round(per_step_launches, 2)
    out["avg_launch_ms"] = round(ms / launches, 4)
    return out


def rooflines(cfg, phases, precision, algo, steps):
    """Roofline entries of the phases, largest share of the step first (the
    first is the dominant kernel)."""
    if not phases:
        return {}
    out = {ph: roofline_of(cfg, phases, precision, algo, ph, steps) for ph in ROOFLINE_PHASES}
    order = sorted(out, key=lambda ph: -phases[ph][0])  # shares of the step from the all-phase pass
    return {ph: out[ph] for ph in order if out[ph] is not None}


def roofline(cfg, phases, precision, algo, steps):
    """The dominant kernel's roofline: of the VHS build and the exchange (the
    contractions the metric names), the one with the larger share of the step."""
    r = rooflines(cfg, phases, precision, algo, steps)
    for ph in r:
        if ph in ("vhs", "exchange"):
            return r[ph]
    return None


def host_description():
    """CPU model, BLAS library and its thread count on this host."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas, threads = None, None
    try:
        from threadpoolctl import threadpool_info

        for d in threadpool_info():
            if d.get("user_api") == "blas":
                blas = f"{d.get('internal_api')} {d.get('version')}"
                threads = d.get("num_threads")
                break
    except Exception:
        pass
    return model, blas, threads


def energy_errors(oh, states):
    """Per-walker energy error of each GPU path against the oracle's local
    energy of the same (GPU) walkers: max |dE| in Ha and relative to
    S = |E1| + |EJ| + |EK|."""
    from oracle import afqmc_oracle as orc

    out = {}
    for prec, (pa, pb, e_gpu) in states.items():
        e_ref = orc.local_energy(oh, pa, pb)
        S = np.abs(e_ref).sum(axis=1)
        err = np.abs(e_gpu.sum(axis=1) - e_ref.sum(axis=1))
        out[prec] = {"max_abs_Ha": float(err.max()), "max_rel_to_S": float((err / S).max()),
                     "walkers": int(len(err)), "E_scale_Ha": float(np.abs(e_ref.sum(axis=1)).max())}
    return out


def cpu_baseline_and_energy_error(cfg, h1, L, phiT, gpu_states, sample, x_steps):
    """The FP64 oracle: its walker-step rate on a bounded sample (the median
    of several full steps of `sample` walkers), and the per-walker energy
    error of each GPU path against it on sampled walkers."""
    from oracle import afqmc_oracle as orc

    t = time.time()
    oh = orc.setup(h1, L, phiT, phiT, dt=cfg.dt, taylor_order=cfg.taylor_order)
    log(f"oracle setup {time.time() - t:.1f} s")
    out = energy_errors(oh, gpu_states)
    for prec, v in out.items():
        log(f"energy error {cfg.name} {prec}: {v['max_abs_Ha']:.3e} Ha ({v['max_rel_to_S']:.2e} of S)")
    # timed oracle sample: consecutive full steps (propagate, QR, energy) of
    # `sample` walkers from the trial
    pa = np.repeat(phiT[None].astype(np.complex128), sample, axis=0)
    pb = pa.copy()
    lo = orc.overlap(oh, pa, pb)
    lw = np.zeros(sample)
    times = []
    for x in x_steps:
        t = time.time()
        pa, pb, lo, lw, _ = orc.step(oh, pa, pb, lo, lw, x[:sample], do_qr=True)
        times.append(time.time() - t)
    med = float(np.median(times))
    model, blas, threads = host_description()
    cpu = {"value": round(sample / med, 3), "unit": "walker-steps/s",
           "cores": threads or os.cpu_count(), "kind": "oracle",
           "sample": f"{sample} walkers x {len(times)} consecutive full steps (propagate, QR, local energy) of the "
                     f"same workload from the trial, FP64 NumPy oracle; median step {med:.2f} s "
                     f"(steps {', '.join(f'{x:.2f}' for x in times)} s); setup not timed",
           "cpu_model": model, "blas": blas, "host_cpus": os.cpu_count()}
    log(f"oracle: {sample} walkers, median step {med:.2f} s over {len(times)} steps ({model}; {blas})")
    return cpu, out


def run_config_leg(name, precisions, steps, warmup, device, sample=6):
    """Another workload at its own size (one fused step per walker per step,
    QR on its schedule, energy every step): walker-steps/s of each path and
    the per-walker energy error of its last step against the oracle."""
    import torch

    from oracle import afqmc_oracle as orc
    from paper_2209_04015_amd import inputs

    cfg = inputs.CONFIGS[name]
    h1, L = inputs.hamiltonian(cfg.N, cfg.K, cfg.decay, seed=0)
    phiT = inputs.trial(h1, cfg.n)
    fields_dev = torch.as_tensor(inputs.fields(cfg.W, cfg.K, warmup + steps, seed=0), device=device)
    res, states = {}, {}
    for prec in precisions:
        ham, w, e, ms, _, st, extra, stt = run_gpu(cfg, h1, L, phiT, prec, steps, warmup, fields_dev, None, device,
                                                    sample=sample, secondary=False, profile=False)
        res[prec] = {"value": round(cfg.W * steps / (ms * 1e-3), 2), "unit": "walker-steps/s",
                     "ms_per_step": round(ms / steps, 4), "status": st,
                     "exchange_algorithm": extra["exchange_algorithm"]}
        states[prec] = stt
        ham.close()
        del w, e
        torch.cuda.empty_cache()
    oh = orc.setup(h1, L, phiT, phiT, dt=cfg.dt, taylor_order=cfg.taylor_order)
    for prec, v in energy_errors(oh, states).items():
        res[prec]["energy_error_vs_fp64_oracle"] = v
        log(f"energy error {name} {prec}: {v['max_abs_Ha']:.3e} Ha ({v['max_rel_to_S']:.2e} of S)")
    return {"workload": f"{name}: N={cfg.N}, na=nb={cfg.n}, K={cfg.K}, {cfg.W} walkers, dt={cfg.dt}, QR every "
                        f"{cfg.qr_interval} step(s), energy every step; {steps} timed steps after {warmup}",
            "paths": res}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--config", default="n290")
    ap.add_argument("--cpu-sample", type=int, default=4, help="walkers in the timed oracle sample")
    ap.add_argument("--cpu-steps", type=int, default=5, help="consecutive oracle steps timed (median reported)")
    ap.add_argument("--energy-sample", type=int, default=8, help="walkers compared with the oracle's energy")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--only", choices=MODES, help="run one path only (profiling runs)")
    ap.add_argument("--headline", choices=MODES[1:], default="fp16x3",
                    help="mixed path reported as value (the others are on the same line)")
    ap.add_argument("--exchange", choices=("auto", "direct", "pair"), default="auto",
                    help="exchange algorithm of the main paths (profiling runs)")
    ap.add_argument("--msd-only", action="store_true",
                    help="time the multi-determinant trial calls only (profiling runs)")
    ap.add_argument("--msd-dets", type=int, default=MSD_DETS, help="determinants of the multi-determinant trial")
    ap.add_argument("--batch-only", action="store_true", help="time the uneven multi-system batch only")
    ap.add_argument("--no-legs", action="store_true", help="skip the other workloads (n100, n200, MSD, batch)")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the walker-parallel "
              "multi-GPU layout (walkers split across GPUs, each with a copy of the Hamiltonian) is not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2209_04015_amd import inputs

    cfg = inputs.CONFIGS[args.config]
    device = torch.device("cuda:0")
    t = time.time()
    h1, L = inputs.hamiltonian(cfg.N, cfg.K, cfg.decay, seed=0)
    phiT = inputs.trial(h1, cfg.n)
    nsteps = args.warmup + args.steps
    fields = inputs.fields(cfg.W, cfg.K, max(nsteps, args.cpu_steps), seed=0)
    fields_dev = torch.as_tensor(fields, device=device)
    block_fields_dev = torch.as_tensor(inputs.fields(cfg.W, cfg.K, BLOCK_STEPS, seed=1), device=device)
    log(f"inputs {cfg.name}: N={cfg.N} n={cfg.n} K={cfg.K} W={cfg.W} generated in {time.time() - t:.1f} s")

    if args.calib_copy:
        n = args.calib_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=device)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy} MiB read + {args.calib_copy} MiB written")
        del src, dst

    if args.msd_only:
        print(json.dumps({"msd": run_msd(cfg, h1, L, device, args.steps, args.msd_dets)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"uneven_batch": run_batch(device, args.steps)}), flush=True)
        return

    results = {}
    extras = {}
    states = {}
    esample = min(args.energy_sample, cfg.W)
    for precision in MODES:
        if args.only and precision != args.only:
            continue
        ham, w, e, ms, phases, status, extra, st = run_gpu(cfg, h1, L, phiT, precision, args.steps, args.warmup,
                                                           fields_dev, block_fields_dev, device,
                                                           exchange=args.exchange, sample=esample)
        results[precision] = (ms, phases, status)
        extras[precision] = extra
        states[precision] = st
        ham.close()
        del w, e
        torch.cuda.empty_cache()

    def phase_table(phases):
        return {k: round(v[0] / args.steps, 4) for k, v in phases.items() if not k.startswith("_") and v[1] > 0}

    if args.only:
        ms, ph, st = results[args.only]
        algo = extras[args.only]["exchange_algorithm"]
        print(json.dumps({"metric": METRIC, "value": round(cfg.W * args.steps / (ms * 1e-3), 2),
                          "unit": "walker-steps/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 4),
                          "only": args.only,
                          "roofline": roofline(cfg, ph, args.only, algo, args.steps),
                          "rooflines": rooflines(cfg, ph, args.only, algo, args.steps),
                          **extras[args.only],
                          "phases_ms_per_step": phase_table(ph)}), flush=True)
        return

    # the paper's direct exchange algorithm on the headline path, for comparison
    ham, w, e, ms_d, ph_d, st_d, ex_d, _ = run_gpu(cfg, h1, L, phiT, args.headline, args.steps, args.warmup,
                                                  fields_dev, block_fields_dev, device, exchange="direct",
                                                  secondary=False)
    direct = {"exchange_algorithm": "direct", "value": round(cfg.W * args.steps / (ms_d * 1e-3), 2),
              "unit": "walker-steps/s", "ms_per_step": round(ms_d / args.steps, 4),
              "roofline": rooflines(cfg, ph_d, args.headline, "direct", args.steps).get("exchange"),
              "phases_ms_per_step": phase_table(ph_d)}
    ham.close()
    del w, e
    torch.cuda.empty_cache()

    legs = {}
    msd = batch = None
    if not args.no_legs:
        # the paper's other workload sizes beside the headline one: the FP64
        # GPU comparison size (n100) and the mixed-precision size (n200)
        legs["n100"] = run_config_leg("n100", ("fp64", args.headline), 10, 2, device)
        legs["n200"] = run_config_leg("n200", ("fp64", "fp32", "bf16x3", "fp16x3"), 10, 2, device)
        msd = run_msd(cfg, h1, L, device, args.steps, args.msd_dets)
        batch = run_batch(device, args.steps)

    cpu = None
    eerr = None
    if not args.no_cpu:
        cpu, eerr = cpu_baseline_and_energy_error(cfg, h1, L, phiT, states, args.cpu_sample,
                                                  fields[:args.cpu_steps])

    W = cfg.W

    def rate(ms):
        return W * args.steps / (ms * 1e-3)

    head = args.headline
    msh, phh, sth = results[head]
    ms64, ph64, st64 = results["fp64"]
    fl = step_flops(cfg, extras[head]["exchange_algorithm"])
    paths = {}
    for p in MODES:
        ms, ph, st = results[p]
        algo = extras[p]["exchange_algorithm"]
        paths[p] = {"value": round(rate(ms), 2), "unit": "walker-steps/s",
                    "ms_per_step": round(ms / args.steps, 4),
                    "roofline": roofline(cfg, ph, p, algo, args.steps),
                    "rooflines": rooflines(cfg, ph, p, algo, args.steps),
                    "phases_ms_per_step": phase_table(ph), "status": st,
                    "energy_error_vs_fp64_oracle": (eerr or {}).get(p), **extras[p]}
    dtypes = {"fp32": "f32 (MFMA) contractions and one-body half steps",
              "fp16x3": "f16 hi/lo x3 (MFMA) force bias, VHS, exchange and the propagation P T6(VHS) P in one launch "
                        "(Horner's rule, f32 sums)",
              "bf16x3": "bf16 hi/lo x3 (MFMA) exchange; f32 (MFMA) force bias, VHS, Taylor and one-body half steps"}
    line = {
        "metric": METRIC,
        "value": round(rate(msh), 2),
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(msh / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtypes[head] + "; f64 walkers, overlaps, solves, QR, weights and energy sums",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: ph-AFQMC full walker step (propagate + QR + local energy every "
                        f"step), N={cfg.N} orbitals, na=nb={cfg.n}, K={cfg.K} Cholesky vectors, "
                        f"{W} walkers, dt={cfg.dt}, Taylor order {cfg.taylor_order}, QR every "
                        f"{cfg.qr_interval} step(s); exchange energy algorithm: "
                        f"{extras[head]['exchange_algorithm']}",
            "exchange_algorithm": extras[head]["exchange_algorithm"],
            "walkers": W, "N": cfg.N, "n_per_spin": cfg.n, "K": cfg.K, "headline_path": head,
        },
        "roofline": roofline(cfg, phh, head, extras[head]["exchange_algorithm"], args.steps),
        "rooflines": rooflines(cfg, phh, head, extras[head]["exchange_algorithm"], args.steps),
        "roofline_note": "achieved = algorithmic work of the phase's launches in one step / their time, measured "
                         "with HIP events around the phase's launches in a pass of the same steps in which only "
                         "that phase is timed; phases_ms_per_step comes from a pass with every phase timed; value "
                         "and ms_per_step come from the pass without events",
        "cpu_baseline": cpu,
        "fp64": paths["fp64"],
        "mixed_over_fp64": round(ms64 / msh, 3),
        "energy_error_vs_fp64_oracle": (eerr or {}).get(head),
        **extras[head],
        "phases_ms_per_step": phase_table(phh),
        "direct_exchange": direct,
        "config_legs": legs,
        "multi_determinant_trial": msd,
        "uneven_batch": batch,
        "paths": paths,
        "algorithmic_gflop_per_walker_step": {k: round(v / 1e9, 4) for k, v in fl.items()},
        "status": sth,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
