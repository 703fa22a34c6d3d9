"""Throughput of the phaseless-AFQMC walker step on one MI355X.

One step = one full walker step for every walker: Green's function, force
bias, VHS, propagation (two one-body half steps around a 6-term Taylor
series), overlap ratio and phaseless weight, QR re-orthogonalisation on the
workload's schedule, and the local energy (E1, EJ, EK) of every walker.

The headline is the FP16X3 path (16-bit hi/lo split contractions on the
matrix cores, FP32 elsewhere in the contractions, FP64 for overlaps, solves,
QR, weights and energy sums); the FP64, FP32 and BF16X3 paths run on the
same seeded inputs and are reported beside it, with the roofline of the
dominant kernel, the oracle's CPU rate and the energy error against the
oracle.  Also on the line: the paper's direct exchange algorithm, the
propagation-only and 25-step block rates, the multi-determinant trial's
calls, and the uneven multi-system batch.  Inputs are synthetic (seeded
generators), resident in HBM before timing starts.

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
            exchange="auto", sample=1):
    import torch

    from paper_2209_04015_amd import afqmc

    W = cfg.W
    t = time.time()
    ham = afqmc.Hamiltonian(h1, L, phiT, phiT, dt=cfg.dt, max_walkers=W, precision=precision, exchange=exchange,
                            taylor_order=cfg.taylor_order)
    log(f"{precision}: init {time.time() - t:.1f} s, exchange algorithm {ham.exchange}")
    pa = torch.as_tensor(np.repeat(phiT[None].astype(np.complex128), W, axis=0), device=device)
    w = afqmc.Walkers(pa, pa.clone())
    ham.overlap(w)
    e = torch.empty((W, 3), dtype=torch.complex128, device=device)
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        ham.step(w, fields_dev[i], do_qr=((i + 1) % cfg.qr_interval == 0), energy_out=e, reuse=(i > 0))
    torch.cuda.synchronize()
    log(f"{precision}: warmup done")
    ham.profile_enable(steps * 40)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for i in range(warmup, warmup + steps):
        ham.step(w, fields_dev[i], do_qr=((i + 1) % cfg.qr_interval == 0), energy_out=e, reuse=True)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    phases = ham.profile_read()
    ham.profile_enable(0)
    status = ham.status()
    log(f"{precision}: {steps} steps in {ms:.1f} ms ({ms / steps:.2f} ms/step), status {status}")
    # the oracle comparison uses the walkers and energies of the last timed step
    # (re-orthogonalised every step), before the secondary runs below move them
    sample_state = (w.phi_a[:sample].cpu().numpy(), w.phi_b[:sample].cpu().numpy(), e[:sample].cpu().numpy())
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
    blk_fields = block_fields_dev
    start.record(stream)
    ham.block(w, blk_fields, 0.5, energy_out=e, reuse=True)
    stop.record(stream)
    torch.cuda.synchronize()
    ms_block = start.elapsed_time(stop)
    log(f"{precision}: propagation only {ms_prop / steps:.2f} ms/step; block of {BLOCK_STEPS} "
        f"steps {ms_block:.1f} ms")
    extra = {"exchange_algorithm": ham.exchange,
             "propagation_only": {"value": round(W * steps / (ms_prop * 1e-3), 2), "unit": "walker-steps/s",
                                  "ms_per_step": round(ms_prop / steps, 4)},
             "block": {"value": round(W * BLOCK_STEPS / (ms_block * 1e-3), 2), "unit": "walker-steps/s",
                       "ms_per_block": round(ms_block, 3),
                       "definition": f"{BLOCK_STEPS} steps, QR and local energy at the last, "
                                     "global energy, comb population control"}}
    return ham, w, e, ms, phases, status, extra, sample_state


MSD_DETS = 10000


def msd_flops_per_walker(N, n):
    """Algorithmic FP64 flops per walker of the Green's function call beyond
    the determinant sums: Y = C_virt^T theta (4 N nv n), M Y (8 n^2 nv),
    Q (4 N n (n + nv)) and G = theta Q^T (8 N^2 n), per spin."""
    nv = N - n
    return 2 * (4 * N * nv * n + 8 * n * n * nv + 4 * N * n * (n + nv) + 8 * N * N * n)


def run_msd(cfg, h1, L, device, steps, ndet=MSD_DETS):
    """Multi-determinant trial (Sec. III.A): overlap, Green's function and
    force bias of every walker against a synthetic ndet-determinant expansion
    in the eigenvector basis of the workload's h1, timed over `steps` calls
    each on the current stream.  The force bias contracts with the packed L
    of an FP64 Hamiltonian of the same workload."""
    import torch

    from paper_2209_04015_amd import afqmc, inputs

    N, n, W, K = cfg.N, cfg.n, cfg.W, cfg.K
    t = time.time()
    C = inputs.orbitals(h1)
    coeff, rank, orbs = inputs.msd_expansion(N, n, n, ndet, max_rank=4, seed=5)
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
    trial.close()
    torch.cuda.empty_cache()
    log(f"msd: overlap {ms_o:.3f} ms, Green's function {ms_g:.3f} ms, force bias {ms_f:.3f} ms per call, "
        f"step {ms_s:.3f} ms (FP32 path {ms_s32:.3f} ms), status {status}")
    gbytes = W * 2 * N * N * 16
    npk = N * (N + 1) // 2
    return {"workload": f"multi-determinant trial: {ndet} determinants (ranks <= 4 per spin) in the eigenvector "
                        f"basis of the {cfg.name} h1, {N} orbitals, na=nb={n}, {W} walkers, K={K} for the force "
                        f"bias, FP64",
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
            "status": status}


def run_batch(device, steps, precision="fp16x3"):
    """The uneven multi-system workload (8 systems, N = 40 .. 200) advanced
    together by one hipGraph launch per step (autotuned exchange tile order),
    QR and local energy every step; and the same steps taken system after
    system with afqmc_step on one stream, for comparison."""
    import torch

    from paper_2209_04015_amd import afqmc, inputs

    t = time.time()
    systems = inputs.uneven_batch()
    hams, ws, fs, es, starts = [], [], [], [], []
    for (N, n, K, decay, W, seed) in systems:
        h1, L = inputs.hamiltonian(N, K, decay, seed=seed)
        phiT = inputs.trial(h1, n)
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
    b.autotune()
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    b.step(fs, es, do_qr=True)          # capture + first replays (untimed)
    torch.cuda.synchronize()
    start.record(stream)
    b.step(fs, es, do_qr=True)
    stop.record(stream)
    torch.cuda.synchronize()
    ms_b = start.elapsed_time(stop)
    st_b = sum(h.status() for h in hams)
    b.close()
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
    log(f"batch: {steps} steps in {ms_b:.1f} ms (graph) vs {ms_s:.1f} ms (systems in turn)")
    return {"workload": "uneven multi-system batch: 8 systems, N = 40, 60, ..., 160, 200, n = N/5, K = 4N, "
                        f"walkers {[s[4] for s in systems]}, {precision}, QR and local energy every step, "
                        "one hipGraph launch per step, autotuned exchange tile order",
            "value": round(wtot * steps / (ms_b * 1e-3), 1), "unit": "walker-steps/s",
            "ms_per_step": round(ms_b / steps, 4), "status": st_b,
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


# kernel (and its template instance in the rocprofv3 summaries) per phase,
# precision and exchange algorithm
def _kernel_of(phase, precision, algo):
    split = precision in ("fp16x3", "bf16x3")
    H = {"fp16x3": "HalfF16", "bf16x3": "HalfBF16"}.get(precision)
    T = {"fp32": "float", "fp64": "double", "bf16x3": "float"}.get(precision)
    if phase == "exchange":
        base = ("exchange_pair" if algo == "pair" else "exchange") + ("_split_kernel" if split else "_kernel")
        return base, f"{base}<{H if split else T}>"
    if precision == "fp16x3":   # the VHS runs on split operands only in FP16X3
        return "vhs_split_kernel", "vhs_split_kernel<HalfF16>"
    # tile template arguments of the FP32 / FP64 VHS instances (step_kernels.hip)
    return "vhs_kernel", {"double": "vhs_kernel<double, 64, 64, 16, 2, 2>",
                          "float": "vhs_kernel<float, 64, 64, 32, 2, 2>"}[T]


def roofline_of(cfg, phases, precision, algo, phase):
    ms, launches = phases[phase]
    if launches == 0:
        return None
    avg_ms = ms / launches
    flops = (exchange_flops_per_launch(cfg, cfg.W, algo) if phase == "exchange"
             else vhs_flops_per_launch(cfg, cfg.W))
    achieved = flops / (avg_ms * 1e-3) / 1e12
    kernel, instance = _kernel_of(phase, precision, algo)
    note = None
    if "split" in kernel:
        # three 16-bit products per algorithmic multiply-add
        peak = round(PEAK_TFLOPS[precision[:4]] / 3.0, 1)
        note = f"{precision[:4]} dense peak / 3 products"
    else:
        peak = PEAK_TFLOPS["fp64" if precision == "fp64" else "fp32"]
    out = {"kernel": kernel, "bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
           "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
           "traffic": hbm_traffic(kernel, instance, cfg.name),
           "avg_launch_ms": round(avg_ms, 4), "launches_per_step_share_ms": round(ms, 3),
           "flops_per_launch": flops}
    if note:
        out["peak_note"] = note
    return out


def rooflines(cfg, phases, precision, algo):
    """Roofline entries of the exchange and VHS kernels; the first is the one with
    the larger share of the step (the dominant kernel)."""
    out = {ph: roofline_of(cfg, phases, precision, algo, ph) for ph in ("exchange", "vhs")}
    order = sorted(out, key=lambda ph: -phases[ph][0])
    return {ph: out[ph] for ph in order if out[ph] is not None}


def roofline(cfg, phases, precision, algo):
    r = rooflines(cfg, phases, precision, algo)
    return next(iter(r.values())) if r else None


def cpu_baseline_and_energy_error(cfg, h1, L, phiT, gpu_states, sample, x_sample):
    """The FP64 oracle: its walker-step rate on a bounded sample, and the per-walker
    energy error of each GPU path against it on sampled walkers."""
    from oracle import afqmc_oracle as orc

    t = time.time()
    oh = orc.setup(h1, L, phiT, phiT, dt=cfg.dt, taylor_order=cfg.taylor_order)
    log(f"oracle setup {time.time() - t:.1f} s")
    out = {}
    for prec, (pa, pb, e_gpu) in gpu_states.items():
        e_ref = orc.local_energy(oh, pa, pb)
        S = np.abs(e_ref).sum(axis=1)
        err = np.abs(e_gpu.sum(axis=1) - e_ref.sum(axis=1))
        out[prec] = {"max_abs_Ha": float(err.max()), "max_rel_to_S": float((err / S).max()),
                     "walkers": int(len(err)), "E_scale_Ha": float(np.abs(e_ref.sum(axis=1)).max())}
        log(f"energy error {prec}: {err.max():.3e} Ha ({(err / S).max():.2e} of S)")
    # timed oracle sample: full steps (propagate, QR, energy) of `sample` walkers
    pa = np.repeat(phiT[None].astype(np.complex128), sample, axis=0)
    pb = pa.copy()
    lo = orc.overlap(oh, pa, pb)
    lw = np.zeros(sample)
    t = time.time()
    orc.step(oh, pa, pb, lo, lw, x_sample, do_qr=True)
    dt = time.time() - t
    threads = None
    try:
        from threadpoolctl import threadpool_info

        threads = max((d.get("num_threads", 0) for d in threadpool_info()), default=None)
    except Exception:
        pass
    cpu = {"value": round(sample / dt, 3), "unit": "walker-steps/s",
           "cores": threads or os.cpu_count(), "kind": "oracle",
           "sample": f"{sample} walkers x 1 full step (propagate, QR, local energy) of the same "
                     f"workload, FP64 NumPy oracle; setup not timed; {dt:.1f} s"}
    log(f"oracle: {sample} walker-steps in {dt:.1f} s")
    return cpu, out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="n290")
    ap.add_argument("--cpu-sample", type=int, default=12, help="walkers in the timed oracle sample")
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
    fields = inputs.fields(cfg.W, cfg.K, nsteps, seed=0)
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
    sample = min(args.cpu_sample, cfg.W)
    for precision in MODES:
        if args.only and precision != args.only:
            continue
        ham, w, e, ms, phases, status, extra, st = run_gpu(cfg, h1, L, phiT, precision, args.steps, args.warmup,
                                                           fields_dev, block_fields_dev, device,
                                                           exchange=args.exchange, sample=sample)
        results[precision] = (ms, phases, status)
        extras[precision] = extra
        states[precision] = st
        ham.close()
        del w, e
        torch.cuda.empty_cache()

    # the paper's direct exchange algorithm on the headline path, for comparison
    direct = None
    if not args.only:
        ham, w, e, ms_d, ph_d, st_d, ex_d, _ = run_gpu(cfg, h1, L, phiT, args.headline, args.steps, args.warmup,
                                                      fields_dev, block_fields_dev, device, exchange="direct")
        direct = {"exchange_algorithm": "direct", "value": round(cfg.W * args.steps / (ms_d * 1e-3), 2),
                  "unit": "walker-steps/s", "ms_per_step": round(ms_d / args.steps, 4),
                  "roofline": roofline(cfg, ph_d, args.headline, "direct"),
                  "phases_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in ph_d.items() if v[1] > 0}}
        ham.close()
        del w, e
        torch.cuda.empty_cache()

    msd = None if args.only else run_msd(cfg, h1, L, device, args.steps, args.msd_dets)
    batch = None if args.only else run_batch(device, args.steps)

    if args.only:
        ms, ph, st = results[args.only]
        print(json.dumps({"metric": METRIC, "value": round(cfg.W * args.steps / (ms * 1e-3), 2),
                          "unit": "walker-steps/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 4),
                          "only": args.only,
                          "roofline": roofline(cfg, ph, args.only, extras[args.only]["exchange_algorithm"]),
                          "rooflines": rooflines(cfg, ph, args.only, extras[args.only]["exchange_algorithm"]),
                          **extras[args.only],
                          "phases_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in ph.items()
                                                 if v[1] > 0}}), flush=True)
        return

    cpu = None
    eerr = None
    if not args.no_cpu:
        cpu, eerr = cpu_baseline_and_energy_error(cfg, h1, L, phiT, states, sample,
                                                  fields[0, :sample])

    W = cfg.W
    def rate(ms):
        return W * args.steps / (ms * 1e-3)

    def phase_table(phases):
        return {k: round(v[0] / args.steps, 4) for k, v in phases.items() if v[1] > 0}

    head = args.headline
    msh, phh, sth = results[head]
    ms64, ph64, st64 = results["fp64"]
    fl = step_flops(cfg, extras[head]["exchange_algorithm"])
    paths = {}
    for p in MODES:
        ms, ph, st = results[p]
        paths[p] = {"value": round(rate(ms), 2), "unit": "walker-steps/s",
                    "ms_per_step": round(ms / args.steps, 4),
                    "roofline": roofline(cfg, ph, p, extras[p]["exchange_algorithm"]),
                    "rooflines": rooflines(cfg, ph, p, extras[p]["exchange_algorithm"]),
                    "phases_ms_per_step": phase_table(ph), "status": st,
                    "energy_error_vs_fp64_oracle": (eerr or {}).get(p), **extras[p]}
    dtypes = {"fp32": "f32 contractions (MFMA)",
              "fp16x3": "f16 hi/lo x3 exchange and VHS + f32 contractions (MFMA)",
              "bf16x3": "bf16 hi/lo x3 exchange + f32 contractions (MFMA)"}
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
        "dtype": dtypes[head] + " + f64 overlaps/solves/QR/weights/energy sums",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: ph-AFQMC full walker step (propagate + QR + local energy every "
                        f"step), N={cfg.N} orbitals, na=nb={cfg.n}, K={cfg.K} Cholesky vectors, "
                        f"{W} walkers, dt={cfg.dt}, Taylor order {cfg.taylor_order}, QR every "
                        f"{cfg.qr_interval} step(s); exchange energy through pair integrals "
                        f"({extras[head]['exchange_algorithm']})",
            "exchange_algorithm": extras[head]["exchange_algorithm"],
            "walkers": W, "N": cfg.N, "n_per_spin": cfg.n, "K": cfg.K, "headline_path": head,
        },
        "roofline": roofline(cfg, phh, head, extras[head]["exchange_algorithm"]),
        "rooflines": rooflines(cfg, phh, head, extras[head]["exchange_algorithm"]),
        "cpu_baseline": cpu,
        "fp64": paths["fp64"],
        "mixed_over_fp64": round(ms64 / msh, 3),
        "energy_error_vs_fp64_oracle": (eerr or {}).get(head),
        **extras[head],
        "phases_ms_per_step": phase_table(phh),
        "direct_exchange": direct,
        "multi_determinant_trial": msd,
        "uneven_batch": batch,
        "paths": paths,
        "algorithmic_gflop_per_walker_step": {k: round(v / 1e9, 4) for k, v in fl.items()},
        "status": sth,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
