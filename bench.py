"""Throughput of the radiation spectral synthesis on one MI355X.

Headline workload: the mixed-precision form -- particles of the filamentation-
jitter generator (electrons of two gamma0 = 3 counter-streaming beams, kT = 0.01
rest-frame spread, Boris-pushed through a static random-filament field, k^-2 over
[0.5, 8], deflection parameter 0.3), 2048 samples each, seen from 16 directions
(head-on, 15/30/45 degrees oblique at four azimuths, three perpendicular) on 2048
log-spaced frequencies over [0.1, 1e3] omega_p.  The ensemble has 1e6 particles
(6.71e13 terms, 123 GB of trajectories, generated on the device); one step is one
lw_accumulate over all of it with the trajectories already resident in HBM
(--particles takes a slice instead).

metric: terms/s, a term being one (particle, sample, direction, frequency)
product of the spectral sum.  The headline path is the matrix-core contraction
with FP16 hi/lo operands and three products; the other matrix-core variants
(one and two FP16 products, BF16 hi/lo) are timed on the same tensors, the FP32
path on its first 5e4 particles, and every path's band-integrated error against
the FP64 oracle is measured on 8 particles of the same workload.

Legs (each its own JSON object): the FP32 and FP16 hi/lo paths on the
1e5-particle, 4096-sample, 4-direction, 1024-frequency jitter ensemble, with
coherent, in-situ and coupled recording; the batched uneven three-species workload (64 directions) with
per-CU busy spread; the learned surrogate (training on 1.25e5 particles' exact
spectra, inference on 1e6 particles with fallback and a 1 % held-out judge); and
the FP64 oracle on the host cores.

Prints one JSON line.  Options: --steps K --warmup W --particles P --paths ...
--no-surrogate and the other --no-* switches.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)



def fp32_term_peak():
    """Issue-bound ceiling of the FP32 path (terms/s).

    Per term a wave64 issues 8 full-rate VALU instructions (FP64 multiply,
    round-to-integer and FMA for the turn fraction; FP64->FP32 convert; four
    FP32 FMAs) at 4 cycles each and two half-rate transcendentals (sin, cos)
    at 8 cycles each: 48 SIMD cycles per 64 terms.  With 4 SIMDs per CU,
    256 CUs and 2.4 GHz this is 4 * 64/48 * 256 * 2.4e9 = 3.28e12 terms/s.
    """
    return 4.0 * 64.0 / 48.0 * 256 * 2.4e9


PEAK_MFMA_TFLOPS = 2500.0  # dense FP16/BF16 matrix peak of one MI355X
PEAK_HBM_GBS = 8000.0  # HBM3E bandwidth of one MI355X
PEAK_FP32_VECTOR_TFLOPS = 157.3  # FP32 vector peak of one MI355X (with packed FP32 math)


def spread_width(products):
    """Taps W of the spreading kernel: 10 for the hi/lo operand split, 8 for one product."""
    return 10 if products == 3 else 8


def spread_flops_per_unit(w, bands=1):
    """Counted arithmetic of the spreading step for one (sample, direction, band) with W taps.

    Per band, FP32: the W tap weights times the demodulated integrand into 2 polarisations x
    (re, im), 4W FMAs = 8W; the tap weights, W/2 mirrored pairs of degree-8 polynomials in
    z = 2 frac(u) - 1 evaluated as even and odd parts in z^2 (4 + 3 Horner FMAs and 2 FMAs
    to combine), 9W, plus 3 for z and z^2; the demodulation of both polarisations by (cos,
    sin), 4.  FP64: the turn fraction of w_c tau 2, the grid coordinate and its fraction 4.
    Per sample and direction, shared by the (at most two) bands one work-group spreads:
    the integrand e.(n x ((n - beta) x a)) / kappa^2 for both polarisations, 35 (FP32), kappa
    6 and the retarded time 9 (FP64).  Sine, cosine and reciprocal are not counted.  Total
    17 W + 13 + 50 / g with g the mean bands per work-group (208 at W = 10 with two bands).
    This is instruction work, reported beside the algorithmic figure below.
    """
    nb = max(1, bands)
    groups = (nb + 1) // 2
    return 17 * w + 13 + 50.0 * groups / nb


# Algorithmic work of the spread per (sample, direction, band): 8 taps x 2 polarisations
# multiply-adds, 32 FLOP (the figure the roofline's frac uses); the contraction's
# algorithmic work is one product's multiply-adds, however many hi/lo products run.
SPREAD_ALGO_FLOPS = 32
C3_PARTICLES = 1_000_000
C3_TERMS = C3_PARTICLES * 2048 * 16 * 2048  # the full mixed-precision ensemble: 6.7e13 terms


def split_path(name):
    """'mfma_f16x3' -> ('mfma_f16', 3); 'fp32' -> ('fp32', 1)."""
    for k in (1, 2, 3):
        if name.endswith(f"x{k}"):
            return name[:-2], k
    return name, 1


def mfma_options(ctx, bands, path, products):
    """Band count and product count of one matrix-core path (the other type keeps three)."""
    if path == "mfma_bf16":
        ctx.set_mfma_options(bands, 3, products)
    else:
        ctx.set_mfma_options(bands, products, 3)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("c3", "c2"), default="c3",
                    help="headline workload: c3 = the mixed-precision form (2048 steps, 16 directions, "
                         "2048 frequencies; a slice of its 1e6 particles per step); c2 = the jitter "
                         "ensemble (4096 steps, 4 directions, 1024 frequencies)")
    ap.add_argument("--particles", type=int, default=0,
                    help="particles per step of the headline workload (default: all of it, 1e6 for c3 and "
                         "1e5 for c2)")
    ap.add_argument("--other-path-steps", type=int, default=3,
                    help="timed steps of the non-headline paths on the headline workload")
    ap.add_argument("--fp32-particles", type=int, default=50_000,
                    help="particles of the headline workload timed on the FP32 path (speedup at equal shape)")
    ap.add_argument("--c2-particles", type=int, default=100_000, help="particles of the jitter (c2) leg")
    ap.add_argument("--c2-steps", type=int, default=3, help="timed steps of the FP32 path on the c2 leg")
    ap.add_argument("--chunk", type=int, default=8192, help="particles generated per host chunk")
    ap.add_argument("--paths", default="mfma_f16x1,mfma_f16x2,mfma_bf16x3,mfma_f16x3",
                    help="comma list of fp32, mfma_f16[x1|x2|x3], mfma_bf16[x1|x3]; the last one is the headline")
    ap.add_argument("--bands", type=int, default=2,
                    help="frequency bands of the matrix-core paths (2 measured fastest on both workloads: "
                         "the upper band keeps the grid, the lower one is ~9x coarser)")
    ap.add_argument("--tile", type=int, default=0,
                    help="contraction tile: 1 = 128x128, 2 = 256x128, 3 = 128x256, 4 = 256x256 "
                         "(0: library default)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-insitu", action="store_true")
    ap.add_argument("--no-coupled", action="store_true")
    ap.add_argument("--coupled-windows", type=int, default=10)
    ap.add_argument("--coupled-steps", type=int, default=40, help="simulation steps per window")
    ap.add_argument("--windows", type=int, default=4, help="time windows of the in-situ leg")
    ap.add_argument("--batched-particles", type=int, default=50_000,
                    help="particles of the uneven three-species workload in the batched leg")
    ap.add_argument("--batched-tune-particles", type=int, default=8000,
                    help="the first particles of the batched leg the autotuner times its candidates on")
    ap.add_argument("--surrogate-infer", type=int, default=1_000_000)
    ap.add_argument("--surrogate-chunk", type=int, default=100_000)
    ap.add_argument("--surrogate-fallback-path", choices=("fp32", "mfma_f16"), default="mfma_f16",
                    help="exact path of the surrogate's fallback (mfma_f16: FP16 hi/lo, three products, on a "
                         "gathered copy of the flagged particles)")
    ap.add_argument("--surrogate-judge-path", choices=("fp32", "mfma_f16"), default="fp32",
                    help="exact path of the held-out judge")
    ap.add_argument("--surrogate-steps", type=int, default=1500)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (scales HBM byte counters)")
    ap.add_argument("--host-generator", action="store_true",
                    help="generate the throughput ensemble on the host (default: on the device)")
    return ap.parse_args()


def band_integrated_error(S, ref, om, n_bands=16, floor=1e-4):
    worst = 0.0
    idx = np.array_split(np.arange(om.size), n_bands)
    for s, r in zip(S.reshape(-1, om.size), ref.reshape(-1, om.size)):
        pr = np.array([np.trapezoid(r[i] * om[i], np.log(om[i])) for i in idx])
        ps = np.array([np.trapezoid(s[i] * om[i], np.log(om[i])) for i in idx])
        m = pr >= floor * pr.max()
        worst = max(worst, float(np.max(np.abs(ps[m] - pr[m]) / pr[m])))
    return worst


TRAFFIC_PROFILES = {
    "c2": os.path.join(ROOT, "profiles", "lw_dft_mfma_r128__jitter_1e5x4096_4dir_1024w.md"),
    "c3": os.path.join(ROOT, "profiles", "lw_mfma__mixed_precision_1e6x2048_16dir_2048w.md"),
}
PROFILED_PARTICLES = {"c2": 100_000, "c3": 1_000_000}
TRAFFIC_FIELDS = {"contraction": "traffic_bytes_per_launch", "spread": "spread_traffic_bytes_per_launch"}


def kernel_code_digest(src):
    """SHA-256 of a source file's code: line comments and all whitespace removed (the file
    has no block comments and no "//" inside string literals)."""
    import hashlib
    import re

    code = re.sub(r"//[^\n]*", "", src)
    return hashlib.sha256(re.sub(r"\s+", "", code).encode()).hexdigest()


def profiled_traffic(path, tile, particles, workload="c3", bands=2, kernel="contraction"):
    """HBM bytes per launch of the contraction (or the spreading kernel) from the committed
    counter profile of this exact configuration (the default launch of the workload), or None
    when there is no such profile or the kernel code or the band count differs from the
    profiled run."""
    if path != "mfma_f16x3" or tile not in (0, 4) or workload not in TRAFFIC_PROFILES:
        return None
    if particles != PROFILED_PARTICLES[workload]:
        return None
    try:
        text = open(TRAFFIC_PROFILES[workload]).read()
        src = open(os.path.join(ROOT, "paper_1003_1140_amd", "csrc", "lw_mfma.hip")).read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines()
                  if line.startswith(tuple(f + ":" for f in (*TRAFFIC_FIELDS.values(), "kernel_code_sha256",
                                                             "bands"))))
    if fields.get("kernel_code_sha256", "").strip() != kernel_code_digest(src):
        return None
    if fields.get("bands", "").strip() != str(bands):
        return None
    value = fields.get(TRAFFIC_FIELDS[kernel])
    return float(value) if value is not None else None


def attach_traffic(r, path, tile, particles, workload, bands):
    """Profiled HBM bytes per launch on both kernels' rooflines of a timed matrix-core path, and
    its `roofline` again the dominant kernel's (copied before the traffic was known)."""
    for kernel in ("contraction", "spread"):
        r["roofline_" + kernel]["traffic"] = profiled_traffic(path, tile, particles, workload, bands, kernel)
    r["roofline"] = dict(r["roofline_spread" if r["roofline"]["bound"] == "alu" else "roofline_contraction"])


def SPREAD_KERNEL(w):
    return f"lw_spread_kernel<{w}>"


TILE_KERNELS = {0: "lw_dft_mfma_r128_kernel<WN=4, MI=4, NJ=2> (256 x 256 tiles, eight waves)",
                1: "lw_dft_mfma_r128_kernel<WN=2, MI=2, NJ=2> (128 x 128 tiles)",
                2: "lw_dft_mfma_kernel (256 x 128 tiles)",
                3: "lw_dft_mfma_r128_kernel<WN=4, MI=2, NJ=2> (128 x 256 tiles)",
                4: "lw_dft_mfma_r128_kernel<WN=4, MI=4, NJ=2> (256 x 256 tiles, eight waves)"}


def time_path(ctx, batch, name, steps, warmup, terms_per_step, bands, tile=0):
    import torch

    path, products = split_path(name)
    mfma_options(ctx, bands, path, products)
    ws = ctx.workspace(batch, path)
    for _ in range(warmup):
        ctx.accumulate(batch, path, workspace=ws)
    torch.cuda.synchronize()
    ctx.reset()
    ctx.profile_read()  # clear
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.accumulate(batch, path, workspace=ws)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.profile_read()
    S = ctx.read_spectra() / steps
    assert np.all(np.isfinite(S))
    res = {"terms_per_s": terms_per_step * steps / el, "ms_per_step": el / steps * 1e3,
           "kernel_ms_per_step": {k: prof[k] / steps for k in ("direct_ms", "spread_ms", "gemm_ms")}}
    if path == "fp32":
        per_launch_ms = prof["direct_ms"] / max(prof["direct_launches"], 1)
        ach = terms_per_step * steps / prof["direct_launches"] / (per_launch_ms * 1e-3)
        peak = fp32_term_peak()
        # the same rate as counted arithmetic: four FP32 FMAs (8 FLOPs) per term
        res["roofline"] = {"bound": "alu", "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "Tterm/s",
                           "frac": ach / peak, "traffic": None, "kernel": "lw_direct_f32_kernel<4>",
                           "avg_launch_ms": per_launch_ms,
                           "counted_tflops": 8 * ach / 1e12,
                           "frac_of_fp32_vector_peak": 8 * ach / 1e12 / PEAK_FP32_VECTOR_TFLOPS}
    else:
        # the library counts each product's multiply-adds; one product is the useful work
        executed = prof["gemm_flops"] / (prof["gemm_ms"] * 1e-3) / 1e12
        ach = executed / products
        peak = PEAK_MFMA_TFLOPS
        contraction = {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                       "frac": ach / peak, "traffic": None, "kernel": TILE_KERNELS[tile],
                       "avg_launch_ms": prof["gemm_ms"] / max(prof["gemm_launches"], 1),
                       "launches_per_step": prof["gemm_launches"] / steps,
                       "products": products, "executed_tflops": executed,
                       "executed_frac": executed / peak}
        # every band spreads every sample once per direction (the plan holds 1 to 16 bands,
        # at most one per frequency)
        w = spread_width(products)
        nb = max(1, min(bands, 16, ctx.nw))
        units = float(batch.n_samples_host) * ctx.nd * nb * steps
        sec = prof["spread_ms"] * 1e-3
        ach = units * SPREAD_ALGO_FLOPS / sec / 1e12
        counted = units * spread_flops_per_unit(w, nb) / sec / 1e12
        spread = {"bound": "alu", "achieved": ach, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                  "frac": ach / PEAK_FP32_VECTOR_TFLOPS, "traffic": None, "kernel": SPREAD_KERNEL(w),
                  "avg_launch_ms": prof["spread_ms"] / max(prof["spread_launches"], 1),
                  "launches_per_step": prof["spread_launches"] / steps,
                  "algorithmic_flops_per_sample_direction_band": SPREAD_ALGO_FLOPS,
                  "units_per_step": units / steps,
                  "counted_flops_per_sample_direction_band": spread_flops_per_unit(w, nb),
                  "counted_tflops": counted, "counted_frac": counted / PEAK_FP32_VECTOR_TFLOPS}
        res["roofline_contraction"] = contraction
        res["roofline_spread"] = spread
        # the headline roofline is the kernel that takes longer in the step
        res["roofline"] = dict(spread if prof["spread_ms"] > prof["gemm_ms"] else contraction)
    return res, S


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline(recipe, dirs, om, target_s, label):
    import oracle
    import workloads

    nthreads = oracle.max_threads()
    ncal = 2 * nthreads  # enough particles to occupy every thread
    cal = workloads.generate(recipe, 10_000_000, ncal)
    t = time.perf_counter()
    oracle.spectrum(cal, dirs, om, n_species=1, nthreads=nthreads)
    dt_cal = time.perf_counter() - t
    per_particle = dt_cal / ncal
    n = int(max(2, min(2048, target_s / max(per_particle, 1e-6))))
    sample = workloads.generate(recipe, 10_000_000, n)
    t = time.perf_counter()
    oracle.spectrum(sample, dirs, om, n_species=1, nthreads=nthreads)
    el = time.perf_counter() - t
    terms = sample.n_samples * len(dirs) * len(om)
    return {"value": terms / el, "unit": "terms/s", "cores": nthreads, "kind": "oracle",
            "cpu_model": cpu_model(), "logical_cpus_visible": os.cpu_count(),
            "sample": f"{n} particles of the {label} x {sample.n_samples // n} samples x {len(dirs)} dirs x "
                      f"{len(om)} freqs, FP64 libm sin/cos, {el:.1f} s"}


def oracle_check(recipe, dirs, om, paths, bands, n_particles=8):
    """The first particles of the headline workload, generated on the host (the same bytes
    go to the device): every path's spectrum against the FP64 oracle -- band-integrated
    error (16 log bands per direction, bands holding >= 1e-4 of the strongest) and the
    largest per-bin error over bins >= 1e-4 of the direction's peak."""
    import oracle
    import workloads
    from paper_1003_1140_amd import Context, DeviceBatch

    host = workloads.generate(recipe, 0, n_particles)
    t = time.perf_counter()
    ref = oracle.spectrum(host, dirs, om, n_species=1)
    t_oracle = time.perf_counter() - t
    dev = DeviceBatch.from_host(host)
    out = {"particles": n_particles, "directions": len(dirs), "frequencies": len(om),
           "samples": int(host.n_samples), "oracle_seconds": t_oracle}
    for name in paths:
        path, products = split_path(name)
        c = Context(0)
        c.set_directions(dirs)
        c.set_frequencies(om)
        mfma_options(c, bands, path, products)
        c.accumulate(dev, path, workspace=c.workspace(dev, path))
        S = c.read_spectra()
        c.close()
        out[name] = {"band_integrated_err": band_integrated_error(S, ref, om),
                     "per_bin_max_err": band_relative(S, ref)}
    return out


def upload_ensemble(recipe, n, chunk, dev, host=False):
    """The whole ensemble in device memory, generated on the device (or on the host)."""
    from paper_1003_1140_amd import DeviceBatch

    if host:
        from workloads.device import upload_chunks

        tensors, ns = upload_chunks(recipe, n, chunk, dev)
    else:
        from workloads.gpu import generate_device

        tensors, ns = generate_device(recipe, 0, n, dev)
    b = DeviceBatch(tensors, n)
    b.n_samples_host = ns
    return b


def window_batches(batch, n_windows, dev):
    """Split a batch of equal-length trajectories into n_windows consecutive time windows
    (each particle's t0 moved to the window's first sample), as an in-situ recorder sees
    the run between snapshots."""
    import torch

    from paper_1003_1140_amd import DeviceBatch

    P = batch.n_particles
    offs = batch.t["offsets"].cpu().numpy()
    L = int(offs[1] - offs[0]) if P else 0
    assert np.all(np.diff(offs) == L), "window_batches needs equal trajectory lengths"
    edges = [round(i * L / n_windows) for i in range(n_windows + 1)]
    out = []
    for k0, k1 in zip(edges[:-1], edges[1:]):
        t = {}
        for k, v in batch.t.items():
            if k in ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az"):
                t[k] = v.view(P, L)[:, k0:k1].contiguous().view(-1)
            elif k == "offsets":
                t[k] = torch.arange(P + 1, dtype=torch.int64, device=dev) * (k1 - k0)
            elif k == "t0":
                t[k] = v + k0 * batch.t["dt"]
            else:
                t[k] = v
        out.append(DeviceBatch(t, P))
    return out


def insitu_leg(a, batch, terms_per_step, dirs, om, S_fp32, log):
    """Coherent synthesis and in-situ recording on the headline ensemble (FP32 path).

    coherent: one pass adding w q A_p into the summed species amplitude.
    in-situ: the run cut into time windows; each window's amplitudes are added to a
    per-particle FP64 state and a spectrum snapshot is taken from the state after
    every window (what the recording scheme does between simulation steps); the last
    snapshot must equal the one-pass spectrum."""
    import torch

    from paper_1003_1140_amd import Context

    dev = torch.device("cuda:0")
    res = {}
    c = Context(0)
    c.set_directions(dirs)
    c.set_frequencies(om)
    c.set_coherent(True)
    ws = c.workspace(batch, "fp32")
    c.accumulate(batch, "fp32", workspace=ws)  # warm-up
    torch.cuda.synchronize()
    c.reset()
    steps = max(1, min(a.steps, 2))
    t0 = time.perf_counter()
    for _ in range(steps):
        c.accumulate(batch, "fp32", workspace=ws)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    S_coh = c.read_spectra()
    res["coherent_terms_per_s"] = terms_per_step * steps / el
    # the same on the matrix-core path (FP16 hi/lo), checked against the FP32 coherent pass
    c.set_mfma_options(a.bands, 3, 3)
    wsm = c.workspace(batch, "mfma_f16")
    c.reset()
    c.accumulate(batch, "mfma_f16", workspace=wsm)  # warm-up
    torch.cuda.synchronize()
    c.reset()
    t0 = time.perf_counter()
    for _ in range(steps):
        c.accumulate(batch, "mfma_f16", workspace=wsm)
    torch.cuda.synchronize()
    el_m = time.perf_counter() - t0
    res["coherent_mfma_f16x3_terms_per_s"] = terms_per_step * steps / el_m
    res["coherent_mfma_vs_fp32_band_err"] = float(np.max(band_integrated_error(c.read_spectra(), S_coh, om)))
    del wsm
    log(f"[bench] coherent mfma_f16x3: {res['coherent_mfma_f16x3_terms_per_s']:.3e} terms/s, band error vs "
        f"coherent fp32 {res['coherent_mfma_vs_fp32_band_err']:.2e}")
    res["coherent_over_incoherent_peak"] = float(S_coh.max() / (steps * steps) / S_fp32.max())
    log(f"[bench] coherent: {res['coherent_terms_per_s']:.3e} terms/s")
    del ws
    c.close()

    wins = window_batches(batch, a.windows, dev)
    c = Context(0)
    c.set_directions(dirs)
    c.set_frequencies(om)
    state = c.amplitude_state(batch.n_particles)
    ws = torch.empty(max(256, c.amplitude_workspace_size(batch.n_particles)), dtype=torch.uint8, device=dev)
    c.accumulate_amplitudes(wins[0], state)  # warm-up
    c.spectrum_from_amplitudes(batch, state, ws)
    torch.cuda.synchronize()
    state.zero_()
    snap_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    snaps = []
    for w in wins:
        c.accumulate_amplitudes(w, state)
        c.reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        c.spectrum_from_amplitudes(batch, state, ws)
        e1.record()
        snaps.append(c.read_spectra())
        snap_ms.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t1 = time.perf_counter()
    avg, diag = c.spectral_diagnostics(weights=None)
    diag_ms = (time.perf_counter() - t1) * 1e3
    state_bytes = state.numel() * 8
    ms = float(np.mean(snap_ms))
    gbs = state_bytes / (ms * 1e-3) / 1e9
    res.update({
        "windows": a.windows,
        "insitu_terms_per_s": terms_per_step / el,
        "insitu_ms_per_step": el * 1e3,
        "state_bytes": state_bytes,
        "snapshot_ms": ms,
        "snapshot_roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                              "frac": gbs / PEAK_HBM_GBS, "traffic": None,
                              "kernel": "lw_amp_reduce_kernel + lw_reduce_partials"},
        "last_snapshot_vs_one_pass_band_err": band_relative(snaps[-1], S_fp32),
        "diagnostics_ms": diag_ms,
        "observer_average": {"omega_peak": float(diag[0, -1, 2]), "alpha": float(diag[0, -1, 4]),
                             "beta": float(diag[0, -1, 6])},
        "per_observer_omega_peak": [float(x) for x in diag[0, :-1, 2]],
    })
    log(f"[bench] in-situ ({a.windows} windows, snapshot after each): {res['insitu_terms_per_s']:.3e} "
        f"terms/s, snapshot {ms:.2f} ms ({gbs:.0f} GB/s), last vs one pass "
        f"{res['last_snapshot_vs_one_pass_band_err']:.2e}")
    # the same recording with the windows' amplitudes from the matrix-core path (FP16 hi/lo)
    c.set_mfma_options(a.bands, 3, 3)
    wsm = c.workspace(wins[0], "mfma_f16")
    state.zero_()
    c.accumulate_amplitudes(wins[0], state, "mfma_f16", wsm)  # warm-up
    torch.cuda.synchronize()
    state.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for w in wins:
        c.accumulate_amplitudes(w, state, "mfma_f16", wsm)
        c.reset()
        c.spectrum_from_amplitudes(batch, state, ws)
        last = c.read_spectra()
    torch.cuda.synchronize()
    el_m = time.perf_counter() - t0
    res["insitu_mfma_f16x3_terms_per_s"] = terms_per_step / el_m
    res["insitu_mfma_last_snapshot_vs_one_pass_band_integrated_err"] = float(
        band_integrated_error(last, S_fp32, om))
    log(f"[bench] in-situ on mfma_f16x3: {res['insitu_mfma_f16x3_terms_per_s']:.3e} terms/s, last vs FP32 "
        f"one pass (band-integrated) {res['insitu_mfma_last_snapshot_vs_one_pass_band_integrated_err']:.2e}")
    del wsm
    del state, ws, wins
    c.close()
    return res


def coupled_leg(a, dirs, om, log):
    """In-situ coupling: a device pusher advances the jitter ensemble window by window
    (simulation steps of 10 synthesis steps, growing filament amplitude) and every window
    goes straight into the recorder (per-particle amplitude state) with a snapshot after
    each window.  Times the pusher and the recording separately with HIP events on the
    stream both use."""
    import torch

    from paper_1003_1140_amd import Context, DeviceBatch, Recorder
    from workloads import configs
    from workloads.gpu import InsituSim

    n, n_steps, n_sub, n_win = a.particles, a.coupled_steps, 10, a.coupled_windows
    res = {"workload": f"{n} particles of the jitter recipe advanced in situ: {n_win} windows of "
                       f"{n_steps} simulation steps x {n_sub} synthesis steps (dt_synth = "
                       f"{configs.DT}), filament amplitude growing 0.01 -> 1 at rate 0.4; 4 dirs, "
                       f"{len(om)} log omega; snapshot after every window",
           "terms": float(n) * n_steps * n_sub * n_win * len(dirs) * len(om)}
    for path in ("fp32", "mfma_f16"):
        sim = InsituSim(configs.jitter_recipe(), 0, n, "cuda")
        c = Context(0)
        c.set_directions(dirs)
        c.set_frequencies(om)
        c.set_mfma_options(a.bands, 3, 3)
        rec = Recorder(c, n, coherent=False, path=path)
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(n_win)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for w in range(n_win):
            e = ev[w]
            e[0].record()
            t = sim.window(n_steps, n_sub)
            e[1].record()
            rec.record(DeviceBatch(t, n))
            e[2].record()
            S = rec.snapshot()
            e[3].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        push = sum(e[0].elapsed_time(e[1]) for e in ev)
        record = sum(e[1].elapsed_time(e[2]) for e in ev)
        snap = sum(e[2].elapsed_time(e[3]) for e in ev)
        assert np.all(np.isfinite(S))
        sim_steps = n_win * n_steps
        res[path] = {"wall_s": wall, "push_ms": push, "record_ms": record, "snapshot_ms": snap,
                     "recording_terms_per_s": res["terms"] / ((record + snap) * 1e-3),
                     "synthesis_ms_per_simulation_step": (record + snap) / sim_steps,
                     "push_ms_per_simulation_step": push / sim_steps}
        log(f"[bench] coupled in situ ({path}): push {push:.0f} ms, recording {record:.0f} ms, snapshots "
            f"{snap:.0f} ms over {sim_steps} simulation steps; recording "
            f"{res[path]['recording_terms_per_s']:.3e} terms/s")
        if path == "fp32":  # pitch cones of the final momenta (Section 3.2 analysis)
            ux, uy, uz = (sim.state[3 + k].contiguous() for k in range(3))
            theta = [m * np.pi / 8 for m in range(5)]
            edges = np.exp(np.linspace(0.0, np.log(2500.0), 41))
            c.pitch_cones(ux, uy, uz, [1.0, 0.0, 0.0], theta, 1.0 / 3.0, edges, member=True)  # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            counts, dev, _ = c.pitch_cones(ux, uy, uz, [1.0, 0.0, 0.0], theta, 1.0 / 3.0, edges, member=True)
            res["pitch_cones_ms"] = (time.perf_counter() - t1) * 1e3
            res["pitch_cone_counts"] = [int(x) for x in counts.sum(axis=1)]
        del rec, sim
        c.close()
        torch.cuda.empty_cache()
    return res


def band_relative(S, ref, floor=1e-4):
    S = np.asarray(S).reshape(-1, np.shape(S)[-1])
    ref = np.asarray(ref).reshape(-1, np.shape(ref)[-1])
    worst = 0.0
    for s_, r_ in zip(S, ref):
        m = r_ >= floor * r_.max()
        if m.any():
            worst = max(worst, float(np.max(np.abs(s_[m] - r_[m]) / r_[m])))
    return worst


def batched_leg(a, log):
    """Uneven multi-species workload: plain grid vs persistent launch vs autotuned shape, and
    a captured graph of the tuned launch (FP32 path), plus the tuned matrix-core path.  The
    tuner times its candidates on the first particles; the chosen shape then runs the whole
    slice.  The persistent launch records each compute unit's busy time (load balance)."""
    import torch

    from paper_1003_1140_amd import Context, DeviceBatch
    from workloads import configs
    from workloads.gpu import generate_device

    n = a.batched_particles
    rec = configs.uneven_recipe()
    t, ns = generate_device(rec, 0, n)
    b = DeviceBatch(t, n)
    nt = min(n, a.batched_tune_particles)
    bt = b.head(nt)
    dirs, om = configs.dirs_equal_area(), configs.log_grid(0.1, 1e3, 1024)
    terms = float(ns) * len(dirs) * len(om)
    ctx = Context(0)
    ctx.set_directions(dirs)
    ctx.set_frequencies(om)
    ctx.set_species(3)
    ctx.set_profiling(True)

    def timed(fn, reps=1):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    out = {"workload": f"{n} of the 4e5 particles of the uneven workload (47.5 % e-, 47.5 % e+, 5 % ions of "
                       f"mass 16; gamma0 2/5/15; lengths U[256, 8192]; {ns} samples), 64 equal-area "
                       f"directions, 1024 log omega in [0.1, 1e3], 3 species; tuner candidates timed on the "
                       f"first {nt} particles", "terms": terms}
    ws = ctx.workspace(b, "fp32")
    ctx.set_tuning(persistent=0)
    s_plain = timed(lambda: ctx.accumulate(b, "fp32", workspace=ws))
    S_plain = ctx.read_spectra() / 2.0
    ctx.reset()
    ctx.set_tuning(persistent=1)
    ctx.plan_batch(b, "fp32")
    s_pers = timed(lambda: ctx.accumulate(b, "fp32", workspace=ws))
    busy_default = ctx.profile_cu_busy()
    t0 = time.perf_counter()
    rep_fp32 = ctx.tune(bt, "fp32", repeats=1)
    t_tune = time.perf_counter() - t0
    if rep_fp32["best"].get("persistent"):
        ctx.plan_batch(b, "fp32")  # the tuned shape, planned for the whole slice
    ws = ctx.workspace(b, "fp32")  # the tuned shape may need a different workspace
    ctx.reset()
    ctx.profile_read()
    s_tuned = timed(lambda: ctx.accumulate(b, "fp32", workspace=ws))
    prof = ctx.profile_read()
    busy_tuned = ctx.profile_cu_busy() if rep_fp32["best"].get("persistent") else None
    S_tuned = ctx.read_spectra() / 2.0
    m = S_plain > 1e-4 * S_plain.max(axis=-1, keepdims=True)
    tuned_vs_plain = float(np.max(np.abs(S_tuned - S_plain)[m] / S_plain[m]))
    g = ctx.graph_capture(b, "fp32", workspace=ws)
    s_graph = timed(g.launch)
    g.close()
    rep_mfma = ctx.tune(bt, "mfma_f16", repeats=1)
    wsm = ctx.workspace(b, "mfma_f16")
    ctx.reset()
    s_mfma = timed(lambda: ctx.accumulate(b, "mfma_f16", workspace=wsm))
    S_mfma = ctx.read_spectra() / 2.0
    out.update({"fp32_plain_grid_terms_per_s": terms / s_plain, "fp32_persistent_terms_per_s": terms / s_pers,
                "fp32_tuned_terms_per_s": terms / s_tuned, "fp32_tuned_graph_terms_per_s": terms / s_graph,
                "mfma_f16x3_tuned_terms_per_s": terms / s_mfma, "tuner_seconds_fp32": t_tune,
                "tuned_fp32": rep_fp32["best"], "tuned_mfma": rep_mfma["best"],
                "fp32_tuned_kernel_ms": prof["direct_ms"] / max(prof["direct_launches"], 1),
                "fp32_tuned_vs_plain_max_rel": tuned_vs_plain,
                "mfma_vs_fp32_band_integrated": band_integrated_error(S_mfma, S_plain, om),
                "cu_busy_persistent_default": busy_default,
                "cu_busy_spread_persistent_default": (busy_default["max_ms"] - busy_default["min_ms"])
                / busy_default["mean_ms"],
                "cu_busy_persistent_tuned": busy_tuned})
    if busy_tuned:
        out["cu_busy_spread_persistent_tuned"] = (busy_tuned["max_ms"] - busy_tuned["min_ms"]) / busy_tuned["mean_ms"]
    log(f"[bench] batched: plain {terms / s_plain:.3e}, persistent {terms / s_pers:.3e}, tuned "
        f"{terms / s_tuned:.3e}, graph {terms / s_graph:.3e}, mfma {terms / s_mfma:.3e} terms/s; per-CU busy "
        f"{busy_default['min_ms']:.1f}..{busy_default['max_ms']:.1f} ms over {busy_default['cus']} CUs")
    return out


def surrogate_leg(a, log):
    """Train the surrogate, then time it against the exact path on 1e6 particles."""
    import torch

    from paper_1003_1140_amd import Context, DeviceBatch
    from paper_1003_1140_amd import surrogate as sg
    from workloads import configs
    from workloads.gpu import generate_device

    cfg = configs.WORKLOADS["surrogate"]
    rec = configs.surrogate_recipe(cfg["steps"])
    dirs, om = configs.dirs_jitter(), configs.log_grid(*cfg["omega"])
    ctxs = []
    for _ in range(1 + 3):  # surrogate pipeline, then exact subsamples at 1/16, 1/8, 1/4
        c = Context(0)
        c.set_directions(dirs)
        c.set_frequencies(om)
        ctxs.append(c)
    ctx, subs = ctxs[0], ctxs[1:]
    fracs = (1 / 16, 1 / 8, 1 / 4)
    exact = Context(0)
    exact.set_directions(dirs)
    exact.set_frequencies(om)
    exact_m = Context(0)  # the matrix-core exact path (FP16 hi/lo) on the same particles
    exact_m.set_directions(dirs)
    exact_m.set_frequencies(om)
    exact_m.set_mfma_options(1, 3, 3)
    t = time.perf_counter()
    tt, _ = generate_device(rec, 0, cfg["n_train"])
    tc, _ = generate_device(rec, cfg["n_train"], cfg["n_calib"])
    log(f"[bench] surrogate: generated {cfg['n_train']} + {cfg['n_calib']} particles in "
        f"{time.perf_counter() - t:.1f} s")
    sur = sg.train(ctx, DeviceBatch(tt, cfg["n_train"]), DeviceBatch(tc, cfg["n_calib"]),
                   steps=a.surrogate_steps, fallback_fraction=cfg["fallback"], log=log)
    del tt, tc
    torch.cuda.empty_cache()
    ctx.reset()
    judge = sg.Judge(ctx, exact_path=a.surrogate_judge_path)
    n, chunk, first = a.surrogate_infer, min(a.surrogate_chunk, a.surrogate_infer), cfg["infer_first_id"]
    t_exact = t_pipe = t_mfma = 0.0
    fallback = 0
    terms = 0.0
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        tb, ns = generate_device(rec, first + c0, m)
        b = DeviceBatch(tb, m)
        terms += float(ns) * len(dirs) * len(om)
        held = sg.held_out_indices(m, first + c0, cfg["held_out"], 11406)
        if c0 == 0:  # allocate the network's activation workspace before timing
            sur.net.forward(ctx.features(b).view(-1, 16))
            ctx.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        exact.accumulate(b, "fp32")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = sg.infer_chunk(ctx, sur, b, judge=judge, held=held, exact_path=a.surrogate_fallback_path)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ws_m = exact_m.workspace(b, "mfma_f16")  # plans the grids (synchronises) before timing
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        exact_m.accumulate(b, "mfma_f16", workspace=ws_m)
        torch.cuda.synchronize()
        t_mfma += time.perf_counter() - t3
        del ws_m
        t_exact += t1 - t0
        t_pipe += t2 - t1
        fallback += r["fallback"]
        for f, sc in zip(fracs, subs):
            sc.accumulate(b.head(max(1, int(round(f * m)))), "fp32")
        del tb, b
    S_pipe, S_exact = ctx.read_spectra(), exact.read_spectra()
    S_mfma = exact_m.read_spectra()
    Se, Sp, Ss = judge.spectra()
    held_err = sg.held_out_errors(Se, Sp)
    floor = sg.split_half_floor(Se, judge.half_spectrum())
    sur_only = sg.held_out_errors(Se, Ss)
    ens = sg.held_out_errors(S_exact, S_pipe)
    sub = {f"{f:.4f}": sg.held_out_errors(S_exact, sc.read_spectra() / f)["per_bin_median"]
           for f, sc in zip(fracs, subs)}
    return {
        "workload": f"{n} particles (ids from {first}) of the surrogate ensemble, 4096 steps, 4 dirs, "
                    f"256 log omega in [0.1,1e3]; trained on {cfg['n_train']} particles' exact spectra "
                    f"({sur.stats['train_pairs']} pairs), calibrated on {cfg['n_calib']}",
        "equivalent_terms_per_s": terms / t_pipe, "exact_terms_per_s": terms / t_exact,
        "gain_vs_exact": t_exact / t_pipe, "seconds_pipeline": t_pipe, "seconds_exact": t_exact,
        "exact_mfma_f16x3_terms_per_s": terms / t_mfma, "gain_vs_exact_mfma": t_mfma / t_pipe,
        "exact_mfma_vs_fp32_band_integrated": band_integrated_error(S_mfma, S_exact, om),
        "fallback_fraction": fallback / n, "fallback_path": a.surrogate_fallback_path,
        "judge_path": a.surrogate_judge_path, "held_out_particles": judge.n,
        "held_out_per_bin_max": held_err["per_bin_max"], "held_out_per_bin_median": held_err["per_bin_median"],
        "held_out_split_half_floor_per_bin_max": floor["per_bin_max"],
        "held_out_split_half_floor_per_bin_median": floor["per_bin_median"],
        "held_out_band_integrated_max": band_integrated_error(Sp, Se, om),
        "held_out_surrogate_only_per_bin_max": sur_only["per_bin_max"],
        "held_out_surrogate_only_per_bin_median": sur_only["per_bin_median"],
        "ensemble_per_bin_max": ens["per_bin_max"], "ensemble_per_bin_median": ens["per_bin_median"],
        "ensemble_band_integrated_max": band_integrated_error(S_pipe, S_exact, om),
        "exact_subsample_per_bin_median": sub,
        "train": {k: v for k, v in sur.stats.items()},
    }


def headline_workload(name):
    from workloads import configs

    if name == "c3":
        return configs.wide_recipe(), configs.dirs_wide(), configs.log_grid(0.1, 1e3, 2048), 2048
    return configs.jitter_recipe(), configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 1024), 4096


def time_paths(ctx, batch, paths, steps, warmup, terms_per_step, a, log):
    results, spectra = {}, {}
    for path in paths:
        results[path], spectra[path] = time_path(ctx, batch, path, steps, warmup, terms_per_step,
                                                 a.bands, a.tile)
        log(f"[bench] {path}: {results[path]['terms_per_s']:.3e} terms/s")
    return results, spectra


def c2_leg(a, log):
    """The jitter ensemble (1e5 particles x 4096 samples, 4 directions, 1024 frequencies): the
    FP32 path's own configuration, the headline matrix-core path on it, and the coherent,
    in-situ and coupled recording legs."""
    import torch

    from paper_1003_1140_amd import Context

    dev = torch.device("cuda:0")
    recipe, dirs, om, steps_per_particle = headline_workload("c2")
    batch = upload_ensemble(recipe, a.c2_particles, a.chunk, dev, host=a.host_generator)
    terms = float(batch.n_samples_host) * len(dirs) * len(om)
    ctx = Context(0)
    ctx.set_directions(dirs)
    ctx.set_frequencies(om)
    ctx.set_profiling(True)
    if a.tile:
        ctx.set_tuning(tile=a.tile)
    out = {"workload": f"filamentation-jitter ensemble: {a.c2_particles} e- of gamma0=3 counter-streaming "
                       "beams, 4096 Boris steps, 4 dirs (+x,-x,+y,+z), 1024 log omega in [0.1,1e3]",
           "terms_per_step": terms}
    res, spec = time_paths(ctx, batch, ["fp32"], a.c2_steps, 1, terms, a, log)
    res2, spec2 = time_paths(ctx, batch, ["mfma_f16x3"], max(a.steps, 2), 1, terms, a, log)
    res.update(res2)
    spec.update(spec2)
    res["mfma_f16x3"]["band_integrated_err_vs_fp32"] = band_integrated_error(spec["mfma_f16x3"], spec["fp32"], om)
    res["mfma_f16x3"]["speedup_vs_fp32"] = res["mfma_f16x3"]["terms_per_s"] / res["fp32"]["terms_per_s"]
    attach_traffic(res["mfma_f16x3"], "mfma_f16x3", a.tile, a.c2_particles, "c2", a.bands)
    out["paths"] = res
    ctx.close()
    if not a.no_insitu:
        out["insitu"] = insitu_leg(a, batch, terms, dirs, om, spec["fp32"], log)
    del batch
    torch.cuda.empty_cache()
    if not a.no_coupled:
        out["coupled"] = coupled_leg(a, dirs, om, log)
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (no multi-GPU path); --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_1003_1140_amd import Context

    def log(m):
        print(m, file=sys.stderr, flush=True)

    torch.cuda.init()
    dev = torch.device("cuda:0")
    if a.copy_probe_mib > 0:
        n = a.copy_probe_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {n} bytes read and {n} bytes written")
        del src, dst
    recipe, dirs, om, n_steps = headline_workload(a.workload)
    if a.particles <= 0:
        a.particles = C3_PARTICLES if a.workload == "c3" else 100_000
    t = time.perf_counter()
    batch = upload_ensemble(recipe, a.particles, a.chunk, dev, host=a.host_generator)
    terms_per_step = float(batch.n_samples_host) * len(dirs) * len(om)
    log(f"[bench] generated and uploaded {a.particles} particles ({batch.n_samples_host} samples) "
        f"in {time.perf_counter() - t:.1f} s")

    ctx = Context(0)
    ctx.set_directions(dirs)
    ctx.set_frequencies(om)
    ctx.set_profiling(True)
    if a.tile:
        ctx.set_tuning(tile=a.tile)
    paths = [p for p in a.paths.split(",") if p]
    head = paths[-1]
    results, spectra = {}, {}
    for path in paths:  # the headline path gets the requested steps, the others a few
        st, wu = (a.steps, a.warmup) if path == head else (min(a.steps, a.other_path_steps), 1)
        r_, s_ = time_paths(ctx, batch, [path], st, wu, terms_per_step, a, log)
        results.update(r_)
        spectra.update(s_)
    r = results[head]
    # the FP32 path on the first particles of the same workload: speedup at equal shape, and
    # every matrix-core path's spectrum on those particles against it
    fp32_cmp = None
    if "fp32" not in results and a.fp32_particles > 0:
        sub = batch.head(min(a.fp32_particles, a.particles))
        sub.n_samples_host = int(sub.t["offsets"][sub.n_particles].item() - sub.t["offsets"][0].item())
        terms_sub = float(sub.n_samples_host) * len(dirs) * len(om)
        rf, sf = time_path(ctx, sub, "fp32", 2, 1, terms_sub, a.bands, a.tile)
        fp32_cmp = {"particles": sub.n_particles, "terms_per_s": rf["terms_per_s"],
                    "ms_per_step": rf["ms_per_step"], "roofline": rf["roofline"]}
        for name in paths:
            path, products = split_path(name)
            mfma_options(ctx, a.bands, path, products)
            ctx.reset()
            ctx.accumulate(sub, path, workspace=ctx.workspace(sub, path))
            fp32_cmp[name + "_band_integrated_err_vs_fp32"] = band_integrated_error(ctx.read_spectra(), sf, om)
            results[name]["speedup_vs_fp32_same_workload"] = results[name]["terms_per_s"] / rf["terms_per_s"]
        log(f"[bench] fp32 on {sub.n_particles} particles of the same workload: {rf['terms_per_s']:.3e} terms/s")
        del sub
    if "roofline_contraction" in r:
        attach_traffic(r, head, a.tile, a.particles, a.workload, a.bands)
    ctx.close()
    del batch
    torch.cuda.empty_cache()
    path_dtype = {"fp32": "f32 (f64 phase)", "mfma_f16": "f16 hi/lo operands, f32 acc",
                  "mfma_bf16": "bf16 hi/lo operands, f32 acc"}[split_path(head)[0]]
    if split_path(head)[1] == 1 and head != "fp32":
        path_dtype = path_dtype.replace(" hi/lo", "")
    if split_path(head)[1] == 2:
        path_dtype = "f16 operands (F hi/lo, table once), f32 acc"
    if a.workload == "c3":
        whole = a.particles == C3_PARTICLES
        config = {"workload": ("mixed-precision form: " + ("all of its" if whole else f"a slice of {a.particles} of its")
                               + " 1e6 particles per step, jitter generator (gamma0=3 counter-streaming e- beams, "
                               "kT=0.01, static random-filament B_y, deflection 0.3), 2048 Boris steps, 16 dirs "
                               "(head-on, 15/30/45 deg at 4 azimuths, 3 perpendicular), 2048 log omega in [0.1,1e3]"),
                  "particles_per_step": a.particles, "full_ensemble_particles": C3_PARTICLES,
                  "samples_per_particle": 2048, "directions": len(dirs), "frequencies": 2048,
                  "path": head, "bands": a.bands}
    else:
        config = {"workload": f"filamentation-jitter ensemble: {a.particles} e- of gamma0=3 counter-streaming "
                              "beams, 4096 Boris steps, 4 dirs (+x,-x,+y,+z), 1024 log omega in [0.1,1e3]; "
                              "1 step = the whole ensemble",
                  "particles": a.particles, "samples_per_particle": 4096, "directions": 4,
                  "frequencies": 1024, "path": head, "bands": a.bands}
    out = {
        "metric": "LW spectral terms/s (particle x step x omega x n)",
        "value": r["terms_per_s"],
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": path_dtype,
        "data": "synthetic",
        "config": config,
        "roofline": r["roofline"],
        **({"roofline_contraction": r["roofline_contraction"], "roofline_spread": r["roofline_spread"]}
           if "roofline_contraction" in r else {}),
        "paths": results,
    }
    if a.workload == "c3":
        out["full_c3_seconds"] = C3_TERMS / r["terms_per_s"]
    if fp32_cmp is not None:
        out["fp32_same_workload"] = fp32_cmp
    if not a.no_oracle_check:
        out["oracle_check"] = oracle_check(recipe, dirs, om, ["fp32"] + [p for p in paths if p != "fp32"], a.bands)
        log(f"[bench] oracle check on 8 particles: " + ", ".join(
            f"{k} {v['band_integrated_err']:.2e}" for k, v in out["oracle_check"].items() if isinstance(v, dict)))
    if not a.no_c2 and a.workload == "c3":
        out["c2"] = c2_leg(a, log)
        torch.cuda.empty_cache()
    if not a.no_batched:
        out["batched"] = batched_leg(a, log)
        torch.cuda.empty_cache()
    if not a.no_surrogate:
        torch.cuda.empty_cache()
        out["surrogate"] = surrogate_leg(a, log)
        log(f"[bench] surrogate: {out['surrogate']['equivalent_terms_per_s']:.3e} equivalent terms/s, "
            f"gain {out['surrogate']['gain_vs_exact']:.2f}x over exact FP32, "
            f"{out['surrogate']['gain_vs_exact_mfma']:.2f}x over exact MFMA")
    if not a.no_cpu_baseline:
        log("[bench] running CPU oracle baseline")
        label = "mixed-precision form" if a.workload == "c3" else "jitter ensemble"
        out["cpu_baseline"] = cpu_baseline(recipe, dirs, om, a.cpu_seconds, label)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
