"""Throughput of the radiation spectral synthesis on one MI355X.

Workload: the filamentation-jitter ensemble -- electrons of two gamma0 = 3
counter-streaming beams (kT = 0.01 rest-frame spread), 4096 Boris samples
each through a static random-filament field (k^-2 over [0.5, 8], deflection
parameter 0.3), observed along +x, -x, +y, +z on 1024 log-spaced frequencies
over [0.1, 1e3] omega_p.  One step = one lw_accumulate over the whole
1e5-particle ensemble (prepass, accumulation, particle reduction) with its
trajectories (25 GB) already resident in HBM.

metric: terms/s, a term being one (particle, sample, direction, frequency)
product of the spectral sum.

Prints one JSON line.  Options: --steps K --warmup W --particles P --path fp32.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--particles", type=int, default=100_000)
    ap.add_argument("--chunk", type=int, default=8192, help="particles generated per host chunk")
    ap.add_argument("--path", default="fp32", choices=["fp32"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def cpu_baseline(recipe, dirs, om, target_s):
    import oracle
    import workloads

    nthreads = oracle.max_threads()
    cal = workloads.generate(recipe, 10_000_000, 2)
    t = time.perf_counter()
    oracle.spectrum(cal, dirs, om, n_species=1, nthreads=nthreads)
    dt_cal = time.perf_counter() - t
    per_particle = dt_cal / 2
    n = int(max(2, min(512, target_s / max(per_particle, 1e-6))))
    sample = workloads.generate(recipe, 10_000_000, n)
    t = time.perf_counter()
    oracle.spectrum(sample, dirs, om, n_species=1, nthreads=nthreads)
    el = time.perf_counter() - t
    terms = sample.n_samples * len(dirs) * len(om)
    return {"value": terms / el, "unit": "terms/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n} jitter particles x {sample.n_samples // n} samples x {len(dirs)} dirs x "
                      f"{len(om)} freqs, FP64 libm sin/cos, {el:.1f} s"}


def upload_ensemble(recipe, n, chunk, dev):
    """The whole ensemble in device memory, generated on the host chunk by chunk."""
    from paper_1003_1140_amd import DeviceBatch
    from workloads.device import upload_chunks

    tensors, ns = upload_chunks(recipe, n, chunk, dev)
    b = DeviceBatch(tensors, n)
    b.n_samples_host = ns
    return b


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import workloads
    from workloads import configs
    from paper_1003_1140_amd import Context, DeviceBatch

    torch.cuda.init()
    dev = torch.device("cuda:0")
    recipe = configs.jitter_recipe()
    dirs = configs.dirs_jitter()
    om = configs.log_grid(0.1, 1e3, 1024)
    t = time.perf_counter()
    batch = upload_ensemble(recipe, a.particles, a.chunk, dev)
    terms_per_step = float(batch.n_samples_host) * len(dirs) * len(om)
    print(f"[bench] generated and uploaded {a.particles} particles ({batch.n_samples_host} samples) "
          f"in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)

    ctx = Context(0)
    ctx.set_directions(dirs)
    ctx.set_frequencies(om)
    ws = ctx.workspace(batch, a.path)
    stream = torch.cuda.current_stream(dev)
    for i in range(a.warmup):
        ctx.accumulate(batch, a.path, workspace=ws)
    torch.cuda.synchronize()
    print(f"[bench] warmup done", file=sys.stderr, flush=True)

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        ev[i][0].record(stream)
        ctx.accumulate(batch, a.path, workspace=ws)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    S = ctx.read_spectra()
    assert np.all(np.isfinite(S))
    launch_s = [e0.elapsed_time(e1) * 1e-3 for e0, e1 in ev]
    timed_terms = terms_per_step * a.steps
    value = timed_terms / el
    per_launch = timed_terms / a.steps
    achieved = per_launch / (sum(launch_s) / len(launch_s))
    peak = fp32_term_peak()
    out = {
        "metric": "LW spectral terms/s (particle x step x omega x n)",
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": el / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 phase)",
        "data": "synthetic",
        "config": {"workload": f"filamentation-jitter ensemble: {a.particles} e- of gamma0=3 "
                               "counter-streaming beams, 4096 Boris steps, 4 dirs (+x,-x,+y,+z), "
                               "1024 log omega in [0.1,1e3]; 1 step = the whole ensemble",
                   "particles": a.particles, "samples_per_particle": 4096, "directions": 4,
                   "frequencies": 1024, "path": a.path},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "Tterm/s", "frac": achieved / peak, "traffic": None,
                     "kernel": "lw_direct_f32_kernel<4>"},
    }
    if not a.no_cpu_baseline:
        print(f"[bench] timed {a.steps} steps in {el:.2f} s; running CPU oracle baseline",
              file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(recipe, dirs, om, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
