"""Learned spectrum surrogate, driven through the C ABI.

Every arithmetic step runs in the library's kernels: features, network forward,
backward and AdamW, training targets, the surrogate sum, the fallback list and
the exact accumulations.  Torch holds device memory and gathers minibatch rows;
the normalisation statistics and the per-bin calibration are computed once on
the host in FP64 from copies.

* targets: each (particle, direction)'s own spectrum from the exact FP32 path
  (per-particle output) as y = log10(S_p / (w q^2) + 1e-30) on the surrogate's
  frequency grid;
* inputs: the 16 trajectory features, normalised in FP32 inside the network
  (shift and scale from the training set; constant features get scale 0);
* network: 16 -> 3 x 256 (GELU) -> n_omega on BF16 matrix cores with FP32
  accumulation, AdamW with a cosine learning-rate schedule; the last layer starts
  from the per-bin mean and spread of the targets;
* calibration split (particles the network never saw): the error head learns
  each pair's RMS log10 error, the fallback threshold is the quantile that sends
  a chosen fraction of particles to the exact path, and a per-bin factor removes
  the bias of 10^<log S> against <S> in the summed spectra;
* inference: unflagged particles add their predicted spectra, flagged ones are
  accumulated exactly; a seeded held-out fraction is also accumulated exactly
  and by the surrogate alone, on judge contexts, and compared.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from .lw import MLP, Context, DeviceBatch

FLOOR = 1e-30


def exact_log_spectra(ctx: Context, batch: DeviceBatch) -> torch.Tensor:
    """Training targets: device [P * nd, nw] log10 of each pair's spectrum / (w q^2)."""
    P = batch.n_particles
    pp = torch.zeros((P, ctx.nd, ctx.nw), dtype=torch.float32, device=f"cuda:{ctx.device}")
    ctx.accumulate(batch, "fp32", per_particle=pp)
    ctx.read_spectra()
    ctx.reset()
    return ctx.surrogate_targets(batch, pp, FLOOR).view(P * ctx.nd, ctx.nw)


def _host(t) -> np.ndarray:
    return t.detach().to("cpu").numpy().astype(np.float64)


@dataclass
class Surrogate:
    net: MLP             # network with its error head and input normalisation
    threshold: float     # error-head threshold of the exact fallback
    train_loss: list = field(default_factory=list)
    head_loss: list = field(default_factory=list)
    stats: dict = field(default_factory=dict)


def train(ctx: Context, batch: DeviceBatch, calib: DeviceBatch, steps=1500, batch_rows=4096, lr=1e-3,
          weight_decay=1e-5, fallback_fraction=0.05, head_steps=600, head_lr=3e-3, seed=1,
          log=None) -> Surrogate:
    """Train the network on `batch` and its error head and calibration on `calib`."""
    dev = torch.device(f"cuda:{ctx.device}")
    t_start = time.perf_counter()
    x = ctx.features(batch).view(-1, 16).contiguous()
    y = exact_log_spectra(ctx, batch)
    torch.cuda.synchronize(dev)
    t_targets = time.perf_counter() - t_start
    xh, yh = _host(x), _host(y)
    mu_x, sd_x = xh.mean(0), xh.std(0)
    scale_x = np.where(sd_x > 1e-6 * (np.abs(mu_x) + 1.0), 1.0 / np.maximum(sd_x, 1e-300), 0.0)
    mu_y, sd_y = yh.mean(0), np.maximum(yh.std(0), 1e-3)
    net = MLP(ctx, 16, 256, 3, ctx.nw, seed=seed)
    net.set_input_norm(mu_x, scale_x)
    p, head = net.get_params()
    n_out = ctx.nw
    off_last = p.size - (n_out * 256 + n_out)
    p[off_last: off_last + n_out * 256] *= np.repeat(sd_y, 256).astype(np.float32)
    p[-n_out:] = mu_y
    net.set_params(p, head)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    rows = x.shape[0]
    nb = min(batch_rows, rows)
    losses = []
    t0 = time.perf_counter()
    for step in range(steps):
        idx = torch.randint(0, rows, (nb,), device=dev, generator=g)
        lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * step / steps))
        losses.append(net.train_step(x[idx].contiguous(), y[idx].contiguous(), lr=float(lr_t),
                                     weight_decay=weight_decay))
        if log and (step % 250 == 0 or step == steps - 1):
            log(f"[surrogate] step {step} loss {losses[-1]:.5f} ({time.perf_counter() - t0:.1f} s)")
    t_train = time.perf_counter() - t0
    # calibration split: realised errors, error head, per-bin bias, threshold
    xc = ctx.features(calib).view(-1, 16).contiguous()
    yc = exact_log_spectra(ctx, calib)
    pred = net.forward(xc)
    ph, ych = _host(pred), _host(yc)
    rms = np.sqrt(np.mean((ph - ych) ** 2, axis=1))
    rms_d = torch.from_numpy(rms.astype(np.float32)).to(dev)
    head_losses = []
    for step in range(head_steps):
        idx = torch.randint(0, xc.shape[0], (min(batch_rows, xc.shape[0]),), device=dev, generator=g)
        head_losses.append(net.train_head_step(xc[idx].contiguous(), rms_d[idx].contiguous(), lr=head_lr))
    ratio = (10.0 ** ych).sum(0) / (10.0 ** ph).sum(0)
    p, head = net.get_params()
    p = p.astype(np.float64)
    p[-n_out:] += np.log10(ratio)
    net.set_params(p.astype(np.float32), head)
    _, err = net.forward(xc, with_error=True)
    per_particle = _host(err).reshape(-1, ctx.nd).max(1)
    thr = float(np.quantile(per_particle, 1.0 - fallback_fraction)) if fallback_fraction > 0 else float("inf")
    stats = {"train_pairs": int(rows), "calib_pairs": int(xc.shape[0]), "steps": steps,
             "final_train_loss": float(np.mean(losses[-50:])) if losses else None,
             "calib_rms_log10_median": float(np.median(rms)), "calib_rms_log10_p90": float(np.quantile(rms, 0.9)),
             "calib_bias_log10_max": float(np.max(np.abs(np.log10(ratio)))), "threshold": thr,
             "seconds_targets": t_targets, "seconds_train": t_train}
    return Surrogate(net=net, threshold=thr, train_loss=losses, head_loss=head_losses, stats=stats)


class Judge:
    """Exact and surrogate-only accumulators of the held-out particles."""

    def __init__(self, ctx: Context):
        om = ctx.get_frequencies()
        self.exact = Context(ctx.device)
        self.sur = Context(ctx.device)
        for c in (self.exact, self.sur):
            c.set_directions(ctx.dirs)
            c.set_frequencies(om)
            c.set_species(ctx.ns)
        self.n = 0

    def add(self, batch: DeviceBatch, ylog, held_idx):
        """held_idx: device int64 indices (increasing) of the chunk's held-out particles."""
        if held_idx.numel() == 0:
            return
        self.exact.accumulate_subset(batch, held_idx)
        mask = torch.ones(batch.n_particles, self.sur.nd, dtype=torch.float32, device=ylog.device)
        mask[held_idx] = 0.0
        self.sur.surrogate_accumulate(batch, ylog, mask, 0.5)
        self.n += int(held_idx.numel())

    def spectra(self):
        return self.exact.read_spectra(), self.sur.read_spectra()


def infer_chunk(ctx: Context, sur: Surrogate, batch: DeviceBatch, judge: Judge | None = None, held_idx=None,
                threshold=None) -> dict:
    """Add the surrogate estimate of one chunk to ctx's S (exact for flagged particles)."""
    thr = sur.threshold if threshold is None else threshold
    x = ctx.features(batch).view(-1, 16)
    ylog, err = sur.net.forward(x, with_error=True)
    _, idx, cnt = ctx.surrogate_accumulate(batch, ylog, err, thr, compact=True)
    n_flag = int(cnt.item())
    if n_flag:
        ctx.accumulate_subset(batch, idx[:n_flag])
    if judge is not None and held_idx is not None:
        judge.add(batch, ylog, held_idx)
    return {"fallback": n_flag}


def held_out_errors(S_exact, S_sur, floor=1e-4):
    """Per-bin relative error of the summed held-out spectrum (bins >= floor of each direction's peak)."""
    worst, med = [], []
    for se, ss in zip(S_exact.reshape(-1, S_exact.shape[-1]), S_sur.reshape(-1, S_sur.shape[-1])):
        m = se >= floor * se.max()
        rel = np.abs(ss[m] - se[m]) / se[m]
        worst.append(float(rel.max()))
        med.append(float(np.median(rel)))
    return {"per_bin_max": max(worst), "per_bin_median": float(np.median(med)), "per_direction_max": worst}


def held_out_indices(n_particles: int, first_id: int, fraction: float, seed: int) -> np.ndarray:
    """Seeded held-out subset of particle ids first_id .. first_id + n - 1 (chunk-local, increasing)."""
    rng = np.random.Generator(np.random.Philox(key=seed + (first_id << 20)))
    return np.flatnonzero(rng.random(n_particles) < fraction).astype(np.int64)
