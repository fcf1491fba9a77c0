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
  accumulation, AdamW with a cosine learning-rate schedule.  Feature 11 is the
  log of the energy radiated towards n, which by Parseval's theorem is the
  frequency integral of the pair's spectrum; it is added to every output, so
  the network learns the spectral shape, log10(S / E), while the heavy-tailed
  amplitude comes from the trajectory exactly.  The last layer starts from the
  per-bin mean and spread of that shape;
* calibration split (particles the network never saw): the error head learns
  the log10 of each pair's share in the error of the summed spectrum, the mean
  over bins of |S_pred - S| / <S>_d (with <S>_d the mean per-pair spectrum of
  the direction on the training set), so that the fallback goes to the pairs
  that would damage the ensemble most, not to those whose own log error is
  large; the fallback threshold is the quantile that sends a chosen fraction of
  particles to the exact path, and a factor per direction and bin, fitted on
  the particles the threshold keeps on the surrogate, removes the bias of
  10^<log S> against <S> in their summed spectra (applied by the surrogate sum);
* inference: unflagged particles add their predicted spectra, flagged ones are
  accumulated exactly; a seeded held-out fraction is also accumulated exactly
  and by the pipeline (surrogate, or exact where flagged), on judge contexts,
  and compared.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from .lw import MLP, Context, DeviceBatch

FLOOR = 1e-30
ENERGY_FEATURE = 11  # ln(E + 1e-30)
LOG10E = 1.0 / np.log(10.0)


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
    calib: object = None  # device [nd][nw] log10 correction of the summed predictions
    train_loss: list = field(default_factory=list)
    head_loss: list = field(default_factory=list)
    stats: dict = field(default_factory=dict)


def train(ctx: Context, batch: DeviceBatch, calib: DeviceBatch, steps=1500, batch_rows=4096, lr=1e-3,
          weight_decay=1e-5, fallback_fraction=0.05, head_steps=1000, head_lr=3e-3, seed=1,
          log=None) -> Surrogate:
    """Train the network on `batch` and its error head and calibration on `calib`."""
    dev = torch.device(f"cuda:{ctx.device}")
    t_start = time.perf_counter()
    x = ctx.features(batch).view(-1, 16).contiguous()
    y = exact_log_spectra(ctx, batch)
    torch.cuda.synchronize(dev)
    t_targets = time.perf_counter() - t_start
    # statistics on the device: feature moments, <S>_d per (direction, bin), and the moments of
    # the spectral shape (targets minus the Parseval skip); the host only sets the network's
    # normalisation parameters from them
    fx = _host(ctx.column_stats(x))[0]
    mu_x = fx[:, 0]
    sd_x = np.sqrt(np.maximum(fx[:, 1] - mu_x * mu_x, 0.0))
    scale_x = np.where(sd_x > 1e-6 * (np.abs(mu_x) + 1.0), 1.0 / np.maximum(sd_x, 1e-300), 0.0)
    s_mean = ctx.column_stats(y, groups=ctx.nd, exp10=True)
    fy = _host(ctx.column_stats(y, row_add=x[:, ENERGY_FEATURE], row_add_stride=x.shape[1],
                                row_add_coeff=-LOG10E))[0]
    mu_y = fy[:, 0]
    sd_y = np.maximum(np.sqrt(np.maximum(fy[:, 1] - mu_y * mu_y, 0.0)), 1e-3)
    net = MLP(ctx, 16, 256, 3, ctx.nw, seed=seed)
    net.set_input_norm(mu_x, scale_x)
    net.set_output_skip(ENERGY_FEATURE, LOG10E)
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
    rms = np.sqrt(np.mean((_host(pred) - _host(yc)) ** 2, axis=1))  # reported only
    # error-head targets: each pair's share in the error of the summed spectrum
    share_d = ctx.error_share(pred, yc, ctx.nd, s_mean, FLOOR)
    p, head = net.get_params()
    head[:] = 0.0
    head[-1] = float(_host(ctx.column_stats(share_d.view(-1, 1)))[0, 0, 0])
    net.set_params(p, head)
    head_losses = []
    for step in range(head_steps):
        idx = torch.randint(0, xc.shape[0], (min(batch_rows, xc.shape[0]),), device=dev, generator=g)
        lr_t = head_lr * 0.5 * (1.0 + np.cos(np.pi * step / head_steps))
        head_losses.append(net.train_head_step(xc[idx].contiguous(), share_d[idx].contiguous(), lr=float(lr_t)))
    _, err = net.forward(xc, with_error=True)
    # fallback threshold: the quantile of the per-particle largest predicted error; then the
    # per-bin calibration 10^<log S> -> <S> over the particles the threshold keeps
    thr = ctx.quantile_of_maxima(err, ctx.nd, 1.0 - fallback_fraction) if fallback_fraction > 0 else float("inf")
    sh = ctx.column_stats(yc, groups=ctx.nd, exp10=True, err=err, threshold=thr)
    sp = ctx.column_stats(pred, groups=ctx.nd, exp10=True, err=err, threshold=thr)
    calib_d = ctx.log_ratio(sh, sp)
    ratio = 10.0 ** _host(calib_d).reshape(ctx.nd, ctx.nw)  # reported only
    stats = {"train_pairs": int(rows), "calib_pairs": int(xc.shape[0]), "steps": steps,
             "final_train_loss": float(np.mean(losses[-50:])) if losses else None,
             "calib_rms_log10_median": float(np.median(rms)), "calib_rms_log10_p90": float(np.quantile(rms, 0.9)),
             "calib_bias_log10_max": float(np.max(np.abs(np.log10(ratio)))), "threshold": thr,
             "head_loss_first": head_losses[0] if head_losses else None,
             "head_loss_last": float(np.mean(head_losses[-50:])) if head_losses else None,
             "seconds_targets": t_targets, "seconds_train": t_train}
    sur = Surrogate(net=net, threshold=thr, calib=calib_d, train_loss=losses, head_loss=head_losses,
                    stats=stats)
    sur.input_shift, sur.input_scale, sur.calib_ratio = mu_x, scale_x, ratio
    return sur


def exact_subset(ctx: Context, batch: DeviceBatch, idx, path="fp32"):
    """Exact sum of the particles listed in idx (device int64) into ctx's S: the FP32 kernel
    walking the list, or another exact path ("mfma_f16": FP16 hi/lo operands, three products)
    on a copy of those particles gathered into a batch of their own."""
    if path == "fp32":
        ctx.accumulate_subset(batch, idx)
    else:
        ctx.accumulate(batch.gather(ctx, idx), path)


class Judge:
    """Accumulators of the held-out particles: exact, as the pipeline estimates them
    (surrogate, exact where flagged), and surrogate alone.  The exact sum is kept as two
    halves (every other held-out particle, counting across chunks, and the rest), so that the
    sampling noise of the held-out sum can be measured on the same particles (split-half
    floor) without summing any particle twice."""

    def __init__(self, ctx: Context, exact_path="fp32"):
        om = ctx.get_frequencies()
        self.exact_path = exact_path
        self.half, self.rest = Context(ctx.device), Context(ctx.device)
        self.pipe, self.sur = Context(ctx.device), Context(ctx.device)
        for c in (self.half, self.rest, self.pipe, self.sur):
            c.set_directions(ctx.dirs)
            c.set_frequencies(om)
            c.set_species(ctx.ns)
        self.n = 0

    def add(self, batch: DeviceBatch, ylog, held, flagged, calib=None):
        """held: host int64 indices (increasing) of the chunk's held-out particles;
        flagged: host int64 indices of the particles the pipeline computed exactly."""
        if held.size == 0:
            return
        dev = ylog.device
        P, nd = batch.n_particles, self.sur.nd
        held_d = torch.from_numpy(held).to(dev, non_blocking=True)
        # every other held-out particle (counting across chunks), and the rest
        first = self.n % 2
        exact_subset(self.half, batch, held_d[first::2].contiguous(), self.exact_path)
        rest = held_d[1 - first::2].contiguous()
        if rest.numel():
            exact_subset(self.rest, batch, rest, self.exact_path)
        # an "error" of 0 keeps a particle on the surrogate sum, 1 leaves it out (threshold 0.5)
        keep = torch.ones((P, nd), dtype=torch.float32, device=dev)
        keep[held_d] = 0.0
        self.sur.surrogate_accumulate(batch, ylog, keep, 0.5, calib=calib)
        held_flagged = np.intersect1d(held, flagged, assume_unique=True)
        if held_flagged.size:
            hf = torch.from_numpy(held_flagged).to(dev, non_blocking=True)
            keep[hf] = 1.0
            exact_subset(self.pipe, batch, hf, self.exact_path)
        self.pipe.surrogate_accumulate(batch, ylog, keep, 0.5, calib=calib)
        self.n += int(held.size)

    def spectra(self):
        """(exact, pipeline, surrogate-only) spectra of the held-out particles."""
        return (self.half.read_spectra() + self.rest.read_spectra(), self.pipe.read_spectra(),
                self.sur.read_spectra())

    def half_spectrum(self):
        """Exact spectrum of every other held-out particle."""
        return self.half.read_spectra()


def infer_chunk(ctx: Context, sur: Surrogate, batch: DeviceBatch, judge: Judge | None = None, held=None,
                threshold=None, exact_path="fp32") -> dict:
    """Add the surrogate estimate of one chunk to ctx's S (exact for flagged particles, on
    exact_path: see exact_subset).

    held: host int64 indices (increasing) of the chunk's held-out particles, judged when
    a Judge is given."""
    thr = sur.threshold if threshold is None else threshold
    x = ctx.features(batch).view(-1, 16)
    ylog, err = sur.net.forward(x, with_error=True)
    _, idx, cnt = ctx.surrogate_accumulate(batch, ylog, err, thr, compact=True, calib=sur.calib)
    n_flag = int(cnt.item())
    if n_flag:
        exact_subset(ctx, batch, idx[:n_flag], exact_path)
    if judge is not None and held is not None:
        flagged = idx[:n_flag].cpu().numpy() if n_flag else np.zeros(0, dtype=np.int64)
        judge.add(batch, ylog, np.asarray(held, dtype=np.int64), flagged, calib=sur.calib)
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


def split_half_floor(S_exact, S_half, floor=1e-4):
    """Sampling noise of the held-out sum, measured on the same particles: with S_a the exact
    sum of every other held-out particle and S_b = S - S_a the rest, |S_a - S_b| / S per bin
    has the spread of the difference between the held-out sum and a perfect prediction of its
    mean (the two halves are independent and each carries half the variance).  Per-bin max
    and median over the bins held_out_errors scores."""
    worst, med = [], []
    for se, sa in zip(S_exact.reshape(-1, S_exact.shape[-1]), S_half.reshape(-1, S_half.shape[-1])):
        m = se >= floor * se.max()
        rel = np.abs(2.0 * sa[m] - se[m]) / se[m]
        worst.append(float(rel.max()))
        med.append(float(np.median(rel)))
    return {"per_bin_max": max(worst), "per_bin_median": float(np.median(med)), "per_direction_max": worst}


def held_out_indices(n_particles: int, first_id: int, fraction: float, seed: int) -> np.ndarray:
    """Seeded held-out subset of particle ids first_id .. first_id + n - 1 (chunk-local, increasing)."""
    rng = np.random.Generator(np.random.Philox(key=seed + (first_id << 20)))
    return np.flatnonzero(rng.random(n_particles) < fraction).astype(np.int64)
