"""Helpers shared by the GPU parity tests: run the library through the C ABI and score it.

The score follows the accuracy statement of the FP32 path: per (species,
direction), the largest relative error over frequency bins whose reference
value is at least 1e-4 of that direction's peak.
"""
from __future__ import annotations

import numpy as np


def gpu_spectrum(batch, dirs, omega, path="fp32", n_species=1, per_particle=False, ctx=None):
    import torch

    from paper_1003_1140_amd import Context, DeviceBatch

    c = ctx or Context(0)
    c.set_directions(dirs)
    c.set_frequencies(omega)
    c.set_species(n_species)
    db = DeviceBatch.from_host(batch)
    pp = None
    if per_particle:
        pp = torch.zeros((batch.n_particles, len(np.atleast_2d(dirs)), len(omega)), dtype=torch.float32,
                         device="cuda")
    c.accumulate(db, path, per_particle=pp)
    S = c.read_spectra()
    if per_particle:
        return S, pp.cpu().numpy().astype(np.float64)
    return S


def band_relative_error(S, ref, floor=1e-4):
    """Max over (species, direction) of max_j |S - ref| / ref over bins with ref >= floor * max."""
    S = np.asarray(S, dtype=np.float64).reshape(-1, np.shape(S)[-1])
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, np.shape(ref)[-1])
    worst = 0.0
    for s, r in zip(S, ref):
        if r.max() <= 0:
            assert np.all(s == 0)
            continue
        m = r >= floor * r.max()
        worst = max(worst, float(np.max(np.abs(s[m] - r[m]) / r[m])))
    return worst


def all_bins_relative_error(S, ref):
    S = np.asarray(S, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    m = ref > 0
    return float(np.max(np.abs(S[m] - ref[m]) / ref[m])) if m.any() else 0.0


def band_integrated_errors(S, ref, omega, n_bands=16, floor=1e-4):
    """Relative error of the band-integrated power, per (species, direction) row.

    The frequency list is cut into ``n_bands`` equal runs; each band's power is
    the trapezoid integral of S d(omega) in ln(omega) (S * omega d ln omega).  Bands
    whose reference power is below ``floor`` of the row's strongest band are
    left out.  Returns the worst error of each row.
    """
    S = np.asarray(S, dtype=np.float64).reshape(-1, np.shape(S)[-1])
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, np.shape(ref)[-1])
    om = np.asarray(omega, dtype=np.float64)
    idx = np.array_split(np.arange(om.size), n_bands)
    worst = []
    for s, r in zip(S, ref):
        pr = np.array([np.trapezoid(r[i] * om[i], np.log(om[i])) if len(i) > 1 else r[i].sum()
                       for i in idx])
        ps = np.array([np.trapezoid(s[i] * om[i], np.log(om[i])) if len(i) > 1 else s[i].sum()
                       for i in idx])
        if pr.max() <= 0:
            worst.append(0.0 if np.all(s == 0) else np.inf)
            continue
        m = pr >= floor * pr.max()
        worst.append(float(np.max(np.abs(ps[m] - pr[m]) / pr[m])))
    return np.array(worst)
