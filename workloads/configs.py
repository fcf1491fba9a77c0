"""Workload definitions: direction sets, frequency grids and generator recipes.

Five workloads, all in PIC units (c = m_e = q_e = 1, omega in omega_p):

* ``synchrotron``: one electron, gamma = 10, uniform circular motion (omega0 = 1),
  2000 samples over one orbit period, one observer in the orbit plane, 512
  log-spaced frequencies over [0.01, 10] omega_c.
* ``jitter``: 1e5 electrons, gamma0 = 3 counter-streaming beams with a
  kT = 0.01 rest-frame spread, 4096 Boris steps through a static random
  filament field (k^-2 over [0.5, 8], deflection parameter 0.3); directions
  +x, -x, +y, +z; 1024 log frequencies over [0.1, 1e3].
* ``jitter_wide``: 1e6 particles of the same generator, 2048 steps, 16
  directions (head-on, 15/30/45 degrees oblique at four azimuths, three
  perpendicular), 2048 log frequencies over [0.1, 1e3].
* ``uneven``: 4e5 particles, 47.5 % electrons, 47.5 % positrons, 5 % ions
  (mass 16), gamma0 in {2, 5, 15}, lengths uniform in [256, 8192], 64
  equal-area directions, 1024 log frequencies.
* ``surrogate``: the jitter generator with its own seed, 256 log frequencies
  over [0.1, 1e3].  Training, calibration and inference particles are disjoint
  id ranges of one ensemble, so they move through the same filament field (one
  simulation, as for an in-situ diagnostic); ``surrogate_recipe_other_field``
  draws a second field realisation for the cross-field check.
"""
from __future__ import annotations

import numpy as np

from . import make_recipe

SEEDS = {"jitter": 11401, "jitter_wide": 11402, "uneven": 11403, "surrogate": 11405,
         "surrogate_other_field": 11406}
DT = 0.005  # sample spacing: a tenth of a Courant-limited PIC step on a 0.1 c/omega_p grid


def log_grid(wmin, wmax, n):
    """omega_j = wmin (wmax/wmin)^(j/(n-1)), endpoints included."""
    j = np.arange(n, dtype=np.float64)
    return wmin * (wmax / wmin) ** (j / (n - 1))


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def dirs_jitter():
    return unit(np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64))


def dirs_wide():
    """Head-on +x; theta in {15, 30, 45} deg from +x at azimuths 0/90/180/270; 3 perpendicular."""
    out = [[1.0, 0.0, 0.0]]
    for th in (15.0, 30.0, 45.0):
        for ph in (0.0, 90.0, 180.0, 270.0):
            t, p = np.radians(th), np.radians(ph)
            out.append([np.cos(t), np.sin(t) * np.cos(p), np.sin(t) * np.sin(p)])
    for ph in (0.0, 120.0, 240.0):
        p = np.radians(ph)
        out.append([0.0, np.cos(p), np.sin(p)])
    return unit(np.array(out))


def dirs_equal_area(n_bands=8, n_az=8):
    """Cell centres of an equal-area sphere grid: bands equal in z, equal azimuth sectors."""
    out = []
    for i in range(n_bands):
        zc = -1.0 + (2 * i + 1) / n_bands
        rr = np.sqrt(1 - zc * zc)
        for j in range(n_az):
            ph = 2 * np.pi * (j + 0.5) / n_az
            out.append([rr * np.cos(ph), rr * np.sin(ph), zc])
    return unit(np.array(out))


def synchrotron_setup(gamma=10.0, n_samples=2000, n_omega=512):
    """One electron on a circle (omega0 = 1), one orbit period, observer +x in the orbit plane."""
    beta = np.sqrt(1 - 1 / gamma**2)
    omega_c = 1.5 * gamma**3 / beta  # critical frequency for omega0 = 1 (rho = beta)
    T = 2 * np.pi
    return dict(gamma=gamma, omega0=1.0, n=n_samples, dt=T / n_samples, omega_c=omega_c,
                dirs=np.array([[1.0, 0.0, 0.0]]),
                omega=log_grid(0.01 * omega_c, 10 * omega_c, n_omega))


def jitter_recipe(seed=SEEDS["jitter"], steps=4096):
    return make_recipe(seed, steps=steps, gammas=(3.0,), dt=DT)


def jitter_2d_recipe(seed=SEEDS["jitter"], steps=4096):
    """The jitter ensemble in 2D2V: motion confined to the x-z plane of the field."""
    return make_recipe(seed, steps=steps, gammas=(3.0,), dt=DT, two_d=True)


def dirs_paper(two_d=False):
    """Six far observers spread uniformly in angle from head-on (along the stream, +x) to
    edge-on (Section 2.2): in the x-z plane of the motion for 2D runs, in the x-y plane
    otherwise (the paper gives no azimuth for 3D)."""
    th = np.linspace(0.0, 0.5 * np.pi, 6)
    side = np.stack([np.cos(th), np.zeros(6), np.sin(th)], axis=1) if two_d else \
        np.stack([np.cos(th), np.sin(th), np.zeros(6)], axis=1)
    return unit(side)


def wide_recipe(seed=SEEDS["jitter_wide"], steps=2048):
    return make_recipe(seed, steps=steps, gammas=(3.0,), dt=DT)


def uneven_recipe(seed=SEEDS["uneven"]):
    return make_recipe(seed, gammas=(2.0, 5.0, 15.0), dt=DT, frac_pos=0.475, frac_ion=0.05,
                       ion_mass=16.0, len_range=(256, 8192))


def surrogate_recipe(steps=4096):
    return make_recipe(SEEDS["surrogate"], steps=steps, gammas=(3.0,), dt=DT)


def surrogate_recipe_other_field(steps=4096):
    return make_recipe(SEEDS["surrogate_other_field"], steps=steps, gammas=(3.0,), dt=DT)


WORKLOADS = {
    "synchrotron": dict(n_particles=1, dirs=None, n_omega=512),
    "jitter": dict(n_particles=100_000, steps=4096, dirs=dirs_jitter, omega=(0.1, 1e3, 1024)),
    "jitter_wide": dict(n_particles=1_000_000, steps=2048, dirs=dirs_wide, omega=(0.1, 1e3, 2048)),
    "uneven": dict(n_particles=400_000, steps=None, dirs=dirs_equal_area, omega=(0.1, 1e3, 1024),
                   n_species=3),
    "surrogate": dict(n_train=125_000, n_calib=200_000, n_infer=1_000_000, infer_first_id=1 << 20,
                      steps=4096, dirs=dirs_jitter, omega=(0.1, 1e3, 256), held_out=0.01,
                      fallback=0.05),
}
