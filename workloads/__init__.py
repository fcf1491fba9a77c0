"""Seeded synthetic inputs shared by the HIP library's tests/bench and the oracle.

This package holds no part of the radiation computation.  It produces

* ``Batch``: a particle batch in the structure-of-arrays layout the library
  and the oracle both read (positions and velocities FP64, accelerations FP32,
  per-particle start time, step, charge, weight and species);
* analytic test orbits (``orbits``): uniform circular motion, straight
  motion, a driven oscillator and a Gaussian-enveloped oscillator;
* the filamentation-jitter ensemble generator (``filaments.c``): beams through
  a static random-filament magnetic field, pushed with the Boris scheme;
* direction sets and frequency grids of the workloads (``configs``).

Units are the paper's PIC units: c = m_e = q_e = 1, times in 1/omega_p.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libworkloads.so")


def build(force: bool = True) -> str:
    """Compile filaments.c into libworkloads.so (gcc, FP64, OpenMP)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
               os.path.join(_HERE, "filaments.c"), "-o", _SO + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        _lib = ctypes.CDLL(_SO)
        _lib.wl_generate.restype = ctypes.c_int
        _lib.wl_field_info.restype = ctypes.c_int
        _lib.wl_field_eval.restype = ctypes.c_int
        _lib.wl_field_coeffs.restype = ctypes.c_int
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Batch:
    """Particles in structure-of-arrays layout.

    Particle p owns samples ``offsets[p] .. offsets[p+1]-1``; sample k of a
    particle sits at time ``t0[p] + k * dt[p]``.  ``bx, by, bz`` is beta = v/c,
    ``ax, ay, az`` is d(beta)/dt.
    """

    offsets: np.ndarray  # int64 [P+1]
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    bx: np.ndarray
    by: np.ndarray
    bz: np.ndarray
    ax: np.ndarray  # float32 for the library (float64 allowed for oracle-only use)
    ay: np.ndarray
    az: np.ndarray
    t0: np.ndarray  # float64 [P]
    dt: np.ndarray  # float64 [P]
    charge: np.ndarray  # float32 [P]
    weight: np.ndarray  # float32 [P]
    species: np.ndarray  # int32 [P]
    meta: dict = field(default_factory=dict)

    @property
    def n_particles(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_samples(self) -> int:
        return int(self.offsets[-1] - self.offsets[0])

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def select(self, idx) -> "Batch":
        """Sub-batch of the given particle indices (copies)."""
        idx = np.asarray(idx, dtype=np.int64)
        lens = self.lengths()[idx]
        offs = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(lens, out=offs[1:])
        take = np.concatenate([np.arange(self.offsets[i], self.offsets[i + 1]) for i in idx]) \
            if len(idx) else np.zeros(0, dtype=np.int64)
        sub = {k: getattr(self, k)[take] for k in ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az")}
        per = {k: getattr(self, k)[idx] for k in ("t0", "dt", "charge", "weight", "species")}
        return Batch(offsets=offs, meta=dict(self.meta), **sub, **per)

    def time_window(self, k0, k1) -> "Batch":
        """Samples k0 .. k1-1 of every particle (clipped to its length), each particle's
        t0 moved to the window's first sample: the chunk an in-situ recorder sees between
        two snapshots."""
        lens = self.lengths()
        a = np.minimum(lens, k0)
        b = np.minimum(lens, np.maximum(k1, k0))
        offs = np.zeros(len(lens) + 1, dtype=np.int64)
        np.cumsum(b - a, out=offs[1:])
        take = np.concatenate([np.arange(self.offsets[i] + a[i], self.offsets[i] + b[i])
                               for i in range(len(lens))]) if len(lens) else np.zeros(0, dtype=np.int64)
        sub = {k: getattr(self, k)[take] for k in ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az")}
        per = {k: getattr(self, k).copy() for k in ("dt", "charge", "weight", "species")}
        return Batch(offsets=offs, meta=dict(self.meta), t0=self.t0 + a * self.dt, **sub, **per)

    @staticmethod
    def concat(batches) -> "Batch":
        lens = np.concatenate([b.lengths() for b in batches])
        offs = np.zeros(len(lens) + 1, dtype=np.int64)
        np.cumsum(lens, out=offs[1:])
        cat = {k: np.concatenate([getattr(b, k) for b in batches])
               for k in ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az",
                         "t0", "dt", "charge", "weight", "species")}
        return Batch(offsets=offs, meta=dict(batches[0].meta), **cat)

    def with_f32_accel(self) -> "Batch":
        return Batch(offsets=self.offsets, x=self.x, y=self.y, z=self.z, bx=self.bx, by=self.by,
                     bz=self.bz, ax=self.ax.astype(np.float32), ay=self.ay.astype(np.float32),
                     az=self.az.astype(np.float32), t0=self.t0, dt=self.dt, charge=self.charge,
                     weight=self.weight, species=self.species, meta=dict(self.meta))


def single_particle(x, y, z, bx, by, bz, ax, ay, az, t0=0.0, dt=1.0, charge=-1.0, weight=1.0,
                    species=0, accel_dtype=np.float64) -> Batch:
    n = len(x)
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    fa = lambda a: np.ascontiguousarray(a, dtype=accel_dtype)
    return Batch(offsets=np.array([0, n], dtype=np.int64), x=f64(x), y=f64(y), z=f64(z),
                 bx=f64(bx), by=f64(by), bz=f64(bz), ax=fa(ax), ay=fa(ay), az=fa(az),
                 t0=np.array([t0], dtype=np.float64), dt=np.array([dt], dtype=np.float64),
                 charge=np.array([charge], dtype=np.float32),
                 weight=np.array([weight], dtype=np.float32),
                 species=np.array([species], dtype=np.int32))


class Recipe(ctypes.Structure):
    """Mirror of ``wl_recipe`` in filaments.c."""

    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("dt", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("box", ctypes.c_double),
        ("kmin", ctypes.c_double),
        ("kmax", ctypes.c_double),
        ("n_gamma", ctypes.c_int32),
        ("gamma0", ctypes.c_double * 4),
        ("frac_pos", ctypes.c_double),
        ("frac_ion", ctypes.c_double),
        ("ion_mass", ctypes.c_double),
        ("len_min", ctypes.c_int32),
        ("len_max", ctypes.c_int32),
        ("two_d", ctypes.c_int32),
    ]


def make_recipe(seed, steps=4096, gammas=(3.0,), dt=0.005, kT=0.01, delta=0.3,
                box=4.0 * np.pi, kmin=0.5, kmax=8.0, frac_pos=0.0, frac_ion=0.0,
                ion_mass=16.0, len_range=None, two_d=False) -> Recipe:
    r = Recipe()
    r.seed = int(seed)
    r.dt = dt
    r.kT = kT
    r.delta = delta
    r.box = box
    r.kmin = kmin
    r.kmax = kmax
    r.n_gamma = len(gammas)
    for i, g in enumerate(gammas):
        r.gamma0[i] = g
    r.frac_pos = frac_pos
    r.frac_ion = frac_ion
    r.ion_mass = ion_mass
    lo, hi = len_range if len_range is not None else (steps, steps)
    r.len_min = int(lo)
    r.len_max = int(hi)
    r.two_d = 1 if two_d else 0
    return r


def particle_meta(recipe: Recipe, first_id: int, n: int):
    lib = _load()
    lens = np.zeros(n, dtype=np.int32)
    spec = np.zeros(n, dtype=np.int32)
    g0 = np.zeros(n, dtype=np.float64)
    q = np.zeros(n, dtype=np.float32)
    m = np.zeros(n, dtype=np.float32)
    lib.wl_particle_meta(ctypes.byref(recipe), ctypes.c_int64(first_id), ctypes.c_int64(n),
                         _ptr(lens), _ptr(spec), _ptr(g0), _ptr(q), _ptr(m))
    return lens, spec, g0, q, m


def generate(recipe: Recipe, first_id: int, n: int, nthreads: int = 0) -> Batch:
    """Particles first_id .. first_id+n-1 of the workload (any slice regenerates identically)."""
    lib = _load()
    lens, _, _, _, _ = particle_meta(recipe, first_id, n)
    offs = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    ns = int(offs[-1])
    arrs = {k: np.empty(ns, dtype=np.float64) for k in ("x", "y", "z", "bx", "by", "bz")}
    arrs.update({k: np.empty(ns, dtype=np.float32) for k in ("ax", "ay", "az")})
    per = dict(t0=np.empty(n, np.float64), dt=np.empty(n, np.float64),
               charge=np.empty(n, np.float32), weight=np.empty(n, np.float32),
               species=np.empty(n, np.int32))
    st = lib.wl_generate(ctypes.byref(recipe), ctypes.c_int64(first_id), ctypes.c_int64(n),
                         _ptr(offs), *[_ptr(arrs[k]) for k in ("x", "y", "z", "bx", "by", "bz",
                                                               "ax", "ay", "az")],
                         _ptr(per["t0"]), _ptr(per["dt"]), _ptr(per["charge"]),
                         _ptr(per["weight"]), _ptr(per["species"]), ctypes.c_int(nthreads))
    if st != 0:
        raise RuntimeError(f"wl_generate failed with status {st}")
    return Batch(offsets=offs, meta={"seed": int(recipe.seed), "first_id": int(first_id)},
                 **arrs, **per)


def field_info(recipe: Recipe):
    lib = _load()
    nm = ctypes.c_int32()
    brms = ctypes.c_double()
    kbar = ctypes.c_double()
    lib.wl_field_info(ctypes.byref(recipe), ctypes.byref(nm), ctypes.byref(brms), ctypes.byref(kbar))
    return nm.value, brms.value, kbar.value


def field_eval(recipe: Recipe, x, z):
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.empty_like(x)
    lib.wl_field_eval(ctypes.byref(recipe), ctypes.c_int64(x.size), _ptr(x), _ptr(z), _ptr(out))
    return out


def philox4x32_10(ctr, key):
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.wl_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out
