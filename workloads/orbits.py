"""Analytic test orbits (exact r(t), beta(t), d(beta)/dt sampled at t_k = t0 + k dt).

These are inputs, not the method: each returns a one-particle ``Batch`` whose
accelerations are kept in FP64 (for oracle-only closed-form tests) unless
``accel_dtype=np.float32`` is asked for.
"""
from __future__ import annotations

import numpy as np

from . import single_particle


def _times(n, dt, t0):
    return t0 + np.arange(n, dtype=np.float64) * dt


def circular(gamma, omega0, n, dt, phase0=np.pi / 2, t0=0.0, charge=-1.0, weight=1.0,
             accel_dtype=np.float64):
    """Uniform circular motion in the x-y plane, counter-clockwise.

    r = rho (cos phi, sin phi, 0), phi = omega0 t + phase0, rho = beta / omega0.
    With phase0 = pi/2 the velocity at t = 0 points along -x.
    """
    beta = np.sqrt(1.0 - 1.0 / gamma**2)
    rho = beta / omega0
    t = _times(n, dt, t0)
    phi = omega0 * t + phase0
    c, s = np.cos(phi), np.sin(phi)
    zero = np.zeros(n)
    return single_particle(rho * c, rho * s, zero, -beta * s, beta * c, zero,
                           -beta * omega0 * c, -beta * omega0 * s, zero, t0=t0, dt=dt,
                           charge=charge, weight=weight, accel_dtype=accel_dtype)


def straight(beta_vec, r0, n, dt, t0=0.0, charge=-1.0, weight=1.0, accel_dtype=np.float64):
    """Uniform straight motion r = r0 + beta (t - t0)."""
    b = np.asarray(beta_vec, dtype=np.float64)
    t = _times(n, dt, t0) - t0
    zero = np.zeros(n)
    return single_particle(r0[0] + b[0] * t, r0[1] + b[1] * t, r0[2] + b[2] * t,
                           np.full(n, b[0]), np.full(n, b[1]), np.full(n, b[2]),
                           zero, zero, zero, t0=t0, dt=dt, charge=charge, weight=weight,
                           accel_dtype=accel_dtype)


def driven_oscillator(beta_d, beta1, omega0, n, dt, t0=0.0, charge=-1.0, weight=1.0,
                      accel_dtype=np.float64):
    """Drift along z with a transverse oscillation along x.

    beta = beta_d z + beta1 cos(omega0 t) x,  r = beta_d t z + (beta1/omega0) sin(omega0 t) x.
    """
    t = _times(n, dt, t0)
    zero = np.zeros(n)
    return single_particle((beta1 / omega0) * np.sin(omega0 * t), zero, beta_d * t,
                           beta1 * np.cos(omega0 * t), zero, np.full(n, beta_d),
                           -beta1 * omega0 * np.sin(omega0 * t), zero, zero, t0=t0, dt=dt,
                           charge=charge, weight=weight, accel_dtype=accel_dtype)


def gaussian_oscillator(amp, omega0, sigma, beta_d, n, dt, t0=None, charge=-1.0, weight=1.0,
                        accel_dtype=np.float64):
    """x(t) = amp exp(-t^2 / (2 sigma^2)) sin(omega0 t), z(t) = beta_d t.

    A smooth, time-limited orbit whose spectrum is band-limited (used for the
    continuous Parseval and Larmor checks).  Velocity and acceleration are the
    exact first and second derivatives.
    """
    if t0 is None:
        t0 = -0.5 * (n - 1) * dt
    t = _times(n, dt, t0)
    e = np.exp(-t**2 / (2 * sigma**2))
    s, c = np.sin(omega0 * t), np.cos(omega0 * t)
    x = amp * e * s
    v = amp * e * (omega0 * c - t / sigma**2 * s)
    a = amp * e * (-(omega0**2) * s - 2 * omega0 * t / sigma**2 * c
                   + (t**2 / sigma**4 - 1 / sigma**2) * s)
    zero = np.zeros(n)
    return single_particle(x, zero, beta_d * t, v, zero, np.full(n, beta_d), a, zero, zero,
                           t0=t0, dt=dt, charge=charge, weight=weight, accel_dtype=accel_dtype)


def zigzag(beta0, phi_m, big_omega, n, dt, t0=0.0, charge=-1.0, weight=1.0,
           accel_dtype=np.float64):
    """Constant speed beta0 with a velocity direction that swings in the x-y plane.

    beta = beta0 (cos phi, sin phi, 0), phi = phi_m sin(W t) (W = big_omega), so gamma is
    constant and d(beta)/dt = beta0 phi' (-sin phi, cos phi, 0) is perpendicular to beta.
    Positions are the exact integrals of beta, from the Bessel expansions
    cos(a sin x) = J0(a) + 2 sum_k J_2k(a) cos(2k x) and
    sin(a sin x) = 2 sum_k J_(2k+1)(a) sin((2k+1) x), truncated where the terms
    fall below 1e-18.
    """
    import scipy.special as sp

    t = _times(n, dt, t0)
    ph = phi_m * np.sin(big_omega * t)
    dph = phi_m * big_omega * np.cos(big_omega * t)
    x = beta0 * sp.jv(0, phi_m) * t
    y = np.zeros(n)
    for k in range(1, 40):
        je, jo = sp.jv(2 * k, phi_m), sp.jv(2 * k - 1, phi_m)
        x = x + beta0 * 2 * je * np.sin(2 * k * big_omega * t) / (2 * k * big_omega)
        y = y - beta0 * 2 * jo * np.cos((2 * k - 1) * big_omega * t) / ((2 * k - 1) * big_omega)
        if abs(je) < 1e-18 and abs(jo) < 1e-18:
            break
    zero = np.zeros(n)
    return single_particle(x, y, zero, beta0 * np.cos(ph), beta0 * np.sin(ph), zero,
                           -beta0 * dph * np.sin(ph), beta0 * dph * np.cos(ph), zero, t0=t0,
                           dt=dt, charge=charge, weight=weight, accel_dtype=accel_dtype)


def rotate(batch, R):
    """Rotate positions, velocities and accelerations of a batch by the 3x3 matrix R."""
    from . import Batch

    def rot(a, b, c, dtype):
        m = np.stack([a, b, c], axis=0).astype(np.float64)
        out = R @ m
        return [np.ascontiguousarray(out[i], dtype=dtype) for i in range(3)]

    x, y, z = rot(batch.x, batch.y, batch.z, np.float64)
    bx, by, bz = rot(batch.bx, batch.by, batch.bz, np.float64)
    ax, ay, az = rot(batch.ax, batch.ay, batch.az, batch.ax.dtype)
    return Batch(offsets=batch.offsets.copy(), x=x, y=y, z=z, bx=bx, by=by, bz=bz, ax=ax, ay=ay,
                 az=az, t0=batch.t0.copy(), dt=batch.dt.copy(), charge=batch.charge.copy(),
                 weight=batch.weight.copy(), species=batch.species.copy(), meta=dict(batch.meta))
