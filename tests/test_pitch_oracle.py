"""Pins of the pitch-cone oracle (CPU): closed forms and a Monte-Carlo isotropy check."""
import math

import numpy as np

from oracle import pitch

AX = np.array([1.0, 0.0, 0.0])
THETA = [m * math.pi / 8 for m in range(5)]
EDGES = np.exp(np.linspace(0.0, np.log(400.0), 13))


def _at(theta, phi, umag):
    """Momenta at pitch angle theta from +x (azimuth phi about x)."""
    return (umag * np.cos(theta), umag * np.sin(theta) * np.cos(phi), umag * np.sin(theta) * np.sin(phi))


def test_isotropic_momenta_give_no_deviation():
    rng = np.random.default_rng(7)
    n = 2_000_000
    v = rng.normal(size=(3, n))
    v /= np.linalg.norm(v, axis=0)
    umag = np.exp(rng.uniform(0, np.log(15.0), n))
    counts, dev, _ = pitch.pitch_cones(*(v * umag), AX, THETA, 1.0 / 6.0, EDGES)
    frac = pitch.cone_bounds(THETA, 1.0 / 6.0)
    frac = frac[:, 1] - frac[:, 0]
    for m in range(5):
        for b in range(EDGES.size - 1):
            N = counts[5, b]
            if N < 20000:
                continue
            sigma = math.sqrt(frac[m] * (1 - frac[m]) / N) / frac[m]
            assert abs(dev[m, b] - 1.0) < 5 * sigma, (m, b, dev[m, b], sigma)


def test_cone_fraction_closed_form():
    # the folded pitch angle of isotropic directions has density sin(theta) on [0, pi/2]
    b = pitch.cone_bounds([math.pi / 4], 0.1)[0]
    numeric = np.trapezoid(np.sin(np.linspace(math.pi / 4 - 0.1, math.pi / 4 + 0.1, 20001)),
                           np.linspace(math.pi / 4 - 0.1, math.pi / 4 + 0.1, 20001))
    assert abs((b[1] - b[0]) - numeric) < 1e-9
    # the cone around the axis is clipped at 0, the one around pi/2 at pi/2
    b0, b4 = pitch.cone_bounds([0.0, math.pi / 2], 0.1)
    assert b0[1] == 1.0 and abs(b4[0] - math.cos(math.pi / 2)) < 1e-16


def test_exact_angles_both_beams_and_outside():
    u = [[], [], []]
    want = []
    for m, t in enumerate(THETA):
        for sgn in (1.0, -1.0):  # both beams fold to the same pitch angle
            x, y, z = _at(t, 0.3 * m, 5.0)
            u[0].append(sgn * x)
            u[1].append(y)
            u[2].append(z)
            want.append(m)
    for t in (math.pi / 16, 3 * math.pi / 16):  # between cones of half width 0.05
        x, y, z = _at(t, 1.0, 5.0)
        u[0].append(x)
        u[1].append(y)
        u[2].append(z)
        want.append(-1)
    counts, _, member = pitch.pitch_cones(*u, AX, THETA, 0.05, EDGES)
    assert list(member) == want
    assert counts[5].sum() == len(want) and all(counts[m].sum() == 2 for m in range(5))


def test_gamma_squared_bins_are_closed_below():
    u = np.array([0.0, 1.0, 2.0, 3.0, 0.5])  # gamma^2 = 1, 2, 5, 10, 1.25 exactly
    counts, _, _ = pitch.pitch_cones(u, 0 * u, 0 * u, AX, THETA, 0.1, [1.0, 2.0, 5.0, 10.0])
    assert list(counts[5]) == [2, 1, 1]  # [1, 2) holds 1 and 1.25; 10 is past the top edge
