"""Pins of the coherent-synthesis oracle (CPU).

Coherent synthesis adds the amplitudes w_p q_p A_p of a species before squaring
(Section 2.2, the sum over particles inside the squared modulus).  What fixes it:
one particle is its own incoherent spectrum; N copies radiate N^2 times one; opposite
charges on one trajectory cancel exactly; a copy delayed by D interferes as
2 (1 + cos w D); species stay separate; and the summed amplitude is additive over
time windows, which is what an in-situ recorder accumulates between snapshots.
"""
import numpy as np

import oracle
from workloads import Batch, orbits

OM = np.linspace(0.2, 6.0, 97)
DIRS = [[0.0, 0.0, 1.0], [0.6, 0.0, 0.8], [1.0, 0.0, 0.0]]


def _one(t0=0.0, charge=-1.0, weight=1.0):
    return orbits.driven_oscillator(0.3, 0.2, 1.7, 300, 0.04, t0=t0, charge=charge, weight=weight)


def test_single_particle_is_its_incoherent_spectrum():
    b = _one()
    np.testing.assert_allclose(oracle.coherent_spectrum(b, DIRS, OM, n_species=1),
                               oracle.spectrum(b, DIRS, OM, n_species=1), rtol=1e-13, atol=0)
    # a macro-particle of weight w is w charges on one trajectory: w^2 coherent, w incoherent
    bw = _one(weight=2.5)
    np.testing.assert_allclose(oracle.coherent_spectrum(bw, DIRS, OM, n_species=1),
                               2.5 * oracle.spectrum(bw, DIRS, OM, n_species=1), rtol=1e-13, atol=0)


def test_copies_add_coherently():
    b1 = _one()
    b3 = Batch.concat([b1, b1, b1])
    s1 = oracle.spectrum(b1, DIRS, OM, n_species=1)
    np.testing.assert_allclose(oracle.coherent_spectrum(b3, DIRS, OM, n_species=1), 9.0 * s1, rtol=1e-12)
    np.testing.assert_allclose(oracle.spectrum(b3, DIRS, OM, n_species=1), 3.0 * s1, rtol=1e-12)


def test_opposite_charges_on_one_trajectory_cancel_exactly():
    b = Batch.concat([_one(charge=-1.0), _one(charge=1.0)])
    assert np.all(oracle.coherent_spectrum(b, DIRS, OM, n_species=1) == 0.0)


def test_delayed_copy_interferes():
    delay = 0.37
    late = _one()
    late.t0 = late.t0 + delay  # same samples, emitted delay later
    b = Batch.concat([_one(), late])
    s1 = oracle.spectrum(_one(), DIRS, OM, n_species=1)
    expect = s1 * 2.0 * (1.0 + np.cos(OM * delay))
    np.testing.assert_allclose(oracle.coherent_spectrum(b, DIRS, OM, n_species=1), expect,
                               rtol=1e-10, atol=1e-12 * s1.max())


def test_species_stay_separate():
    a, c = _one(), orbits.circular(3.0, 1.3, 200, 0.02, phase0=0.4)
    b = Batch.concat([a, c])
    b.species = np.array([0, 1], dtype=np.int32)
    S = oracle.coherent_spectrum(b, DIRS, OM, n_species=2)
    np.testing.assert_allclose(S[0], oracle.spectrum(a, DIRS, OM, n_species=1)[0], rtol=1e-13)
    np.testing.assert_allclose(S[1], oracle.spectrum(c, DIRS, OM, n_species=1)[0], rtol=1e-13)


def test_summed_amplitude_is_additive_over_time_windows():
    b = Batch.concat([_one(), orbits.circular(3.0, 1.3, 250, 0.02, phase0=0.4, weight=0.7)])
    _, A = oracle.coherent_spectrum(b, DIRS, OM, n_species=1, with_amplitude=True)
    _, A1 = oracle.coherent_spectrum(b.time_window(0, 120), DIRS, OM, n_species=1, with_amplitude=True)
    _, A2 = oracle.coherent_spectrum(b.time_window(120, 10_000), DIRS, OM, n_species=1, with_amplitude=True)
    np.testing.assert_allclose(A1 + A2, A, rtol=0, atol=1e-12 * np.abs(A).max())
    # snapshot spectra P(t1) and P(t2) are the squared partial sums
    S1 = oracle.coherent_spectrum(b.time_window(0, 120), DIRS, OM, n_species=1)
    np.testing.assert_allclose(S1, np.sum(np.abs(A1) ** 2, axis=-1) / (4 * np.pi**2), rtol=1e-12)
