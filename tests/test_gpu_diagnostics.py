"""GPU parity of the spectral diagnostics (observer average, omega_peak, slopes alpha and beta).

The GPU kernel and the oracle read the same FP64 spectrum and form the observer
average with the same operations in the same order, so the average is bit-exact.
Integer results (the
peak index and the bin counts of the two fits) are decided in FP64 on both
sides from the same values and must agree exactly; the floating results differ
only by the order of the sums and by the last bit of log/exp, so they are held
to 1e-10 relative (NaN where the oracle has NaN).
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import diagnostics as dg
from workloads import configs

pytestmark = pytest.mark.gpu
RTOL = 1e-10


def _ctx(dirs, omega, ns=1):
    from paper_1003_1140_amd import Context

    c = Context(0)
    c.set_directions(dirs)
    c.set_frequencies(omega)
    c.set_species(ns)
    return c


def _check(avg, diag, avg_ref, diag_ref):
    np.testing.assert_array_equal(avg, avg_ref)  # same products and sums in the same order
    for f in (0, 5, 7):  # k, n_alpha, n_beta
        np.testing.assert_array_equal(diag[..., f], diag_ref[..., f])
    np.testing.assert_array_equal(diag[..., 1], diag_ref[..., 1])  # w_k: the grid value itself
    for f in (2, 3, 4, 6):
        np.testing.assert_allclose(diag[..., f], diag_ref[..., f], rtol=RTOL, atol=0, equal_nan=True)


def test_analytic_spectra():
    om = np.exp(np.linspace(np.log(0.1), np.log(1e3), 401))
    x = np.log(om / om[200])
    rows = [np.exp(np.where(x < 0, x, -1.5 * x)),                        # broken power law
            5.0 * np.exp(-(np.log(om) - np.log(3.7)) ** 2 / (2 * 0.4**2)),  # peak between grid points
            om ** -2.0,                                                     # peak at the first bin
            np.zeros(om.size),                                              # empty row
            np.where(np.isin(np.arange(om.size), [50, 300]), 2.0, 1.0)]     # tie: first wins
    dirs = [[0, 0, 1], [1, 0, 0], [0, 1, 0], [0.6, 0, 0.8], [0, 0.6, 0.8]]
    S = np.stack(rows)[None]
    c = _ctx(dirs, om)
    c.load_accumulator(S)
    w = np.array([1.0, 0.0, 2.0, 0.5, 3.0])
    for weights, ar, br in ((None, None, None), (w, (0.05, 0.5), (2.0, 10.0))):
        avg, diag = c.spectral_diagnostics(weights=weights, alpha_range=ar, beta_range=br)
        avg_ref, diag_ref = dg.spectral_diagnostics(S, om, weights, ar or (1e-2, 0.3), br or (3.0, 30.0))
        _check(avg, diag, avg_ref, diag_ref)
    assert diag[0, 0, 0] == 200 and abs(diag[0, 0, 4] - 1.0) < 1e-12
    c.close()


def test_accumulated_spectra_several_species_and_a_snapshot_difference():
    import torch

    from paper_1003_1140_amd import DeviceBatch

    b = workloads.generate(configs.uneven_recipe(), 0, 30)
    dirs = configs.dirs_equal_area()[::4]
    om = configs.log_grid(0.1, 1e3, 700)
    c = _ctx(dirs, om, ns=3)
    c.accumulate(DeviceBatch.from_host(b.select(np.arange(15))))
    S1 = c.read_spectra()
    c.accumulate(DeviceBatch.from_host(b.select(np.arange(15, 30))))
    S2 = c.read_spectra()
    weights = np.sin(np.linspace(0.1, 1.5, len(dirs)))
    avg, diag = c.spectral_diagnostics(weights=weights)
    _check(avg, diag, *dg.spectral_diagnostics(S2, om, weights))
    # diagnostics of a difference of two snapshots, passed as a device array
    dS = torch.from_numpy(S2 - S1).cuda().contiguous()
    avg, diag = c.spectral_diagnostics(S=dS)
    _check(avg, diag, *dg.spectral_diagnostics(S2 - S1, om))
    c.close()


def test_coherent_context_spectrum():
    from paper_1003_1140_amd import DeviceBatch

    b = workloads.generate(configs.jitter_recipe(), 0, 12)
    dirs, om = configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 512)
    c = _ctx(dirs, om)
    c.set_coherent(True)
    c.accumulate(DeviceBatch.from_host(b))
    avg, diag = c.spectral_diagnostics()
    S = c.read_spectra()
    _check(avg, diag, *dg.spectral_diagnostics(S, om))
    # the oracle's own FP64 coherent spectrum peaks in the same bin of the average
    ref = oracle.coherent_spectrum(b, dirs, om, n_species=1)
    _, dref = dg.spectral_diagnostics(ref, om)
    assert abs(diag[0, -1, 0] - dref[0, -1, 0]) <= 1
    c.close()


def test_argument_errors():
    from paper_1003_1140_amd import LWError

    om = configs.log_grid(0.1, 1e3, 64)
    c = _ctx([[0, 0, 1], [1, 0, 0]], om)
    for kw in ({"weights": [1.0, -1.0]}, {"weights": [0.0, 0.0]}, {"alpha_range": (0.5, 0.1)},
               {"beta_range": (0.0, 3.0)}):
        with pytest.raises(LWError) as ei:
            c.spectral_diagnostics(**kw)
        assert ei.value.status == -1
    c.close()
