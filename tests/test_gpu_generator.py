"""The device twin of the workload generator against the host generator (inputs only)."""
import numpy as np
import pytest

import workloads
from workloads import configs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("recipe", [configs.jitter_recipe(steps=512), configs.uneven_recipe(),
                                    configs.jitter_2d_recipe(steps=512)])
def test_device_generator_matches_host_over_short_horizons(recipe):
    from workloads.gpu import generate_device

    n = 24
    host = workloads.generate(recipe, 3000, n)
    dev, ns = generate_device(recipe, 3000, n)
    assert ns == host.n_samples
    for k in ("t0", "dt", "charge", "weight", "species"):
        assert np.array_equal(dev[k].cpu().numpy(), getattr(host, k)), k
    offs = host.offsets
    worst = 0.0
    for p in range(n):
        s = slice(offs[p], offs[p] + 64)  # first 64 samples, before chaos amplifies rounding
        for k in ("x", "z", "bx", "bz"):
            d = dev[k].cpu().numpy()[s]
            h = getattr(host, k)[s]
            worst = max(worst, float(np.max(np.abs(d - h))))
    print(f"[generator] device vs host, first 64 samples: max abs diff {worst:.2e}", flush=True)
    assert worst < 1e-9
    # whole trajectories stay physical
    bx, by, bz = (dev[k].cpu().numpy() for k in ("bx", "by", "bz"))
    assert np.all(bx * bx + by * by + bz * bz < 1.0)


def test_two_d_device_ensemble_and_its_spectrum():
    """2D2V on the device: in-plane motion, and both paths match the oracle for in-plane observers."""
    import oracle
    from paper_1003_1140_amd import Context, DeviceBatch
    from workloads.gpu import generate_device, to_host
    from _parity import band_integrated_errors, band_relative_error

    r = configs.jitter_2d_recipe(steps=1024)
    t, _ = generate_device(r, 0, 24)
    for k in ("y", "by", "ay"):
        assert float(t[k].abs().max()) == 0.0, k
    dirs, om = configs.dirs_paper(two_d=True), configs.log_grid(0.1, 1e3, 512)
    ref = oracle.spectrum(to_host(t), dirs, om, n_species=1)
    c = Context(0)
    c.set_directions(dirs)
    c.set_frequencies(om)
    db = DeviceBatch(t, 24)
    c.accumulate(db)
    assert band_relative_error(c.read_spectra(), ref) <= 1e-5
    c.reset()
    c.accumulate(db, "mfma_f16")
    assert band_integrated_errors(c.read_spectra()[0], ref[0], om).max() <= 1e-5
    c.close()
