"""The device twin of the workload generator against the host generator (inputs only)."""
import numpy as np
import pytest

import workloads
from workloads import configs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("recipe", [configs.jitter_recipe(steps=512), configs.uneven_recipe()])
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
