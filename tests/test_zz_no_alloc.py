"""GPU test of the allocation-free entry point lw_accumulate_noalloc.

It must give lw_accumulate's FP32 result on the same batch bit for bit (same kernels, same
partial-sum layout, same reduction order), on two calls in a row of which the second is
smaller (the static scratch keeps the first call's contents), stay within the FP32 path's
bar of the oracle, and refuse a batch whose partial sums exceed the scratch before any
launch.
"""
import numpy as np
import pytest

import oracle
import workloads
from workloads import configs, orbits

from _parity import band_relative_error

pytestmark = pytest.mark.gpu


def _ctx(dirs, om, ns=1):
    from paper_1003_1140_amd import Context

    c = Context(0)
    c.set_directions(dirs)
    c.set_frequencies(om)
    c.set_species(ns)
    return c


def test_noalloc_equals_workspace_path_on_two_calls():
    from paper_1003_1140_amd import DeviceBatch

    dirs = configs.dirs_jitter()
    om = configs.log_grid(0.1, 1e3, 300)
    big = workloads.generate(configs.uneven_recipe(), 7, 24)
    small = big.select(range(5))
    noalloc = _ctx(dirs, om, ns=3)
    for host in (big, small):  # second call smaller than the first
        db = DeviceBatch.from_host(host)
        ref_ctx = _ctx(dirs, om, ns=3)
        ref_ctx.accumulate(db, "fp32")
        S_ref = ref_ctx.read_spectra()
        noalloc.reset()
        noalloc.accumulate_noalloc(db)
        S = noalloc.read_spectra()
        print(f"[noalloc] {host.n_particles} particles: max |S - S_workspace| = {np.abs(S - S_ref).max():.3e}",
              flush=True)
        assert np.array_equal(S, S_ref)
    # and the oracle's bar on the smaller batch
    ref = oracle.spectrum(small, dirs, om, n_species=3)
    err = band_relative_error(S, ref)
    print(f"[noalloc] vs oracle: {err:.2e}", flush=True)
    assert err <= 1e-5


def test_noalloc_refuses_a_batch_larger_than_its_scratch():
    from paper_1003_1140_amd import LW_ENOMEM, DeviceBatch, LWError

    # 5000 two-sample particles, 64 directions, 4096 frequencies: partial sums far above 64 MiB
    parts = [orbits.straight([0.1, 0.0, 0.0], [0, 0, 0], 2, 0.01)] * 5000
    db = DeviceBatch.from_host(workloads.Batch.concat(parts))
    c = _ctx(configs.dirs_equal_area(), configs.log_grid(0.1, 1e3, 4096))
    with pytest.raises(LWError) as e:
        c.accumulate_noalloc(db)
    assert e.value.status == LW_ENOMEM and "static scratch" in str(e.value)
    assert np.all(c.read_spectra() == 0.0)
