"""GPU tests of the batched launches: persistent ticket queue over uneven lengths and
several species, HIP-graph capture and replay, and the launch-shape autotuner.

The uneven workload mixes electrons, positrons and ions (mass 16) from three
bulk Lorentz factors with trajectory lengths from 256 to 8192 samples.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from workloads import configs

from _parity import band_integrated_errors, band_relative_error

pytestmark = pytest.mark.gpu
TOL = 1e-5


def ctx_for(dirs, om, ns=3):
    from paper_1003_1140_amd import Context

    c = Context(0)
    c.set_directions(dirs)
    c.set_frequencies(om)
    c.set_species(ns)
    return c


@pytest.fixture(scope="module")
def uneven_small():
    b = workloads.generate(configs.uneven_recipe(), 100, 40)
    dirs = configs.dirs_equal_area()[::4]
    om = configs.log_grid(0.1, 1e3, 1024)
    return b, dirs, om


def test_persistent_plan_matches_oracle(uneven_small):
    from paper_1003_1140_amd import DeviceBatch

    b, dirs, om = uneven_small
    ref = oracle.spectrum(b, dirs, om, n_species=3)
    c = ctx_for(dirs, om)
    db = DeviceBatch.from_host(b)
    c.plan_batch(db, "fp32")
    c.accumulate(db, "fp32")
    S = c.read_spectra()
    err = band_relative_error(S, ref)
    print(f"[parity] persistent fp32, uneven 40 particles x 16 dirs x 3 species: {err:.3e}", flush=True)
    assert err <= TOL
    # the matrix-core path on the same batch
    c2 = ctx_for(dirs, om)
    c2.plan_batch(db, "mfma_f16")
    c2.accumulate(db, "mfma_f16")
    be = band_integrated_errors(c2.read_spectra(), ref, om)
    print(f"[parity] mfma f16 x3, uneven 40 particles: band-integrated {be.max():.3e}", flush=True)
    assert be.max() <= TOL


def test_persistent_equals_plain_grid_on_a_larger_batch():
    from paper_1003_1140_amd import DeviceBatch

    b = workloads.generate(configs.uneven_recipe(), 5000, 1500)
    dirs = configs.dirs_equal_area()
    om = configs.log_grid(0.1, 1e3, 1024)
    db = DeviceBatch.from_host(b)
    c = ctx_for(dirs, om)
    c.set_tuning(persistent=0)
    c.accumulate(db, "fp32")
    S_grid = c.read_spectra()
    c.reset()
    c.set_tuning(persistent=1)
    c.plan_batch(db, "fp32")
    c.accumulate(db, "fp32")
    S_pers = c.read_spectra()
    c.reset()
    c.accumulate(db, "fp32")
    assert np.array_equal(c.read_spectra(), S_pers)  # the persistent launch is deterministic
    np.testing.assert_allclose(S_pers, S_grid, rtol=1e-9, atol=0)
    assert S_pers[2].max() > 0  # ions present


@pytest.mark.parametrize("path", ["fp32", "mfma_f16"])
def test_graph_replays_match_eager(uneven_small, path):
    """After k replays S equals, bit for bit, S after k eager lw_accumulate calls; eager work
    on another context and synchronisations run between the replays."""
    import torch

    from paper_1003_1140_amd import DeviceBatch

    b, dirs, om = uneven_small
    db = DeviceBatch.from_host(b)
    other = DeviceBatch.from_host(workloads.generate(configs.uneven_recipe(), 900, 7))
    c = ctx_for(dirs, om)
    c.plan_batch(db, path)
    ws = c.workspace(db, path)
    eager = []
    for _ in range(3):
        c.accumulate(db, path, workspace=ws)
        eager.append(c.read_spectra())
    c.reset()
    g = c.graph_capture(db, path, workspace=ws)
    side = ctx_for(dirs, om)
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(c.read_spectra(), eager[rep]), f"replay {rep + 1}"
        side.accumulate(other, "fp32")
        side.read_spectra()
    g.close()


def test_autotuner_leaves_spectra_unchanged_and_picks_a_shape(uneven_small, tmp_path):
    from paper_1003_1140_amd import DeviceBatch

    b, dirs, om = uneven_small
    db = DeviceBatch.from_host(b)
    c = ctx_for(dirs, om)
    c.accumulate(db, "fp32")
    before = c.read_spectra()
    cache = str(tmp_path / "tune.json")
    rep = c.tune(db, "fp32", repeats=1, cache_json=cache)
    assert np.array_equal(c.read_spectra(), before)
    assert rep["best"] is not None and all(cd["ms"] > 0 for cd in rep["candidates"])
    print("[tune] fp32 best", json.dumps(rep["best"]), flush=True)
    assert os.path.exists(cache)
    c.reset()
    c.accumulate(db, "fp32")
    ref = oracle.spectrum(b, dirs, om, n_species=3)
    assert band_relative_error(c.read_spectra(), ref) <= TOL
    # the tuned shape reloads into a fresh context
    c2 = ctx_for(dirs, om)
    c2.load_tuning(cache)
    c2.accumulate(db, "fp32")
    assert band_relative_error(c2.read_spectra(), ref) <= TOL
    rep = c.tune(db, "mfma_f16", repeats=1)
    print("[tune] mfma best", json.dumps(rep["best"]), flush=True)
    assert rep["best"] is not None


def test_stale_graphs_are_refused(uneven_small):
    """A graph whose accumulators or tables were reallocated is refused on the host (it is never
    launched); a fresh capture works again."""
    from paper_1003_1140_amd import DeviceBatch, LWError

    b, dirs, om = uneven_small
    db = DeviceBatch.from_host(b.select(range(8)))
    c = ctx_for(dirs, om)
    g = c.graph_capture(db, "fp32")
    g.launch()
    c.set_species(3)  # reallocates S
    with pytest.raises(LWError) as ei:
        g.launch()
    assert ei.value.status == -4
    g.close()
    # matrix-core: a products change switches the kernel shape and rebuilds the tables
    c.reset()
    c.set_mfma_options(1, 3, 3)
    c.plan_batch(db, "mfma_f16")
    ws = c.workspace(db, "mfma_f16")
    g = c.graph_capture(db, "mfma_f16", workspace=ws)
    g.launch()
    first = c.read_spectra()
    c.set_mfma_options(1, 1, 3)
    c.accumulate(db, "mfma_f16", workspace=c.workspace(db, "mfma_f16"))
    with pytest.raises(LWError) as ei:
        g.launch()
    assert ei.value.status == -4
    g.close()
    c.set_mfma_options(1, 3, 3)
    c.reset()
    c.plan_batch(db, "mfma_f16")
    ws = c.workspace(db, "mfma_f16")
    g = c.graph_capture(db, "mfma_f16", workspace=ws)
    g.launch()
    np.testing.assert_allclose(c.read_spectra(), first, rtol=1e-12, atol=0)
    g.close()
    c.close()
