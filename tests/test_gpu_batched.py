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


def test_uneven_bench_slice_sampled_bins():
    """The benchmark's batched launch at its size: 5e4 particles of the uneven workload
    (device-generated as the benchmark does, lengths 256..8192, three species), 64 equal-area
    directions, 1024 log frequencies; the persistent FP32 launch on its planned ticket queue,
    then the matrix-core path.  The oracle recomputes two sampled (direction, frequency) bins
    per species over all 5e4 particles from host copies of the same trajectories.  Bars: the
    FP32 path's 1e-5 per bin, 1e-4 per sampled bin for the matrix-core path."""
    from types import SimpleNamespace

    from paper_1003_1140_amd import DeviceBatch
    from workloads.gpu import generate_device

    n = 50_000
    t, _ = generate_device(configs.uneven_recipe(), 0, n)
    b = DeviceBatch(t, n)
    dirs, om = configs.dirs_equal_area(), configs.log_grid(0.1, 1e3, 1024)
    c = ctx_for(dirs, om)
    c.set_tuning(persistent=1)
    c.plan_batch(b, "fp32")
    c.accumulate(b, "fp32")
    S32 = c.read_spectra()
    c.reset()
    c.accumulate(b, "mfma_f16")
    S16 = c.read_spectra()
    # per species a forward and an oblique direction, a low and a high frequency, each moved
    # down to the nearest bin holding at least 1e-3 of its (species, direction) peak (chosen
    # from the FP32 spectrum; the expected values come from the oracle alone)
    picks = []
    for s in range(3):
        for d, j in ((0, 200), (37, 900)):
            peak = S32[s, d].max()
            while j > 0 and S32[s, d, j] < 1e-3 * peak:
                j -= 1
            picks.append((s, d, j))
    ref = np.zeros(len(picks))
    offs = t["offsets"].cpu().numpy()
    per_sample = ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az")
    per_particle = ("t0", "dt", "charge", "weight", "species")
    step = 8192
    for p0 in range(0, n, step):
        p1 = min(n, p0 + step)
        s0, s1 = int(offs[p0]), int(offs[p1])
        h = SimpleNamespace(n_particles=p1 - p0, offsets=offs[p0:p1 + 1],
                            **{k: t[k][s0:s1].cpu().numpy() for k in per_sample},
                            **{k: t[k][p0:p1].cpu().numpy() for k in per_particle})
        for s in range(3):
            idx = [i for i, (sp, _, _) in enumerate(picks) if sp == s]
            ref[idx] += oracle.sampled_bins(h, dirs[[picks[i][1] for i in idx]], om[[picks[i][2] for i in idx]],
                                            species=s)
    r32 = np.array([abs(S32[s, d, j] / ref[i] - 1.0) for i, (s, d, j) in enumerate(picks)])
    r16 = np.array([abs(S16[s, d, j] / ref[i] - 1.0) for i, (s, d, j) in enumerate(picks)])
    print(f"[parity] uneven workload, 5e4 particles, sampled bins: fp32 persistent "
          f"{[f'{x:.2e}' for x in r32]}, mfma f16 x3 {[f'{x:.2e}' for x in r16]}", flush=True)
    assert r32.max() <= TOL
    assert r16.max() <= 1e-4


@pytest.mark.parametrize("f64_accel", [False, True])
def test_gathered_subset_is_a_batch_of_its_own(f64_accel):
    """lw_subset_offsets and lw_gather_particles: an unsorted list of 300 of 800 uneven
    particles (three species, lengths 256..8192, d(beta)/dt in FP32 or FP64) gathered into a
    batch of its own equals the host selection bit for bit; the FP32 sum of it equals
    lw_accumulate_subset on the same list bit for bit (same particles, same positions); the
    matrix-core path on it meets its 1e-5 band-integrated bar against that sum.  An empty
    list gathers nothing; an index outside the batch is refused."""
    import torch

    from paper_1003_1140_amd import LW_EINVAL, DeviceBatch, LWError

    host = workloads.generate(configs.uneven_recipe(), 300, 800)
    db = DeviceBatch.from_host(host, f64_accel=f64_accel)
    dirs = configs.dirs_equal_area()[::8]
    om = configs.log_grid(0.1, 1e3, 512)
    c = ctx_for(dirs, om)
    rng = np.random.default_rng(17)
    pick = rng.choice(800, 300, replace=False)  # unsorted
    idx = torch.from_numpy(pick.astype(np.int64)).cuda()
    sub = db.gather(c, idx)
    assert sub.n_particles == 300
    sel = host.select(pick)
    np.testing.assert_array_equal(sub.t["offsets"].cpu().numpy(), sel.offsets - sel.offsets[0])
    for k in ("x", "y", "z", "bx", "by", "bz", "t0", "dt", "charge", "weight", "species"):
        np.testing.assert_array_equal(sub.t[k].cpu().numpy(), getattr(sel, k), err_msg=k)
    for k in ("ax", "ay", "az"):
        want = getattr(sel, k).astype(np.float64 if f64_accel else np.float32)
        np.testing.assert_array_equal(sub.t[k].cpu().numpy(), want, err_msg=k)
    c.set_tuning(persistent=0)
    c.accumulate(sub, "fp32")
    S_gather = c.read_spectra()
    c.reset()
    c.accumulate_subset(db, idx)
    S_list = c.read_spectra()
    np.testing.assert_array_equal(S_gather, S_list)
    c.reset()
    c.accumulate(sub, "mfma_f16")
    S16 = c.read_spectra()
    assert band_integrated_errors(S16, S_list, om).max() <= 1e-5
    empty = db.gather(c, idx[:0])
    assert empty.n_particles == 0 and empty.t["offsets"].cpu().tolist() == [0]
    # particles without samples: lengths 0 in the gathered offsets, and a list of only those
    t0 = dict(db.t)
    t0["offsets"] = torch.tensor([0, 0, 3, 3, 5], dtype=torch.int64, device="cuda")
    db0 = DeviceBatch(t0, 4)
    g0 = db0.gather(c, torch.tensor([3, 0, 1, 2], dtype=torch.int64, device="cuda"))
    assert g0.t["offsets"].cpu().tolist() == [0, 2, 2, 5, 5]
    np.testing.assert_array_equal(g0.t["x"][:5].cpu().numpy(), db.t["x"][[3, 4, 0, 1, 2]].cpu().numpy())
    g1 = db0.gather(c, torch.tensor([0, 2], dtype=torch.int64, device="cuda"))
    assert g1.t["offsets"].cpu().tolist() == [0, 0, 0]
    bad = torch.tensor([3, 800, 5], dtype=torch.int64, device="cuda")
    with pytest.raises(LWError) as e:
        db.gather(c, bad)
    assert e.value.status == LW_EINVAL
    torch.cuda.synchronize()
