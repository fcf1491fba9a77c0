"""GPU tests of the C-ABI boundary calls beyond plain accumulation.

* LW_PATH_AUTO takes the matrix-core path on long frequency lists and the FP32 path
  otherwise (or when per-particle output is asked for), with each path's own result.
* LW_BATCH_F64_ACCEL: d(beta)/dt handed over in FP64.
* A planned batch accumulates on the matrix-core path without synchronising: the call
  is captured into a HIP graph with no synchronisation before it, and the replays equal
  the eager call; a batch that outgrew its plan is reported at the next read.
* Decreasing offsets are a data error.
* Accumulator and network snapshots round-trip through files and refuse foreign or
  corrupted ones.
* The per-CU busy record of the persistent launch.
"""
import os

import numpy as np
import pytest

import oracle
import workloads
from workloads import configs, orbits

from _parity import band_integrated_errors, band_relative_error

pytestmark = pytest.mark.gpu


def ctx_for(dirs, om, ns=1):
    from paper_1003_1140_amd import Context

    c = Context(0)
    c.set_directions(dirs)
    c.set_frequencies(om)
    c.set_species(ns)
    return c


@pytest.fixture(scope="module")
def jitter8():
    return workloads.generate(configs.jitter_recipe(steps=1024), 0, 8)


def test_auto_path_picks_by_frequency_count(jitter8):
    import torch

    from paper_1003_1140_amd import DeviceBatch

    db = DeviceBatch.from_host(jitter8)
    dirs = configs.dirs_jitter()
    for nw, expect in ((512, "mfma_f16"), (64, "fp32")):
        om = configs.log_grid(0.1, 1e3, nw)
        S = {}
        for path in ("auto", expect):
            c = ctx_for(dirs, om)
            c.accumulate(db, path)
            S[path] = c.read_spectra()
            c.close()
        print(f"[auto] nw {nw}: picks {expect}", flush=True)
        assert np.array_equal(S["auto"], S[expect])
    # per-particle output is an FP32-path feature: AUTO takes that path for it
    om = configs.log_grid(0.1, 1e3, 512)
    c = ctx_for(dirs, om)
    pp = torch.zeros((8, len(dirs), 512), dtype=torch.float32, device="cuda")
    c.accumulate(db, "auto", per_particle=pp)
    S_auto = c.read_spectra()
    c2 = ctx_for(dirs, om)
    c2.accumulate(db, "fp32")
    assert np.array_equal(S_auto, c2.read_spectra())
    assert float(pp.sum()) > 0


def test_f64_acceleration_flag(jitter8):
    """FP64 d(beta)/dt: equal to the FP32 input when the values are the FP32-rounded ones
    (both are widened to FP64), and within the FP32 path's bar of the oracle when they are
    the full FP64 values."""
    import copy

    from paper_1003_1140_amd import DeviceBatch

    dirs = configs.dirs_jitter()
    om = configs.log_grid(0.1, 1e3, 256)
    b32 = jitter8
    b64 = copy.deepcopy(b32)
    for k in ("ax", "ay", "az"):
        setattr(b64, k, getattr(b32, k).astype(np.float64))
    d32 = DeviceBatch.from_host(b32)
    d64 = DeviceBatch.from_host(b64, f64_accel=True)
    assert d64.struct.flags == 1 and d32.struct.flags == 0
    for path in ("fp32", "mfma_f16"):
        c = ctx_for(dirs, om)
        c.accumulate(d32, path)
        S32 = c.read_spectra()
        c.reset()
        c.accumulate(d64, path)
        S64 = c.read_spectra()
        assert np.array_equal(S32, S64), path
    # an orbit with exact FP64 accelerations, against the oracle on the same FP64 values
    circ = orbits.circular(3.0, 1.0, 3000, 2 * np.pi / 3000)
    ref = oracle.spectrum(circ, [[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]], om, n_species=1)
    c = ctx_for([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]], om)
    c.accumulate(DeviceBatch.from_host(circ, f64_accel=True), "fp32")
    err = band_relative_error(c.read_spectra(), ref)
    print(f"[f64 accel] circular orbit, fp32 path vs oracle: {err:.2e}", flush=True)
    assert err <= 1e-5


def test_planned_mfma_accumulate_is_captured_without_synchronisation(jitter8):
    """After planning (lw_workspace_size), lw_accumulate on the matrix-core path issues no
    synchronisation: a stream capture around it succeeds (a synchronisation would break the
    capture), and replays of the captured graph, with eager work between them, each add the
    eager spectrum."""
    import torch

    from paper_1003_1140_amd import DeviceBatch

    dirs = configs.dirs_wide()[:6]
    om = configs.log_grid(0.1, 1e3, 512)
    db = DeviceBatch.from_host(jitter8)
    eager = ctx_for(dirs, om)
    eager.set_mfma_options(2, 3, 3)
    eager.accumulate(db, "mfma_f16")
    S1 = eager.read_spectra()

    c = ctx_for(dirs, om)
    c.set_mfma_options(2, 3, 3)
    ws = c.workspace(db, "mfma_f16")  # plans the batch (the one synchronising call)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        c.set_stream(s)
        with torch.cuda.graph(g, stream=s):
            c.accumulate(db, "mfma_f16", workspace=ws)
    c.set_stream(None)
    c.reset()
    torch.cuda.synchronize()
    for k in range(1, 4):
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda") * 2.0  # eager work between replays
        del junk
        S = c.read_spectra()
        print(f"[capture] replay {k}: max |S - k S1| / max S1 = "
              f"{np.abs(S - k * S1).max() / S1.max():.2e}", flush=True)
        np.testing.assert_allclose(S, k * S1, rtol=1e-12, atol=1e-14 * S1.max())


def test_batch_that_outgrew_its_plan_is_reported(jitter8):
    """The same offsets pointer with a longer retarded-time span (every step tripled in
    place) is taken as planned; the spreading kernel records the overflow and the read says
    so.  Planning again gives the right spectrum."""
    import torch

    from paper_1003_1140_amd import LW_ESTATE, DeviceBatch, LWError

    dirs = configs.dirs_jitter()
    om = configs.log_grid(0.1, 1e3, 256)
    b = jitter8
    db = DeviceBatch.from_host(b)
    c = ctx_for(dirs, om)
    ws = c.workspace(db, "mfma_f16")
    db.t["dt"].mul_(3.0)
    for k in ("x", "y", "z"):
        db.t[k].mul_(3.0)  # positions of the stretched trajectories (beta unchanged)
    c.accumulate(db, "mfma_f16", workspace=ws)
    with pytest.raises(LWError) as e:
        c.read_spectra()
    assert e.value.status == LW_ESTATE and "outgrew" in str(e.value)
    c.reset()
    ws = c.workspace(db, "mfma_f16")
    c.accumulate(db, "mfma_f16", workspace=ws)
    S = c.read_spectra()
    ref_ctx = ctx_for(dirs, om)
    ref_ctx.accumulate(db, "fp32")
    ref = ref_ctx.read_spectra()
    be = band_integrated_errors(S, ref, om).max()
    print(f"[overflow] after re-planning: band-integrated vs fp32 {be:.2e}", flush=True)
    assert be <= 1e-5
    torch.cuda.synchronize()


def test_decreasing_offsets_are_a_data_error():
    from paper_1003_1140_amd import LW_ERANGE, DeviceBatch

    b = workloads.Batch.concat([orbits.circular(3.0, 1.0, 100, 0.01), orbits.circular(4.0, 1.0, 100, 0.01),
                                orbits.circular(5.0, 1.0, 100, 0.01)])
    b.offsets = np.array([0, 100, 50, 300], dtype=np.int64)  # particle 1 runs backwards
    db = DeviceBatch.from_host(b)
    for path in ("fp32", "mfma_f16"):
        c = ctx_for([[1.0, 0.0, 0.0]], configs.log_grid(0.1, 100.0, 64))
        c.accumulate(db, path)
        st, S, msg = c.read_spectra_status()
        print(f"[offsets] {path}: status {st} ({msg})", flush=True)
        assert st == LW_ERANGE and msg.startswith("particle 1 ")


def test_accumulator_file_round_trip(tmp_path, jitter8):
    from paper_1003_1140_amd import LW_EINVAL, DeviceBatch, LWError

    dirs = configs.dirs_jitter()
    om = configs.log_grid(0.1, 1e3, 128)
    db = DeviceBatch.from_host(jitter8)
    for coherent in (False, True):
        c = ctx_for(dirs, om, ns=2)
        c.set_coherent(coherent)
        c.accumulate(db, "fp32")
        S = c.read_spectra()
        f = str(tmp_path / f"acc_{int(coherent)}.lwacc")
        c.save_accumulator(f)
        c.reset()
        c.load_accumulator_file(f)
        assert np.array_equal(c.read_spectra(), S)
        # resuming adds on top of the loaded state
        c.accumulate(db, "fp32")
        if not coherent:
            np.testing.assert_allclose(c.read_spectra(), 2 * S, rtol=1e-14)
        # another grid, another mode, a corrupted or a short file: refused, state unchanged
        other = ctx_for(dirs, configs.log_grid(0.1, 1e3, 128) * (1 + 1e-12), ns=2)
        other.set_coherent(coherent)
        with pytest.raises(LWError) as e:
            other.load_accumulator_file(f)
        assert e.value.status == LW_EINVAL
        flipped = ctx_for(dirs, om, ns=2)
        flipped.set_coherent(not coherent)
        with pytest.raises(LWError):
            flipped.load_accumulator_file(f)
        raw = bytearray(open(f, "rb").read())
        raw[100] ^= 1
        bad = str(tmp_path / "bad.lwacc")
        open(bad, "wb").write(bytes(raw))
        with pytest.raises(LWError, match="checksum"):
            c.load_accumulator_file(bad)
        open(bad, "wb").write(bytes(raw[:80]))
        with pytest.raises(LWError, match="shorter"):
            c.load_accumulator_file(bad)


def test_network_file_round_trip(tmp_path):
    """Save after some training, load into a fresh network: same outputs bit for bit, and
    training continues identically (AdamW moments and step counts come back too)."""
    import torch

    from paper_1003_1140_amd import MLP, LWError

    c = ctx_for([[1.0, 0.0, 0.0]], [1.0])
    gen = torch.Generator(device="cuda").manual_seed(3)
    x = torch.randn((512, 16), device="cuda", generator=gen)
    t = torch.randn((512, 64), device="cuda", generator=gen)
    a = MLP(c, 16, 64, 2, 64, seed=7)
    a.set_input_norm(np.full(16, 0.1, dtype=np.float32), np.full(16, 2.0, dtype=np.float32))
    a.set_output_skip(3, 0.5)
    for _ in range(5):
        a.train_step(x, t, lr=1e-3)
    f = str(tmp_path / "net.lwmlp")
    a.save(f)
    b = MLP(c, 16, 64, 2, 64, seed=99)
    b.load(f)
    ya, ea = a.forward(x, with_error=True)
    yb, eb = b.forward(x, with_error=True)
    assert torch.equal(ya, yb) and torch.equal(ea, eb)
    la = [a.train_step(x, t, lr=1e-3) for _ in range(3)]
    lb = [b.train_step(x, t, lr=1e-3) for _ in range(3)]
    assert la == lb
    wrong = MLP(c, 16, 32, 2, 64, seed=1)
    with pytest.raises(LWError, match="shape"):
        wrong.load(f)


def test_persistent_launch_records_per_cu_busy_time():
    from paper_1003_1140_amd import DeviceBatch

    b = workloads.generate(configs.uneven_recipe(), 0, 300)
    db = DeviceBatch.from_host(b)
    c = ctx_for(configs.dirs_equal_area()[:16], configs.log_grid(0.1, 1e3, 256), ns=3)
    c.set_profiling(True)
    c.plan_batch(db, "fp32")
    c.accumulate(db, "fp32")
    r = c.profile_cu_busy()
    print(f"[cu busy] {r}", flush=True)
    assert 0 < r["cus"] <= 1024
    assert 0 < r["min_ms"] <= r["mean_ms"] <= r["max_ms"]


def test_product_counts_accepted_and_refused():
    """FP16 takes one, two or three products, BF16 one or three; anything else is refused."""
    from paper_1003_1140_amd import LW_EINVAL, Context, LWError

    c = Context(0)
    for f16, bf16 in ((1, 1), (2, 3), (3, 1), (2, 1)):
        c.set_mfma_options(2, f16, bf16)
    for f16, bf16 in ((0, 3), (4, 3), (3, 2), (3, 0)):
        with pytest.raises(LWError) as e:
            c.set_mfma_options(2, f16, bf16)
        assert e.value.status == LW_EINVAL
    c.close()
