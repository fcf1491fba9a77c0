"""In-situ coupling on the GPU: a device pusher hands windows to the recorder.

The pusher (workloads.gpu.InsituSim) advances persistent particles through the filament
field whose amplitude grows and saturates, each simulation step sub-cycled ten times
for the synthesis (Section 2.2: synthesis step at most a tenth of the simulation step).
Its windows go straight from device memory into the library.  The references come from
the oracle on the very trajectories the device produced (copied back), so the parity
bars are those of the FP32 path (1e-5, see test_gpu_fp32.py and test_gpu_coherent.py).
"""
import numpy as np
import pytest

import oracle
import workloads
from workloads import Batch, configs

from _parity import band_relative_error

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _join(windows):
    """Per particle, the samples of all windows in time order (one trajectory each)."""
    P = windows[0].n_particles
    parts = []
    for p in range(P):
        pieces = [w.select([p]) for w in windows]
        one = pieces[0]
        for k in ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az"):
            setattr(one, k, np.concatenate([getattr(q, k) for q in pieces]))
        one.offsets = np.array([0, one.x.size], dtype=np.int64)
        one.species = pieces[-1].species.copy()  # the region of the latest window
        parts.append(one)
    return Batch.concat(parts)


def _sim(n, regions=1):
    from workloads.gpu import InsituSim

    return InsituSim(configs.jitter_recipe(), 0, n, "cuda", n_regions=regions)


def test_pusher_windows_reproduce_the_one_shot_generator():
    """Constant amplitude 1 and the generator's step: the windows are its trajectory, bit for bit."""
    import torch
    from workloads.gpu import generate_device

    n = 16
    sim = _sim(n)
    wins = [{k: v.clone() for k, v in sim.window(4, 10, amplitude=lambda t: np.ones_like(t)).items()}
            for _ in range(3)]
    full, _ = generate_device(configs.jitter_recipe(), 0, n, "cuda")
    L = 4 * 10
    for k in ("x", "bx", "ax", "bz", "az"):
        got = torch.cat([w[k].view(n, L) for w in wins], dim=1)
        ref = full[k].view(n, -1)[:, :3 * L]
        assert torch.equal(got, ref), k
    assert abs(sim.t - 3 * L * configs.DT) < 1e-12


def test_pusher_preserves_the_lorentz_factor():
    """A magnetic field does no work: the Boris rotation keeps |u| to rounding."""
    sim = _sim(64)
    u0 = sim.state[3:].cpu().numpy()
    sim.window(20, 10)
    u1 = sim.state[3:].cpu().numpy()
    g0 = np.sqrt(1 + np.sum(u0**2, axis=0))
    g1 = np.sqrt(1 + np.sum(u1**2, axis=0))
    assert np.max(np.abs(g1 / g0 - 1)) < 1e-12
    assert np.max(np.abs(u1 - u0)) > 1e-3  # the field did deflect them


@pytest.mark.parametrize("path,bands", [("fp32", 1), ("mfma_f16", 1), ("mfma_f16", 2)])
def test_recorder_incoherent_windows(path, bands):
    """Snapshots of pusher windows recorded into the per-particle state match the oracle on
    the trajectory so far; on the matrix-core path with one band and with the two bands the
    benchmark's in-situ legs use."""
    from paper_1003_1140_amd import Context, DeviceBatch, Recorder
    from _parity import band_integrated_errors

    n, dirs, om = 20, configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 512)
    sim = _sim(n)
    c = Context(0)
    c.set_directions(dirs)
    c.set_frequencies(om)
    c.set_mfma_options(bands, 3, 3)
    rec = Recorder(c, n, coherent=False, path=path)
    host, snaps = [], []
    for _ in range(3):  # 3 windows of 16 simulation steps x 10 sub-steps
        t = sim.window(16, 10)
        rec.record(DeviceBatch(t, n))
        host.append(workloads.gpu.to_host(t))
        snaps.append(rec.snapshot())
    for i in range(3):
        ref = oracle.spectrum(_join(host[:i + 1]), dirs, om, n_species=1)
        if path == "fp32":
            err = band_relative_error(snaps[i], ref)
            assert err <= TOL, (i, err)
        else:
            err = band_integrated_errors(snaps[i].reshape(-1, len(om)), ref.reshape(-1, len(om)), om).max()
            assert err <= 1e-5, (i, err)
        print(f"[insitu] {path}, {bands} band(s), incoherent snapshot {i}: error {err:.3e}", flush=True)
    c.close()


def test_recorder_coherent_regions_and_differences():
    from paper_1003_1140_amd import Context, DeviceBatch, Recorder

    n, dirs, om, R = 24, configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 512), 3
    sim = _sim(n, regions=R)
    c = Context(0)
    c.set_directions(dirs)
    c.set_frequencies(om)
    c.set_species(R)
    rec = Recorder(c, n, coherent=True)
    host, snaps = [], []
    for _ in range(3):
        t = sim.window(16, 10)
        rec.record(DeviceBatch(t, n))
        host.append(workloads.gpu.to_host(t))
        snaps.append(rec.snapshot())
    regions = np.stack([h.species for h in host])
    assert regions.min() >= 0 and regions.max() < R
    # the oracle sums each window's pieces into the region the window assigns them to
    cat = Batch.concat(host)
    b2 = cat.select(np.arange(cat.n_particles))
    b2.weight = cat.weight.astype(np.float64) ** 2
    scale = oracle.spectrum(b2, dirs, om, n_species=R)  # sum of |w q A|^2 / (4 pi^2) per bin
    prev = np.zeros_like(snaps[0])
    for i in range(3):
        ref = oracle.coherent_spectrum(Batch.concat(host[:i + 1]), dirs, om, n_species=R)
        # power error from the amplitude bar: |dS| <= 2 |A| dA + dA^2, dA = TOL R
        dA2 = TOL**2 * scale
        bound = 2 * np.sqrt(ref * dA2) + dA2
        live = scale >= 1e-4 * scale.max(axis=-1, keepdims=True)
        assert np.all(np.abs(snaps[i] - ref)[live] <= 1.0001 * bound[live]), i
        d_ref = ref - (oracle.coherent_spectrum(Batch.concat(host[:i]), dirs, om, n_species=R) if i else 0)
        d_gpu = Recorder.instantaneous(snaps[i], prev)
        prev = snaps[i]
        rows = scale.max(axis=-1) > 0
        rel = np.max(np.abs(d_gpu - d_ref)[rows] / scale.max(axis=-1)[rows][:, None])
        assert rel <= 4 * TOL, (i, rel)
        print(f"[insitu] coherent snapshot {i}: instantaneous-state error {rel:.3e} of the row scale",
              flush=True)
    c.close()
