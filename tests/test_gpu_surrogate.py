"""GPU tests of the learned surrogate: features and network against the CPU
oracles, training, the surrogate sum, the fallback list, and the gain over the
exact path alone.

Tolerances.  Features are FP64 sums rounded once to FP32 (rtol 2e-5); counts
of reversals and of in-cone samples are FP64 decisions on the same inputs on
both sides (they may differ by at most one sample on an exact tie).  The
network multiplies BF16-rounded operands (unit roundoff u = 2^-8) with FP32
accumulation: outputs and gradients are compared element by element with a
reference that rounds the same operands to BF16 in FP64 (tests/_mlp_emul.py, pinned
to the FP64 oracle), each element within its rigorous bound -- FP32 accumulation,
BF16 rounding boundaries within reach, GELU evaluation -- on networks with one
hidden layer, and within four BF16 units of the RMS (and 99.9 % within the bound)
on deeper ones, where worst-case accumulation bounds outgrow the values.  A purely linear layer on
operands that are already BF16 values is exact up to FP32 accumulation (bar
1e-5).
"""
import time

import numpy as np
import pytest

import oracle
import workloads
from oracle import features as oracle_features
from workloads import configs

from _parity import band_integrated_errors

pytestmark = pytest.mark.gpu


def _bf16_round(a):
    """Round FP32 values to the nearest BF16 value (ties to even), kept as FP32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _ctx(dirs, omega, ns=1):
    from paper_1003_1140_amd import Context

    c = Context(0)
    c.set_directions(dirs)
    c.set_frequencies(omega)
    c.set_species(ns)
    return c


# ---------------------------------------------------------------- features
@pytest.mark.parametrize("dirs_name", ["jitter", "six"])
def test_features_match_oracle(dirs_name):
    import torch

    from paper_1003_1140_amd import DeviceBatch

    recipe = configs.jitter_recipe(steps=700)
    host = workloads.generate(recipe, 500, 5)
    dirs = configs.dirs_jitter() if dirs_name == "jitter" else configs.dirs_wide()[:6]
    c = _ctx(dirs, configs.log_grid(0.1, 1e3, 8))
    f = c.features(DeviceBatch.from_host(host)).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    ref = oracle_features.features(host, dirs)
    assert f.shape == ref.shape
    T = host.dt[0] * 700
    for j in range(16):
        if j == 8:
            np.testing.assert_allclose(f[..., j], ref[..., j], rtol=2e-5, atol=1.0 / T + 1e-6)
        elif j == 15:
            np.testing.assert_allclose(f[..., j], ref[..., j], rtol=0, atol=1.0 / 700 + 1e-6)
        else:
            np.testing.assert_allclose(f[..., j], ref[..., j], rtol=2e-5, atol=1e-6, err_msg=f"feature {j}")


def test_features_of_uneven_lengths():
    from paper_1003_1140_amd import DeviceBatch

    recipe = configs.uneven_recipe()
    host = workloads.generate(recipe, 0, 4)
    dirs = configs.dirs_jitter()
    c = _ctx(dirs, configs.log_grid(0.1, 1e3, 8))
    f = c.features(DeviceBatch.from_host(host)).cpu().numpy().astype(np.float64)
    ref = oracle_features.features(host, dirs)
    keep = [j for j in range(16) if j not in (8, 15)]
    np.testing.assert_allclose(f[..., keep], ref[..., keep], rtol=2e-5, atol=1e-6)


# ---------------------------------------------------------------- calibration statistics
def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_column_stats_match_numpy():
    """Grouped column moments of x, of x + c row_add and of 10^(...), over all particles and
    over those whose largest err is within a threshold: 700 particles (slices of 256 and a
    ragged one), 4 groups, 37 columns (part of one 64-column block), against NumPy in FP64."""
    c = _ctx(configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 8))
    rng = np.random.default_rng(17)
    P, G, C = 700, 4, 37
    x = rng.normal(size=(P * G, C)).astype(np.float32)
    ra = rng.normal(size=(P * G, 5)).astype(np.float32)
    err = rng.normal(size=P * G).astype(np.float32)
    x64 = x.astype(np.float64)
    out = c.column_stats(_dev(x)).cpu().numpy()
    np.testing.assert_allclose(out[0, :, 0], x64.mean(0), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(out[0, :, 1], (x64 ** 2).mean(0), rtol=1e-12)
    pmax = err.reshape(P, G).max(1)
    thr = float(np.sort(pmax)[int(0.8 * P)])  # a value the maxima take exactly
    keep = pmax <= thr
    out = c.column_stats(_dev(x), groups=G, row_add=_dev(ra)[:, 2], row_add_stride=5, row_add_coeff=-0.4,
                         exp10=True, err=_dev(err), threshold=thr).cpu().numpy()
    v = (10.0 ** (x64 - 0.4 * ra[:, 2:3].astype(np.float64))).reshape(P, G, C)[keep]
    np.testing.assert_allclose(out[:, :, 0], v.mean(0), rtol=1e-12)
    np.testing.assert_allclose(out[:, :, 1], (v ** 2).mean(0), rtol=1e-12)
    # no particle kept: zeros
    out = c.column_stats(_dev(x), groups=G, err=_dev(err), threshold=float(pmax.min()) - 1.0).cpu().numpy()
    assert np.all(out == 0.0)


def test_quantile_of_maxima_is_exact():
    """The q-quantile of per-particle maxima (linear interpolation, as NumPy's default) on
    values with negatives and many ties (rounded to 1/8), against np.quantile in FP64."""
    c = _ctx(configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 8))
    rng = np.random.default_rng(23)
    for P, G in ((1, 1), (2, 3), (999, 4), (25000, 4)):
        v = (np.round(rng.normal(size=(P, G)) * 8) / 8).astype(np.float32)
        pmax = v.max(1).astype(np.float64)
        for q in (0.0, 0.05, 0.37, 0.5, 0.95, 1.0):
            got = c.quantile_of_maxima(_dev(v), G, q)
            ref = float(np.quantile(pmax, q))
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (P, G, q, got, ref)


def test_error_share_and_log_ratio_match_numpy():
    c = _ctx(configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 8))
    rng = np.random.default_rng(29)
    P, G, C = 300, 4, 130
    y = rng.normal(scale=0.7, size=(P * G, C)).astype(np.float32)
    pr = (y + rng.normal(scale=0.2, size=y.shape)).astype(np.float32)
    y64, p64 = y.astype(np.float64), pr.astype(np.float64)
    smean = c.column_stats(_dev(y), groups=G, exp10=True)
    share = c.error_share(_dev(pr), _dev(y), G, smean, 1e-3).cpu().numpy()
    sm = (10.0 ** y64).reshape(P, G, C).mean(0)
    ref = np.log10(np.mean(np.abs(10.0 ** p64 - 10.0 ** y64) / np.tile(sm, (P, 1)), axis=1) + 1e-3)
    np.testing.assert_allclose(share, ref, rtol=1e-6, atol=1e-6)
    sp = c.column_stats(_dev(pr), groups=G, exp10=True)
    lr = c.log_ratio(smean, sp).cpu().numpy()
    a, b = smean.cpu().numpy()[..., 0].ravel(), sp.cpu().numpy()[..., 0].ravel()
    np.testing.assert_allclose(lr, np.log10(a / b), rtol=1e-6, atol=1e-7)


def test_column_stats_refuses_rows_not_a_multiple_of_groups():
    from paper_1003_1140_amd.lw import LWError

    c = _ctx(configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 8))
    x = np.zeros((10, 3), dtype=np.float32)
    with pytest.raises(LWError):
        c.column_stats(_dev(x), groups=4)


# ---------------------------------------------------------------- network vs oracle
def _net(c, shape, seed=3):
    from paper_1003_1140_amd import MLP

    return MLP(c, *shape, seed=seed)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_linear_layer_is_exact_on_bf16_operands():
    import torch

    c = _ctx(configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 8))
    shape = (16, 8, 0, 40)  # no hidden layer: y = x W^T + b
    net = _net(c, shape)
    rng = np.random.default_rng(5)
    p = _bf16_round(rng.normal(size=net.n_params))
    net.set_params(p)
    for rows in (64, 100, 1):
        x = _bf16_round(rng.normal(size=(rows, 16)))
        y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
        ref = oracle.mlp_forward_backward(shape, p.astype(np.float64), x.astype(np.float64))["y"]
        np.testing.assert_allclose(y, ref, rtol=1e-5, atol=1e-5)


def _params(net, rng, head=False):
    """The network's initial weights with small random biases (and an error head), as FP32."""
    p0, _ = net.get_params()
    p = p0 + rng.normal(scale=0.02, size=p0.size).astype(np.float32)
    h = rng.normal(scale=0.05, size=net.shape[1] + 1).astype(np.float32) if head else None
    net.set_params(p, h)
    return p.astype(np.float64), (h.astype(np.float64) if head else None)


def _check(name, got, ref, bound, rigorous):
    """Element-wise comparison with the BF16 emulation.  Rigorous: every element within its
    bound.  Otherwise (deep networks, where worst-case accumulation bounds grow past the
    values): every element within 2^-6 of the tensor's RMS (four BF16 units) and at least
    99.9 % of them within their bound."""
    d = np.abs(got - ref)
    r = d / np.maximum(bound, 1e-300)
    rms = float(np.sqrt(np.mean(ref ** 2)))
    inside = float(np.mean(d <= bound))
    print(f"[mlp emul] {name}: max |diff| / bound {r.max():.3f}, within bound {inside * 100:.3f} %, "
          f"max |diff| / rms {d.max() / rms:.2e}, median bound / |value| "
          f"{np.median(bound / np.maximum(np.abs(ref), 1e-300)):.1e}", flush=True)
    if rigorous:
        assert r.max() <= 1.0, name
    else:
        assert d.max() <= 2.0 ** -6 * rms, name
        assert inside >= 0.999, name


@pytest.mark.parametrize("shape,rows,rigorous", [((16, 64, 1, 32), 64, True), ((16, 64, 1, 32), 150, True),
                                                 ((16, 64, 1, 32), 4100, True), ((16, 64, 3, 48), 4100, False),
                                                 ((16, 256, 3, 256), 4100, False)])
def test_training_path_matches_bf16_emulation(shape, rows, rigorous):
    """The layered forward (z, GELU), the loss gradient and the backward products (split inner
    dimension for the weight gradients) against the BF16-emulating reference of
    tests/_mlp_emul.py, which is pinned to the FP64 oracle on the CPU."""
    import torch

    import _mlp_emul as E

    c = _ctx(configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 8))
    net = _net(c, shape)
    rng = np.random.default_rng(rows + shape[1])
    p, _ = _params(net, rng)
    x = rng.normal(size=(rows, shape[0])).astype(np.float32)
    t = rng.normal(size=(rows, shape[3])).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    loss, g = net.loss_grad(xd, td)
    ref = E.forward_backward(shape, p, x.astype(np.float64), t.astype(np.float64))
    fp64 = oracle.mlp_forward_backward(shape, p, x.astype(np.float64), t.astype(np.float64), want_grad=True)
    _check(f"gradient {shape} x {rows}", g.astype(np.float64), ref["grad"], ref["egrad"], rigorous)
    assert abs(loss - fp64["loss"]) <= 2e-2 * fp64["loss"]


@pytest.mark.parametrize("shape,rows,rigorous", [((16, 256, 1, 256), 4100, True), ((32, 128, 1, 32), 129, True),
                                                 ((16, 64, 2, 96), 150, False), ((16, 256, 3, 256), 64, False),
                                                 ((16, 256, 3, 256), 4100, False)])
def test_inference_matches_bf16_emulation(shape, rows, rigorous):
    """Inference (lw_mlp_forward) runs the whole network per tile of 128 rows in one kernel for
    these shapes: one tile, a ragged last tile, many tiles; with an input normalisation, an
    output skip and the error head.  Outputs and head against the BF16 emulation."""
    import torch

    import _mlp_emul as E

    c = _ctx(configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 8))
    net = _net(c, shape, seed=rows)
    rng = np.random.default_rng(rows + shape[1])
    n_in = shape[0]
    p, head = _params(net, rng, head=True)
    shift = rng.normal(size=n_in).astype(np.float32)
    scale = rng.uniform(0.5, 2.0, size=n_in).astype(np.float32)
    net.set_input_norm(shift, scale)
    skip, coeff = 3, 0.75
    net.set_output_skip(skip, coeff)
    x = (rng.normal(size=(rows, n_in)) * 2.0).astype(np.float32)
    y, e = net.forward(torch.from_numpy(x).cuda(), with_error=True)
    # the network's input as the kernel forms it: (x - shift) * scale in FP32
    xn = ((x - shift) * scale).astype(np.float32).astype(np.float64)
    ref = E.forward(shape, p, xn, skip=(x[:, skip].astype(np.float64), coeff), head=head)
    _check(f"output {shape} x {rows}", y.cpu().numpy().astype(np.float64), ref["y"], ref["ey"], rigorous)
    _check(f"error head {shape} x {rows}", e.cpu().numpy().astype(np.float64), ref["e"], ref["ee"], rigorous)


@pytest.mark.parametrize("which", ["x", "y"])
def test_inference_with_unaligned_rows_runs_layer_by_layer(which):
    """An input or output array that is not 16-byte aligned takes the layered path instead of
    the single kernel (which reads and writes rows 16 bytes at a time); its outputs and error
    head meet the same emulation bars, with the normalisation and the output skip."""
    import torch

    import _mlp_emul as E

    shape, rows = (16, 64, 2, 96), 150
    c = _ctx(configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 8))
    net = _net(c, shape, seed=11)
    rng = np.random.default_rng(11)
    n_in, n_out = shape[0], shape[3]
    p, head = _params(net, rng, head=True)
    shift = rng.normal(size=n_in).astype(np.float32)
    scale = rng.uniform(0.5, 2.0, size=n_in).astype(np.float32)
    net.set_input_norm(shift, scale)
    net.set_output_skip(3, 0.75)
    x = (rng.normal(size=(rows, n_in)) * 2.0).astype(np.float32)
    xb = torch.zeros(rows * n_in + 4, device="cuda")
    yb = torch.zeros(rows * n_out + 4, device="cuda")
    k = 1 if which == "x" else 0
    xd = xb[k:k + rows * n_in].view(rows, n_in)
    xd.copy_(torch.from_numpy(x))
    k = 1 if which == "y" else 0
    yd = yb[k:k + rows * n_out].view(rows, n_out)
    e = torch.zeros(rows, device="cuda")
    assert (xd.data_ptr() % 16 != 0) == (which == "x") and (yd.data_ptr() % 16 != 0) == (which == "y")
    c._check(c.lib.lw_mlp_forward(net.h, net._ptr(xd), rows, net._ptr(yd), net._ptr(e)))
    xn = ((x - shift) * scale).astype(np.float32).astype(np.float64)
    ref = E.forward(shape, p, xn, skip=(x[:, 3].astype(np.float64), 0.75), head=head)
    _check(f"unaligned {which} output", yd.cpu().numpy().astype(np.float64), ref["y"], ref["ey"], False)
    _check(f"unaligned {which} error head", e.cpu().numpy().astype(np.float64), ref["e"], ref["ee"], False)


def test_input_normalisation_matches_oracle_on_normalised_inputs():
    import torch

    c = _ctx(configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 8))
    shape = (16, 32, 2, 24)
    net = _net(c, shape)
    rng = np.random.default_rng(9)
    shift = rng.normal(size=16).astype(np.float32) * 100 + 1000  # large offsets
    scale = (1.0 / rng.uniform(0.5, 2.0, size=16)).astype(np.float32)
    scale[3] = 0.0  # a dropped feature
    net.set_input_norm(shift, scale)
    x = (shift + rng.normal(size=(80, 16)) / scale.clip(1e-3)).astype(np.float32)
    t = rng.normal(size=(80, 24)).astype(np.float32)
    p, _ = net.get_params()
    xn = (x.astype(np.float64) - shift) * scale
    ref = oracle.mlp_forward_backward(shape, p.astype(np.float64), xn, t.astype(np.float64), want_grad=True)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    y = net.forward(xd).cpu().numpy()
    _, g = net.loss_grad(xd, td)
    assert _rel(y, ref["y"]) < 2e-2
    assert _rel(g, ref["grad"]) < 5e-2


def test_training_reduces_the_loss_and_error_head_learns():
    import torch

    c = _ctx(configs.dirs_jitter(), configs.log_grid(0.1, 1e3, 8))
    shape = (16, 128, 3, 32)
    net = _net(c, shape, seed=7)
    rng = np.random.default_rng(11)
    teacher = rng.normal(size=(16, 32)) / 4.0
    x = rng.normal(size=(4096, 16)).astype(np.float32)
    t = np.sin(x @ teacher).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    first = net.train_step(xd, td, lr=2e-3)
    for _ in range(300):
        last = net.train_step(xd, td, lr=2e-3)
    print(f"[mlp] training loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < 0.1 * first
    # error head: learn |x_0| (a function of the input the trunk has features for)
    e_t = torch.from_numpy(np.abs(x[:, 0]).astype(np.float32)).cuda()
    h0 = net.train_head_step(xd, e_t, lr=3e-3)
    for _ in range(300):
        h1 = net.train_head_step(xd, e_t, lr=3e-3)
    print(f"[mlp] head loss {h0:.4f} -> {h1:.4f}", flush=True)
    assert h1 < 0.5 * h0
    _, e = net.forward(xd, with_error=True)
    assert np.isfinite(e.cpu().numpy()).all()


# ---------------------------------------------------------------- surrogate sum, fallback, targets
def _small_chunk(n=300, steps=512, first_id=0):
    from paper_1003_1140_amd import DeviceBatch
    from workloads.gpu import generate_device

    recipe = configs.surrogate_recipe(steps=steps)
    t, _ = generate_device(recipe, first_id, n)
    return DeviceBatch(t, n)


def test_surrogate_sum_compaction_and_targets():
    import torch

    omega = configs.log_grid(0.1, 1e3, 64)
    c = _ctx(configs.dirs_jitter(), omega)
    b = _small_chunk(n=2500)
    P, nd, nw = b.n_particles, c.nd, c.nw
    rng = np.random.default_rng(2)
    ylog = rng.normal(-2.0, 1.0, size=(P, nd, nw)).astype(np.float32)
    err = rng.uniform(0, 1, size=(P, nd)).astype(np.float32)
    yd, ed = torch.from_numpy(ylog).cuda(), torch.from_numpy(err).cuda()
    flags, idx, cnt = c.surrogate_accumulate(b, yd, ed, 0.9, compact=True)
    S = c.read_spectra()[0]
    fl = flags.cpu().numpy()
    want = (err > 0.9).any(1)
    assert np.array_equal(fl != 0, want)
    n = int(cnt.item())
    assert np.array_equal(idx[:n].cpu().numpy(), np.flatnonzero(want))
    w = b.t["weight"].cpu().numpy().astype(np.float64)
    q = b.t["charge"].cpu().numpy().astype(np.float64)
    keep = ~want
    ref = np.einsum("p,pdj->dj", (w * q * q)[keep], 10.0 ** ylog[keep].astype(np.float64))
    np.testing.assert_allclose(S, ref, rtol=1e-12)
    # targets from per-particle exact spectra
    c.reset()
    pp = torch.zeros((P, nd, nw), dtype=torch.float32, device="cuda")
    c.accumulate(b, "fp32", per_particle=pp)
    c.read_spectra()
    tg = c.surrogate_targets(b, pp).cpu().numpy()
    ref_t = np.log10(pp.cpu().numpy().astype(np.float64) / (w * q * q)[:, None, None] + 1e-30)
    np.testing.assert_allclose(tg, ref_t, rtol=0, atol=2e-6)


def test_fallback_extremes_reduce_to_exact_and_to_surrogate():
    import torch

    from paper_1003_1140_amd import surrogate as sg

    omega = configs.log_grid(0.1, 1e3, 32)
    c = _ctx(configs.dirs_jitter(), omega)
    b = _small_chunk(n=400)
    c.accumulate(b, "fp32")
    S_exact = c.read_spectra()
    c.reset()
    from paper_1003_1140_amd import MLP

    net = MLP(c, 16, 64, 3, c.nw, seed=1)
    sur = sg.Surrogate(net=net, threshold=0.0)
    # threshold -inf: everything falls back to the exact path
    r = sg.infer_chunk(c, sur, b, threshold=float("-inf"))
    assert r["fallback"] == b.n_particles
    np.testing.assert_allclose(c.read_spectra(), S_exact, rtol=1e-12)
    # the same on the matrix-core exact path (a gathered copy of the flagged particles): the
    # matrix-core sum of the whole chunk, exactly (the same particles in the same order)
    c.reset()
    c.accumulate(b, "mfma_f16")
    S_mfma = c.read_spectra()
    c.reset()
    r = sg.infer_chunk(c, sur, b, threshold=float("-inf"), exact_path="mfma_f16")
    assert r["fallback"] == b.n_particles
    np.testing.assert_array_equal(c.read_spectra(), S_mfma)
    assert float(np.max(band_integrated_errors(S_mfma[0], S_exact[0], omega))) <= 1e-5
    # threshold +inf: nothing falls back; S is the plain surrogate sum
    c.reset()
    r = sg.infer_chunk(c, sur, b, threshold=float("inf"))
    assert r["fallback"] == 0
    x = c.features(b).view(-1, 16)
    y = net.forward(x).cpu().numpy().astype(np.float64).reshape(b.n_particles, c.nd, c.nw)
    w = (b.t["weight"] * b.t["charge"] ** 2).cpu().numpy().astype(np.float64)
    ref = np.einsum("p,pdj->dj", w, 10.0 ** y)
    np.testing.assert_allclose(c.read_spectra()[0], ref, rtol=1e-6)
    torch.cuda.synchronize()


def test_trained_surrogate_is_judged_and_gains_over_exact():
    """End to end at reduced size: train on exact spectra, infer with the error-head
    fallback and a held-out judge, and time the pipeline against the exact path
    alone on the same particles."""
    import torch

    from paper_1003_1140_amd import surrogate as sg

    omega = configs.log_grid(0.1, 1e3, 256)
    c = _ctx(configs.dirs_jitter(), omega)
    train_b = _small_chunk(n=20000, steps=4096)
    calib = _small_chunk(n=5000, steps=4096, first_id=20000)
    sur = sg.train(c, train_b, calib, steps=1500, batch_rows=4096, fallback_fraction=0.05,
                   log=lambda m: print(m, flush=True))
    print(f"[surrogate] {sur.stats}", flush=True)
    assert sur.train_loss[-1] < 0.25 * sur.train_loss[0]
    del train_b, calib
    first = 1 << 20  # inference ids, disjoint from the training and calibration ids
    b = _small_chunk(n=40000, steps=4096, first_id=first)
    held = sg.held_out_indices(b.n_particles, first, 0.05, 7)
    # exact path alone
    c.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.accumulate(b, "fp32")
    S_exact = c.read_spectra()
    t_exact = time.perf_counter() - t0
    # pipeline (warm once for the network workspace and the judge's index plumbing)
    c.reset()
    sg.infer_chunk(c, sur, b, judge=sg.Judge(c), held=held)
    c.reset()
    judge = sg.Judge(c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = sg.infer_chunk(c, sur, b, judge=judge, held=held)
    S_pipe = c.read_spectra()
    Se, Sp, Ss = judge.spectra()
    t_pipe = time.perf_counter() - t0
    held_err = sg.held_out_errors(Se, Sp)
    sur_only = sg.held_out_errors(Se, Ss)
    floor = sg.split_half_floor(Se, judge.half_spectrum())
    ens = sg.held_out_errors(S_exact, S_pipe)
    band = float(np.max(band_integrated_errors(Sp, Se, omega)))
    for d in range(c.nd):
        live = S_exact[0, d] >= 1e-4 * S_exact[0, d].max()
        worst = int(np.argmax(np.where(live, np.abs(S_pipe[0, d] / S_exact[0, d] - 1), 0.0)))
        print(f"[surrogate] dir {d}: whole chunk worst bin {worst} (omega {omega[worst]:.3g}) ratio "
              f"{S_pipe[0, d, worst] / S_exact[0, d, worst]:.3f}; held-out per-bin max "
              f"{held_err['per_direction_max'][d]:.3f}, surrogate-only {sur_only['per_direction_max'][d]:.3f}",
              flush=True)
    print(f"[surrogate] fallback {r['fallback']} of {b.n_particles}; held-out ({judge.n}) per-bin max "
          f"{held_err['per_bin_max']:.3e} median {held_err['per_bin_median']:.3e}, band-integrated max "
          f"{band:.3e}; whole chunk per-bin max {ens['per_bin_max']:.3e} median {ens['per_bin_median']:.3e}; "
          f"exact {t_exact * 1e3:.1f} ms, pipeline {t_pipe * 1e3:.1f} ms, gain {t_exact / t_pipe:.2f}x",
          flush=True)
    print(f"[surrogate] held-out split-half floor: per-bin max {floor['per_bin_max']:.3e}, median "
          f"{floor['per_bin_median']:.3e}", flush=True)
    assert r["fallback"] <= 0.15 * b.n_particles
    # The target is 5 % per bin of the summed held-out spectrum.  Two thousand held-out
    # particles are too few for it in the perpendicular directions, where a few particles
    # carry much of the power: even a perfect prediction of each particle's mean spectrum
    # would miss their sum by the sampling noise, measured on the same particles as the
    # split-half floor.  The per-bin maximum must meet the target or stay within twice
    # that floor (the largest of several hundred noisy bins fluctuates by tens of percent
    # between two samples); the median bin must meet the target outright.
    assert held_err["per_bin_max"] <= max(0.05, 2.0 * floor["per_bin_max"])
    assert held_err["per_bin_median"] < 0.05
    assert ens["per_bin_max"] < 0.15
    assert ens["per_bin_median"] < 0.03
    assert float(np.max(band_integrated_errors(S_pipe, S_exact, omega))) < 0.1
    assert t_exact / t_pipe > 1.5
