"""CPU checks of the BF16-emulating network reference used by the GPU network tests.

* BF16 rounding (round to nearest, ties to even) on hand-picked values;
* with rounding off, the emulation reproduces the FP64 oracle (forward and gradients), which
  pins its layout, activation and loss to the oracle's definition;
* a CPU simulation of the GPU arithmetic -- operands rounded to BF16, products accumulated in
  FP32 (NumPy's order, not the GPU's), FP32 bias, GELU, loss gradient -- lies within the
  emulation's element-wise bounds, so that the bounds hold for an accumulation order other
  than the emulation's own.
"""
import numpy as np
import pytest

import oracle

import _mlp_emul as E


def test_bf16_rounding_ties_to_even():
    u = 2.0 ** -7  # BF16 spacing on [1, 2)
    cases = {1.0: 1.0, 1.0 + u / 2: 1.0, 1.0 + 1.5 * u: 1.0 + 2 * u, 1.0 + 0.51 * u: 1.0 + u,
             -(1.0 + 1.5 * u): -(1.0 + 2 * u), 3.0e-3: None}
    for v, want in cases.items():
        got = float(E.bf16(v))
        if want is None:
            assert abs(got - v) <= 2.0 ** -8 * abs(v)
        else:
            assert got == want, (v, got, want)
    nom, span = E.bf16_span(np.array([1.0 + 0.25 * u, 1.0 + 0.5 * u]), np.array([1e-6, 1e-6]))
    assert list(nom) == [1.0, 1.0] and span[0] == 0.0 and span[1] == u


def _random_net(shape, seed):
    rng = np.random.default_rng(seed)
    widths = [shape[0]] + [shape[1]] * shape[2] + [shape[3]]
    p = []
    for l in range(shape[2] + 1):
        din, dout = widths[l], widths[l + 1]
        p += [rng.normal(size=(dout, din)).ravel() / np.sqrt(din), rng.normal(scale=0.02, size=dout)]
    p = np.concatenate(p).astype(np.float32).astype(np.float64)
    x = rng.normal(size=(97, shape[0])).astype(np.float32).astype(np.float64)
    t = rng.normal(size=(97, shape[3])).astype(np.float32).astype(np.float64)
    return p, x, t


@pytest.mark.parametrize("shape", [(16, 32, 1, 24), (16, 64, 3, 48)])
def test_unrounded_emulation_is_the_oracle(shape):
    p, x, t = _random_net(shape, 3)
    ref = oracle.mlp_forward_backward(shape, p, x, t, want_grad=True)
    e = E.forward_backward(shape, p, x, t, bf=False)
    np.testing.assert_allclose(e["y"], ref["y"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(e["grad"], ref["grad"], rtol=1e-10, atol=1e-16)
    assert abs(e["loss"] - ref["loss"]) <= 1e-12 * ref["loss"]


def _simulated_gpu(shape, p, x, t):
    """The GPU's arithmetic on the CPU: BF16 operands, FP32 accumulation and epilogues."""
    f32 = np.float32
    layers = E.layers_of(shape, p)
    L = len(layers) - 1
    bf = lambda v: E.bf16(v).astype(f32)
    gelu = lambda z: E.gelu(z.astype(np.float64)).astype(f32)
    gp = lambda z: E.gelu_grad(z.astype(np.float64)).astype(f32)
    a, acts, zs = x.astype(f32), [x.astype(f32)], []
    for l, (W, b) in enumerate(layers):
        z = (bf(a) @ bf(W.T)).astype(f32) + b.astype(f32)
        zs.append(z)
        if l < L:
            a = gelu(z)
            acts.append(a)
    y = zs[L]
    d = ((2.0 / y.size) * (y.astype(np.float64) - t)).astype(f32)
    grads = [None] * (L + 1)
    for l in range(L, -1, -1):
        W, _ = layers[l]
        dW = (bf(d).T @ bf(acts[l])).astype(f32)
        db = d.astype(np.float64).sum(0).astype(f32)
        grads[l] = np.concatenate([dW.ravel(), db])
        if l > 0:
            d = ((bf(d) @ bf(W)).astype(f32) * gp(zs[l - 1])).astype(f32)
    return y.astype(np.float64), np.concatenate(grads).astype(np.float64)


@pytest.mark.parametrize("shape,seed", [((16, 32, 1, 24), 1), ((16, 64, 1, 32), 2), ((8, 256, 1, 64), 3)])
def test_fp32_simulation_lies_within_the_bounds(shape, seed):
    p, x, t = _random_net(shape, seed)
    e = E.forward_backward(shape, p, x, t)
    y, g = _simulated_gpu(shape, p, x, t)
    assert np.all(np.abs(y - e["y"]) <= e["ey"])
    assert np.all(np.abs(g - e["grad"]) <= e["egrad"])
    # and the bounds are tight enough to matter: far below the values for most elements
    assert np.median(e["ey"] / np.abs(e["y"])) < 1e-3
