"""BF16-emulating reference of the surrogate network, with rigorous element-wise bounds.

The GPU network rounds every product operand to BF16 (round to nearest even), accumulates in
FP32, and keeps everything else (bias and skip additions, GELU, GELU', the loss gradient) in
FP32.  This module evaluates the same network in FP64 with the operands rounded to BF16 at
the same points, and carries for every element a bound on |GPU value - emulated value|:

* a product of inner length K with BF16 operands: the FP32 accumulation error
  gamma_K sum_k |a_k b_k| (gamma_K = K u / (1 - K u), u = 2^-24), plus the operands'
  own differences propagated through the other operand;
* rounding to BF16: the GPU's FP32 value lies within delta (+ its own FP32 rounding) of the
  emulated value; if no BF16 rounding boundary lies in that interval both round to the same
  BF16 number and the difference vanishes, otherwise it is at most the span of BF16 values
  the interval reaches (one unit in the last place);
* GELU and GELU': the difference of the argument times the largest slope over the
  interval, plus the FP32 evaluation error (a few units of FP32 and the 1.5e-7 absolute
  error of a rational erf).

Bounds of this kind stay near the FP32 accumulation level however deep the network, and a
mis-indexed element or a wrong rounding point exceeds them by orders of magnitude.  With
`bf16=False` the emulation is plain FP64 and must reproduce the FP64 oracle
(`oracle.mlp_forward_backward`), which pins its structure (layout, activation, loss).
"""
import numpy as np
from scipy import special as sp

U32 = 2.0 ** -24
ERF_ABS = 1.5e-7      # absolute error allowed for the GPU's erf (rational form or library)
GELU1 = 1.1289        # max |GELU'|
GELU2 = 0.7979        # max |GELU''|


def bf16(x):
    """Round to the nearest BF16 value (ties to even), elementwise, via FP32."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_span(v, delta, exact=False):
    """(BF16 value of v, max |difference| between the BF16 roundings of the FP32 values the
    GPU may hold: any x with |x - v| <= delta, rounded to FP32 and then to BF16).  exact:
    v is the GPU's FP32 value itself (weights, inputs), so the span is 0."""
    if exact:
        return bf16(v), np.zeros(np.shape(v))
    d = delta + 2.0 * U32 * np.abs(v) + 1e-45
    lo, hi, nom = bf16(v - d), bf16(v + d), bf16(v)
    return nom, np.maximum(np.abs(hi - nom), np.abs(nom - lo))


def gelu(z):
    return 0.5 * z * (1.0 + sp.erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + sp.erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def _matmul(a, sa, b, sb):
    """C = a @ b for BF16 nominal operands a, b with spans sa, sb; returns (C, bound)."""
    K = a.shape[1]
    g = K * U32 / (1.0 - K * U32)
    aa, ab = np.abs(a), np.abs(b)
    c = a @ b
    bound = sa @ ab + aa @ sb + sa @ sb + g * ((aa + sa) @ (ab + sb))
    return c, bound


def layers_of(shape, p):
    n_in, hidden, n_hidden, n_out = shape
    widths = [n_in] + [hidden] * n_hidden + [n_out]
    out, off = [], 0
    for l in range(n_hidden + 1):
        din, dout = widths[l], widths[l + 1]
        out.append((p[off:off + din * dout].reshape(dout, din), p[off + din * dout: off + din * dout + dout]))
        off += din * dout + dout
    return out


def forward(shape, p, x, bf=True, skip=None, head=None):
    """Emulated forward.  x: the network's input as the GPU forms it (after normalisation,
    FP32 values).  skip = (raw column values, coeff) added to every output.  head: the error
    head [hidden + 1].  Returns dict(y, ey, z, ez, a, ea, e, ee) with z/a per layer (the
    GPU's stored FP32 values and their bounds)."""
    layers = layers_of(shape, p)
    L = len(layers) - 1
    rnd = bf16_span if bf else (lambda v, d, exact=False: (v, d))
    a, ea = np.asarray(x, dtype=np.float64), np.zeros(np.shape(x))
    zs, ezs, acts, eacts = [], [], [a], [ea]
    for l, (W, b) in enumerate(layers):
        an, san = rnd(a, ea, exact=(l == 0))
        Wn, sWn = rnd(W.T, np.zeros_like(W.T), exact=True)
        z, ez = _matmul(an, san, Wn, sWn)
        z = z + b
        ez = ez + U32 * np.abs(z)            # the bias addition in FP32
        zs.append(z)
        ezs.append(ez)
        if l < L:
            a = gelu(z)
            ea = GELU1 * ez + 4.0 * U32 * np.abs(a) + ERF_ABS * 0.5 * np.abs(z)
            if not bf:
                ea = np.zeros_like(a)
            acts.append(a)
            eacts.append(ea)
    y, ey = zs[L], ezs[L]
    if skip is not None:
        raw, coeff = skip
        y = y + coeff * raw[:, None]
        ey = ey + U32 * (np.abs(y) + np.abs(coeff * raw[:, None]))
    out = {"y": y, "ey": ey if bf else np.zeros_like(y), "z": zs, "ez": ezs, "a": acts, "ea": eacts}
    if head is not None:
        h, eh = acts[L], eacts[L]
        K = h.shape[1]
        g = (K + 1) * U32 / (1.0 - (K + 1) * U32)
        w = np.asarray(head[:-1], dtype=np.float64)
        out["e"] = h @ w + head[-1]
        out["ee"] = eh @ np.abs(w) + g * (np.abs(h) @ np.abs(w) + abs(float(head[-1])))
    return out


def forward_backward(shape, p, x, t, bf=True):
    """Emulated forward, mean-squared loss against t and backward, as the layered GPU
    path computes them.  Returns dict(y, ey, grad, egrad) with grad laid out like p."""
    f = forward(shape, p, x, bf=bf)
    layers = layers_of(shape, p)
    L = len(layers) - 1
    rnd = bf16_span if bf else (lambda v, d, exact=False: (v, d))
    y, ey = f["y"], f["ey"]
    rows, n_out = y.shape
    scale = 2.0 / (rows * n_out)
    # dY = FP32(2 (y - t) / count), formed in FP64 from the FP32 y and t
    d = scale * (y - t)
    ed = scale * ey + U32 * np.abs(d)
    grads, bounds = [None] * (L + 1), [None] * (L + 1)
    for l in range(L, -1, -1):
        W, _ = layers[l]
        inp, einp = f["a"][l], f["ea"][l]
        dn, sdn = rnd(d, ed)
        inn, sinn = rnd(inp, einp, exact=(l == 0))
        dW, edW = _matmul(dn.T, sdn.T, inn, sinn)     # [dout][din]
        # bias gradient: column sums of the FP32 d in double precision
        db = d.sum(0)
        edb = ed.sum(0) + rows * 2.0 ** -53 * np.abs(d).sum(0) + U32 * np.abs(db)
        grads[l] = np.concatenate([dW.ravel(), db])
        bounds[l] = np.concatenate([edW.ravel(), edb])
        if l > 0:
            Wn, sWn = rnd(W, np.zeros_like(W), exact=True)
            back, eback = _matmul(dn, sdn, Wn, sWn)   # [rows][din]
            z, ez = f["z"][l - 1], f["ez"][l - 1]
            gp = gelu_grad(z)
            egp = GELU2 * ez + 10.0 * U32 + ERF_ABS
            d = back * gp
            ed = eback * (np.abs(gp) + egp) + np.abs(back) * egp + U32 * np.abs(d)
            if not bf:
                ed = np.zeros_like(d)
    return {"y": y, "ey": ey, "grad": np.concatenate(grads), "egrad": np.concatenate(bounds),
            "loss": float(np.mean((y - t) ** 2))}
