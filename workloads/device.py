"""Generate a workload on the host chunk by chunk and upload it into device tensors.

Returns the tensors of the structure-of-arrays batch layout (names as in
``workloads.Batch``) so that the caller can wrap them for the library, and
lets the caller look at every host chunk (e.g. to feed the oracle) before it
is dropped, so host memory stays at one chunk.
"""
from __future__ import annotations

import numpy as np

from . import generate, particle_meta

F64 = ("x", "y", "z", "bx", "by", "bz")
F32 = ("ax", "ay", "az")
PER_PARTICLE = {"t0": "float64", "dt": "float64", "charge": "float32", "weight": "float32",
                "species": "int32"}


def upload_chunks(recipe, n, chunk, device, on_chunk=None, first_id=0):
    import torch

    lens = particle_meta(recipe, first_id, n)[0].astype(np.int64)
    offs = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    ns = int(offs[-1])
    t = {"offsets": torch.from_numpy(offs).to(device)}
    for k in F64:
        t[k] = torch.empty(ns, dtype=torch.float64, device=device)
    for k in F32:
        t[k] = torch.empty(ns, dtype=torch.float32, device=device)
    for k, dt in PER_PARTICLE.items():
        t[k] = torch.empty(n, dtype=getattr(torch, dt), device=device)
    for p0 in range(0, n, chunk):
        p1 = min(n, p0 + chunk)
        h = generate(recipe, first_id + p0, p1 - p0)
        s0, s1 = int(offs[p0]), int(offs[p1])
        for k in F64 + F32:
            t[k][s0:s1].copy_(torch.from_numpy(getattr(h, k)))
        for k in PER_PARTICLE:
            t[k][p0:p1].copy_(torch.from_numpy(getattr(h, k)))
        if on_chunk is not None:
            on_chunk(h)
    torch.cuda.synchronize()
    return t, ns
