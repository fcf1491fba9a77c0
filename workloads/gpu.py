"""Device twin of the filament-ensemble generator (inputs only, not the method).

``generate_device(recipe, first_id, n, device)`` writes particles
first_id .. first_id+n-1 straight into device tensors (the structure-of-arrays
layout of ``workloads.Batch``), for ensembles too large to pass through the host.
The host generator remains the source of every oracle input.
"""
from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import numpy as np

from . import _load as _load_host
from . import particle_meta

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libworkloads_gpu.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
        if not os.path.exists(hipcc):
            hipcc = shutil.which("hipcc") or hipcc
        cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-ffp-contract=off",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument",
               os.path.join(_HERE, "filaments_gpu.hip"), "-o", _SO + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is missing: run workloads.gpu.build()")
        import torch  # noqa: F401  (share torch's HIP runtime)

        _lib = ctypes.CDLL(_SO)
        _lib.wl_generate_gpu.restype = ctypes.c_int
    return _lib


def field_coeffs(recipe):
    host = _load_host()
    cap = 64 * 129
    cre = np.zeros(cap)
    cim = np.zeros(cap)
    k0 = ctypes.c_double()
    imax = host.wl_field_coeffs(ctypes.byref(recipe), cre.ctypes.data_as(ctypes.c_void_p),
                                cim.ctypes.data_as(ctypes.c_void_p), ctypes.c_int64(cap),
                                ctypes.byref(k0))
    if imax < 0:
        raise RuntimeError("field coefficient table too large")
    cells = (imax + 1) * (2 * imax + 1)
    return imax, k0.value, cre[:cells].copy(), cim[:cells].copy()


def generate_device(recipe, first_id, n, device="cuda"):
    """Returns (dict of device tensors in the Batch layout, number of samples)."""
    import torch

    lib = _load()
    dev = torch.device(device)
    lens = particle_meta(recipe, first_id, n)[0].astype(np.int64)
    offs = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    ns = int(offs[-1])
    imax, k0, cre, cim = field_coeffs(recipe)
    t = {"offsets": torch.from_numpy(offs).to(dev)}
    for k in ("x", "y", "z", "bx", "by", "bz"):
        t[k] = torch.empty(ns, dtype=torch.float64, device=dev)
    for k in ("ax", "ay", "az"):
        t[k] = torch.empty(ns, dtype=torch.float32, device=dev)
    t["t0"] = torch.empty(n, dtype=torch.float64, device=dev)
    t["dt"] = torch.empty(n, dtype=torch.float64, device=dev)
    t["charge"] = torch.empty(n, dtype=torch.float32, device=dev)
    t["weight"] = torch.empty(n, dtype=torch.float32, device=dev)
    t["species"] = torch.empty(n, dtype=torch.int32, device=dev)
    dcre = torch.from_numpy(cre).to(dev)
    dcim = torch.from_numpy(cim).to(dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    p = lambda ten: ctypes.c_void_p(ten.data_ptr())
    st = lib.wl_generate_gpu(ctypes.byref(recipe), ctypes.c_int64(first_id), ctypes.c_int64(n),
                             p(t["offsets"]), ctypes.c_int32(imax), ctypes.c_double(k0), p(dcre),
                             p(dcim), *[p(t[k]) for k in ("x", "y", "z", "bx", "by", "bz", "ax",
                                                           "ay", "az", "t0", "dt", "charge",
                                                           "weight", "species")],
                             p(status), ctypes.c_void_p(stream))
    if st != 0:
        raise RuntimeError(f"wl_generate_gpu failed ({st})")
    torch.cuda.synchronize(dev)
    if int(status.item()) != 0:
        raise RuntimeError("device generator: particle lengths disagree with the offsets")
    return t, ns
