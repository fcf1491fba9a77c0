"""Device twin of the filament-ensemble generator (inputs only, not the method).

``generate_device(recipe, first_id, n, device)`` writes particles
first_id .. first_id+n-1 straight into device tensors (the structure-of-arrays
layout of ``workloads.Batch``), for ensembles too large to pass through the host.
The host generator remains the source of every oracle input.

``InsituSim`` is the in-situ stand-in: the same particles kept on the device and
advanced window by window through the filament field with an amplitude that grows
and saturates in time (linear filamentation growth, then saturation, Section 3.1),
each simulation step sub-cycled for the synthesis (Section 2.2).  Its windows are
what a PIC code would hand the diagnostic between two recordings; ``to_host`` copies
one back so that the oracle sees exactly the trajectories the device produced.
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
        _lib.wl_insitu_init_gpu.restype = ctypes.c_int
        _lib.wl_insitu_push_gpu.restype = ctypes.c_int
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


def to_host(tensors):
    """A workloads.Batch (numpy) copy of device tensors in the Batch layout."""
    from . import Batch

    h = {k: v.cpu().numpy() for k, v in tensors.items()}
    return Batch(offsets=h["offsets"] - h["offsets"][0], x=h["x"], y=h["y"], z=h["z"], bx=h["bx"],
                 by=h["by"], bz=h["bz"], ax=h["ax"], ay=h["ay"], az=h["az"], t0=h["t0"], dt=h["dt"],
                 charge=h["charge"], weight=h["weight"], species=h["species"])


def growth_amplitude(t, a0=0.01, gamma=0.4, a_sat=1.0):
    """Filament field amplitude: exponential growth at rate gamma from a0, saturating at a_sat
    (a_sat / sqrt(1 + (a_sat^2 / a0^2 - 1) e^{-2 gamma t}))."""
    t = np.asarray(t, dtype=np.float64)
    return a_sat / np.sqrt(1.0 + (a_sat**2 / a0**2 - 1.0) * np.exp(-2.0 * gamma * t))


class InsituSim:
    """Particles first_id .. first_id+n-1 of ``recipe`` advanced window by window on the device.

    ``window(n_steps, n_sub, amplitude)`` advances n_steps simulation steps of n_sub
    synthesis steps of recipe.dt each, with the field amplitude ``amplitude(t)`` taken at
    the simulation step boundaries, and returns the window's samples as device tensors in
    the Batch layout (species = collection region, the z-slab at the window start).  The
    tensors are reused by the next window of the same shape.
    """

    def __init__(self, recipe, first_id, n, device="cuda", n_regions=1):
        import torch

        self.lib = _load()
        self.recipe = recipe
        self.n = int(n)
        self.dev = torch.device(device)
        self.n_regions = int(n_regions)
        self.imax, self.k0, cre, cim = field_coeffs(recipe)
        self.cre = torch.from_numpy(cre).to(self.dev)
        self.cim = torch.from_numpy(cim).to(self.dev)
        self.state = torch.empty((6, self.n), dtype=torch.float64, device=self.dev)
        self.charge = torch.empty(self.n, dtype=torch.float32, device=self.dev)
        self.mass = torch.empty(self.n, dtype=torch.float32, device=self.dev)
        self.t = 0.0
        self._buf = None
        st = self.lib.wl_insitu_init_gpu(ctypes.byref(recipe), ctypes.c_int64(first_id),
                                         ctypes.c_int64(self.n), self._p(self.state),
                                         self._p(self.charge), self._p(self.mass), self._stream())
        if st != 0:
            raise RuntimeError(f"wl_insitu_init_gpu failed ({st})")

    @staticmethod
    def _p(t):
        return ctypes.c_void_p(t.data_ptr())

    def _stream(self):
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)

    def _buffers(self, L):
        import torch

        if self._buf is not None and self._buf[0] == L:
            return self._buf[1]
        n, dev = self.n, self.dev
        t = {"offsets": torch.arange(n + 1, dtype=torch.int64, device=dev) * L}
        for k in ("x", "y", "z", "bx", "by", "bz"):
            t[k] = torch.empty(n * L, dtype=torch.float64, device=dev)
        for k in ("ax", "ay", "az"):
            t[k] = torch.empty(n * L, dtype=torch.float32, device=dev)
        for k, dt in (("t0", torch.float64), ("dt", torch.float64), ("charge", torch.float32),
                      ("weight", torch.float32), ("species", torch.int32)):
            t[k] = torch.empty(n, dtype=dt, device=dev)
        self._buf = (L, t)
        return t

    def window(self, n_steps, n_sub, amplitude=growth_amplitude):
        import torch

        dt = self.recipe.dt
        L = int(n_steps) * int(n_sub)
        t = self._buffers(L)
        bounds = self.t + dt * n_sub * np.arange(n_steps + 1)
        amp = torch.from_numpy(np.ascontiguousarray(amplitude(bounds), dtype=np.float64)).to(self.dev)
        st = self.lib.wl_insitu_push_gpu(
            ctypes.c_int32(self.imax), ctypes.c_double(self.k0), self._p(self.cre), self._p(self.cim),
            ctypes.c_int64(self.n), self._p(self.state), self._p(self.charge), self._p(self.mass),
            self._p(amp), ctypes.c_int32(n_steps), ctypes.c_int32(n_sub), ctypes.c_double(dt),
            ctypes.c_double(self.t), ctypes.c_double(self.recipe.box), ctypes.c_int32(self.n_regions),
            *[self._p(t[k]) for k in ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az", "t0", "dt",
                                       "charge", "weight", "species")],
            self._stream())
        if st != 0:
            raise RuntimeError(f"wl_insitu_push_gpu failed ({st})")
        self.t += dt * L
        return t  # (amp is freed in stream order: the caching allocator reuses it only after)
