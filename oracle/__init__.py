"""FP64 CPU oracle of the radiation spectral synthesis.

TEST INFRASTRUCTURE.  Only tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP library
(``paper_1003_1140_amd``) neither imports it nor shares code with it.

``lw_oracle.c`` is the plain definition of the discretised Lienard-Wiechert
spectral integral (paper, Section 2.2): for every particle, direction n and
frequency w,

    A_p(n, w) = sum_k n x ((n - beta_k) x betadot_k) / (1 - n.beta_k)^2
                      * exp(i w (t_k - n.r_k)) * dt
    S(s, n, w) = sum_{p in s} w_p q_p^2 |A_p|^2 / (4 pi^2)

in FP64 with libm sin/cos.  ``mlp_oracle.c`` is the FP64 reference of the
spectrum surrogate network (forward and backward).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liblw_oracle.so")
_SOURCES = ["lw_oracle.c", "mlp_oracle.c"]

LWO_OK, LWO_EINVAL, LWO_ENOMEM, LWO_ERANGE = 0, -1, -2, -5


class OracleError(RuntimeError):
    def __init__(self, status, where=-1):
        super().__init__(f"oracle status {status} (first offending particle {where})")
        self.status = status
        self.where = where


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", *srcs, "-o", _SO + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        _lib = ctypes.CDLL(_SO)
        for name in ("lwo_amplitude", "lwo_spectrum", "lwo_sampled_bins", "lwo_max_threads",
                     "lwo_coherent_spectrum"):
            getattr(_lib, name).restype = ctypes.c_int
        _lib.mlpo_num_params.restype = ctypes.c_int64
        _lib.mlpo_forward_backward.restype = ctypes.c_double
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def max_threads() -> int:
    return int(_load().lwo_max_threads())


def amplitude(batch, p, direction, omega):
    """Complex amplitude A_p(n, w) of particle p: array [nw, 3] complex128."""
    lib = _load()
    o0, o1 = int(batch.offsets[p]), int(batch.offsets[p + 1])
    arrs = [_f64(getattr(batch, k)[o0:o1]) for k in ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az")]
    om = _f64(np.atleast_1d(omega))
    d = _f64(direction)
    out = np.zeros((om.size, 3, 2), dtype=np.float64)
    bad = ctypes.c_int64(-1)
    st = lib.lwo_amplitude(ctypes.c_int64(o1 - o0), *[_p(a) for a in arrs],
                           ctypes.c_double(float(batch.t0[p])), ctypes.c_double(float(batch.dt[p])),
                           _p(d), ctypes.c_int32(om.size), _p(om), _p(out), ctypes.byref(bad))
    if st != LWO_OK:
        raise OracleError(st, bad.value)
    return out[..., 0] + 1j * out[..., 1]


def spectrum(batch, dirs, omega, n_species=None, per_particle=False, nthreads=0):
    """S[s, d, j] (and optionally the per-particle terms [P, nd, nw])."""
    lib = _load()
    dirs = _f64(np.atleast_2d(dirs))
    om = _f64(omega)
    spec = np.ascontiguousarray(batch.species, dtype=np.int32)
    if n_species is None:
        n_species = int(spec.max()) + 1 if spec.size else 1
    P = batch.n_particles
    S = np.zeros((n_species, dirs.shape[0], om.size), dtype=np.float64)
    pp = np.zeros((P, dirs.shape[0], om.size), dtype=np.float64) if per_particle else None
    arrs = [_f64(getattr(batch, k)) for k in ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az")]
    offs = np.ascontiguousarray(batch.offsets - batch.offsets[0], dtype=np.int64)
    bad = ctypes.c_int64(-1)
    st = lib.lwo_spectrum(ctypes.c_int64(P), _p(offs), *[_p(a) for a in arrs], _p(_f64(batch.t0)),
                          _p(_f64(batch.dt)), _p(_f64(batch.charge)), _p(_f64(batch.weight)),
                          _p(spec), ctypes.c_int32(n_species), _p(dirs),
                          ctypes.c_int32(dirs.shape[0]), _p(om), ctypes.c_int32(om.size), _p(S),
                          _p(pp), ctypes.c_int(nthreads), ctypes.byref(bad))
    if st != LWO_OK:
        raise OracleError(st, bad.value)
    return (S, pp) if per_particle else S


def coherent_spectrum(batch, dirs, omega, n_species=None, with_amplitude=False, nthreads=0):
    """Coherent S[s, d, j] = |sum_p w_p q_p A_p|^2 / (4 pi^2) (and the summed amplitude
    [s, d, j, 3] complex when asked)."""
    lib = _load()
    dirs = _f64(np.atleast_2d(dirs))
    om = _f64(omega)
    spec = np.ascontiguousarray(batch.species, dtype=np.int32)
    if n_species is None:
        n_species = int(spec.max()) + 1 if spec.size else 1
    S = np.zeros((n_species, dirs.shape[0], om.size), dtype=np.float64)
    A = np.zeros((n_species, dirs.shape[0], om.size, 3, 2), dtype=np.float64) if with_amplitude else None
    arrs = [_f64(getattr(batch, k)) for k in ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az")]
    offs = np.ascontiguousarray(batch.offsets - batch.offsets[0], dtype=np.int64)
    bad = ctypes.c_int64(-1)
    st = lib.lwo_coherent_spectrum(ctypes.c_int64(batch.n_particles), _p(offs), *[_p(a) for a in arrs],
                                   _p(_f64(batch.t0)), _p(_f64(batch.dt)), _p(_f64(batch.charge)),
                                   _p(_f64(batch.weight)), _p(spec), ctypes.c_int32(n_species), _p(dirs),
                                   ctypes.c_int32(dirs.shape[0]), _p(om), ctypes.c_int32(om.size), _p(S),
                                   _p(A), ctypes.c_int(nthreads), ctypes.byref(bad))
    if st != LWO_OK:
        raise OracleError(st, bad.value)
    return (S, A[..., 0] + 1j * A[..., 1]) if with_amplitude else S


def sampled_bins(batch, dirs, omega, species=-1, nthreads=0):
    """Spectrum at a list of (direction, frequency) pairs, summed over the batch."""
    lib = _load()
    dirs = _f64(np.atleast_2d(dirs))
    om = _f64(np.atleast_1d(omega))
    assert dirs.shape[0] == om.size
    out = np.zeros(om.size, dtype=np.float64)
    arrs = [_f64(getattr(batch, k)) for k in ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az")]
    offs = np.ascontiguousarray(batch.offsets - batch.offsets[0], dtype=np.int64)
    st = lib.lwo_sampled_bins(ctypes.c_int64(batch.n_particles), _p(offs), *[_p(a) for a in arrs],
                              _p(_f64(batch.t0)), _p(_f64(batch.dt)), _p(_f64(batch.charge)),
                              _p(_f64(batch.weight)),
                              _p(np.ascontiguousarray(batch.species, dtype=np.int32)),
                              ctypes.c_int32(species), ctypes.c_int32(om.size), _p(dirs), _p(om),
                              _p(out), ctypes.c_int(nthreads))
    if st != LWO_OK:
        raise OracleError(st)
    return out


# ---------------------------------------------------------------- surrogate network (FP64)
def mlp_num_params(n_in, hidden, n_hidden, n_out):
    return int(_load().mlpo_num_params(n_in, hidden, n_hidden, n_out))


def mlp_gelu(z):
    z = _f64(z)
    out = np.empty_like(z)
    _load().mlpo_gelu(_p(z), _p(out), ctypes.c_int64(z.size))
    return out


def mlp_forward_backward(shape, params, x, t=None, want_grad=False, want_hidden=False):
    """shape = (n_in, hidden, n_hidden, n_out).  Returns dict(y, loss, grad, hidden)."""
    n_in, hidden, n_hidden, n_out = shape
    lib = _load()
    params = _f64(params)
    x = _f64(x)
    rows = x.shape[0]
    y = np.zeros((rows, n_out))
    tt = _f64(t) if t is not None else None
    grad = np.zeros(params.size) if want_grad else None
    hid = np.zeros((rows, hidden)) if want_hidden else None
    loss = lib.mlpo_forward_backward(n_in, hidden, n_hidden, n_out, _p(params), _p(x), _p(tt),
                                     ctypes.c_int64(rows), _p(y), _p(grad), _p(hid))
    return {"y": y, "loss": float(loss), "grad": grad, "hidden": hid}
