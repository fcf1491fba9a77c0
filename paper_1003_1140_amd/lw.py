"""ctypes binding of include/lw.h (argument marshalling only).

Functions keep the C names (``lw_create``, ``lw_accumulate`` ...).  PyTorch
supplies device memory and the HIP stream; no torch operation touches the
accumulation itself.  The binding raises if liblw.so has not been built --
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblw.so")

LW_OK, LW_EINVAL, LW_ENOMEM, LW_EDEVICE, LW_ESTATE, LW_ERANGE, LW_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
LW_PATH_FP32, LW_PATH_MFMA_F16, LW_PATH_MFMA_BF16, LW_PATH_AUTO = 0, 1, 2, 3
PATHS = {"fp32": LW_PATH_FP32, "mfma_f16": LW_PATH_MFMA_F16, "mfma_bf16": LW_PATH_MFMA_BF16,
         "auto": LW_PATH_AUTO}
LW_BATCH_F64_ACCEL = 1
LW_AUTO_MIN_FREQUENCIES = 256

EXPORTED = ("lw_create", "lw_destroy", "lw_last_error", "lw_set_stream", "lw_set_directions",
            "lw_set_frequencies", "lw_set_log_frequencies", "lw_get_frequencies", "lw_set_species",
            "lw_workspace_size", "lw_accumulate", "lw_read_spectra", "lw_reset",
            "lw_load_accumulator", "lw_stats", "lw_set_mfma_options", "lw_set_mfma_chunk_bytes",
            "lw_mfma_plan_info", "lw_set_profiling",
            "lw_profile_read", "lw_plan_batch", "lw_set_tuning", "lw_tune", "lw_graph_capture",
            "lw_graph_launch", "lw_graph_destroy", "lw_accumulate_subset", "lw_subset_offsets",
            "lw_gather_particles", "lw_features",
            "lw_mlp_create", "lw_mlp_destroy", "lw_mlp_num_params", "lw_mlp_get_params",
            "lw_mlp_set_params", "lw_mlp_set_input_norm", "lw_mlp_set_output_skip",
            "lw_mlp_forward", "lw_mlp_loss_grad", "lw_mlp_train_step",
            "lw_mlp_train_head_step", "lw_surrogate_accumulate", "lw_surrogate_targets",
            "lw_set_coherent", "lw_get_basis", "lw_read_amplitudes", "lw_load_amplitudes",
            "lw_accumulate_amplitudes", "lw_amplitude_workspace_size", "lw_spectrum_from_amplitudes",
            "lw_spectral_diagnostics", "lw_pitch_cones", "lw_profile_cu_busy", "lw_save_accumulator",
            "lw_load_accumulator_file", "lw_mlp_save", "lw_mlp_load", "lw_accumulate_noalloc",
            "lw_column_stats", "lw_error_share", "lw_quantile_of_maxima", "lw_log_ratio")


class LWError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"lw status {status}: {message}")
        self.status = status


class lw_batch(ctypes.Structure):
    _fields_ = [
        ("n_particles", ctypes.c_int64),
        ("offsets", ctypes.c_void_p),
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
        ("bx", ctypes.c_void_p), ("by", ctypes.c_void_p), ("bz", ctypes.c_void_p),
        ("ax", ctypes.c_void_p), ("ay", ctypes.c_void_p), ("az", ctypes.c_void_p),
        ("t0", ctypes.c_void_p), ("dt", ctypes.c_void_p),
        ("charge", ctypes.c_void_p), ("weight", ctypes.c_void_p),
        ("species", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
    ]


_lib = None


def load_library():
    """Load liblw.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_1003_1140_amd/build.py`")
        lib = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        sig = {
            "lw_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int, P]),
            "lw_destroy": (None, [P]),
            "lw_last_error": (ctypes.c_char_p, [P]),
            "lw_set_stream": (ctypes.c_int, [P, P]),
            "lw_set_directions": (ctypes.c_int, [P, P, I32]),
            "lw_set_frequencies": (ctypes.c_int, [P, P, I32]),
            "lw_set_log_frequencies": (ctypes.c_int, [P, D, D, I32]),
            "lw_get_frequencies": (ctypes.c_int, [P, P]),
            "lw_set_species": (ctypes.c_int, [P, I32]),
            "lw_workspace_size": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), ctypes.c_int, ctypes.POINTER(SZ)]),
            "lw_accumulate": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), ctypes.c_int, P, SZ, P]),
            "lw_read_spectra": (ctypes.c_int, [P, P]),
            "lw_reset": (ctypes.c_int, [P]),
            "lw_load_accumulator": (ctypes.c_int, [P, P]),
            "lw_stats": (ctypes.c_int, [P, ctypes.POINTER(I64)]),
            "lw_set_mfma_options": (ctypes.c_int, [P, I32, I32, I32]),
            "lw_set_mfma_chunk_bytes": (ctypes.c_int, [P, I64]),
            "lw_mfma_plan_info": (ctypes.c_int, [P, P, ctypes.c_int, P]),
            "lw_set_profiling": (ctypes.c_int, [P, I32]),
            "lw_plan_batch": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), ctypes.c_int]),
            "lw_set_tuning": (ctypes.c_int, [P, I32, I32, I32, I32, I32]),
            "lw_tune": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), ctypes.c_int, I32, ctypes.c_char_p,
                                       ctypes.c_char_p, SZ]),
            "lw_graph_capture": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), ctypes.c_int, P, SZ,
                                                ctypes.POINTER(P)]),
            "lw_graph_launch": (ctypes.c_int, [P]),
            "lw_graph_destroy": (None, [P]),
            "lw_accumulate_subset": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), P, I64, P, SZ, P]),
            "lw_subset_offsets": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), P, I64, P, ctypes.POINTER(I64)]),
            "lw_gather_particles": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), P, I64, ctypes.POINTER(lw_batch)]),
            "lw_features": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), P]),
            "lw_surrogate_accumulate": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), P, P, P, ctypes.c_float,
                                                       P, P, P, P, SZ]),
            "lw_surrogate_targets": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), P, D, P]),
            "lw_column_stats": (ctypes.c_int, [P, P, I64, I32, I32, P, I64, D, I32, P, ctypes.c_float, P, P,
                                               SZ]),
            "lw_error_share": (ctypes.c_int, [P, P, P, I64, I32, I32, P, I64, D, P]),
            "lw_quantile_of_maxima": (ctypes.c_int, [P, P, I64, I32, D, ctypes.POINTER(D), P, SZ]),
            "lw_log_ratio": (ctypes.c_int, [P, P, I64, P, I64, I64, P]),
            "lw_mlp_create": (ctypes.c_int, [P, I32, I32, I32, I32, ctypes.c_uint64, ctypes.POINTER(P)]),
            "lw_mlp_destroy": (None, [P]),
            "lw_mlp_num_params": (ctypes.c_int, [P, ctypes.POINTER(I64)]),
            "lw_mlp_get_params": (ctypes.c_int, [P, P, I64, P]),
            "lw_mlp_set_params": (ctypes.c_int, [P, P, I64, P]),
            "lw_mlp_set_input_norm": (ctypes.c_int, [P, P, P]),
            "lw_mlp_set_output_skip": (ctypes.c_int, [P, I32, ctypes.c_float]),
            "lw_mlp_forward": (ctypes.c_int, [P, P, I64, P, P]),
            "lw_mlp_loss_grad": (ctypes.c_int, [P, P, P, I64, P, ctypes.POINTER(D)]),
            "lw_mlp_train_step": (ctypes.c_int, [P, P, P, I64, ctypes.c_float, ctypes.c_float,
                                                 ctypes.POINTER(D)]),
            "lw_mlp_train_head_step": (ctypes.c_int, [P, P, P, I64, ctypes.c_float, ctypes.POINTER(D)]),
            "lw_profile_read": (ctypes.c_int, [P, P]),
            "lw_set_coherent": (ctypes.c_int, [P, I32]),
            "lw_get_basis": (ctypes.c_int, [P, P]),
            "lw_read_amplitudes": (ctypes.c_int, [P, P]),
            "lw_load_amplitudes": (ctypes.c_int, [P, P]),
            "lw_accumulate_amplitudes": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), ctypes.c_int, P, SZ, P]),
            "lw_amplitude_workspace_size": (ctypes.c_int, [P, I64, ctypes.POINTER(SZ)]),
            "lw_spectrum_from_amplitudes": (ctypes.c_int, [P, ctypes.POINTER(lw_batch), P, P, SZ]),
            "lw_spectral_diagnostics": (ctypes.c_int, [P, P, P, P, P, P]),
            "lw_pitch_cones": (ctypes.c_int, [P, I64, P, P, P, P, P, I32, D, P, I32, P, P, P]),
            "lw_profile_cu_busy": (ctypes.c_int, [P, P]),
            "lw_save_accumulator": (ctypes.c_int, [P, ctypes.c_char_p]),
            "lw_load_accumulator_file": (ctypes.c_int, [P, ctypes.c_char_p]),
            "lw_mlp_save": (ctypes.c_int, [P, ctypes.c_char_p]),
            "lw_mlp_load": (ctypes.c_int, [P, ctypes.c_char_p]),
            "lw_accumulate_noalloc": (ctypes.c_int, [P, ctypes.POINTER(lw_batch)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _checked_indices(indices):
    """Index lists go to the device as pointers: a device int64 tensor, made contiguous (a
    copy stays valid for the stream-ordered call: torch reuses its memory only for later work
    on the same stream)."""
    if not isinstance(indices, torch.Tensor) or not indices.is_cuda or indices.dtype != torch.int64:
        raise TypeError("indices must be a device (cuda) int64 tensor")
    return indices.contiguous()


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class DeviceBatch:
    """A particle batch resident in device memory (torch tensors) plus its lw_batch view.

    ``host`` is any object with the numpy arrays offsets, x, y, z, bx, by, bz,
    ax, ay, az (float32), t0, dt, charge, weight and species.
    """

    F64 = ("x", "y", "z", "bx", "by", "bz", "t0", "dt")
    F32 = ("ax", "ay", "az", "charge", "weight")

    def __init__(self, tensors: dict, n_particles: int):
        self.t = tensors
        self.n_particles = int(n_particles)
        self.struct = lw_batch()
        self.struct.n_particles = self.n_particles
        for name, _ in lw_batch._fields_[1:-1]:
            ten = tensors.get(name)
            setattr(self.struct, name, ten.data_ptr() if ten is not None else None)
        # FP64 accelerations (all three, or none) are passed as such with the batch flag
        f64 = [tensors[k].dtype == torch.float64 for k in ("ax", "ay", "az") if k in tensors]
        if any(f64) and not all(f64):
            raise ValueError("ax, ay, az must share one dtype")
        self.struct.flags = LW_BATCH_F64_ACCEL if f64 and all(f64) else 0

    @classmethod
    def from_host(cls, host, device="cuda", with_species=True, f64_accel=False):
        """f64_accel: pass d(beta)/dt as FP64 (LW_BATCH_F64_ACCEL) instead of rounding it to FP32."""
        dev = torch.device(device)
        t = {"offsets": torch.from_numpy(np.ascontiguousarray(host.offsets, dtype=np.int64)).to(dev)}
        for k in cls.F64:
            t[k] = torch.from_numpy(np.ascontiguousarray(getattr(host, k), dtype=np.float64)).to(dev)
        for k in cls.F32:
            dt = np.float64 if (f64_accel and k in ("ax", "ay", "az")) else np.float32
            t[k] = torch.from_numpy(np.ascontiguousarray(getattr(host, k), dtype=dt)).to(dev)
        if with_species:
            t["species"] = torch.from_numpy(np.ascontiguousarray(host.species, dtype=np.int32)).to(dev)
        return cls(t, len(host.offsets) - 1)

    def gather(self, ctx: "Context", indices) -> "DeviceBatch":
        """The particles listed in `indices` (device int64) as a batch of their own, copied by
        lw_subset_offsets and lw_gather_particles (ctx's stream; synchronises once)."""
        idx = _checked_indices(indices)
        n = int(idx.numel())
        dev = self.t["offsets"].device
        offs = torch.empty(n + 1, dtype=torch.int64, device=dev)
        total = ctypes.c_int64()
        ctx._check(ctx.lib.lw_subset_offsets(ctx.h, ctypes.byref(self.struct), ctypes.c_void_p(idx.data_ptr()), n,
                                             ctypes.c_void_p(offs.data_ptr()), ctypes.byref(total)))
        t = {"offsets": offs}
        # at least one element, so that a list of empty particles still has arrays to point at
        for k in ("x", "y", "z", "bx", "by", "bz", "ax", "ay", "az"):
            t[k] = torch.empty(max(total.value, 1), dtype=self.t[k].dtype, device=dev)
        for k in ("t0", "dt", "charge", "weight"):
            t[k] = torch.empty(n, dtype=self.t[k].dtype, device=dev)
        if self.t.get("species") is not None:
            t["species"] = torch.empty(n, dtype=torch.int32, device=dev)
        out = DeviceBatch(t, n)
        ctx._check(ctx.lib.lw_gather_particles(ctx.h, ctypes.byref(self.struct), ctypes.c_void_p(idx.data_ptr()), n,
                                               ctypes.byref(out.struct)))
        return out

    def head(self, n: int) -> "DeviceBatch":
        """The first n particles (a view sharing the arrays)."""
        assert 0 <= n <= self.n_particles
        return DeviceBatch(self.t, n)

    @property
    def n_samples(self) -> int:
        o = self.t["offsets"]
        return int((o[-1] - o[0]).item())


class Context:
    """One lw_ctx: grids, the FP64 accumulator and the device error record."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = load_library()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        st = self.lib.lw_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream))
        if st != LW_OK:
            raise LWError(st, "lw_create failed")
        self.h = h
        self.nd = self.nw = 0
        self.ns = 1
        self.coherent = False
        self.dirs = None
        self._children = weakref.WeakSet()  # networks and graphs, destroyed before the context

    def _check(self, st):
        if st != LW_OK:
            raise LWError(st, self.lib.lw_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            for child in list(getattr(self, "_children", ())):
                child.close()
            self.lib.lw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_directions(self, dirs):
        d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        self._check(self.lib.lw_set_directions(self.h, _np_ptr(d), d.shape[0]))
        self.nd = d.shape[0]
        self.dirs = d.copy()

    def set_frequencies(self, omega):
        w = np.ascontiguousarray(omega, dtype=np.float64)
        self._check(self.lib.lw_set_frequencies(self.h, _np_ptr(w), w.size))
        self.nw = w.size

    def set_log_frequencies(self, wmin, wmax, nw):
        self._check(self.lib.lw_set_log_frequencies(self.h, wmin, wmax, nw))
        self.nw = nw

    def get_frequencies(self):
        out = np.zeros(self.nw, dtype=np.float64)
        self._check(self.lib.lw_get_frequencies(self.h, _np_ptr(out)))
        return out

    def set_species(self, ns):
        self._check(self.lib.lw_set_species(self.h, ns))
        self.ns = ns

    def workspace_size(self, batch: DeviceBatch, path="fp32") -> int:
        n = ctypes.c_size_t()
        self._check(self.lib.lw_workspace_size(self.h, ctypes.byref(batch.struct), PATHS.get(path, path),
                                               ctypes.byref(n)))
        return n.value

    def workspace(self, batch: DeviceBatch, path="fp32"):
        n = self.workspace_size(batch, path)
        return torch.empty(max(n, 256), dtype=torch.uint8, device=f"cuda:{self.device}")

    def accumulate(self, batch: DeviceBatch, path="fp32", workspace=None, per_particle=None):
        if workspace is None:
            workspace = self.workspace(batch, path)
        pp = per_particle.data_ptr() if per_particle is not None else None
        self._check(self.lib.lw_accumulate(self.h, ctypes.byref(batch.struct), PATHS.get(path, path),
                                           ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                           ctypes.c_void_p(pp) if pp else None))
        return workspace

    def accumulate_noalloc(self, batch: DeviceBatch):
        """FP32 path with the library's static scratch for partial sums: no allocation."""
        self._check(self.lib.lw_accumulate_noalloc(self.h, ctypes.byref(batch.struct)))

    def read_spectra(self):
        out = np.zeros((self.ns, self.nd, self.nw), dtype=np.float64)
        self._check(self.lib.lw_read_spectra(self.h, _np_ptr(out)))
        return out

    def read_spectra_status(self):
        """(status, S, message) without raising on LW_ERANGE."""
        out = np.zeros((self.ns, self.nd, self.nw), dtype=np.float64)
        st = self.lib.lw_read_spectra(self.h, _np_ptr(out))
        return st, out, self.lib.lw_last_error(self.h).decode()

    def reset(self):
        self._check(self.lib.lw_reset(self.h))

    def load_accumulator(self, S):
        s = np.ascontiguousarray(S, dtype=np.float64)
        assert s.size == self.ns * self.nd * self.nw
        self._check(self.lib.lw_load_accumulator(self.h, _np_ptr(s)))

    # ---- coherent synthesis and in-situ recording ----
    def set_stream(self, stream):
        """Order later calls on this stream (a torch.cuda.Stream, a raw hipStream_t, or None)."""
        raw = getattr(stream, "cuda_stream", stream)
        self._check(self.lib.lw_set_stream(self.h, ctypes.c_void_p(raw) if raw else None))

    def save_accumulator(self, path):
        self._check(self.lib.lw_save_accumulator(self.h, os.fsencode(path)))

    def load_accumulator_file(self, path):
        self._check(self.lib.lw_load_accumulator_file(self.h, os.fsencode(path)))

    def profile_cu_busy(self) -> dict:
        out = np.zeros(4, dtype=np.float64)
        self._check(self.lib.lw_profile_cu_busy(self.h, _np_ptr(out)))
        return {"cus": int(out[0]), "min_ms": out[1], "mean_ms": out[2], "max_ms": out[3]}

    def set_coherent(self, coherent=True):
        self._check(self.lib.lw_set_coherent(self.h, 1 if coherent else 0))
        self.coherent = bool(coherent)

    def get_basis(self):
        """[nd][3][3]: n, e1, e2 per direction."""
        out = np.zeros((self.nd, 9), dtype=np.float64)
        self._check(self.lib.lw_get_basis(self.h, _np_ptr(out)))
        return out.reshape(self.nd, 3, 3)

    def read_amplitudes(self):
        """Summed amplitudes [ns][nd][nw][4]: (Re, Im) on e1, then on e2 (coherent mode)."""
        out = np.zeros((self.ns, self.nd, self.nw, 4), dtype=np.float64)
        self._check(self.lib.lw_read_amplitudes(self.h, _np_ptr(out)))
        return out

    def load_amplitudes(self, A):
        a = np.ascontiguousarray(A, dtype=np.float64)
        assert a.size == 4 * self.ns * self.nd * self.nw
        self._check(self.lib.lw_load_amplitudes(self.h, _np_ptr(a)))

    def amplitude_state(self, n_particles):
        """A zeroed per-particle amplitude state, device FP64 [n_particles][nd][nw][4]."""
        return torch.zeros((n_particles, self.nd, self.nw, 4), dtype=torch.float64,
                           device=f"cuda:{self.device}")

    def accumulate_amplitudes(self, batch: DeviceBatch, state, path="fp32", workspace=None):
        assert state.dtype == torch.float64 and state.is_contiguous()
        assert state.numel() == batch.n_particles * self.nd * self.nw * 4
        path = PATHS.get(path, path)
        if workspace is None and path != LW_PATH_FP32:
            workspace = self.workspace(batch, path)
        wp = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
        nb = workspace.numel() if workspace is not None else 0
        self._check(self.lib.lw_accumulate_amplitudes(self.h, ctypes.byref(batch.struct), path, wp, nb,
                                                      ctypes.c_void_p(state.data_ptr())))
        return workspace

    def amplitude_workspace_size(self, n_particles) -> int:
        n = ctypes.c_size_t()
        self._check(self.lib.lw_amplitude_workspace_size(self.h, n_particles, ctypes.byref(n)))
        return n.value

    def spectrum_from_amplitudes(self, batch: DeviceBatch, state, workspace=None):
        assert state.dtype == torch.float64 and state.is_contiguous()
        assert state.numel() == batch.n_particles * self.nd * self.nw * 4
        if workspace is None:
            workspace = torch.empty(max(self.amplitude_workspace_size(batch.n_particles), 256),
                                    dtype=torch.uint8, device=f"cuda:{self.device}")
        self._check(self.lib.lw_spectrum_from_amplitudes(self.h, ctypes.byref(batch.struct),
                                                         ctypes.c_void_p(state.data_ptr()),
                                                         ctypes.c_void_p(workspace.data_ptr()),
                                                         workspace.numel()))
        return workspace

    def spectral_diagnostics(self, S=None, weights=None, alpha_range=None, beta_range=None):
        """(average [ns][nw], rows [ns][nd + 1][8]) of S (device FP64 [ns][nd][nw] tensor) or of
        the context's spectrum; each row {k, w_k, omega_peak, S_k, alpha, n_alpha, beta, n_beta}."""
        avg = np.zeros((self.ns, self.nw), dtype=np.float64)
        diag = np.zeros((self.ns, self.nd + 1, 8), dtype=np.float64)
        sp = None
        if S is not None:
            assert S.dtype == torch.float64 and S.is_contiguous() and S.numel() == self.ns * self.nd * self.nw
            sp = ctypes.c_void_p(S.data_ptr())
        wp = None
        if weights is not None:
            wa = np.ascontiguousarray(weights, dtype=np.float64)
            assert wa.size == self.nd
            wp = _np_ptr(wa)
        rp = None
        if alpha_range is not None or beta_range is not None:
            ra = np.array([*(alpha_range or (1e-2, 0.3)), *(beta_range or (3.0, 30.0))], dtype=np.float64)
            rp = _np_ptr(ra)
        self._check(self.lib.lw_spectral_diagnostics(self.h, sp, wp, rp, _np_ptr(avg), _np_ptr(diag)))
        return avg, diag

    def pitch_cones(self, ux, uy, uz, axis, theta_c, dtheta, edges, member=False):
        """(counts [n_cones + 1][n_bins], deviation [n_cones][n_bins], member or None) for device
        FP64 momenta ux, uy, uz (u = gamma beta)."""
        n = int(ux.numel())
        for t in (ux, uy, uz):
            assert t.dtype == torch.float64 and t.is_contiguous() and t.numel() == n
        ax = np.ascontiguousarray(axis, dtype=np.float64)
        th = np.ascontiguousarray(theta_c, dtype=np.float64)
        ed = np.ascontiguousarray(edges, dtype=np.float64)
        counts = np.zeros((th.size + 1, ed.size - 1), dtype=np.int64)
        dev = np.zeros((th.size, ed.size - 1), dtype=np.float64)
        mem = torch.empty(n, dtype=torch.int32, device=ux.device) if member else None
        self._check(self.lib.lw_pitch_cones(self.h, n, ctypes.c_void_p(ux.data_ptr()), ctypes.c_void_p(uy.data_ptr()),
                                            ctypes.c_void_p(uz.data_ptr()), _np_ptr(ax), _np_ptr(th), th.size,
                                            float(dtheta), _np_ptr(ed), ed.size - 1, _np_ptr(counts), _np_ptr(dev),
                                            ctypes.c_void_p(mem.data_ptr()) if member else None))
        return counts, dev, mem

    def set_mfma_options(self, bands=1, products_f16=3, products_bf16=3):
        self._check(self.lib.lw_set_mfma_options(self.h, bands, products_f16, products_bf16))

    def set_mfma_chunk_bytes(self, nbytes=0):
        self._check(self.lib.lw_set_mfma_chunk_bytes(self.h, int(nbytes)))

    def mfma_plan_info(self, batch, path="mfma_f16"):
        """{particles_per_chunk, chunks, bands, workspace_bytes} of the batch (plans it)."""
        out = np.zeros(4, dtype=np.int64)
        self._check(self.lib.lw_mfma_plan_info(self.h, ctypes.byref(batch.struct), PATHS.get(path, path),
                                               _np_ptr(out)))
        return {"particles_per_chunk": int(out[0]), "chunks": int(out[1]), "bands": int(out[2]),
                "workspace_bytes": int(out[3])}

    def set_profiling(self, enable=True):
        self._check(self.lib.lw_set_profiling(self.h, 1 if enable else 0))

    def profile_read(self) -> dict:
        out = np.zeros(7, dtype=np.float64)
        self._check(self.lib.lw_profile_read(self.h, _np_ptr(out)))
        return {"direct_ms": out[0], "spread_ms": out[1], "gemm_ms": out[2], "gemm_flops": out[3],
                "direct_launches": int(out[4]), "gemm_launches": int(out[5]),
                "spread_launches": int(out[6])}

    def plan_batch(self, batch: DeviceBatch, path="fp32"):
        self._check(self.lib.lw_plan_batch(self.h, ctypes.byref(batch.struct), PATHS.get(path, path)))

    def set_tuning(self, wpt=0, pb=0, persistent=1, bands=0, tile=0):
        """tile: 0 keep, 1 = 128 x 128, 2 = 256 x 128, 3 = 128 x 256, 4 = 256 x 256 contraction tiles."""
        self._check(self.lib.lw_set_tuning(self.h, wpt, pb, persistent, bands, tile))

    def tune(self, batch: DeviceBatch, path="fp32", repeats=2, cache_json=None) -> dict:
        import json

        buf = ctypes.create_string_buffer(1 << 16)
        self._check(self.lib.lw_tune(self.h, ctypes.byref(batch.struct), PATHS.get(path, path), repeats,
                                     cache_json.encode() if cache_json else None, buf, len(buf)))
        return json.loads(buf.value.decode())

    def load_tuning(self, cache_json):
        """Apply the choice recorded by tune(..., cache_json=...)."""
        import json

        with open(cache_json) as f:
            best = json.load(f)["best"]
        self.set_tuning(best["wpt"], best["pb"], best["persistent"], best["bands"], best["tile"])

    def graph_capture(self, batch: DeviceBatch, path="fp32", workspace=None) -> "Graph":
        if workspace is None:
            workspace = self.workspace(batch, path)
        g = ctypes.c_void_p()
        self._check(self.lib.lw_graph_capture(self.h, ctypes.byref(batch.struct), PATHS.get(path, path),
                                              ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                              ctypes.byref(g)))
        return Graph(self, g, workspace, batch)

    def accumulate_subset(self, batch: DeviceBatch, indices, workspace=None, per_particle=None):
        """Exact FP32 accumulation of the particles in `indices` (device int64 tensor)."""
        indices = _checked_indices(indices)
        n = int(indices.numel())
        if workspace is None:
            sub = lw_batch()
            ctypes.memmove(ctypes.byref(sub), ctypes.byref(batch.struct), ctypes.sizeof(lw_batch))
            sub.n_particles = n
            sz = ctypes.c_size_t()
            self._check(self.lib.lw_workspace_size(self.h, ctypes.byref(sub), LW_PATH_FP32, ctypes.byref(sz)))
            workspace = torch.empty(max(sz.value, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        pp = ctypes.c_void_p(per_particle.data_ptr()) if per_particle is not None else None
        self._check(self.lib.lw_accumulate_subset(self.h, ctypes.byref(batch.struct),
                                                  ctypes.c_void_p(indices.data_ptr()), n,
                                                  ctypes.c_void_p(workspace.data_ptr()),
                                                  workspace.numel(), pp))
        return workspace

    def surrogate_accumulate(self, batch: DeviceBatch, ylog, err, threshold, compact=False, calib=None):
        """Add 10^(ylog + calib) of unflagged particles to S (calib: device [nd][nw] or None).

        Returns the device flags [n_particles]; with compact=True also the device
        int64 list of flagged particles (increasing) and its device count [1]."""
        P = batch.n_particles
        flags = torch.empty(P, dtype=torch.int32, device=ylog.device)
        need = ((P + 127) // 128) * self.ns * self.nd * self.nw * 8
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=ylog.device)
        ep = ctypes.c_void_p(err.data_ptr()) if err is not None else None
        idx = cnt = None
        if compact:
            idx = torch.empty(max(P, 1), dtype=torch.int64, device=ylog.device)
            cnt = torch.empty(1, dtype=torch.int64, device=ylog.device)
        cp = ctypes.c_void_p(calib.data_ptr()) if calib is not None else None
        self._check(self.lib.lw_surrogate_accumulate(self.h, ctypes.byref(batch.struct),
                                                     ctypes.c_void_p(ylog.data_ptr()), cp, ep,
                                                     float(threshold), ctypes.c_void_p(flags.data_ptr()),
                                                     ctypes.c_void_p(idx.data_ptr()) if compact else None,
                                                     ctypes.c_void_p(cnt.data_ptr()) if compact else None,
                                                     ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        return (flags, idx, cnt) if compact else flags

    def surrogate_targets(self, batch: DeviceBatch, per_particle, floor=1e-30):
        """log10(per-particle spectrum / (w q^2) + floor), device [n_particles][nd][nw]."""
        out = torch.empty_like(per_particle)
        self._check(self.lib.lw_surrogate_targets(self.h, ctypes.byref(batch.struct),
                                                  ctypes.c_void_p(per_particle.data_ptr()), float(floor),
                                                  ctypes.c_void_p(out.data_ptr())))
        return out

    def features(self, batch: DeviceBatch):
        out = torch.empty((batch.n_particles, self.nd, 16), dtype=torch.float32,
                          device=f"cuda:{self.device}")
        self._check(self.lib.lw_features(self.h, ctypes.byref(batch.struct), ctypes.c_void_p(out.data_ptr())))
        return out


    def column_stats(self, x, groups=1, row_add=None, row_add_stride=1, row_add_coeff=0.0, exp10=False,
                     err=None, threshold=0.0):
        """Device double [groups][cols][2]: mean and mean square per group and column of x
        (device float [rows][cols], row r = p groups + g), of x + coeff row_add or of 10 to that,
        over the particles whose largest err (device float [rows]) is <= threshold."""
        rows, cols = int(x.shape[0]), int(x.shape[1])
        P = rows // groups
        slices = max(1, (P + 255) // 256)
        ws = torch.empty(max(slices * groups * cols * 3 * 8, 256), dtype=torch.uint8, device=x.device)
        out = torch.empty((groups, cols, 2), dtype=torch.float64, device=x.device)
        ra = ctypes.c_void_p(row_add.data_ptr()) if row_add is not None else None
        ep = ctypes.c_void_p(err.data_ptr()) if err is not None else None
        self._check(self.lib.lw_column_stats(self.h, ctypes.c_void_p(x.data_ptr()), rows, cols, groups, ra,
                                             row_add_stride, float(row_add_coeff), int(bool(exp10)), ep,
                                             float(threshold), ctypes.c_void_p(out.data_ptr()),
                                             ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        return out

    def error_share(self, pred, y, groups, smean, floor):
        """Device float [rows]: log10 of each row's mean |10^pred - 10^y| / smean[r mod groups]
        plus floor; smean = device double [groups][cols][2] (the means are used)."""
        rows, cols = int(pred.shape[0]), int(pred.shape[1])
        share = torch.empty(rows, dtype=torch.float32, device=pred.device)
        self._check(self.lib.lw_error_share(self.h, ctypes.c_void_p(pred.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                            rows, cols, groups, ctypes.c_void_p(smean.data_ptr()), 2,
                                            float(floor), ctypes.c_void_p(share.data_ptr())))
        return share

    def quantile_of_maxima(self, v, groups, q):
        """q-quantile of the per-particle maxima of v (device float [n][groups])."""
        n = int(v.numel()) // groups
        ws = torch.empty(((4 * n + 255) // 256) * 256 + 1280, dtype=torch.uint8, device=v.device)
        out = ctypes.c_double()
        self._check(self.lib.lw_quantile_of_maxima(self.h, ctypes.c_void_p(v.data_ptr()), n, groups, float(q),
                                                   ctypes.byref(out), ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        return out.value

    def log_ratio(self, num, den, stride=2):
        """Device float [n]: log10(num / den) of the strided device doubles where both are positive."""
        n = int(num.numel()) // stride
        out = torch.empty(n, dtype=torch.float32, device=num.device)
        self._check(self.lib.lw_log_ratio(self.h, ctypes.c_void_p(num.data_ptr()), stride,
                                          ctypes.c_void_p(den.data_ptr()), stride, n,
                                          ctypes.c_void_p(out.data_ptr())))
        return out
    def stats(self) -> int:
        calls = ctypes.c_int64()
        self._check(self.lib.lw_stats(self.h, ctypes.byref(calls)))
        return calls.value


class Graph:
    """A captured lw_accumulate; keeps its workspace and batch alive."""

    def __init__(self, ctx: Context, handle, workspace, batch):
        self.ctx, self.h, self.workspace, self.batch = ctx, handle, workspace, batch
        ctx._children.add(self)

    def launch(self):
        st = self.ctx.lib.lw_graph_launch(self.h)
        if st != LW_OK:
            raise LWError(st, self.ctx.lib.lw_last_error(self.ctx.h).decode())

    def close(self):
        if self.h and self.ctx.h:
            self.ctx.lib.lw_graph_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """lw_mlp: the surrogate network (BF16 matrix-core kernels, FP32 master weights)."""

    def __init__(self, ctx: Context, n_in=16, hidden=256, n_hidden=3, n_out=256, seed=1):
        self.ctx = ctx
        self.shape = (n_in, hidden, n_hidden, n_out)
        h = ctypes.c_void_p()
        ctx._check(ctx.lib.lw_mlp_create(ctx.h, n_in, hidden, n_hidden, n_out, seed, ctypes.byref(h)))
        self.h = h
        ctx._children.add(self)
        n = ctypes.c_int64()
        ctx._check(ctx.lib.lw_mlp_num_params(h, ctypes.byref(n)))
        self.n_params = n.value

    def close(self):
        if getattr(self, "h", None) and self.ctx.h:
            self.ctx.lib.lw_mlp_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _ptr(t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else None

    def get_params(self):
        p = np.zeros(self.n_params, dtype=np.float32)
        head = np.zeros(self.shape[1] + 1, dtype=np.float32)
        self.ctx._check(self.ctx.lib.lw_mlp_get_params(self.h, _np_ptr(p), self.n_params, _np_ptr(head)))
        return p, head

    def set_params(self, params, head=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        hd = np.ascontiguousarray(head, dtype=np.float32) if head is not None else None
        self.ctx._check(self.ctx.lib.lw_mlp_set_params(self.h, _np_ptr(p), self.n_params,
                                                       _np_ptr(hd) if hd is not None else None))

    def set_input_norm(self, shift=None, scale=None):
        if shift is None:
            self.ctx._check(self.ctx.lib.lw_mlp_set_input_norm(self.h, None, None))
            return
        sh = np.ascontiguousarray(shift, dtype=np.float32)
        sc = np.ascontiguousarray(scale, dtype=np.float32)
        assert sh.size == self.shape[0] and sc.size == self.shape[0]
        self.ctx._check(self.ctx.lib.lw_mlp_set_input_norm(self.h, _np_ptr(sh), _np_ptr(sc)))

    def set_output_skip(self, input_index=-1, coeff=0.0):
        self.ctx._check(self.ctx.lib.lw_mlp_set_output_skip(self.h, int(input_index), float(coeff)))

    def forward(self, x, with_error=False):
        rows = x.shape[0]
        y = torch.empty((rows, self.shape[3]), dtype=torch.float32, device=x.device)
        e = torch.empty(rows, dtype=torch.float32, device=x.device) if with_error else None
        self.ctx._check(self.ctx.lib.lw_mlp_forward(self.h, self._ptr(x), rows, self._ptr(y), self._ptr(e)))
        return (y, e) if with_error else y

    def loss_grad(self, x, t):
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = ctypes.c_double()
        self.ctx._check(self.ctx.lib.lw_mlp_loss_grad(self.h, self._ptr(x), self._ptr(t), x.shape[0],
                                                      _np_ptr(g), ctypes.byref(loss)))
        return loss.value, g

    def train_step(self, x, t, lr=1e-3, weight_decay=0.0, want_loss=True):
        loss = ctypes.c_double()
        self.ctx._check(self.ctx.lib.lw_mlp_train_step(self.h, self._ptr(x), self._ptr(t), x.shape[0], lr,
                                                       weight_decay, ctypes.byref(loss)))
        return loss.value

    def save(self, path):
        self.ctx._check(self.ctx.lib.lw_mlp_save(self.h, os.fsencode(path)))

    def load(self, path):
        self.ctx._check(self.ctx.lib.lw_mlp_load(self.h, os.fsencode(path)))

    def train_head_step(self, x, err_target, lr=1e-3):
        loss = ctypes.c_double()
        self.ctx._check(self.ctx.lib.lw_mlp_train_head_step(self.h, self._ptr(x), self._ptr(err_target),
                                                            x.shape[0], lr, ctypes.byref(loss)))
        return loss.value
