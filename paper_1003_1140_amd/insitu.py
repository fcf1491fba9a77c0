"""In-situ recording driver (Section 2.2, recording scheme).

The diagnostic integrates the summed retarded field from the start of recording and
squares it when a spectrum is wanted; the spectrum over a later stretch of time is the
difference of two recorded spectra.  ``Recorder`` drives the C ABI for one run:

* coherent: every window is added into the context's summed species amplitudes
  (``lw_accumulate``); a snapshot is their power;
* incoherent: every window's amplitudes are added into a per-particle state
  (``lw_accumulate_amplitudes``); a snapshot turns the state into a spectrum
  (``lw_spectrum_from_amplitudes``) with each particle in the collection region of its
  latest window.

Every step runs in the library; this class only keeps the buffers and the order of calls.
"""
from __future__ import annotations

import numpy as np

from .lw import Context, DeviceBatch, LWError


class Recorder:
    def __init__(self, ctx: Context, n_particles: int, coherent: bool = False, path: str = "fp32"):
        self.ctx = ctx
        self.n = int(n_particles)
        self.coherent = bool(coherent)
        self.path = path
        ctx.set_coherent(self.coherent)
        self.state = None if self.coherent else ctx.amplitude_state(self.n)
        self._ws = None
        self._ws_state = None
        self._last = None
        self.windows = 0

    def record(self, batch: DeviceBatch):
        """Add one window (the same particles, in the same order, every window)."""
        if batch.n_particles != self.n:
            raise ValueError("a window must hold the recorder's particles")
        if self._ws is None and (self.coherent or self.path != "fp32"):
            self._ws = self.ctx.workspace(batch, self.path)
        if self.coherent:
            self.ctx.accumulate(batch, self.path, workspace=self._ws)
        else:
            self.ctx.accumulate_amplitudes(batch, self.state, self.path, self._ws)
        self._last = batch
        self.windows += 1

    def snapshot(self) -> np.ndarray:
        """P(t) since the start of recording, [species or region][direction][frequency]."""
        if self._last is None:
            return np.zeros((self.ctx.ns, self.ctx.nd, self.ctx.nw))
        if self.coherent:
            return self.ctx.read_spectra()
        # the reset below clears the device error record: report what the windows left first
        st, _, msg = self.ctx.read_spectra_status()
        if st != 0:
            raise LWError(st, msg)
        self.ctx.reset()
        self._ws_state = self.ctx.spectrum_from_amplitudes(self._last, self.state, self._ws_state)
        return self.ctx.read_spectra()

    @staticmethod
    def instantaneous(P1: np.ndarray, P0: np.ndarray) -> np.ndarray:
        """The spectral state between two recordings, P(t1) - P(t0)."""
        return np.asarray(P1) - np.asarray(P0)
