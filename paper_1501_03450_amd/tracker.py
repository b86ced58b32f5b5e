"""A small convenience wrapper over the C ABI that keeps the particle state in
torch-owned device tensors.  All tracking work runs in the HIP library."""

from __future__ import annotations

import numpy as np

from . import binding as B


class SpinTracker:
    """Owns one library context, a lattice and a bunch resident on the GPU."""

    def __init__(self, elements, beam, device: int = 0, precision: str = "fp64",
                 report_every: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("SpinTracker needs a ROCm GPU (there is no CPU fallback)")
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.ctx = B.st_create(device)
        self.beam = beam
        self.precision = precision
        self.report_every = report_every
        B.st_load_lattice(self.ctx, elements, beam.G, beam.gamma0, beam.aperture,
                          precision, report_every)
        self.n = 0
        self.q = None

    # -- state -------------------------------------------------------------
    def set_particles(self, z, spin, alive=None):
        t = self.torch
        z = t.as_tensor(np.asarray(z) if not t.is_tensor(z) else z, dtype=t.float64)
        spin = t.as_tensor(np.asarray(spin) if not t.is_tensor(spin) else spin, dtype=t.float64)
        n = z.shape[1]
        if alive is None:
            alive = t.ones(n, dtype=t.int32)
        alive = t.as_tensor(np.asarray(alive) if not t.is_tensor(alive) else alive, dtype=t.int32)
        if z.shape != (6, n) or spin.shape != (3, n) or alive.shape != (n,):
            raise ValueError("expected z[6][n], spin[3][n], alive[n]")
        self.z = z.to(self.device).contiguous()
        self.spin = spin.to(self.device).contiguous()
        self.alive = alive.to(self.device).contiguous()
        self.n = n
        self.q = None
        B.st_bind_particles(self.ctx, n, self.z.data_ptr(), self.spin.data_ptr(), self.alive.data_ptr())

    def bind_tensors(self, z, spin, alive):
        """Bind caller-owned contiguous device tensors without copying."""
        n = z.shape[1]
        self.z, self.spin, self.alive, self.n, self.q = z, spin, alive, n, None
        B.st_bind_particles(self.ctx, n, z.data_ptr(), spin.data_ptr(), alive.data_ptr())

    def enable_quaternions(self):
        t = self.torch
        self.q = t.zeros((4, self.n), dtype=t.float64, device=self.device)
        B.st_bind_quaternions(self.ctx, self.q.data_ptr() if self.n else None)
        return self.q

    # -- work --------------------------------------------------------------
    def _stream(self, stream):
        if stream is None:
            stream = self.torch.cuda.current_stream(self.device)
        return stream.cuda_stream

    def track(self, turns: int, stream=None):
        B.st_track(self.ctx, turns, self._stream(stream))

    def polarization(self, stream=None):
        n = B.st_polarization(self.ctx)
        out = self.torch.zeros((max(n, 1), 4), dtype=self.torch.float64, device=self.device)
        if n:
            B.st_polarization(self.ctx, out.data_ptr(), n, self._stream(stream))
        return out[:n]

    def read(self, stream=None):
        z = np.empty((6, self.n))
        spin = np.empty((3, self.n))
        alive = np.empty(self.n, dtype=np.int32)
        B.st_read_particles(self.ctx, z.ctypes.data, spin.ctypes.data, alive.ctypes.data,
                            self._stream(stream))
        return z, spin, alive

    def close(self):
        if self.ctx is not None:
            B.st_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
