"""One two-star system whose state lives in PyTorch device tensors, driven through libnbody."""

from __future__ import annotations

import numpy as np

from . import (
    LAWS,
    MODES,
    NB_FP64,
    NbBuffers,
    NbParams,
    nb_create,
    nb_destroy,
    nb_diagnostics,
    nb_forces,
    nb_l1_log,
    nb_resort,
    nb_retention,
    nb_scratch_bytes,
    nb_step,
)


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("a ROCm GPU is required (torch.cuda.is_available() is False)")
    return torch


class System:
    """Device-resident system. ``pos``/``vel`` are (n, 3) host arrays; star 1 is rows [0, n1)."""

    def __init__(self, pos, vel, n1, *, G, m, dt, D1, D2, q, a=1.0, R2_0=0.2, growth_rate=1e-4,
                 growth_on=True, mode="kahan", device=None, stream=None, law="contact",
                 eps=0.0, gamma=0.0, beta=1.0):
        torch = _torch()
        self.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        dtype = torch.float64 if self.mode == NB_FP64 else torch.float32
        self.device = torch.device(device if device is not None else "cuda")
        pos = np.asarray(pos)
        vel = np.asarray(vel)
        n = int(pos.shape[0])
        self.n, self.n1 = n, int(n1)
        self.law = LAWS[law] if isinstance(law, str) else int(law)
        self.params = NbParams(n=n, n1=int(n1), G=G, m=m, dt=dt, D1=D1, D2=D2, q=q, a=a,
                               R2_0=R2_0, growth_rate=growth_rate, growth_on=int(bool(growth_on)),
                               mode=self.mode, law=self.law, pad=0, eps=eps, gamma=gamma,
                               beta=beta)
        nbytes = nb_scratch_bytes(self.params)
        k = dict(dtype=dtype, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)

        def col(a, c):
            return torch.from_numpy(np.ascontiguousarray(a[:, c])).to(**k) if n else \
                torch.zeros(1, **k)

        # every upload and allocation is ordered on the system's stream
        with torch.cuda.stream(self.stream):
            self.x, self.y, self.z = col(pos, 0), col(pos, 1), col(pos, 2)
            self.vx, self.vy, self.vz = col(vel, 0), col(vel, 1), col(vel, 2)
            self.ax, self.ay, self.az = (torch.zeros(max(n, 1), **k) for _ in range(3))
            self.side = torch.zeros(max(n, 1), dtype=torch.int8, device=self.device)
            # 256-byte alignment: over-allocate and offset
            self._scratch = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._scratch.data_ptr()
        off = (-base) % 256
        self.buffers = NbBuffers(
            x=self.x.data_ptr(), y=self.y.data_ptr(), z=self.z.data_ptr(),
            vx=self.vx.data_ptr(), vy=self.vy.data_ptr(), vz=self.vz.data_ptr(),
            ax=self.ax.data_ptr(), ay=self.ay.data_ptr(), az=self.az.data_ptr(),
            side=self.side.data_ptr(), scratch=base + off, scratch_bytes=nbytes)
        self.handle = nb_create(self.params, self.buffers, self.stream)

    @classmethod
    def from_ic(cls, ic, *, dt=1e-4, mode="kahan", growth_on=True, growth_rate=1e-4, **kw):
        """From a ``synth.BinaryIC``: positions and velocities rounded once to the mode's type."""
        mode_id = MODES[mode] if isinstance(mode, str) else int(mode)
        if mode_id == NB_FP64:
            pos, vel = ic.f32_as_f64()
        else:
            pos, vel = ic.f32()
        return cls(pos, vel, ic.n1, G=ic.G, m=ic.m, dt=dt, D1=ic.D1, D2=ic.D2, q=ic.q, a=ic.a,
                   R2_0=ic.R2, growth_rate=growth_rate, growth_on=growth_on, mode=mode, **kw)

    # ------------------------------------------------------------ operations

    def forces(self):
        nb_forces(self.handle, self.stream)

    def step(self, n_steps: int = 1):
        nb_step([self.handle], n_steps, self.stream)

    def resort(self):
        """Rebuilds the force kernels' sorted order from the current positions."""
        nb_resort(self.handle, self.stream)

    def diagnostics(self, with_pe: bool = False) -> dict:
        return nb_diagnostics(self.handle, with_pe, self.stream)

    def l1_log(self, max_steps: int = 4096) -> np.ndarray:
        return nb_l1_log(self.handle, max_steps, self.stream)

    def retention(self) -> tuple:
        """(n_past, n_bound) of the current state (see nb_retention)."""
        return nb_retention(self.handle, self.stream)

    def synchronize(self):
        self.stream.synchronize()

    def tensors(self):
        return (self.x, self.y, self.z, self.vx, self.vy, self.vz, self.ax, self.ay, self.az,
                self.side, self._scratch)

    def use_on(self, stream):
        """Marks the device tensors as used on another stream (for PyTorch's allocator)."""
        for t in self.tensors():
            t.record_stream(stream)

    # ------------------------------------------------------------ state read-back
    # Read-backs wait for the system's own stream; work queued for it on another stream (for
    # example a batch stepped on a server's compute stream) must be waited for by the caller.

    def _stack(self, a, b, c) -> np.ndarray:
        self.synchronize()
        return np.stack([t[: self.n].cpu().numpy() for t in (a, b, c)], axis=1)

    def positions(self) -> np.ndarray:
        return self._stack(self.x, self.y, self.z)

    def velocities(self) -> np.ndarray:
        return self._stack(self.vx, self.vy, self.vz)

    def accelerations(self) -> np.ndarray:
        return self._stack(self.ax, self.ay, self.az)

    def sides(self) -> np.ndarray:
        self.synchronize()
        return self.side[: self.n].cpu().numpy()

    def close(self):
        """Destroys the library handle and releases the device tensors (the memory returns to
        PyTorch's allocator at once, whatever other references to this object remain)."""
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.synchronize()
            nb_destroy(self.handle)
            self.handle = None
            for name in ("x", "y", "z", "vx", "vy", "vz", "ax", "ay", "az", "side", "_scratch"):
                setattr(self, name, None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_many(systems, n_steps: int = 1, stream=None):
    """Advances several systems together: one launch per kernel over all systems' work."""
    if not systems:
        return
    st = stream if stream is not None else systems[0].stream
    nb_step([s.handle for s in systems], n_steps, st)
