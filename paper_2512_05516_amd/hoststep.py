"""Whole time steps with the particle records in host memory (Sec. 6, the
pipeline comparison): the records live in pinned host memory and every
step pays its host<->device traffic.

* AoS baseline: the records go to the device once, the plain AoS kernels run
  on them (bin, density, force, kick/drift), the records come back.
* In-place: the records go to the device once, are converted to SoA there,
  all kernels run, the SoA is written back into the records on the device,
  the records come back.
* Streaming: the host builds the cell list; for every kernel the host gathers
  just that kernel's inputs (narrowed and quantised), ships them, runs the
  kernel and scatters its outputs back into the host records.

Every step is a sequence of C-ABI calls; this module only sequences them.
"""
import numpy as np

from . import sphmi
from .pipeline import Pipeline


def pinned_records(rec: np.ndarray):
    """A copy of the records in pinned host memory: (uint8 tensor, numpy
    structured view of the same memory)."""
    import torch
    t = torch.empty(rec.nbytes, dtype=torch.uint8, pin_memory=True)
    view = t.numpy().view(rec.dtype)
    view[:] = rec
    return t, view


class HostStep:
    """Steps over host records `host_t` (a pinned uint8 tensor, see
    pinned_records) with n_c cells per axis. `prec` is the SoA storage of
    the in-place and streaming arrangements; `til` / `sched` the pair-kernel
    tiling (sub-cell order is not used: the host cell list has none)."""

    def __init__(self, host_t, dtype, n_c, prec=None, til=None, sched=None, prm=None,
                 nthreads=0, device="cuda", til_force=None, split=None):
        import torch
        self.torch = torch
        self.host_t = host_t
        self.rec = host_t.numpy().view(dtype)
        self.n = int(self.rec.shape[0])
        self.n_c = int(n_c)
        self.nthreads = int(nthreads)
        # device side: the same buffers the resident pipeline uses
        self.pipe = Pipeline(self.rec, n_c, prec=prec, device=device, til=til, prm=prm,
                             sched=sched, til_force=til_force, split=split)
        self.layout = self.pipe.layout
        n, C = self.n, self.n_c ** 3
        pin = dict(pin_memory=True)
        self._start = torch.empty(C + 1, dtype=torch.int32, **pin)
        self._perm = torch.empty(max(n, 1), dtype=torch.int32, **pin)
        self._cell = torch.empty(max(n, 1), dtype=torch.int32, **pin)
        self._hmax = torch.empty(C, dtype=torch.float32, **pin)
        prec = self.pipe.prec
        st = max(sphmi.host_staging_size(n, n_c, v, prec) for v in ("density", "force_in", "kick_in"))
        wb = max(sphmi.writeback_host_size(n, v) for v in ("density", "force", "kick"))
        self.staging = torch.empty(st, dtype=torch.uint8, **pin)
        self.wb_staging = torch.empty(wb, dtype=torch.uint8, **pin)

    # --- arrangements -----------------------------------------------------------
    def aos_step(self, dt_kick=1e-4, dt_drift=1e-4):
        p = self.pipe
        p.aos.copy_(self.host_t, non_blocking=True)
        p.bin()
        p.density_aos()
        p.force_aos()
        p.kick_drift_aos(dt_kick, dt_drift)
        self.host_t.copy_(p.aos, non_blocking=True)
        self.torch.cuda.synchronize()

    def inplace_step(self, dt_kick=1e-4, dt_drift=1e-4):
        p = self.pipe
        p.aos.copy_(self.host_t, non_blocking=True)
        p.bin()
        p.convert("full")
        p.density()
        p.force()
        p.kick_drift(dt_kick, dt_drift)
        p.writeback("full")
        self.host_t.copy_(p.aos, non_blocking=True)
        self.torch.cuda.synchronize()

    def streaming_step(self, dt_kick=1e-4, dt_drift=1e-4):
        p, n = self.pipe, self.n
        start, perm = self._start.numpy(), self._perm.numpy()[:n]
        cell, hmax = self._cell.numpy()[:n], self._hmax.numpy()
        sphmi.bin_host(self.rec, self.layout, self.n_c, self.nthreads,
                       out=(start, perm, cell, hmax))
        c = p.cells
        c.cell_start.copy_(self._start, non_blocking=True)
        c.perm.copy_(self._perm, non_blocking=True)
        c.cell.copy_(self._cell, non_blocking=True)
        c.hmax.copy_(self._hmax, non_blocking=True)
        p.build_lists()
        args = (self.layout, self.n_c, perm, cell)
        sphmi.gather_host(self.rec, *args, "density", p.soa, self.staging, self.nthreads, p.stream)
        p.density()
        sphmi.writeback_host(p.soa, perm, "density", self.rec, self.layout, self.wb_staging,
                             self.nthreads, p.stream)
        sphmi.gather_host(self.rec, *args, "force_in", p.soa, self.staging, self.nthreads, p.stream)
        p.force()
        sphmi.writeback_host(p.soa, perm, "force", self.rec, self.layout, self.wb_staging,
                             self.nthreads, p.stream)
        sphmi.gather_host(self.rec, *args, "kick_in", p.soa, self.staging, self.nthreads, p.stream)
        p.kick_drift(dt_kick, dt_drift)
        sphmi.writeback_host(p.soa, perm, "kick", self.rec, self.layout, self.wb_staging,
                             self.nthreads, p.stream)

    def step(self, kind, dt_kick=1e-4, dt_drift=1e-4):
        {"aos": self.aos_step, "inplace": self.inplace_step,
         "streaming": self.streaming_step}[kind](dt_kick, dt_drift)

    # --- host<->device bytes of one step ----------------------------------------
    def pcie_bytes(self, kind) -> dict:
        n, C = self.n, self.n_c ** 3
        stride = self.rec.dtype.itemsize
        if kind in ("aos", "inplace"):
            return {"h2d": n * stride, "d2h": n * stride}
        prec = self.pipe.prec
        esz = {sphmi.F32: 4, sphmi.F16: 2, sphmi.BF16: 2}
        pos, vel, mhu = esz[prec.pos], esz[prec.vel], esz[prec.mhu]
        cells = 4 * (C + 1) + 8 * n + 4 * C
        h2d = cells + n * (3 * pos + 3 * mhu)                        # density view
        h2d += n * (3 * pos + 3 * vel + 2 * mhu + 16)                # force view + rho f P c
        h2d += n * (24 + 12 + 4 + 16)                                # kick view + a du
        d2h = n * 28 + n * 24 + n * 40
        return {"h2d": h2d, "d2h": d2h}
