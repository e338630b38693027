"""Host orchestration of the hot path over the C ABI (no arithmetic here).

``Pipeline`` keeps one particle set resident in HBM as AoS records and runs
either the SoA path (bin, convert, density, force, reduce, kick/drift,
writeback) or the plain-AoS path (bin, density, force, kick/drift on the
records) on one HIP stream.
"""
from __future__ import annotations

import numpy as np

from . import sphmi


class Pipeline:
    def __init__(self, aos_np: np.ndarray, n_c: int, prec=None, device="cuda", til=None,
                 prm=None, stream=None, sub_bits: int = 0, sched=None,
                 til_force=None, split=None, tally=False, keep_cells=False, max_cells=1):
        import torch
        self.torch = torch
        self.n = int(aos_np.shape[0])
        self.n_c = int(n_c)
        self.dtype = aos_np.dtype
        self.layout = sphmi.layout_from_dtype(aos_np.dtype)
        raw = np.ascontiguousarray(aos_np).view(np.uint8).reshape(-1)
        self.aos = torch.from_numpy(raw.copy()).to(device)
        self.prec = prec or sphmi.precision()
        self.prm = prm or sphmi.params()
        self.til = til or sphmi.tile()
        self.til_force = til_force or self.til
        self.stream = stream
        # keep_cells: the binning keeps the cell list (and the work lists)
        # while no particle has left its cell or sub-cell since it was built;
        # the kicks count such particles into cells.rebin[0]
        self.cells = sphmi.DeviceCells(self.n, self.n_c, device, sub_bits, tally=tally,
                                       rebin=keep_cells)
        # sched: None (one workgroup per cell) or a work-list schedule, one
        # for both loops or a (density, force) pair; max_cells > 1: the work
        # lists merge up to that many sparse cells along x into one item
        sd, sf = sched if isinstance(sched, (tuple, list)) else (sched, sched)
        self.sched = (sd, sf)
        self.split = dict(split or {})
        self.work = self.work_force = None
        self._lists = []        # (list, occupancy range or None) rebuilt with the cell list
        ti_d = self.til.ti or 64
        ti_f = self.til_force.ti or 64
        # a loop that runs split takes its own lists below; its single-launch
        # list is then built only on demand (smoothing_length)
        if sd:
            self.work = sphmi.DeviceWork(self.n, self.n_c, ti_d, device, sd, max_cells=max_cells)
            if "density" not in self.split:
                self._lists.append((self.work, None))
        if sf:
            if self.work is not None and ti_f == ti_d:
                self.work_force = self.work.with_sched(sf)
                if "force" not in self.split and "density" in self.split:
                    self._lists.append((self.work, None))
            else:
                self.work_force = sphmi.DeviceWork(self.n, self.n_c, ti_f, device, sf,
                                                   max_cells=max_cells)
                if "force" not in self.split:
                    self._lists.append((self.work_force, None))
        # split: per loop ("density" / "force") None or (T, (ti, k), sched)
        # or (T, (ti, k), sched, max_cells): cells with fewer than T
        # particles run as a launch of their own with that tile and schedule
        # (with max_cells > 1, up to that many such cells along x share a
        # work item), the other cells with the loop's own tile and schedule
        self._parts = {}
        shared = {}   # (ti, occupancy range, max_cells) -> list: the two loops may share one

        def part_list(ti, occ, merge, sch):
            key = (ti, occ, merge)
            if key in shared:
                return shared[key].with_sched(sch)
            w = sphmi.DeviceWork(self.n, self.n_c, ti, device, sch, max_cells=merge)
            shared[key] = w
            self._lists.append((w, occ))
            return w

        for loop, main_til, main_sched in (("density", self.til, sd), ("force", self.til_force, sf)):
            sp = self.split.get(loop)
            if not sp:
                continue
            T, (ti, k), small_sched = sp[:3]
            merge = int(sp[3]) if len(sp) > 3 else 1
            big_sched = main_sched or "grid"
            small, big = (0, int(T)), (int(T), 2 ** 31 - 1)
            ws = part_list(ti, small, merge, small_sched)
            wl = part_list(main_til.ti or 64, big, 1, big_sched)
            self._parts[loop] = [(sphmi.tile(ti, k), ws, small), (main_til, wl, big)]
        self.bin_ws = torch.empty(sphmi.bin_workspace_size(self.n, self.n_c), dtype=torch.uint8,
                                  device=device)
        self.soa = sphmi.DeviceSoa(self.n, self.prec, device)
        self.red_ws = torch.empty(sphmi.reduce_workspace_size(self.n), dtype=torch.uint8,
                                  device=device)
        self.red_out = torch.zeros(8, dtype=torch.float64, device=device)
        self.moved = (self.cells.rebin[:1] if keep_cells else
                      torch.zeros(1, dtype=torch.int32, device=device))

    # --- individual stages -------------------------------------------------
    def bin(self):
        sphmi.bin(self.aos, self.layout, self.cells, self.bin_ws, self.stream)
        self.build_lists()

    def build_lists(self):
        """(Re)build every work list the step's loops take from the current
        cell list (each list once, also where both loops share it)."""
        for w, occ in self._lists:
            if occ is None:
                sphmi.worklist(self.cells, w, self.stream)
            else:
                sphmi.worklist(self.cells, w, self.stream, occ)

    def convert(self, view="full"):
        sphmi.convert(self.aos, self.layout, self.cells, view, self.soa, self.stream)

    def smoothing_length(self, eta=sphmi.ETA, tol=1e-4, max_iter=30, write_back=True):
        """Iterate h to the root of h = eta (m / rho(h))^(1/3) for the binned
        and converted particles (H stored in FP32); with write_back the new
        h also goes into the AoS records. Returns (passes, not converged)."""
        if self.work is not None:
            sphmi.worklist(self.cells, self.work, self.stream)
        out = sphmi.smoothing_length(self.soa, self.cells, self.prm, eta, tol, max_iter,
                                     self.til, self.work, None,
                                     self.aos if write_back else None,
                                     self.layout if write_back else None, self.stream)
        self.cells.invalidate()        # h changed; rebuild the lists now
        self.build_lists()             # the passes leave a filtered list behind
        return out

    def density(self):
        if "density" in self._parts:
            for til, w, _ in self._parts["density"]:
                sphmi.density(self.soa, self.cells, self.prm, til, self.stream, w)
            return
        sphmi.density(self.soa, self.cells, self.prm, self.til, self.stream, self.work)

    def force(self):
        if "force" in self._parts:
            for til, w, _ in self._parts["force"]:
                sphmi.force(self.soa, self.cells, self.prm, til, self.stream, w)
            return
        sphmi.force(self.soa, self.cells, self.prm, self.til_force, self.stream, self.work_force)

    def reduce(self):
        sphmi.reduce(self.soa, self.cells, self.red_out, self.red_ws, self.stream)

    def kick_drift(self, dt_kick, dt_drift):
        sphmi.kick_drift(self.soa, self.cells, dt_kick, dt_drift, self.moved, self.stream)

    def writeback(self, view="full"):
        sphmi.writeback(self.soa, self.cells, view, self.aos, self.layout, self.stream)

    def reduce_aos(self):
        sphmi.reduce_aos(self.aos, self.layout, self.cells, self.red_out, self.red_ws, self.stream)

    def density_aos(self):
        for til, w, _ in self._parts.get("density", [(self.til, self.work, None)]):
            sphmi.density_aos(self.aos, self.layout, self.cells, self.prm, til, self.stream, w)

    def force_aos(self):
        for til, w, _ in self._parts.get("force", [(self.til_force, self.work_force, None)]):
            sphmi.force_aos(self.aos, self.layout, self.cells, self.prm, til, self.stream, w)

    def kick_drift_aos(self, dt_kick, dt_drift):
        sphmi.kick_drift_aos(self.aos, self.layout, self.cells, dt_kick, dt_drift, self.moved,
                             self.stream)

    # --- whole steps ----------------------------------------------------------
    def soa_step(self, dt_kick=1e-4, dt_drift=1e-4):
        """bin -> convert(full) -> density -> force -> reduce -> kick/drift -> writeback"""
        self.bin()
        self.convert("full")
        self.density()
        self.force()
        self.reduce()
        self.kick_drift(dt_kick, dt_drift)
        self.writeback("full")

    def aos_step(self, dt_kick=1e-4, dt_drift=1e-4):
        """bin -> density (AoS) -> force (AoS) -> reduce (AoS) -> kick/drift (AoS)"""
        self.bin()
        self.density_aos()
        self.force_aos()
        self.reduce_aos()
        self.kick_drift_aos(dt_kick, dt_drift)

    def kdk_run(self, steps, dt=None, c_cfl=sphmi.C_CFL, dt_max=float("inf")):
        """Leapfrog kick-drift-kick over `steps` steps with h held fixed
        (the sequence of sph_predict / sph_step_totals in the header). dt:
        fixed step size, or None for the Courant step from the last forces
        (capped at dt_max). Returns the history: per step the step size and
        the totals before it, then the totals after the run (dt None)."""
        torch = self.torch
        tot = torch.zeros(8, dtype=torch.float64, device=self.aos.device)

        def totals():
            sphmi.step_totals(self.soa, self.cells, tot, self.red_ws, self.prm, c_cfl,
                              self.stream)
            t = tot.cpu().numpy()
            return {"p": t[0:3].copy(), "ekin": float(t[3]), "eth": float(t[4]),
                    "mass": float(t[5]), "dt_cfl": float(t[6]), "n_vsig": int(t[7])}

        self.bin()
        self.convert("full")
        self.density()
        self.force()
        self.writeback("full")
        hist = []
        for _ in range(steps):
            t = totals()
            step = dt if dt is not None else min(t["dt_cfl"], dt_max)
            hist.append(dict(t, dt=step))
            self.kick_drift(0.5 * step, step)
            self.writeback("kick")
            self.bin()
            self.convert("full")
            sphmi.predict(self.soa, self.cells, self.aos, self.layout, 0.5 * step, self.stream)
            self.density()
            self.force()
            self.kick_drift(0.5 * step, 0.0)
            self.writeback("full")
        hist.append(dict(totals(), dt=None))
        return hist

    # --- readback ---------------------------------------------------------------
    def records(self) -> np.ndarray:
        self.torch.cuda.synchronize()
        return self.aos.cpu().numpy().view(self.dtype).copy()

    def slot(self, name) -> np.ndarray:
        """SoA array in input order (slot k -> particle perm[k])."""
        self.torch.cuda.synchronize()
        t = self.soa[name]
        if t.dtype in (self.torch.float16, self.torch.bfloat16):
            t = t.float()
        vals = t.cpu().numpy()
        perm = self.cells.perm[: self.n].cpu().numpy()
        out = np.empty_like(vals)
        out[perm] = vals
        return out

    def status(self) -> int:
        self.torch.cuda.synchronize()
        return int(self.cells.status.item())


def settle_h(rec: np.ndarray, tol=1e-4, max_iter=30, room=1.6, prm=None, stream=None):
    """Smoothing lengths from the density iteration on the GPU
    (sph_smoothing_length) for AoS records whose h is the start value: the
    records are binned in a cell list `room` times roomier than the largest
    start support radius (so h can grow), iterated, and read back. Returns
    (records with the new h, the cells per axis of the new h, i.e.
    floor(1 / max H), and a dict with the pass count, the particles not
    converged and the start cell count)."""
    import torch
    prm = prm or sphmi.params()
    gk = prm.gamma_k
    n_c0 = int(np.floor(1.0 / (room * gk * float(rec["h"].max()))))
    p0 = Pipeline(rec, n_c0, sched="grid", til=sphmi.tile(32, 2), sub_bits=2, prm=prm,
                  stream=stream)
    p0.bin()
    p0.convert("full")
    passes, left = p0.smoothing_length(tol=tol, max_iter=max_iter)
    out = p0.records()
    del p0
    torch.cuda.empty_cache()
    n_c = int(np.floor(1.0 / (gk * float(out["h"].max()))))
    return out, n_c, {"passes": passes, "not_converged": left, "n_c_during": n_c0}
