"""Serving loop client: cell-pair tasks over particle state resident in HBM.

The server itself (batching, admission, streams, completion) is native code
behind the C ABI (sph_server_*); this module marshals requests and
completion records as numpy structured arrays and builds synthetic task
streams: (kind, ci, cj, i range) tasks whose i and j sides hold 16..512
particles, with Poisson arrivals.
"""
import ctypes as C

import numpy as np

from . import sphmi

REQUEST = np.dtype([("kind", "<i4"), ("ci", "<i4"), ("cj", "<i4"), ("i_begin", "<i4"),
                    ("i_end", "<i4"), ("reserved", "<i4"), ("arrival_ns", "<i8"),
                    ("out", "<u8")])
DONE = np.dtype([("id", "<i8"), ("arrival_ns", "<i8"), ("admit_ns", "<i8"),
                 ("launch_ns", "<i8"), ("done_ns", "<i8"), ("batch", "<i4"),
                 ("batch_tasks", "<i4")])
RESULT = np.dtype([("v", "<f4", (5,)), ("count", "<i4"), ("pad", "<i4", (2,))])
TASK_MAX_I = 1024
assert REQUEST.itemsize == 40 and DONE.itemsize == 48 and RESULT.itemsize == 32


def now_ns() -> int:
    return int(sphmi.lib().sph_now_ns())


class Server:
    """A running server over the resident state of a Pipeline (binned,
    converted, density computed for force tasks). The pipeline must stay
    unchanged while the server runs."""

    def __init__(self, pipe, tile=None, streams=4, max_batch=256, pool_bytes=64 << 20):
        import torch
        self.pipe = pipe
        self.cfg = sphmi.ServerConfig(tile or sphmi.Tile(0, 0), int(streams), int(max_batch),
                                      int(pool_bytes))
        L = sphmi.lib()
        nbytes = C.c_size_t()
        sphmi._check(L.sph_server_workspace_size(C.byref(self.cfg), C.byref(nbytes)))
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=pipe.aos.device)
        self.h = C.c_void_p()
        sphmi._check(L.sph_server_create(C.byref(self.cfg), C.byref(pipe.soa.struct),
                                         C.byref(pipe.soa.prec), C.byref(pipe.cells.struct),
                                         C.byref(pipe.prm), C.c_void_p(self.ws.data_ptr()),
                                         nbytes.value, C.byref(self.h)))

    def submit(self, req: np.ndarray) -> int:
        req = np.ascontiguousarray(req, dtype=REQUEST)
        first = C.c_int64()
        sphmi._check(sphmi.lib().sph_server_submit(self.h, C.c_void_p(req.ctypes.data), len(req),
                                                   C.byref(first)))
        return first.value

    def poll(self, max_records=1 << 16, wait_ms=0) -> np.ndarray:
        out = np.empty(max_records, DONE)
        n = C.c_int32()
        sphmi._check(sphmi.lib().sph_server_poll(self.h, C.c_void_p(out.ctypes.data), max_records,
                                                 C.byref(n), int(wait_ms)))
        return out[: n.value]

    def drain(self, timeout_ms=60000):
        sphmi._check(sphmi.lib().sph_server_drain(self.h, int(timeout_ms)))

    def stats(self) -> dict:
        s = sphmi.ServerStats()
        sphmi._check(sphmi.lib().sph_server_get_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in sphmi.ServerStats._fields_ if k != "reserved"}

    def close(self):
        if self.h:
            sphmi._check(sphmi.lib().sph_server_destroy(self.h))
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def run(self, req: np.ndarray, timeout_ms=30000) -> np.ndarray:
        """Submit all requests, wait until they are done, return their
        completion records ordered by request."""
        first = self.submit(req)
        recs = []
        got = 0
        while got < len(req):
            r = self.poll(wait_ms=min(timeout_ms, 1000))
            recs.append(r)
            got += len(r)
            if len(r) == 0 and now_ns() > int(req["arrival_ns"].max()) + timeout_ms * 1_000_000:
                raise TimeoutError("serving run did not finish")
        done = np.concatenate(recs) if recs else np.empty(0, DONE)
        return done[np.argsort(done["id"] - first)]


def make_tasks(cell_start: np.ndarray, n_c: int, count: int, seed: int, lo=16, hi=512,
               density_fraction=0.5) -> np.ndarray:
    """`count` tasks (kind, ci, cj, i_begin, i_end): i ranges are the cells
    with at least `lo` particles, those above `hi` split into ranges of at
    most `hi`; cj is drawn from the 27 cells around ci that hold at least
    `lo` particles (ci itself included); kind 0 (density) with probability
    density_fraction, else 1 (force)."""
    rng = np.random.default_rng(seed)
    start = np.asarray(cell_start, np.int64)
    occ = np.diff(start)
    ok = np.nonzero(occ >= lo)[0]
    if ok.size == 0:
        raise ValueError("no cell holds enough particles for a task")
    ranges = []
    for c in ok:
        a, b = int(start[c]), int(start[c + 1])
        k = -(-(b - a) // hi)
        edges = np.linspace(a, b, k + 1).round().astype(np.int64)
        ranges += [(c, edges[t], edges[t + 1]) for t in range(k)]
    ranges = np.array(ranges, np.int64)
    pick = ranges[rng.integers(0, len(ranges), count)]
    ci = pick[:, 0]
    cx, cy, cz = ci % n_c, (ci // n_c) % n_c, ci // (n_c * n_c)
    out = np.empty((count, 5), np.int32)
    d = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    for t in range(count):
        nb = (((cx[t] + d[:, 0]) % n_c) + n_c * (((cy[t] + d[:, 1]) % n_c) +
                                                 n_c * ((cz[t] + d[:, 2]) % n_c)))
        nb = nb[occ[nb] >= lo]
        out[t, 2] = nb[rng.integers(0, len(nb))]
    out[:, 0] = (rng.random(count) >= density_fraction).astype(np.int32)
    out[:, 1] = ci
    out[:, 3] = pick[:, 1]
    out[:, 4] = pick[:, 2]
    return out


def poisson_arrivals(count: int, rate: float, t0_ns: int, seed: int) -> np.ndarray:
    """Arrival times (ns) of a Poisson process of `rate` per second from t0."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    return t0_ns + np.round(np.cumsum(gaps) * 1e9).astype(np.int64)


def requests(tasks: np.ndarray, arrivals, out_ptr: int = 0):
    """Request records; with out_ptr (host address of a buffer of
    sum(i_end - i_begin) RESULT records) each task's records go to
    consecutive places in it. Returns (requests, record offset of each)."""
    n = len(tasks)
    req = np.zeros(n, REQUEST)
    for k, name in enumerate(("kind", "ci", "cj", "i_begin", "i_end")):
        req[name] = tasks[:, k]
    req["arrival_ns"] = arrivals
    sizes = (tasks[:, 4] - tasks[:, 3]).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]) if n else np.zeros(0, np.int64)
    if out_ptr:
        req["out"] = out_ptr + offs * RESULT.itemsize
    return req, offs
