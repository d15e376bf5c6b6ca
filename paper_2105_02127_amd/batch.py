"""Many independent meshes advanced together (binding of teno_batch_*).

One SSP-RK3 step of every mesh runs as persistent launches over a shared
work list (see include/teno.h), optionally replayed from a captured HIP
graph.  Graph capture needs a non-default stream, so calls run on a side
stream ordered against the caller's current stream.

`autotune` times the schedule options (one reconstruction launch for all
orders versus one per order, persistent wavefronts per compute unit, work
order) on the actual batch and keeps the fastest, caching the choice in a
JSON file keyed by the batch's (order, cell count) signature.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import itertools
import json
import os

import torch

from . import teno

_vp = C.c_void_p


class Batch:
    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (_vp * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = C.c_void_p()
        teno._check(teno.load().teno_batch_create(arr, len(self.solvers), C.byref(h)))
        self.h = h
        self.side = torch.cuda.Stream(device=self.solvers[0].device)

    def __del__(self):
        if getattr(self, "h", None) and teno._lib is not None:
            teno._lib.teno_batch_destroy(self.h)
            self.h = None

    @property
    def tuning(self) -> dict:
        t = teno.BatchTuning()
        teno._check(teno.load().teno_batch_get_tuning(self.h, C.byref(t)))
        return {k: int(getattr(t, k)) for k, _ in teno.BatchTuning._fields_}

    def set_tuning(self, **kw):
        cur = self.tuning
        cur.update(kw)
        t = teno.BatchTuning(**cur)
        teno._check(teno.load().teno_batch_set_tuning(self.h, C.byref(t)))

    def _ptrs(self, U):
        if len(U) != len(self.solvers):
            raise teno.TenoError("one state per mesh")
        for u, s in zip(U, self.solvers):
            teno._ptr(u, (s.n_cell, 4), torch.float64, "U")
        return (_vp * len(U))(*[u.data_ptr() for u in U])

    def _run(self, fn):
        cur = torch.cuda.current_stream(self.side.device)
        self.side.wait_stream(cur)
        with torch.cuda.stream(self.side):
            fn(C.c_void_p(self.side.cuda_stream))
        cur.wait_stream(self.side)

    def max_dt(self, U, cfl=0.4, dt=None):
        dt = torch.empty(len(U), dtype=torch.float64, device=U[0].device) if dt is None else dt
        ptrs = self._ptrs(U)
        self._run(lambda st: teno._check(teno.load().teno_batch_max_dt(
            self.h, ptrs, float(cfl), C.c_void_p(dt.data_ptr()), st)))
        return dt

    def set_flags(self, flags3):
        """Per-mesh int16 tensors [3, n_cell] that later steps fill with their
        stages' selection flags (uint16 bit patterns); None stops it."""
        if flags3 is None:
            teno._check(teno.load().teno_batch_set_flags(self.h, None))
            self._flags = None
            return
        if len(flags3) != len(self.solvers):
            raise teno.TenoError("one flag tensor per mesh")
        for f, s in zip(flags3, self.solvers):
            teno._ptr(f, (3, s.n_cell), torch.int16, "flags3")
        self._flags = list(flags3)       # keeps the buffers alive
        arr = (_vp * len(flags3))(*[f.data_ptr() for f in flags3])
        teno._check(teno.load().teno_batch_set_flags(self.h, arr))

    @property
    def stats(self) -> dict:
        st = teno.BatchStats()
        teno._check(teno.load().teno_batch_get_stats(self.h, C.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in teno.BatchStats._fields_}

    def rk_step(self, U, dt):
        if dt.dtype != torch.float64 or dt.numel() != len(U) or not dt.is_contiguous():
            raise teno.TenoError("dt must be a contiguous float64 tensor with one entry per mesh")
        ptrs = self._ptrs(U)
        self._run(lambda st: teno._check(teno.load().teno_batch_rk_step(
            self.h, ptrs, C.c_void_p(dt.data_ptr()), st)))

    def signature(self) -> str:
        sig = [(s.order, s.n_cell) for s in self.solvers]
        return hashlib.sha256(json.dumps(sig).encode()).hexdigest()[:16]


CANDIDATES = [dict(order_mode=om, waves_per_cu=w, item_order=io, use_graph=1)
              for om, w, io in itertools.product((0, 1), (0, 4, 8, 16), (0, 1))]


def autotune(batch: Batch, U, dt, steps: int = 3, cache: str | None = None, verbose=False,
             cfl: float | None = 0.4):
    """Times every candidate schedule for `steps` batch steps (on scratch
    copies of U) and applies the fastest; returns (best, timings).  With a
    cfl each timed step is what a simulation loop runs: the per-mesh dt from
    the current states, then the SSP-RK3 step (graph replay)."""
    key = batch.signature()
    if cache and os.path.exists(cache):
        try:
            known = json.load(open(cache))
        except (OSError, ValueError):
            known = {}
        if key in known:
            batch.set_tuning(**known[key])
            return known[key], {}
    work = [u.clone() for u in U]
    timings = {}

    def step():
        if cfl is not None:
            batch.max_dt(work, cfl, dt)
        batch.rk_step(work, dt)

    for cand in CANDIDATES:
        batch.set_tuning(**cand)
        step()                                    # capture + warm-up
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        timings[json.dumps(cand, sort_keys=True)] = ms
        if verbose:
            print(f"[autotune] {cand} {ms:.3f} ms/step", flush=True)
    best = json.loads(min(timings, key=timings.get))
    batch.set_tuning(**best)
    if cache:
        try:
            known = json.load(open(cache)) if os.path.exists(cache) else {}
        except (OSError, ValueError):
            known = {}
        known[key] = best
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as fh:
            json.dump(known, fh, indent=1)
    return best, timings
