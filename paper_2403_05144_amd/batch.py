"""Many independent P-ERK runs advanced together (one stage-tick launch for all of them).

PerkBatch groups PerkSolver runs (2D Euler, degree 2 or 3).  Each run keeps its own mesh,
coefficient family, partition, dt and number of steps; tick t applies stage t mod S of every
unfinished run.  The tile shape (elements per tile, persistent grid size) is chosen by
`autotune`, which times candidate shapes on the batch itself and restores the states.
All arithmetic runs in libperk's batched stage kernel; this module marshals arguments.
"""
from __future__ import annotations

import ctypes
import json
import os
import time

import numpy as np
import torch

from . import _lib as L
from .solver import PerkError, _stream_handle

TILE_CANDIDATES = tuple((m, g) for m in (1, 2, 4) for g in (0, 256, 512, 1024, 2048))


class PerkBatch:
    def __init__(self, solvers):
        self.lib = L.lib()
        self.solvers = list(solvers)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s._ctx.value for s in self.solvers])
        self._b = ctypes.c_void_p()
        st = self.lib.pe_batch_create(ctypes.byref(self._b), arr, len(self.solvers))
        if st != L.PE_OK:
            raise PerkError(f"pe_batch_create: {L.STATUS.get(st, st)}: {self.lib.pe_batch_last_error(None).decode()}")
        self.tiling = (1, 0)
        self.dt = None
        self.n_steps = None

    def _check(self, st, what):
        if st != L.PE_OK:
            raise PerkError(f"{what}: {L.STATUS.get(st, st)}: {self.lib.pe_batch_last_error(self._b).decode()}")

    def __del__(self):
        try:
            if self._b:
                self.lib.pe_batch_destroy(self._b)
                self._b = ctypes.c_void_p()
        except Exception:
            pass

    def set_steps(self, dt, n_steps):
        self.dt = np.ascontiguousarray(np.asarray(dt, dtype=np.float64))
        self.n_steps = np.ascontiguousarray(np.asarray(n_steps, dtype=np.int64))
        if self.dt.shape != (len(self.solvers),) or self.n_steps.shape != (len(self.solvers),):
            raise PerkError("set_steps: one dt and one step count per run")
        self._check(self.lib.pe_batch_set_steps(self._b, self.dt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                self.n_steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
                    "pe_batch_set_steps")

    def set_tiling(self, elems_per_tile_p3, grid_blocks):
        self._check(self.lib.pe_batch_set_tiling(self._b, int(elems_per_tile_p3), int(grid_blocks)),
                    "pe_batch_set_tiling")
        self.tiling = (int(elems_per_tile_p3), int(grid_blocks))

    def info(self):
        nt, es = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.pe_batch_info(self._b, ctypes.byref(nt), ctypes.byref(es)), "pe_batch_info")
        return nt.value, es.value

    @property
    def n_ticks(self):
        return self.info()[0]

    def run(self, tick_begin=0, tick_end=None, stream=None):
        if tick_end is None:
            tick_end = self.n_ticks
        self._check(self.lib.pe_batch_run(self._b, int(tick_begin), int(tick_end), _stream_handle(stream)),
                    "pe_batch_run")

    def autotune(self, candidates=TILE_CANDIDATES, ticks=None, reps=2, cache=None):
        """Time every (elements per tile, grid) candidate on the first `ticks` ticks (default:
        one step of the longest stage count, at least 16) and keep the fastest.  The states
        and evaluation counters of the runs are restored afterwards.  With `cache` (a JSON
        path) a result stored for the same batch signature is reused."""
        key = self.signature()
        if cache and os.path.exists(cache):
            with open(cache) as f:
                stored = json.load(f)
            if key in stored:
                self.set_tiling(*stored[key]["tiling"])
                return stored[key]
        n_ticks = self.n_ticks
        if ticks is None:
            ticks = max(16, max(s.family.S for s in self.solvers))
        ticks = min(ticks, n_ticks)
        saved = [s.u.clone() for s in self.solvers]
        for s in self.solvers:
            s.counters(reset=True)
        timings = {}
        for m, g in candidates:
            self.set_tiling(m, g)
            best = float("inf")
            for _ in range(reps):
                for s, u in zip(self.solvers, saved):
                    s.u.copy_(u)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                self.run(0, ticks)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            timings[(m, g)] = best
        for s, u in zip(self.solvers, saved):
            s.u.copy_(u)
            s.counters(reset=True)
        torch.cuda.synchronize()
        choice = min(timings, key=timings.get)
        self.set_tiling(*choice)
        result = {"tiling": list(choice), "ticks_timed": ticks,
                  "timings_s": {f"{m}x{g}": t for (m, g), t in timings.items()}}
        if cache:
            stored = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    stored = json.load(f)
            stored[key] = result
            with open(cache, "w") as f:
                json.dump(stored, f, indent=1)
        return result

    def signature(self):
        """Runs' (degree, stage count, element count) and the device name: the autotuner key."""
        runs = sorted((s.degree, s.family.S, s.n_elements) for s in self.solvers)
        h = hash(tuple(runs)) & 0xFFFFFFFFFFFF
        return f"{torch.cuda.get_device_name(0)}|{len(runs)}|{h:012x}"
