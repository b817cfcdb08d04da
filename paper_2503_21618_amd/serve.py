"""Serving loop over the batch API: continuous batching of interval eigensolves.

Requests (a pencil, gamma, L, optional poles) arrive over time.  Each scheduling
round
  1. admits waiting requests in arrival order while the batch accepts them: the
     library checks each pencil's persistent bytes (merged CSR and subspace
     blocks) against the free pool and the filter arena needed by the unfinished
     pencils plus the newcomer against the arena, i.e. admission by HBM
     footprint; the first request that does not fit waits (first come, first
     served), and so do the ones behind it;
  2. runs one outer step (one batched filter application for every unfinished
     pencil, then Rayleigh-Ritz and residuals per pencil) on the device, where
     the subspaces stay resident between steps;
  3. collects finished pencils (their results copied out, their pool space
     freed), recording each request's latency from arrival to completion.

All arithmetic runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import binding as lib


@dataclass
class Request:
    rid: int
    A: object
    B: object
    gamma: float
    L: int
    sigma: object = None
    w: object = None
    V0: object = None
    arrival: float = 0.0          # seconds on the server's clock (or step index)


@dataclass
class Completion:
    rid: int
    result: lib.SolveResult
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class Server:
    """Continuous-batching server over one lib.Batch.

    ws_bytes: device workspace (pool + arena); arena_bytes: filter arena shared
    by the unfinished pencils of a step.  clock: returns the current time
    (default: wall clock relative to the server's start); tests pass a step
    counter instead.  make_batch: builds the batch (default lib.Batch); tests
    of the scheduling pass a host-only stand-in with the same methods."""
    ws_bytes: int
    arena_bytes: int
    max_poles: int = 6
    options: object = None
    stream: object = None
    clock: object = None
    make_batch: object = None
    batch: lib.Batch = field(init=False)
    queue: deque = field(init=False, default_factory=deque)
    active: dict = field(init=False, default_factory=dict)
    done: list = field(init=False, default_factory=list)
    steps: int = field(init=False, default=0)
    peak_active: int = field(init=False, default=0)

    def __post_init__(self):
        make = self.make_batch or (lambda: lib.Batch(self.ws_bytes, self.arena_bytes, self.max_poles,
                                                     self.options, stream=self.stream))
        self.batch = make()
        if self.clock is None:
            t0 = time.perf_counter()
            self.clock = lambda: time.perf_counter() - t0

    def submit(self, req: Request):
        self.queue.append(req)

    def admit(self) -> int:
        n = 0
        while self.queue:
            req = self.queue[0]
            pid = self.batch.add(req.A, req.B, req.gamma, req.L, req.sigma, req.w, req.V0, must_fit=False)
            if pid is None:
                if not self.active:
                    raise lib.SlrfError(3, f"request {req.rid} does not fit an empty server")
                break
            self.queue.popleft()
            self.active[pid] = (req, self.clock())
            n += 1
        self.peak_active = max(self.peak_active, len(self.active))
        return n

    def collect(self) -> int:
        n = 0
        for pid in list(self.active):
            finished, _ = self.batch.query(pid)
            if not finished:
                continue
            req, t_adm = self.active.pop(pid)
            res = self.batch.result(pid)
            self.batch.remove(pid)
            self.done.append(Completion(req.rid, res, req.arrival, t_adm, self.clock()))
            n += 1
        return n

    def pump(self) -> int:
        """One scheduling round; returns the number of unfinished pencils after it."""
        self.admit()
        if self.active:
            self.batch.step()
            self.steps += 1
            self.collect()
        return len(self.active)

    def idle(self) -> bool:
        return not self.queue and not self.active

    def close(self):
        self.batch.close()


def latency_stats(done) -> dict:
    lat = np.array([c.latency for c in done])
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
            "mean": float(lat.mean()), "max": float(lat.max())}
