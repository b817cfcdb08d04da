"""Scheduling properties of the continuous-batching server (serve.Server) on the
host, with a stand-in for the device batch: a footprint model and a step
clock, no GPU.

The stand-in admits a pencil only when its persistent bytes fit the pool and
the transient bytes of the unfinished pencils plus its own fit the arena (the
rule the library applies); each pencil finishes after a fixed number of outer
steps.  Under a Poisson trace of requests of mixed sizes:

* the pool and the arena are never over-committed;
* requests are admitted in arrival order (first come, first served);
* every request completes (no starvation), with admission at or after arrival
  and completion after admission;
* a request larger than an empty server is refused loudly.
"""
import numpy as np
import pytest

import pencils


class FakeBatch:
    """Host-only batch: A carries (persistent, transient, steps) of the pencil."""

    def __init__(self, pool, arena):
        self.pool, self.arena = pool, arena
        self.used = self.trans = 0
        self.next = 0
        self.live = {}
        self.order = []
        self.high = (0, 0)

    def add(self, A, B, gamma, L, sigma=None, w=None, V0=None, must_fit=True):
        p, t, steps = A
        if self.used + p > self.pool or self.trans + t > self.arena:
            return None
        pid = self.next
        self.next += 1
        self.live[pid] = [p, t, steps, B]
        self.used += p
        self.trans += t
        self.order.append(B)
        self.high = (max(self.high[0], self.used), max(self.high[1], self.trans))
        return pid

    def step(self):
        for v in self.live.values():
            if v[2] > 0:
                v[2] -= 1
        return sum(1 for v in self.live.values() if v[2] > 0)

    def query(self, pid):
        return self.live[pid][2] == 0, None

    def result(self, pid):
        return ("done", self.live[pid][3])

    def remove(self, pid):
        p, t, _, _ = self.live.pop(pid)
        self.used -= p
        self.trans -= t

    def close(self):
        pass


def run_trace(count, rate, pool, arena, seed):
    import paper_2503_21618_amd.serve as serve
    u = pencils.uniform(seed, 3 * count).reshape(count, 3)
    arrivals = pencils.arrival_times(count, rate, seed=seed + 1)
    fake = FakeBatch(pool, arena)
    clock = {"t": 0.0}
    srv = serve.Server(pool + arena, arena, make_batch=lambda: fake, clock=lambda: clock["t"])
    reqs = []
    for r in range(count):
        p = int(1 + 40 * u[r, 0] ** 2)            # persistent units, a few large ones
        t = int(1 + 30 * u[r, 1] ** 2)            # transient units
        steps = int(3 + 12 * u[r, 2])             # outer steps to converge
        reqs.append(serve.Request(r, (p, t, steps), r, 1.0, 8, arrival=float(arrivals[r])))
    pending = list(reqs)
    guard = 0
    while pending or not srv.idle():
        while pending and pending[0].arrival <= clock["t"]:
            srv.submit(pending.pop(0))
        if not srv.idle():
            srv.pump()
        clock["t"] += 1.0
        guard += 1
        assert guard < 100000
    return srv, fake


@pytest.mark.parametrize("rate,seed", [(0.3, 11), (1.5, 12), (4.0, 13)])
def test_server_never_overcommits_and_serves_in_order(rate, seed):
    pool, arena = 100, 60
    srv, fake = run_trace(300, rate, pool, arena, seed)
    assert fake.high[0] <= pool and fake.high[1] <= arena
    assert fake.order == sorted(fake.order) == list(range(300))        # FIFO admission
    assert sorted(c.rid for c in srv.done) == list(range(300))        # nobody starves
    for c in srv.done:
        assert c.arrival <= c.admitted < c.finished
    # under overload the queue builds up but the server stays busy
    if rate >= 1.5:
        assert srv.peak_active >= 3


def test_server_refuses_a_request_larger_than_empty():
    import paper_2503_21618_amd.serve as serve
    fake = FakeBatch(10, 10)
    srv = serve.Server(20, 10, make_batch=lambda: fake, clock=lambda: 0.0)
    srv.submit(serve.Request(0, (11, 1, 3), 0, 1.0, 8))
    with pytest.raises(Exception):
        srv.pump()
