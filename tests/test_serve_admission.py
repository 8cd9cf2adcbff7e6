"""Host logic of the continuous-batching server, on the CPU: a simulated pool
backend (no device) stands in for hfz_batch so that the admission rules can be
checked directly: the reserved bytes never exceed the budget, every request is
served to its last step, slots are reused, empty pools are released under
memory pressure, requests needing new memory are admitted in arrival order,
and a failing step ends only its own request."""
import contextlib
import threading
import time

import numpy as np
import pytest

import workloads
from paper_1503_07416_amd import hfz
from paper_1503_07416_amd.serve import Server


class FakeStats:
    def __init__(self, done, cycles):
        self.steps_done = done
        self.cycles_last = cycles


class FakeBatch:
    def __init__(self, backend, cfg, capacity):
        self.backend = backend
        self.cfg = cfg
        self.count = capacity
        self.filled = [None] * capacity
        self.E = [0.0] * capacity
        self.closed = False

    def set_state(self, i, rho, u, v):
        assert self.filled[i] is None, "slot loaded twice"
        self.filled[i] = np.array(rho, copy=True)
        self.E[i] = 1.0

    def energy(self, i):
        return [self.E[i], 0, 0, 0, 0]

    def step(self, nsteps, raise_on_error=True):
        with self.backend.lock:
            self.backend.live += 1
            self.backend.max_live = max(self.backend.max_live, self.backend.live)
        time.sleep(self.backend.step_time * (self.cfg.n / 64) ** 2)
        st, rc = [], 0
        for i in range(self.count):
            if self.filled[i] is None:
                st.append(FakeStats(0, 0))
            elif self.backend.fail_when(self.filled[i]):
                st.append(FakeStats(0, 0))
                rc = hfz.ENOCONV
            else:
                self.filled[i] = self.filled[i] + np.array([0.0, 1.0])
                self.E[i] *= 0.5
                st.append(FakeStats(1, 3))
        with self.backend.lock:
            self.backend.live -= 1
        return rc, st

    def get_state(self, i):
        return [self.filled[i]] * 3

    def release(self, i):
        self.filled[i] = None

    def close(self):
        assert all(f is None for f in self.filled), "pool closed with a filled slot"
        self.closed = True


class FakeBackend:
    def __init__(self, step_time=2e-4, fail_when=lambda rho: False):
        self.step_time = step_time
        self.fail_when = fail_when
        self.lock = threading.Lock()
        self.live = 0
        self.max_live = 0
        self.pools = []

    def pool_bytes(self, params, capacity):
        return 4096 + capacity * 100 * params.n * params.n

    def make_pool(self, cfg, capacity):
        b = FakeBatch(self, cfg, capacity)
        self.pools.append(b)
        return b

    def context(self, pool):
        return contextlib.nullcontext()

    def to_host(self, tensors):
        return [np.array(t) for t in tensors]


def stream(count, sizes=(8, 16, 32), steps=(2, 9), seed=3):
    reqs = workloads.serving_stream(count, rate=2000.0, seed=seed, sizes=sizes, steps=steps)
    for r in reqs:
        r.fix_state(np.array([float(r.rid), 0.0]), None, None)   # the fake backend tracks (rid, steps taken)
    return reqs


class WatchedServer(Server):
    """Records the reserved bytes at every pool reservation."""

    def __init__(self, *a, **kw):
        super().__init__(*a, **kw)
        self.trace = []
        self.new_memory = []

    def _new_pool(self, job):
        pool = super()._new_pool(job)
        self.trace.append(self.reserved)
        if pool is not None:
            self.new_memory.append(job.req.rid)
        return pool


def slot(n):
    return 4096 + 100 * n * n


def test_all_served_budget_respected_results_exact():
    be = FakeBackend()
    budget = 3 * slot(32) + 2 * slot(16)
    srv = WatchedServer(budget, backend=be, pool_target_bytes=2 * slot(16), max_slots=4, keep_results=True,
                        check_energy=True)
    reqs = stream(40)
    jobs, rep = srv.run(reqs, realtime=True)
    assert rep["completed"] == 40 and rep["failed"] == 0
    assert max(srv.trace) <= budget and rep["peak_reserved_bytes"] <= budget
    for j in jobs:
        assert j.steps_done == j.req.steps and len(j.lat) == j.req.steps
        # the fake step counts steps: the result is exact for every request
        assert list(j.result[0]) == [j.req.rid, j.req.steps]
        assert len(j.energy) == j.req.steps + 1
    assert rep["energy_increases"] == 0
    assert rep["request_steps"] == sum(r.steps for r in reqs)
    assert be.max_live >= 2, "pools of different classes should step concurrently"
    assert all(p.closed for p in be.pools)
    assert srv.reserved == 0


def test_pools_reused_and_released_under_pressure():
    be = FakeBackend()
    # room for one 32^2 slot: classes must take turns, releasing empty pools
    budget = slot(32) + 10
    srv = WatchedServer(budget, backend=be, pool_target_bytes=1, max_slots=1)
    jobs, rep = srv.run(stream(24), realtime=False)
    assert rep["completed"] == 24
    assert rep["peak_reserved_bytes"] <= budget
    assert rep["pools_released"] >= 1
    assert max(srv.trace) <= budget


def test_memory_admission_in_arrival_order():
    be = FakeBackend()
    budget = slot(32) + slot(8) + 10
    srv = WatchedServer(budget, backend=be, pool_target_bytes=1, max_slots=1)
    reqs = stream(30)
    jobs, rep = srv.run(reqs, realtime=False)
    assert rep["completed"] == 30
    # requests admitted by reserving new memory are admitted in arrival order
    # (others may only pass them by taking a free slot of an existing pool)
    assert srv.new_memory == sorted(srv.new_memory)
    assert len(srv.new_memory) > 3


def test_failure_ends_only_its_request():
    be = FakeBackend(fail_when=lambda st: st[0] == 7 and st[1] == 2)   # request 7 after two steps
    srv = Server(10 * slot(32), backend=be, pool_target_bytes=4 * slot(32), max_slots=4, keep_results=True)
    reqs = stream(12)
    reqs[7].steps = 6
    jobs, rep = srv.run(reqs, realtime=False)
    by = {j.req.rid: j for j in jobs}
    assert by[7].error == hfz.ENOCONV and by[7].steps_done == 2 and by[7].result is None
    assert rep["failed"] == 1 and rep["completed"] == 11
    for rid, j in by.items():
        if rid != 7:
            assert j.error == 0 and list(j.result[0]) == [rid, j.req.steps]


def test_request_larger_than_budget_rejected():
    srv = Server(slot(16), backend=FakeBackend())
    with pytest.raises(ValueError):
        srv.run(stream(3, sizes=(32,)), realtime=False)
