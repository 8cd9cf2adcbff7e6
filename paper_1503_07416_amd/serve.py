"""Continuous-batching server over the batched solver (hfz_batch_* of the C ABI).

A request is one simulation: parameters (model, grid size n, h, s, ...), an
initial state (rho, u, v) and a number of time steps of the scheme of Sec. 5
(Eqs. discrete_a-d).  Requests arrive over time and differ in model and size.

Design
  * Requests whose hfz_params are identical form a class.  A class owns slot
    pools: hfz_batch handles of `capacity` instances whose multigrid
    hierarchies stay resident in device memory for the life of the pool.
  * Admission control (the thread that calls :meth:`Server.run`) places each
    arrived request into a free slot of its class.  With no free slot it
    reserves a new pool if the device-memory budget still holds it, first
    releasing pools that have stood empty; requests that need new memory are
    admitted strictly first come, first served, while a request that finds a
    free slot in an existing pool may pass them (it takes no new memory).
    The sum of the reserved pool workspaces never exceeds the budget.
  * One worker thread per pool advances all filled slots of the pool by one
    time step per call (hfz_batch_step: one launch per level and phase for all
    instances, per-instance stop test), on the pool's own HIP stream, so the
    pools of different classes run concurrently on the device.  A request
    leaves its slot after its last step and the next request of the class
    can take the slot at the following step boundary (continuous batching).
  * Per-step latency of a request is the wall time of the pool step it took
    part in; the report gives p50/p99 of these over every request-step, the
    queueing delay (arrival to admission) and the throughput.

The slot arithmetic is the batched solver's, which gives every instance the
result it gets alone (each keeps its own stop test), so a request's result
does not depend on which other requests share its pool or the device.
"""
import collections
import ctypes
import threading
import time

import numpy as np

from . import hfz


def class_key(params):
    """Hashable identity of an hfz_params: requests with equal keys can share a pool."""
    return tuple(getattr(params, f) for f, _ in hfz.Params._fields_)


class DeviceBackend:
    """Slot pools on a HIP device: each pool is an :class:`hfz.Batch` on a stream of its own."""

    def __init__(self, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.lib = hfz.load()

    def pool_bytes(self, params, capacity):
        arr = (hfz.Params * capacity)(*([params] * capacity))
        nb = ctypes.c_size_t(0)
        hfz.check(self.lib.hfz_batch_workspace_bytes(arr, capacity, ctypes.byref(nb)),
                  "hfz_batch_workspace_bytes")
        return nb.value

    def make_pool(self, cfg, capacity):
        stream = self.torch.cuda.Stream(self.device)  # default priority
        return hfz.Batch([cfg] * capacity, device=self.device, stream=stream)

    def context(self, pool):
        """Context for a pool's worker thread: torch work of the thread goes to the pool's stream."""
        return self.torch.cuda.stream(pool.batch.stream)

    def to_host(self, tensors):
        return [t.cpu().numpy() for t in tensors]


class Job:
    """A request while it is served, and what is measured about it."""

    def __init__(self, req, key):
        self.req = req
        self.key = key
        self.t_arrive = None
        self.t_admit = None
        self.t_done = None
        self.steps_done = 0
        self.cycles = 0
        self.lat = []          # seconds per step
        self.energy = []       # E after set_state and after every step (if checked)
        self.error = 0
        self.result = None


class Pool:
    def __init__(self, key, batch, capacity, nbytes):
        self.key = key
        self.batch = batch
        self.capacity = capacity
        self.nbytes = nbytes
        self.slots = [None] * capacity   # Job assigned by admission control
        self.inbox = []                  # (slot, Job) not yet loaded by the worker
        self.running = {}                # slot -> Job being stepped
        self.closing = False
        self.thread = None
        self.steps = 0

    def free_slot(self):
        for k, j in enumerate(self.slots):
            if j is None:
                return k
        return -1

    def empty(self):
        return all(j is None for j in self.slots) and not self.inbox and not self.running


class Server:
    """Continuous-batching server.

    budget_bytes: device memory that pool workspaces may reserve in total.
    pool_target_bytes: size a new pool aims for (capacity = this // slot bytes,
      clipped to [1, max_slots] and to what the budget has left).
    check_energy: read the discrete energy after every step and count steps
      with E^{k+1} > E^k + energy_tol * max(1, |E^k|) (Thm. thm_energy_stability).
    keep_results: copy each request's final state to host numpy arrays.
    """

    def __init__(self, budget_bytes, backend=None, pool_target_bytes=None, max_slots=32,
                 check_energy=False, energy_tol=1e-10, keep_results=False):
        self.budget = int(budget_bytes)
        self.backend = backend if backend is not None else DeviceBackend()
        self.pool_target = int(pool_target_bytes) if pool_target_bytes else max(1, self.budget // 8)
        self.max_slots = int(max_slots)
        self.check_energy = check_energy
        self.energy_tol = energy_tol
        self.keep_results = keep_results
        self.cv = threading.Condition()
        self.pools = []
        self.reserved = 0
        self.peak_reserved = 0
        self.pools_created = 0
        self.pools_released = 0
        self.ndone = 0
        self.fatal = None
        self._slot_bytes = {}

    # ---- admission control (caller's thread) --------------------------------
    def slot_bytes(self, params):
        k = class_key(params)
        if k not in self._slot_bytes:
            self._slot_bytes[k] = self.backend.pool_bytes(params, 1)
        return self._slot_bytes[k]

    def _capacity_for(self, params, room):
        cap = max(1, min(self.max_slots, self.pool_target // max(1, self.slot_bytes(params))))
        while cap >= 1:
            nb = self.backend.pool_bytes(params, cap)
            if nb <= room:
                return cap, nb
            cap //= 2
        return 0, 0

    def _release_empty_pools(self, need):
        """Releases empty pools (oldest first) until `need` bytes fit; lock held on entry and exit."""
        for pool in list(self.pools):
            if self.budget - self.reserved >= need:
                return
            if pool.empty():
                pool.closing = True
                self.cv.notify_all()
                self.cv.release()
                try:
                    pool.thread.join()
                    pool.batch.close()
                finally:
                    self.cv.acquire()
                self.pools.remove(pool)
                self.reserved -= pool.nbytes
                self.pools_released += 1

    def _new_pool(self, job):
        """Reserves and starts a pool for job's class if the budget allows; lock held."""
        params = job.req_params
        need1 = self.slot_bytes(params)
        if self.budget - self.reserved < need1:
            self._release_empty_pools(need1)
        cap, nb = self._capacity_for(params, self.budget - self.reserved)
        if cap == 0:
            return None
        self.reserved += nb
        assert self.reserved <= self.budget
        self.peak_reserved = max(self.peak_reserved, self.reserved)
        self.cv.release()
        try:
            batch = self.backend.make_pool(job.req.cfg, cap)
        finally:
            self.cv.acquire()
        pool = Pool(job.key, batch, cap, nb)
        pool.thread = threading.Thread(target=self._worker, args=(pool,), daemon=True)
        self.pools.append(pool)
        self.pools_created += 1
        pool.thread.start()
        return pool

    def _assign(self, pool, k, job):
        pool.slots[k] = job
        pool.inbox.append((k, job))
        job.t_admit = time.perf_counter()
        self.cv.notify_all()

    def _admit(self, waiting):
        blocked = False
        for job in list(waiting):
            pool, k = None, -1
            for p in self.pools:
                if p.key == job.key and not p.closing:
                    k = p.free_slot()
                    if k >= 0:
                        pool = p
                        break
            if pool is None:
                if blocked:
                    continue          # only free slots may pass a request blocked on memory
                pool = self._new_pool(job)
                if pool is None:
                    blocked = True
                    continue
                k = pool.free_slot()
            waiting.remove(job)
            self._assign(pool, k, job)

    # ---- workers --------------------------------------------------------------
    def _worker(self, pool):
        try:
            with self.backend.context(pool):
                self._work(pool)
        except BaseException as e:  # noqa: BLE001 - reported to the controller
            with self.cv:
                self.fatal = e
                self.cv.notify_all()

    def _work(self, pool):
        b = pool.batch
        while True:
            with self.cv:
                while not pool.inbox and not pool.running and not pool.closing and self.fatal is None:
                    self.cv.wait()
                if self.fatal is not None:
                    return
                if pool.closing and not pool.inbox and not pool.running:
                    return
                intake, pool.inbox = pool.inbox, []
            for k, job in intake:
                r = job.req
                b.set_state(k, r.rho, r.u, r.v)
                if hasattr(r, "drop_state"):
                    r.drop_state()   # the host copy of the initial state is no longer needed
                if self.check_energy:
                    job.energy.append(b.energy(k)[0])
                pool.running[k] = job
            t = time.perf_counter()
            rc, st = b.step(1, raise_on_error=False)
            dt = time.perf_counter() - t
            pool.steps += 1
            if rc not in (0, hfz.ENOCONV, hfz.ENAN):
                raise hfz.HfzError(rc, "hfz_batch_step")
            finished = []
            for k, job in pool.running.items():
                if st[k].steps_done == 1:
                    job.steps_done += 1
                    job.cycles += st[k].cycles_last
                    job.lat.append(dt)
                    if self.check_energy:
                        job.energy.append(b.energy(k)[0])
                    if job.steps_done >= job.req.steps:
                        finished.append(k)
                else:
                    job.error = rc if rc != 0 else hfz.ENOCONV
                    finished.append(k)
            for k in finished:
                job = pool.running.pop(k)
                if self.keep_results and job.error == 0:
                    job.result = self.backend.to_host(b.get_state(k))
                b.release(k)
                job.t_done = time.perf_counter()
            if finished:
                with self.cv:
                    for k in finished:
                        pool.slots[k] = None
                    self.ndone += len(finished)
                    self.cv.notify_all()

    # ---- driver ---------------------------------------------------------------
    def run(self, requests, realtime=True, poll=0.02, progress_every=None, log=None):
        """Serves `requests` (objects with arrival [s], steps, cfg, rho, u, v);
        arrivals are honoured in wall time if `realtime`, else all arrive at
        once.  With progress_every (seconds), a line of progress goes to `log`
        (a file object) that often.  Returns (jobs in arrival order, report
        dict)."""
        jobs = []
        for r in sorted(requests, key=lambda q: q.arrival):
            p = hfz.make_params(r.cfg)
            j = Job(r, class_key(p))
            j.req_params = p
            if self.slot_bytes(p) > self.budget:
                raise ValueError(f"request {getattr(r, 'rid', '?')} needs {self.slot_bytes(p)} bytes, "
                                 f"more than the budget {self.budget}")
            jobs.append(j)
        arrivals = collections.deque(jobs)
        waiting = []
        t0 = time.perf_counter()
        t_log = t0
        try:
            with self.cv:
                while self.ndone < len(jobs):
                    if self.fatal is not None:
                        raise self.fatal
                    now = time.perf_counter() - t0
                    while arrivals and (not realtime or arrivals[0].req.arrival <= now):
                        j = arrivals.popleft()
                        j.t_arrive = t0 + (j.req.arrival if realtime else 0.0)
                        waiting.append(j)
                    self._admit(waiting)
                    if progress_every and log is not None and time.perf_counter() - t_log >= progress_every:
                        t_log = time.perf_counter()
                        print(f"serve: {self.ndone}/{len(jobs)} requests done, {len(waiting)} waiting, "
                              f"{len(self.pools)} pools, {self.reserved / 2**30:.1f} GiB reserved, "
                              f"{t_log - t0:.1f} s", file=log, flush=True)
                    tmo = poll
                    if arrivals and realtime:
                        tmo = min(tmo, max(0.0, arrivals[0].req.arrival - (time.perf_counter() - t0)))
                    self.cv.wait(timeout=tmo)
                if self.fatal is not None:
                    raise self.fatal
        finally:
            self.shutdown()
        return jobs, self.report(jobs, t0)

    def shutdown(self):
        with self.cv:
            for p in self.pools:
                p.closing = True
            self.cv.notify_all()
        for p in list(self.pools):
            if p.thread is not None:
                p.thread.join()
            p.batch.close()
        with self.cv:
            self.reserved -= sum(p.nbytes for p in self.pools)
            self.pools = []

    def report(self, jobs, t0):
        lat = np.array([x for j in jobs for x in j.lat]) * 1e3
        queue = np.array([j.t_admit - j.t_arrive for j in jobs if j.t_admit is not None]) * 1e3
        done = [j for j in jobs if j.t_done is not None]
        t_first = min(j.t_arrive for j in jobs) if jobs else t0
        t_last = max(j.t_done for j in done) if done else t0
        span = max(t_last - t_first, 1e-12)
        steps = int(sum(j.steps_done for j in jobs))
        violations = 0
        for j in jobs:
            e = j.energy
            for a, c in zip(e[:-1], e[1:]):
                if c > a + self.energy_tol * max(1.0, abs(a)):
                    violations += 1

        def pct(a, q):
            return float(np.percentile(a, q)) if len(a) else None

        return {
            "requests": len(jobs),
            "completed": sum(1 for j in jobs if j.error == 0 and j.t_done is not None),
            "failed": sum(1 for j in jobs if j.error != 0),
            "request_steps": steps,
            "makespan_s": span,
            "steps_per_s": steps / span,
            "requests_per_s": len(done) / span,
            "step_latency_ms_p50": pct(lat, 50),
            "step_latency_ms_p99": pct(lat, 99),
            "queue_ms_p50": pct(queue, 50),
            "queue_ms_p99": pct(queue, 99),
            "budget_bytes": self.budget,
            "peak_reserved_bytes": self.peak_reserved,
            "pools_created": self.pools_created,
            "pools_released": self.pools_released,
            "energy_checked": bool(self.check_energy),
            "energy_increases": violations,
            "cycles_per_step": (sum(j.cycles for j in jobs) / steps) if steps else None,
        }
