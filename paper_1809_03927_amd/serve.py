"""Serving loop for dose requests that arrive over time (one GPU).

An optimiser of 4D-robust plans, the use the paper foresees for the engine
(Sec. 1 and Sec. 4.C), issues many dose calculations of different sizes.
This loop takes such requests as they arrive and

* admits them in arrival order while their phantom, tally, dose and request
  data fit a device-memory budget (the head of the queue waits when it does
  not fit, so no request starves);
* keeps phantoms resident on the device and, when room is needed, unloads
  those no admitted request uses, least recently used first;
* runs admitted requests on the persistent engine in slices of their work
  items (chunks of a spot's histories); before each slice it takes the
  oldest small request (at most `small_histories` histories, by default the
  median request size) if there is one, else the oldest large one: a small
  request arriving behind a large one waits for about one slice, while the
  large requests keep their arrival order and so a latency tail close to
  that of serving everything in arrival order (least-expected-slowdown and
  shortest-remaining-first orders are available too);
* submits the next slice as soon as the running one has handed out its last
  work item (the kernel sets a pinned host flag), on a second stream, so
  that the drain of one persistent launch (its last histories running at
  falling occupancy) overlaps the start of the next instead of idling CUs,
  while the choice of what runs next is made as late as possible (a request
  arriving during a slice can still run next).  With one stream the next
  slice waits for the running one to end.

Slices of one request add into the same integer tally, and a history's random
numbers depend only on (seed, request, spot, history), so the served dose of a
request is bit-identical to the dose of one uninterrupted run, whatever the
schedule.  The comparison engine ("plain-serial") runs every request whole,
in arrival order, with the plain engine (one launch per phase).

The scheduler does not know the device: an executor does the work and a clock
tells time, so the policy is tested on the CPU with a simulated clock.
"""
from __future__ import annotations

import argparse
import concurrent.futures
import dataclasses
import hashlib
import json
import math
import sys
import threading
import time
from collections import OrderedDict, deque
from typing import Callable, Dict, List, Optional

import numpy as np

from . import workloads as W


# ----------------------------------------------------------------------------
# jobs and clocks
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Job:
    index: int
    arrival_s: float
    n_histories: int
    phantom_key: tuple
    nvox: int
    cancel_s: Optional[float] = None     # the requester withdraws it at this time
    n_items: int = 0
    next_item: int = 0                   # first work item not yet submitted
    items_done: int = 0
    in_flight: int = 0                   # slices submitted and not yet completed
    item_hist: Optional[np.ndarray] = None  # histories per work item (sliced runs)
    admitted_s: Optional[float] = None
    first_run_s: Optional[float] = None
    done_s: Optional[float] = None
    cancelled: bool = False
    started: bool = False                # buffers made and request data prepared
    slices: int = 0
    state: Dict = dataclasses.field(default_factory=dict)

    @property
    def remaining(self) -> int:
        if self.item_hist is None:
            return self.n_histories
        return int(self.item_hist[self.next_item:].sum())

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep_until(self, t: float) -> None:
        d = t - self.now()
        if d > 0:
            time.sleep(d)


class FakeClock:
    """Simulated time, advanced by a simulated executor."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def sleep_until(self, t: float) -> None:
        self.t = max(self.t, t)

    def advance(self, dt: float) -> None:
        self.t += dt


class Executor:
    """What the scheduler needs from a device."""

    def phantom_bytes(self, key) -> int:
        raise NotImplementedError

    def job_bytes(self, job: Job) -> int:
        raise NotImplementedError

    def load_phantom(self, key) -> None:
        raise NotImplementedError

    def unload_phantom(self, key) -> None:
        raise NotImplementedError

    def start(self, job: Job, sliced: bool) -> None:
        """Allocate the job's buffers; set job.n_items (and job.item_hist when sliced)."""
        raise NotImplementedError

    def submit(self, job: Job, item_begin: int, item_end: int):
        """Start work items [item_begin, item_end) of the job; return a token."""
        raise NotImplementedError

    def finished(self, token) -> bool:
        """Has the submission completed?  (Does not block.)"""
        raise NotImplementedError

    def drained(self, token) -> bool:
        """Has the submission taken all its work, so that the next one may
        start beside its last histories?  (Does not block.)"""
        return self.finished(token)

    def progress(self, tokens, until: Optional[float] = None) -> None:
        """Block until a token may have drained or finished, or until time
        `until` (a new arrival), whichever comes first."""
        raise NotImplementedError

    def run(self, job: Job, item_begin: int, item_end: int) -> None:
        token = self.submit(job, item_begin, item_end)
        while not self.finished(token):
            self.progress([token])

    def finish(self, job: Job) -> None:
        """Produce the job's dose on the host (the request is served when this returns)."""
        raise NotImplementedError

    def release(self, job: Job) -> None:
        """Free the job's buffers (after finish, or on cancellation)."""
        raise NotImplementedError


# ----------------------------------------------------------------------------
# scheduler
# ----------------------------------------------------------------------------

class Scheduler:
    """Admission by device-memory budget, phantom residency, slice scheduling.

    Sliced policies cut requests into slices of at most `slice_histories`
    histories (at least one work item) and choose, before each slice,
      "small-first": the oldest request of at most `small_histories`
                  histories, else the oldest request;
      "slowdown": the least (remaining histories / rate_hist_per_s) /
                  (time since arrival + slowdown_c_s);
      "srpt":     the fewest remaining histories.
    policy "fifo": every request whole, in arrival order.
    `depth` submissions are kept in flight (completed in submission order).
    """

    POLICIES = ("small-first", "slowdown", "srpt", "fifo")

    def __init__(self, executor: Executor, clock, budget_bytes: int, policy: str = "small-first",
                 slice_histories: int = 4_000_000, log: Optional[Callable[[str], None]] = None,
                 log_every: int = 25, depth: int = 1, rate_hist_per_s: float = 1.3e8,
                 slowdown_c_s: float = 0.05, small_histories: float = 2.2e6, prestart: int = 2):
        if policy not in self.POLICIES:
            raise ValueError(f"unknown policy {policy!r}")
        self.small = float(small_histories)
        self.prestart = int(prestart)
        self.rate = float(rate_hist_per_s)
        self.slowdown_c = float(slowdown_c_s)
        if depth < 1:
            raise ValueError("depth must be >= 1")
        self.depth = depth
        self.ex = executor
        self.clock = clock
        self.budget = int(budget_bytes)
        self.policy = policy
        self.slice_histories = int(slice_histories)
        self.log = log
        self.log_every = log_every
        self.resident: "OrderedDict[tuple, int]" = OrderedDict()  # phantom -> admitted users, LRU order
        self.admitted: List[Job] = []
        self.used = 0
        self.peak_used = 0
        self.evictions = 0
        self.phantom_loads = 0
        self.slices = 0

    # -- memory -----------------------------------------------------------------
    def _need(self, job: Job) -> int:
        need = self.ex.job_bytes(job)
        if job.phantom_key not in self.resident:
            need += self.ex.phantom_bytes(job.phantom_key)
        return need

    def _make_room(self, job: Job) -> bool:
        need = self._need(job)
        for key in list(self.resident):  # least recently used first
            if self.used + need <= self.budget:
                break
            if self.resident[key] == 0 and key != job.phantom_key:
                self.ex.unload_phantom(key)
                self.used -= self.ex.phantom_bytes(key)
                del self.resident[key]
                self.evictions += 1
        return self.used + need <= self.budget

    def _admit(self, job: Job) -> None:
        if job.phantom_key not in self.resident:
            self.ex.load_phantom(job.phantom_key)
            self.used += self.ex.phantom_bytes(job.phantom_key)
            self.resident[job.phantom_key] = 0
            self.phantom_loads += 1
        self.resident[job.phantom_key] += 1
        self.resident.move_to_end(job.phantom_key)
        self.used += self.ex.job_bytes(job)
        self.peak_used = max(self.peak_used, self.used)
        job.admitted_s = self.clock.now()
        self.admitted.append(job)  # its buffers are made when it first runs

    def _retire(self, job: Job) -> None:
        self.ex.release(job)
        self.used -= self.ex.job_bytes(job)
        self.resident[job.phantom_key] -= 1
        self.admitted.remove(job)

    # -- policy -------------------------------------------------------------------
    def _key(self, j: Job, now: float):
        if self.policy == "fifo":
            return (j.arrival_s, j.index)
        if self.policy == "small-first":
            return (j.n_histories > self.small, j.arrival_s, j.index)
        if self.policy == "srpt":
            return (j.remaining, j.arrival_s, j.index)
        return (j.remaining / self.rate / (now - j.arrival_s + self.slowdown_c), j.arrival_s, j.index)

    def _ready(self) -> List[Job]:
        return [j for j in self.admitted if not j.started or j.next_item < j.n_items]

    def _pick(self) -> Optional[Job]:
        ready = self._ready()
        if not ready:
            return None
        now = self.clock.now()
        return min(ready, key=lambda j: self._key(j, now))

    def _prestart(self) -> None:
        """Prepare the next requests in pick order while the device works:
        at most `prestart` prepared requests wait for their first slice (each
        preparation takes host time the loop cannot spend on submissions)."""
        ahead = sum(1 for j in self.admitted if j.started and j.first_run_s is None)
        room = self.prestart - ahead
        if room <= 0:
            return
        now = self.clock.now()
        todo = sorted((j for j in self.admitted if not j.started), key=lambda j: self._key(j, now))
        for j in todo[:room]:
            self.ex.start(j, sliced=self.policy != "fifo")
            j.started = True

    def _slice_end(self, job: Job) -> int:
        if self.policy == "fifo" or job.item_hist is None:
            return job.n_items
        e, acc = job.next_item, 0
        while e < job.n_items and (acc == 0 or acc + int(job.item_hist[e]) <= self.slice_histories):
            acc += int(job.item_hist[e])
            e += 1
        return e

    # -- main loop ------------------------------------------------------------------
    def run(self, jobs: List[Job]) -> List[Job]:
        """Serve `jobs`; return the served ones in completion order."""
        for j in jobs:
            if self.ex.job_bytes(j) + self.ex.phantom_bytes(j.phantom_key) > self.budget:
                raise ValueError(f"request {j.index} needs more than the whole budget")
        waiting = deque(sorted(jobs, key=lambda j: (j.arrival_s, j.index)))
        inflight: deque = deque()  # (job, item_begin, item_end, token): not yet drained
        running: List[tuple] = []  # drained, not yet finished
        done: List[Job] = []
        while waiting or self.admitted:
            now = self.clock.now()
            for j in [j for j in waiting if j.cancel_s is not None and j.cancel_s <= now]:
                waiting.remove(j)
                j.cancelled = True
            for j in [j for j in self.admitted
                      if j.cancel_s is not None and j.cancel_s <= now and j.in_flight == 0]:
                self._retire(j)
                j.cancelled = True
            while waiting and waiting[0].arrival_s <= now and self._make_room(waiting[0]):
                self._admit(waiting.popleft())
            # keep `depth` slices that still have work to hand out
            while len(inflight) < self.depth:
                job = self._pick()
                if job is None:
                    break
                if not job.started:
                    self.ex.start(job, sliced=self.policy != "fifo")
                    job.started = True
                if job.first_run_s is None:
                    job.first_run_s = self.clock.now()
                b, e = job.next_item, self._slice_end(job)
                inflight.append((job, b, e, self.ex.submit(job, b, e)))
                job.next_item = e
                job.in_flight += 1
                job.slices += 1
                self.slices += 1
            if inflight:
                self._prestart()
            moved = False
            while inflight and self.ex.drained(inflight[0][3]):
                running.append(inflight.popleft())
                moved = True
            for sub in [x for x in running if self.ex.finished(x[3])]:
                running.remove(sub)
                moved = True
                job, b, e, _ = sub
                job.in_flight -= 1
                job.items_done += e - b
                if job.items_done == job.n_items:
                    self.ex.finish(job)
                    job.done_s = self.clock.now()
                    self._retire(job)
                    done.append(job)
                    if self.log and len(done) % self.log_every == 0:
                        self.log(f"{self.policy}: {len(done)} served, {len(waiting)} waiting, "
                                 f"{len(self.admitted)} admitted, t={job.done_s:.2f} s")
            if moved:
                continue
            nxt = None
            if waiting:
                nxt = waiting[0].arrival_s
                if waiting[0].cancel_s is not None:
                    nxt = min(nxt, waiting[0].cancel_s)
            if inflight or running:
                self.ex.progress([x[3] for x in inflight] + [x[3] for x in running],
                                 until=nxt if nxt is not None and nxt > now else None)
                continue
            if self.admitted:  # only cancelled-pending work remains: nothing runs it
                raise RuntimeError("admitted requests with no work left to submit")
            if not waiting:
                break
            if waiting[0].arrival_s <= now:
                raise RuntimeError("the queue head does not fit an empty device")
            self.clock.sleep_until(nxt)
        return done


def summarize(done: List[Job], label: str) -> dict:
    lat = np.array([j.latency_s for j in done])
    hist = sum(j.n_histories for j in done)
    t0 = min(j.arrival_s for j in done)
    t1 = max(j.done_s for j in done)
    return {"engine": label, "requests": len(done), "histories": int(hist),
            "makespan_s": t1 - t0, "throughput_hist_per_s": hist / (t1 - t0),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()), "max_latency_s": float(lat.max())}


# ----------------------------------------------------------------------------
# simulated executor (tests of the policy)
# ----------------------------------------------------------------------------

class SimExecutor(Executor):
    """Models a device: running h histories takes overhead_s + h / rate seconds.

    It checks what the scheduler must guarantee: a phantom is loaded before
    use and never unloaded while an admitted job uses it, and every work item
    of a job runs exactly once."""

    def __init__(self, clock: FakeClock, rate_hist_per_s=1e8, overhead_s=1e-3, chunk=256,
                 bytes_per_voxel_phantom=3, bytes_per_voxel_job=16):
        self.clock = clock
        self.rate = rate_hist_per_s
        self.overhead = overhead_s
        self.chunk = chunk
        self.bpv_phantom = bytes_per_voxel_phantom
        self.bpv_job = bytes_per_voxel_job
        self.nvox: Dict[tuple, int] = {}
        self.loaded: set = set()
        self.live: List[Job] = []
        self.calls: List[tuple] = []
        self.peak = 0
        self.busy_until = 0.0

    def _mem(self) -> int:
        return (sum(self.nvox[k] * self.bpv_phantom for k in self.loaded)
                + sum(j.nvox * self.bpv_job for j in self.live))

    def phantom_bytes(self, key) -> int:
        return self.nvox[key] * self.bpv_phantom

    def job_bytes(self, job: Job) -> int:
        self.nvox.setdefault(job.phantom_key, job.nvox)
        return job.nvox * self.bpv_job

    def load_phantom(self, key) -> None:
        assert key not in self.loaded
        self.loaded.add(key)
        self.calls.append(("load", key))

    def unload_phantom(self, key) -> None:
        assert key in self.loaded
        assert all(j.phantom_key != key for j in self.live), "phantom in use unloaded"
        self.loaded.remove(key)
        self.calls.append(("unload", key))

    def start(self, job: Job, sliced: bool) -> None:
        assert job.phantom_key in self.loaded
        self.live.append(job)
        self.peak = max(self.peak, self._mem())
        n = job.n_histories
        h = [self.chunk] * (n // self.chunk) + ([n % self.chunk] if n % self.chunk else [])
        job.item_hist = np.array(h, dtype=np.int64) if sliced else None
        job.n_items = len(h)
        job.state["covered"] = np.zeros(len(h), dtype=np.int32)

    def submit(self, job: Job, item_begin: int, item_end: int):
        assert job in self.live and job.phantom_key in self.loaded
        assert 0 <= item_begin < item_end <= job.n_items
        job.state["covered"][item_begin:item_end] += 1
        h = min(job.n_histories, item_end * self.chunk) - item_begin * self.chunk
        self.calls.append(("run", job.index, item_begin, item_end))
        # the device runs submissions one after another
        self.busy_until = max(self.busy_until, self.clock.now()) + self.overhead + h / self.rate
        return self.busy_until

    def finished(self, token) -> bool:
        return self.clock.now() >= token

    def progress(self, tokens, until: Optional[float] = None) -> None:
        t = min(tokens)
        if until is not None:
            t = min(t, until)
        self.clock.sleep_until(t)

    def finish(self, job: Job) -> None:
        assert np.all(job.state["covered"] == 1), "work items not covered exactly once"
        assert job.in_flight == 0
        self.calls.append(("finish", job.index))

    def release(self, job: Job) -> None:
        self.live = [j for j in self.live if j is not job]
        self.calls.append(("release", job.index))


# ----------------------------------------------------------------------------
# GPU executor
# ----------------------------------------------------------------------------

LUT_BYTES = 4096 * 2 * (4 + 8)  # per phase: density and stopping-power-ratio tables, FP32 and FP64


class GpuExecutor(Executor):
    """Runs jobs through libpmc on the current device; tallies and doses are
    torch-owned device buffers, phantoms and plans live in the context."""

    def __init__(self, ctx, phantoms: Dict[tuple, W.Phase], plans: Dict[int, W.Plan],
                 engine: int, launch: Optional[dict] = None, verify: bool = True,
                 keep_doses: bool = False, n_streams: int = 1, drain_signal: bool = True):
        import torch
        from . import pmc
        self.torch, self.pmc, self.ctx = torch, pmc, ctx
        self.phantoms = phantoms
        self.plans = plans
        self.engine = engine
        self.launch = dict(launch or {})
        self.verify = verify
        self.keep_doses = keep_doses
        self.slot_of: Dict[tuple, int] = {}
        self.free_slots = list(range(1023, -1, -1))
        # buffers, dose conversion and copies run on an I/O stream of their
        # own, and the host waits on events only: work on (or a wait for) the
        # null stream would also wait for the transport running on the others
        self.io = torch.cuda.Stream()
        # submissions go round robin to side streams (default priority): with
        # one stream, slices run back to back on the device while the host
        # prepares the next; with two, consecutive slices may overlap
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.next_stream = 0
        # drain signals of persistent launches (pinned host words the kernel
        # sets when every work item is taken): the scheduler then submits the
        # next slice, which waits on its stream for the running one to end
        persistent = engine == pmc.PMC_ENGINE_PERSISTENT
        self.drain_flags = (torch.zeros(64, dtype=torch.int32, pin_memory=True)
                            if drain_signal and persistent else None)
        self.free_flags = list(range(64))
        self.digests: Dict[int, str] = {}
        self.balances: Dict[int, dict] = {}
        self.doses: Dict[int, np.ndarray] = {}
        # pinned host buffers for the dose copies, by voxel count; a buffer is
        # reused once the digest of its previous dose is taken (worker thread)
        self.pinned: Dict[int, List] = {}
        self.pinned_lock = threading.Lock()
        self.hasher = concurrent.futures.ThreadPoolExecutor(max_workers=2)
        self.pending: List = []
        self.checks: List[tuple] = []  # balance checks waiting for their sums

    def close(self) -> None:
        """Finish the pending balance checks and digests."""
        self._check_balances(wait=True)
        for f in self.pending:
            f.result()
        self.pending.clear()
        self.hasher.shutdown(wait=True)

    def _host_buffer(self, nvox: int):
        with self.pinned_lock:
            free = self.pinned.setdefault(nvox, [])
            if free:
                return free.pop()
        return self.torch.empty(nvox, dtype=self.torch.float64, pin_memory=True)

    def _give_back(self, buf) -> None:
        with self.pinned_lock:
            self.pinned[buf.numel()].append(buf)

    def phantom_bytes(self, key) -> int:
        ph = self.phantoms[key]
        return ph.nvox * (2 + (ph.mask is not None)) + LUT_BYTES

    def job_bytes(self, job: Job) -> int:
        n_spots = len(self.plans[job.index].spots)
        # the library's default work item holds 64 to 256 histories
        items = job.n_histories // max(1, self.launch.get("chunk") or 64) + n_spots
        # tally + dose + counters; spot descriptors and core boxes, work items, LUT copy, targets
        return job.nvox * 16 + 128 + n_spots * 128 + items * 16 + 65536

    def load_phantom(self, key) -> None:
        if not self.free_slots:
            raise RuntimeError("all phase slots are in use")
        slot = self.free_slots.pop()
        self.pmc.pmc_load_phase(self.ctx, slot, self.phantoms[key])
        self.slot_of[key] = slot

    def unload_phantom(self, key) -> None:
        slot = self.slot_of.pop(key)
        self.pmc.pmc_unload_phase(self.ctx, slot)
        self.free_slots.append(slot)

    def start(self, job: Job, sliced: bool) -> None:
        torch, pmc = self.torch, self.pmc
        slot = self.slot_of[job.phantom_key]
        plan = self.plans[job.index]
        spots = plan.spots.copy()
        spots["phase"] = slot
        plan_id = job.index % 1024
        pmc.pmc_load_plan(self.ctx, plan_id, plan.fields, spots)
        persistent = self.engine == pmc.PMC_ENGINE_PERSISTENT
        kw = self.launch if persistent else {}
        req = pmc.Request(job.n_histories, [slot], request_id=job.index, engine=self.engine,
                          plan=plan_id, **kw)
        with torch.cuda.stream(self.io):
            job.state.update(req=req, plan_id=plan_id, slot=slot,
                             tally=torch.zeros(job.nvox, dtype=torch.int64, device="cuda"),
                             dose=torch.empty(job.nvox, dtype=torch.float64, device="cuda"),
                             counters=torch.zeros(pmc.PMC_COUNTERS, dtype=torch.int64, device="cuda"))
            zeroed = torch.cuda.Event()
            zeroed.record(self.io)
        if persistent:
            job.n_items = pmc.pmc_request_items(self.ctx, req)
            if sliced:
                job.item_hist = pmc.pmc_request_item_histories(self.ctx, req)
                if len(job.item_hist) != job.n_items:
                    raise RuntimeError("work-item count differs from the library's")
        else:
            job.n_items = 1
        for s in self.streams:  # the buffers are zero before a slice adds into them
            s.wait_event(zeroed)

    def submit(self, job: Job, item_begin: int, item_end: int):
        pmc, st = self.pmc, job.state
        req = st["req"]
        persistent = self.engine == pmc.PMC_ENGINE_PERSISTENT
        if persistent and (item_begin, item_end) != (0, job.n_items):
            req = req.slice(item_begin, item_end)
        stream = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        flag = None
        if persistent and self.drain_flags is not None and self.free_flags:
            flag = self.free_flags.pop()
            self.drain_flags[flag] = 0
            pmc.pmc_dose_device_notify(self.ctx, req, stream.cuda_stream, [st["tally"].data_ptr()],
                                       st["counters"].data_ptr(), self.drain_flags.data_ptr() + 4 * flag)
        else:
            pmc.pmc_dose_device(self.ctx, req, stream.cuda_stream, [st["tally"].data_ptr()],
                                st["counters"].data_ptr())
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return [ev, flag]

    def finished(self, token) -> bool:
        if not token[0].query():
            return False
        if token[1] is not None:  # the launch is over: its flag is free again
            self.free_flags.append(token[1])
            token[1] = None
        return True

    def drained(self, token) -> bool:
        if token[1] is not None and int(self.drain_flags[token[1]]) != 0:
            return True
        return self.finished(token)

    def progress(self, tokens, until: Optional[float] = None) -> None:
        if self.checks:
            self._check_balances()
        time.sleep(2e-5)

    def finish(self, job: Job) -> None:
        # the job's slices are complete (the scheduler waited for them)
        pmc, st, torch = self.pmc, job.state, self.torch
        pmc.pmc_convert_device(self.ctx, st["slot"], st["tally"].data_ptr(), job.n_histories,
                               self.io.cuda_stream, st["dose"].data_ptr(), None)
        buf = self._host_buffer(job.nvox)
        with torch.cuda.stream(self.io):
            buf.copy_(st["dose"], non_blocking=True)
            done = torch.cuda.Event()
            done.record(self.io)
        done.synchronize()  # served once the dose is on the host
        st["host_dose"] = buf

    def release(self, job: Job) -> None:
        pmc, st, torch = self.pmc, job.state, self.torch
        if not st:  # cancelled before it ever ran
            return
        buf = st.get("host_dose")
        if self.verify and buf is not None:
            # exact energy balance of the served tally, checked once the sums
            # arrive: the reduction may wait for CUs held by the next launch,
            # and the loop must not wait with it
            incident = pmc.pmc_balance_from_counters(self.ctx, st["req"], np.zeros(pmc.PMC_COUNTERS),
                                                     0)["incident"]
            t, counters = st["tally"], st["counters"]
            words = torch.empty(2 + pmc.PMC_COUNTERS, dtype=torch.int64, pin_memory=True)
            with torch.cuda.stream(self.io):
                dev = torch.cat([torch.stack(((t >> 32).sum(), (t & 0xFFFFFFFF).sum())), counters])
                words.copy_(dev, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.io)
            self.checks.append((job.index, job.n_histories, incident, words, ev, buf, (t, counters, dev)))
        elif buf is not None:
            self._give_back(buf)
        pmc.pmc_unload_plan(self.ctx, st["plan_id"])
        st.clear()
        self._check_balances()

    def _check_balances(self, wait: bool = False) -> None:
        """Energy balances whose sums have arrived (all of them with wait)."""
        keep = []
        for chk in self.checks:
            index, n_hist, incident, words, ev, buf, _ = chk
            if not wait and not ev.query():
                keep.append(chk)
                continue
            ev.synchronize()
            w = words.numpy().astype(np.uint64)
            b = self.pmc.balance_from_words(w[2:], (int(w[0]) << 32) + int(w[1]), incident)
            if b["deposited"] + b["escaped"] + b["nuclear"] != b["incident"]:
                raise RuntimeError(f"request {index}: energy balance broken {b}")
            if b["histories"] != n_hist:
                raise RuntimeError(f"request {index}: {b['histories']} histories run")
            self.balances[index] = b
            if self.keep_doses:
                self.doses[index] = buf.numpy().copy()

            def digest(index=index, buf=buf):
                self.digests[index] = hashlib.sha256(buf.numpy().data).hexdigest()
                self._give_back(buf)

            self.pending.append(self.hasher.submit(digest))
        self.checks = keep


# ----------------------------------------------------------------------------
# served stream
# ----------------------------------------------------------------------------

def _make_request_data(r: W.ServedRequest):
    return W.served_phantom(r), W.served_plan(r)


def build_stream(reqs: List[W.ServedRequest], workers: int = 0, log=None):
    """Phantoms and plans of a served stream, generated before serving starts.

    workers > 0 uses a pool of forked processes: call it before this process
    touches the GPU."""
    t0 = time.time()
    if workers > 0:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            data = pool.map(_make_request_data, reqs, chunksize=1)
    else:
        data = [_make_request_data(r) for r in reqs]
    phantoms: Dict[tuple, W.Phase] = {}
    plans: Dict[int, W.Plan] = {}
    for r, (ph, plan) in zip(reqs, data):
        phantoms.setdefault(r.phantom_key, ph)
        plans[r.index] = plan
    if log:
        log(f"generated {len(phantoms)} phantoms and {len(plans)} plans in {time.time() - t0:.1f} s")
    return phantoms, plans


def jobs_of(reqs: List[W.ServedRequest], phantoms) -> List[Job]:
    return [Job(r.index, r.arrival_s, r.n_histories, r.phantom_key, phantoms[r.phantom_key].nvox)
            for r in reqs]


def log_uniform_mean(lo: float, hi: float) -> float:
    return (hi - lo) / math.log(hi / lo)


def serve_gpu(ctx, reqs, phantoms, plans, engine: int, policy: str, budget: int,
              launch: Optional[dict] = None, slice_histories: int = 4_000_000, log=None,
              keep_doses: bool = False, depth: int = 1, rate_hist_per_s: float = 1.3e8,
              n_streams: int = 1, small_histories: float = 2.2e6, drain_signal: bool = True):
    """Serve `reqs` on the GPU in real time; returns (summary, executor, scheduler)."""
    ex = GpuExecutor(ctx, phantoms, plans, engine, launch, keep_doses=keep_doses, n_streams=n_streams,
                     drain_signal=drain_signal)
    sched = Scheduler(ex, WallClock(), budget, policy=policy, slice_histories=slice_histories,
                      log=log, depth=depth, rate_hist_per_s=rate_hist_per_s,
                      small_histories=small_histories)
    done = sched.run(jobs_of(reqs, phantoms))
    ex.close()
    s = summarize(done, policy)
    s["per_request"] = [[j.index, j.n_histories, j.arrival_s, j.first_run_s, j.done_s] for j in done]
    s.update(slices=sched.slices, evictions=sched.evictions, phantom_loads=sched.phantom_loads,
             peak_bytes=sched.peak_used, budget_bytes=budget, slices_in_flight=depth,
             streams=n_streams, drain_signal=ex.drain_flags is not None,
             slice_histories=slice_histories)
    return s, ex, sched


def calibrate_plain(ctx, seed: int, h_lo: float, h_hi: float, log=None, n: int = 12) -> float:
    """Service rate (histories/s) of the plain engine on a calibration set of
    served requests drawn with another seed: each request loaded, run, its
    dose copied to the host and everything freed, one after the other."""
    from . import pmc
    reqs = W.served_stream(n + 1, rate_hz=1.0, seed=seed + 1000, h_lo=h_lo, h_hi=h_hi)
    phantoms, plans = build_stream(reqs)
    ex = GpuExecutor(ctx, phantoms, plans, pmc.PMC_ENGINE_PLAIN, verify=False)
    total_h, total_t = 0, 0.0
    for k, j in enumerate(jobs_of(reqs, phantoms)):
        t0 = time.perf_counter()
        ex.load_phantom(j.phantom_key)
        ex.start(j, sliced=False)
        ex.run(j, 0, 1)
        ex.finish(j)
        ex.release(j)
        ex.unload_phantom(j.phantom_key)
        if k:  # the first request warms up the engine
            total_t += time.perf_counter() - t0
            total_h += j.n_histories
    ex.close()
    rate = total_h / total_t
    if log:
        log(f"plain service rate on the calibration set: {rate:.3g} histories/s")
    return rate


def prebuild(n_requests=200, seed=4, h_lo=1e5, h_hi=5e7, workers=0, log=None):
    """Requests (arrival times of a rate-1 Poisson process), phantoms and
    plans of a served stream; with workers > 0 call it before this process
    touches the GPU (forked generator processes)."""
    reqs0 = W.served_stream(n_requests, rate_hz=1.0, seed=seed, h_lo=h_lo, h_hi=h_hi)
    phantoms, plans = build_stream(reqs0, workers, log)
    return reqs0, phantoms, plans


def run_scenario(n_requests=200, load=0.8, seed=4, budget_bytes=0, h_lo=1e5, h_hi=5e7,
                 slice_histories=4_000_000, launch=None, workers=0, log=None, depth=1,
                 policy="small-first", plain=True, n_streams=2, prebuilt=None, small=2.2e6,
                 drain_signal=True):
    """Serve one Poisson stream with the sliced persistent engine (`policy`,
    `depth` slices in flight) and with the plain engine run serially in
    arrival order.  Arrival rate = load x plain throughput / mean request
    size.  Returns a dict of results."""
    if prebuilt is None:
        prebuilt = prebuild(n_requests, seed, h_lo, h_hi, workers, log)
    reqs0, phantoms, plans = prebuilt
    import torch
    from . import pmc
    free, _ = torch.cuda.mem_get_info()
    budget = int(budget_bytes or 0.9 * free)
    ctx = pmc.pmc_create(0, pmc.PMC_FP32, seed, budget)
    try:
        rate_plain = calibrate_plain(ctx, seed, h_lo, h_hi, log)
        lam = load * rate_plain / log_uniform_mean(h_lo, h_hi)
        # the same requests on the time axis of a rate-lam Poisson process
        reqs = [dataclasses.replace(r, arrival_s=r.arrival_s / lam) for r in reqs0]
        out = {"requests": n_requests, "load": load, "arrival_rate_hz": lam,
               "plain_calibration_hist_per_s": rate_plain, "budget_bytes": budget}
        execs = {}
        engines = [("batched", pmc.PMC_ENGINE_PERSISTENT, policy, depth)]
        if plain:
            engines.append(("plain-serial", pmc.PMC_ENGINE_PLAIN, "fifo", 1))
        for label, engine, pol, d in engines:
            s, ex, _ = serve_gpu(ctx, reqs, phantoms, plans, engine, pol, budget, launch,
                                 slice_histories, log, depth=d, rate_hist_per_s=rate_plain,
                                 n_streams=n_streams if engine == pmc.PMC_ENGINE_PERSISTENT else 1,
                                 small_histories=small, drain_signal=drain_signal)
            for key in list(ex.slot_of):
                ex.unload_phantom(key)
            out[label] = s
            execs[label] = ex
            if log:
                log(f"{label}: p50 {s['p50_latency_s'] * 1e3:.1f} ms, p99 "
                    f"{s['p99_latency_s'] * 1e3:.1f} ms, {s['throughput_hist_per_s']:.3g} histories/s")
        if plain:
            a, b = execs["batched"].digests, execs["plain-serial"].digests
            out["identical_doses"] = int(sum(a[k] == b.get(k) for k in a))
        return out
    finally:
        pmc.pmc_destroy(ctx)


def run_grid(n_requests=200, loads=(0.5, 0.8, 1.2), budgets=(0, 2 << 30), seed=4, h_lo=1e5, h_hi=5e7,
             slice_histories=4_000_000, launch=None, workers=0, log=None, policy="small-first",
             n_streams=2, prebuilt=None, small=2.2e6):
    """The same served stream at several loads and device-memory budgets.
    The plain engine's service rate is calibrated once; per load the stream
    is served once by the plain engine serially in arrival order (one
    request at a time: the budget does not change it) and once per budget by
    the batched loop (budget 0 = 0.9 x free device memory).  Every batched
    run's doses must equal the plain run's request by request."""
    if prebuilt is None:
        prebuilt = prebuild(n_requests, seed, h_lo, h_hi, workers, log)
    reqs0, phantoms, plans = prebuilt
    import torch
    from . import pmc
    free, _ = torch.cuda.mem_get_info()
    full = int(0.9 * free)
    ctx_full = pmc.pmc_create(0, pmc.PMC_FP32, seed, full)
    out = {"requests": n_requests, "scenarios": []}
    try:
        rate_plain = calibrate_plain(ctx_full, seed, h_lo, h_hi, log)
        out["plain_calibration_hist_per_s"] = rate_plain
        for load in loads:
            lam = load * rate_plain / log_uniform_mean(h_lo, h_hi)
            reqs = [dataclasses.replace(r, arrival_s=r.arrival_s / lam) for r in reqs0]
            s_plain, ex_plain, _ = serve_gpu(ctx_full, reqs, phantoms, plans, pmc.PMC_ENGINE_PLAIN, "fifo", full,
                                             None, slice_histories, log, rate_hist_per_s=rate_plain,
                                             n_streams=1, small_histories=small)
            for key in list(ex_plain.slot_of):
                ex_plain.unload_phantom(key)
            if log:
                log(f"load {load}: plain-serial p50 {s_plain['p50_latency_s'] * 1e3:.1f} ms, p99 "
                    f"{s_plain['p99_latency_s'] * 1e3:.1f} ms")
            for budget in budgets:
                b = int(budget or full)
                ctx = ctx_full if not budget else pmc.pmc_create(0, pmc.PMC_FP32, seed, b)
                try:
                    s, ex, _ = serve_gpu(ctx, reqs, phantoms, plans, pmc.PMC_ENGINE_PERSISTENT, policy, b, launch,
                                         slice_histories, log, rate_hist_per_s=rate_plain, n_streams=n_streams,
                                         small_histories=small)
                    for key in list(ex.slot_of):
                        ex.unload_phantom(key)
                finally:
                    if budget:
                        pmc.pmc_destroy(ctx)
                same = int(sum(ex.digests[k] == ex_plain.digests.get(k) for k in ex.digests))
                out["scenarios"].append({"load": load, "budget_bytes": b, "budget": "forced" if budget else "full",
                                         "arrival_rate_hz": lam, "batched": s, "plain_serial": s_plain,
                                         "identical_doses": same})
                if log:
                    log(f"load {load}, budget {b / 2**30:.1f} GiB: batched p50 {s['p50_latency_s'] * 1e3:.1f} ms, "
                        f"p99 {s['p99_latency_s'] * 1e3:.1f} ms, {s['throughput_hist_per_s']:.3g} histories/s; "
                        f"identical doses {same}/{len(ex.digests)}")
        return out
    finally:
        pmc.pmc_destroy(ctx_full)


def main():
    p = argparse.ArgumentParser(description="Serve a Poisson stream of dose requests on one GPU.")
    p.add_argument("--requests", type=int, default=200)
    p.add_argument("--load", type=float, default=0.8)
    p.add_argument("--budget-gb", type=float, default=0.0, help="0 = 0.9 x free device memory")
    p.add_argument("--seed", type=int, default=4)
    p.add_argument("--slice-histories", type=int, default=4_000_000)
    p.add_argument("--workers", type=int, default=8)
    p.add_argument("--depth", type=int, default=1, help="slices handing out work at once")
    p.add_argument("--no-drain-signal", action="store_true",
                   help="submit the next slice only when the running one has finished")
    p.add_argument("--streams", type=int, default=2,
                   help="submission streams (>= 2: the next slice starts while the previous drains)")
    p.add_argument("--policy", choices=["small-first", "slowdown", "srpt", "fifo"], default="small-first")
    p.add_argument("--small", type=float, default=2.2e6, help="small-first: largest small request")
    p.add_argument("--no-plain", action="store_true", help="skip the plain-serial comparison")
    p.add_argument("--block", type=int, default=0, help="persistent-engine block size (0 = library default)")
    p.add_argument("--tally-mode", choices=["auto", "lane", "core"], default="auto",
                   help="persistent-engine tally mode (auto: the library's choice)")
    p.add_argument("--per-request", action="store_true", help="keep per-request times in the output")
    a = p.parse_args()
    res = run_scenario(a.requests, a.load, a.seed, int(a.budget_gb * 2**30),
                       slice_histories=a.slice_histories, workers=a.workers, depth=a.depth,
                       policy=a.policy, plain=not a.no_plain, n_streams=a.streams, small=a.small,
                       drain_signal=not a.no_drain_signal,
                       launch=dict({"block_size": a.block} if a.block else {},
                                   tally_mode=["auto", "lane", "core"].index(a.tally_mode)),
                       log=lambda m: print("[serve]", m, file=sys.stderr, flush=True))
    if not a.per_request:
        for k in ("batched", "plain-serial"):
            if k in res:
                res[k].pop("per_request", None)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
