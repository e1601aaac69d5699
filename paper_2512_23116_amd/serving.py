"""Continuous-batching request loop for independent LES runs on one GPU.

Requests (lattice size, Smagorinsky C, tau0, forcing seed, step count) arrive
over time.  The loop admits a waiting request as soon as a slot is free and its
population state fits the HBM budget, keeps every admitted lattice resident on
the device, and advances all active lattices together with ``lbm_batch_step``
(one captured HIP graph of ``steps_per_graph`` batched launches per call).
The active lattices are stepped in groups whose states together fit the GPU's
last-level cache (256 MB Infinity Cache on MI355X), one batched call per group:
a group then takes its steps on chip instead of every launch streaming all
slots through HBM.
Requests that arrive while others run join at the next call; finished ones
leave and free their slot and memory.  Two batched calls are kept in flight:
the next one is enqueued before the loop waits for the oldest, and lattices are
set up and read out on a side stream, so the device is not idle while the host
admits and completes requests.  Latency = completion - arrival.

The engine behind the loop is pluggable: ``GpuEngine`` drives liblbm.so,
``FakeEngine`` simulates durations on the host so the scheduling logic is
tested without a GPU.
"""
import time
from dataclasses import dataclass, field

import numpy as np

from . import params
from .inputs import random_solenoidal_modes

# State bytes per batched call: below the 256 MB last-level cache of MI355X.
GROUP_BYTES = 192 << 20


@dataclass
class Request:
    rid: int
    N: int
    C: float
    tau0: float
    force_seed: int
    init_seed: int
    arrival: float
    steps: int = 5000
    # filled by the loop
    admit: float = None
    complete: float = None
    done_steps: int = 0
    error: str = None
    result: dict = field(default_factory=dict)

    @property
    def cells(self):
        return self.N ** 3

    @property
    def state_bytes(self):
        return 19 * self.cells * 4          # FP32, AA in place

    @property
    def latency(self):
        return None if self.complete is None else self.complete - self.arrival


def cache_groups(reqs, steps, group_bytes):
    """Split (request, steps) pairs into groups of at most `group_bytes` of state:
    first fit in order of decreasing state size (ties by request id); a state
    larger than `group_bytes` forms a group of its own.  None or 0 = one group."""
    pairs = list(zip(reqs, steps))
    if not group_bytes:
        return [pairs] if pairs else []
    groups, room = [], []
    for r, s in sorted(pairs, key=lambda p: (-p[0].state_bytes, p[0].rid)):
        for g in range(len(groups)):
            if r.state_bytes <= room[g]:
                groups[g].append((r, s))
                room[g] -= r.state_bytes
                break
        else:
            groups.append([(r, s)])
            room.append(group_bytes - r.state_bytes)
    return groups


class GpuEngine:
    """Runs requests as FP32/AA lattices batched through liblbm.so, one batched
    call per cache-sized group of lattices (`group_bytes`, None = all at once).

    The batched calls run on the main stream.  Lattices are set up (allocation,
    force tables, initial state) and read out at the end (statistics, optional
    checkpoint, release) on a side stream, ordered against the main stream by
    events, so neither waits for the batched steps in flight."""

    def __init__(self, max_slots=16, steps_per_graph=64, noise=1e-3, group_bytes=GROUP_BYTES):
        import torch
        from . import lbm
        self.torch = torch
        self.lbm = lbm
        self.stream = torch.cuda.Stream()
        self.side = torch.cuda.Stream()
        self.G = steps_per_graph
        self.noise = noise
        self.group_bytes = group_bytes
        self.batch = lbm.lbm_batch_create(max_slots, steps_per_graph, self.stream.cuda_stream)
        self.lat = {}
        self.calls = []          # (start event, end event) of every batched call

    def admit(self, r):
        F0 = params.forcing_amplitude(r.N)
        modes = random_solenoidal_modes(F0, r.force_seed)
        lat = self.lbm.Lattice((r.N, r.N, r.N), r.tau0, r.C, modes, precision="fp32",
                               streaming="aa", smag_form=params.SMAG_FORM,
                               steps_per_graph=self.G, stream=self.side)
        lat.init(self.lbm.LBM_INIT_NOISE, self.noise, r.init_seed)
        # the main stream runs the lattice's steps after its initial state is written
        self.stream.wait_stream(self.side)
        lat.set_stream(self.stream)
        self.lat[r.rid] = lat

    def step(self, reqs, steps):
        """Enqueue one batched call; returns its token (end event)."""
        ev = self.torch.cuda.Event
        start, end = ev(enable_timing=True), ev(enable_timing=True)
        start.record(self.stream)
        # back-to-back calls on one stream: the library waits for the previous
        # call's slot-table copy before it rewrites the table
        for group in cache_groups(reqs, steps, self.group_bytes):
            self.lbm.lbm_batch_step(self.batch, [self.lat[r.rid].handle for r, _ in group],
                                    [s for _, s in group])
        end.record(self.stream)
        self.calls.append((start, end))
        return end

    def wait(self, token=None):
        if token is None:
            self.stream.synchronize()
        else:
            token.synchronize()

    def finish(self, r, token, keep_state=False):
        """Statistics (and checkpoint) of a request whose last batched call is
        `token`, read on the side stream while later calls run on the main one."""
        lat = self.lat.pop(r.rid)
        self.side.wait_event(token)
        lat.set_stream(self.side)
        st = lat.stats(allow_unstable=True)
        r.result = dict(stats=st)
        if keep_state:
            r.result["state"] = lat.save()[0]
        lat.close()

    def busy_seconds(self):
        """GPU time of the batched calls so far (HIP events on the main stream)."""
        self.stream.synchronize()
        return sum(a.elapsed_time(b) for a, b in self.calls) / 1e3

    def close(self):
        self.wait()
        self.side.synchronize()
        for lat in self.lat.values():
            lat.close()
        self.lat.clear()
        self.lbm.lbm_batch_destroy(self.batch)


class FakeEngine:
    """Host-only engine on a simulated device timeline: a call takes
    sum(cells * steps) / rate seconds and starts when the previous one ends (or
    when it is issued, if later); waiting on its token sleeps until its end."""

    def __init__(self, rate=3e10, max_slots=16, steps_per_graph=64, fail_rids=(),
                 clock=time.perf_counter):
        self.rate = rate
        self.G = steps_per_graph
        self.fail_rids = set(fail_rids)
        self.clock = clock
        self.active = {}
        self.calls = []
        self.spans = []
        self.free_at = 0.0

    def admit(self, r):
        if r.rid in self.fail_rids:
            raise RuntimeError(f"admission of request {r.rid} failed")
        self.active[r.rid] = r

    def step(self, reqs, steps):
        self.calls.append([(r.rid, s) for r, s in zip(reqs, steps)])
        dur = sum(r.cells * s for r, s in zip(reqs, steps)) / self.rate
        start = max(self.clock(), self.free_at)
        self.free_at = start + dur
        self.spans.append((start, self.free_at))
        return self.free_at

    def wait(self, token=None):
        end = self.free_at if token is None else token
        delay = end - self.clock()
        if delay > 0:
            time.sleep(delay)

    def finish(self, r, token, keep_state=False):
        self.active.pop(r.rid, None)
        r.result = dict(stats=None)

    def busy_seconds(self):
        return sum(b - a for a, b in self.spans)

    def close(self):
        self.active.clear()


def serve(requests, engine, max_slots=16, hbm_budget=80e9, keep_state=False, clock=None,
          depth=2):
    """Run the request loop until every request has completed or failed.

    Up to `depth` batched calls are in flight: the next call is enqueued before
    the loop waits for the oldest one, so admissions, completions and the host's
    bookkeeping overlap with device work.  A request's steps are scheduled call
    by call (at most steps_per_graph each); it completes when the call holding
    its last steps has finished, and its result is read while later calls run.

    Returns a summary dict: p50/p99 latency (split into queueing and service),
    aggregate MLUPS over the span from the first arrival, the device-busy
    fraction of that span and of the time work was present (some request
    waiting, active or in flight), and the per-request records.
    """
    from collections import deque
    clock = clock or time.perf_counter
    pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
    waiting = []          # FIFO of arrived, not admitted requests
    active = []           # admitted requests with steps not yet finished
    sched = {}            # rid -> steps enqueued so far
    inflight = deque()    # (token, [(request, steps)])
    used = 0
    t0 = clock()
    i = 0
    cell_updates = 0
    work_s = 0.0
    G = engine.G
    last = clock()
    while i < len(pending) or waiting or active or inflight:
        now = clock()
        if waiting or active or inflight:
            work_s += now - last
        last = now
        now -= t0
        while i < len(pending) and pending[i].arrival <= now:
            waiting.append(pending[i])
            i += 1
        # admission: FIFO, by free slot and HBM budget
        while waiting and len(active) < max_slots and used + waiting[0].state_bytes <= hbm_budget:
            r = waiting.pop(0)
            try:
                engine.admit(r)
            except Exception as e:          # a request that cannot start fails alone
                r.error = str(e)
                r.complete = clock() - t0
                continue
            r.admit = clock() - t0
            sched[r.rid] = 0
            used += r.state_bytes
            active.append(r)
        if waiting and not active and not inflight and waiting[0].state_bytes > hbm_budget:
            r = waiting.pop(0)
            r.error = "state larger than the HBM budget"
            r.complete = clock() - t0
            continue
        todo = [(r, min(G, r.steps - sched[r.rid])) for r in active if sched[r.rid] < r.steps]
        if todo and len(inflight) < depth:
            token = engine.step([r for r, _ in todo], [s for _, s in todo])
            for r, s in todo:
                sched[r.rid] += s
            inflight.append((token, todo))
            continue
        if inflight:
            token, calls = inflight.popleft()
            engine.wait(token)
            for r, s in calls:
                r.done_steps += s
                cell_updates += r.cells * s
            still = []
            for r in active:
                if r.done_steps >= r.steps:
                    engine.finish(r, token, keep_state)
                    r.complete = clock() - t0
                    used -= r.state_bytes
                else:
                    still.append(r)
            active = still
            continue
        if i < len(pending):
            delay = pending[i].arrival - (clock() - t0)
            if delay > 0:
                time.sleep(min(delay, 0.01))
    t_end = clock() - t0
    busy = engine.busy_seconds()
    done = [r for r in requests if r.error is None and r.latency is not None]
    lat = np.array([r.latency for r in done])
    wait = np.array([r.admit - r.arrival for r in done])
    service = np.array([r.complete - r.admit for r in done])
    first = min(r.arrival for r in requests) if requests else 0.0
    span = max(t_end - first, 1e-12)
    return dict(
        n=len(requests), failed=sum(r.error is not None for r in requests),
        p50_s=float(np.percentile(lat, 50)) if lat.size else None,
        p99_s=float(np.percentile(lat, 99)) if lat.size else None,
        mean_s=float(lat.mean()) if lat.size else None,
        # latency = queueing (arrival -> admission) + service (admission -> completion)
        wait_p50_s=float(np.percentile(wait, 50)) if wait.size else None,
        wait_p99_s=float(np.percentile(wait, 99)) if wait.size else None,
        service_p50_s=float(np.percentile(service, 50)) if service.size else None,
        service_p99_s=float(np.percentile(service, 99)) if service.size else None,
        wall_s=t_end, busy_s=busy, busy_frac=busy / span,
        work_s=work_s, busy_frac_when_work=busy / max(work_s, 1e-12),
        cell_updates=cell_updates,
        aggregate_mlups=cell_updates / span / 1e6,
        busy_mlups=cell_updates / max(busy, 1e-12) / 1e6,
    )


def make_requests(n=64, seed=2024, steps=5000, rate=None, sizes=(32, 48, 64, 96, 128)):
    """The seeded serving workload: sizes uniform over ``sizes``, C in [0.08, 0.18],
    tau0 in [0.505, 0.55], per-request forcing and noise seeds, Poisson arrivals."""
    from .inputs import serving_requests
    return [Request(rid=d["rid"], N=d["N"], C=d["C"], tau0=d["tau0"],
                    force_seed=d["force_seed"], init_seed=d["init_seed"],
                    arrival=d["arrival"], steps=steps)
            for d in serving_requests(n, seed, sizes=sizes, rate=rate)]
