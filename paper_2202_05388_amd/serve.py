"""Serving loop: many greedy optimisation jobs resident on one GPU at once.

Jobs arrive over time (seeded Poisson stream).  A job is admitted when a slot is
free and its device footprint (G, E, FP64 diagonal, workspace) fits the HBM
budget; it then lives on its own HIP stream until its greedy trajectory ends
(no improving move) or it reaches its step budget, and its memory is released.
Every scheduler pass issues a chunk of steps to each resident job that has
fewer than two chunks in flight, so kernels of different jobs overlap on the
device, and polls progress without blocking (counters copied asynchronously to
pinned host memory; the copy's event is queried).  A job's refresh_G runs after
every `refresh_every` accepted moves.  Jobs share no device memory and use no
cross-job reductions, so a job's result does not depend on what else runs.

Per-step latency of a job = completion time of its step t minus that of step
t-1 (HIP events recorded after every step); per-job latency = completion of the
last step minus arrival.  `mode="serial"` runs the same jobs one at a time in
arrival order (the comparison point).

Grouped small jobs (`group_below` = N pixels, deferred mode): every resident job
of at most N pixels joins one group that lives on one stream; a step of the
group is one gfo_greedy_steps_table call, which moves every member with one
launch per move for all of them (a small job's move is a few microseconds of
device work, so per-job launches, not the device, bound a burst of them).  The
group's device job table is rebuilt when its membership changes, while none of
its steps is in flight.  A member's results are bit for bit those of the same
job run alone.
"""
from __future__ import annotations

import hashlib
import time
from dataclasses import dataclass, field

import numpy as np

from . import _lib as L
from .hiprt import hip
from .job import Job, JobGroup


@dataclass
class Result:
    job_id: int
    name: str
    arrival: float
    admitted: float = 0.0
    finished: float = 0.0
    steps: int = 0
    stopped: bool = False
    step_done: list = field(default_factory=list)   # completion times (s, serving clock)
    fom: float = 0.0
    digest: str = ""
    status: int = 0
    history: object = None                          # (pixel, material) of every accepted move


def footprint(problem, kmax: int) -> int:
    """Device bytes a job needs (G, E, diagonal, eps, workspace, small buffers)."""
    N = problem.ny * problem.nx
    R = N + problem.n_mon
    ld = (N + 63) // 64 * 64
    esz = 8 if problem.dtype == "c64" else 16
    import ctypes as C
    mon = np.ascontiguousarray(problem.monitor_xy()).reshape(-1)
    eps = np.ascontiguousarray(problem.eps_table, dtype=np.float64)
    pr = L.Problem(ny=problem.ny, nx=problem.nx, n_mon=problem.n_mon,
                   dtype=L.GFO_C64 if problem.dtype == "c64" else L.GFO_C128,
                   wavelength=problem.wavelength, pitch=problem.pitch, eps_bg=1.0,
                   h_mon_xy=mon.ctypes.data_as(C.POINTER(C.c_double)),
                   fom_monitor=problem.fom_monitor, n_eps=len(eps),
                   h_eps_table=eps.ctypes.data_as(C.POINTER(C.c_double)))
    work = L.workspace_size(pr, kmax)
    return R * ld * esz + R * esz + 16 * N + N + 8 * 4 * N + work + (1 << 20)


class _Active:
    def __init__(self, rec, job, stream, target, refresh_every, chunk):
        import torch
        self.rec = rec
        self.job = job
        self.stream = stream
        self.target = target
        self.refresh_every = refresh_every
        self.chunk = chunk
        self.issued = 0                 # step calls issued
        self.inflight = []              # [(event, pinned counters, issued_at_copy)]
        self.events = []                # per-step completion events
        self.accepted = 0
        self.done = False
        self.pinned = [torch.zeros(4, dtype=torch.int32, pin_memory=True) for _ in range(2)]
        self.slot = 0
        self.refreshed_at = 0           # issued-step count at the last refresh
        self.grouped = False            # stepped with the group of small jobs


class Server:
    """delay > 0 serves every job in deferred-update mode (flush every `delay` moves)."""

    def __init__(self, budget_bytes=288e9, max_slots=16, chunk=16, device="cuda:0", delay=0,
                 group_below=0, group_slots=48):
        self.budget = float(budget_bytes)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.device = device
        self.delay = int(delay)
        # jobs of at most `group_below` pixels are stepped as one group (deferred
        # mode only), up to `group_slots` of them at a time
        self.group_below = int(group_below) if delay > 0 else 0
        self.group_slots = int(group_slots)

    # ------------------------------------------------------------------ helpers
    def _issue(self, a: _Active, now_event):
        import torch
        left = a.target - a.issued
        n = min(a.chunk, left)
        if a.refresh_every and a.issued and a.issued % a.refresh_every == 0 \
                and a.refreshed_at != a.issued:
            return                              # wait until the boundary's refresh is enqueued
        if a.refresh_every:
            # stop the chunk at the next refresh boundary, assuming every step is accepted
            n = min(n, a.refresh_every - a.issued % a.refresh_every)
        if n <= 0:
            return
        with torch.cuda.stream(a.stream):
            for _ in range(n):
                # one step per call (fused kernels in deferred mode), so that every
                # step has its own completion event
                a.job.greedy_steps(1, stream=a.stream)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(a.stream)
                a.events.append(ev)
            a.issued += n
            buf = a.pinned[a.slot]
            a.slot ^= 1
            buf.copy_(a.job.counters, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(a.stream)
        a.inflight.append((ev, buf, a.issued))

    def _poll(self, a: _Active):
        """Consume finished progress reports; returns True if the job is complete."""
        while a.inflight and a.inflight[0][0].query():
            ev, buf, issued_at = a.inflight.pop(0)
            acc = int(buf[0].item())
            a.accepted = acc
            if acc < issued_at:                   # a step found no improving move
                a.rec.stopped = True
                return True
            if acc >= a.target:
                return True
            if a.refresh_every and acc % a.refresh_every == 0 and acc == issued_at:
                # every move up to the boundary is accepted and no later step was issued
                a.job.refresh(stream=a.stream)
                a.refreshed_at = issued_at
        return False

    def _finish(self, a: _Active, start_ev, t0):
        import torch
        a.stream.synchronize()
        acc = a.job.n_flips()
        rec = a.rec
        rec.steps = acc
        rec.status = a.job.status()
        rec.fom = a.job.fom()
        times = [start_ev.elapsed_time(ev) * 1e-3 for ev in a.events[:acc]]
        rec.step_done = times
        rec.finished = times[-1] if times else time.perf_counter() - t0
        E = a.job.E.cpu().numpy().tobytes()
        hist = a.job.history()
        rec.history = hist
        rec.digest = hashlib.sha256(E + hist.tobytes()).hexdigest()
        del a.job

    # ------------------------------------------------------------------ grouped jobs
    def _group_issue(self):
        """One chunk of steps for every member of the group (one table call per
        step, each followed by a completion event shared by the members)."""
        import torch
        members = self.members
        gs = self.gstream
        n = self.chunk
        for a in members:
            n = min(n, a.target - a.issued)
            if a.refresh_every:
                if a.issued and a.issued % a.refresh_every == 0 and a.refreshed_at != a.issued:
                    return                          # a member's refresh is not enqueued yet
                n = min(n, a.refresh_every - a.issued % a.refresh_every)
        if n <= 0:
            return
        with torch.cuda.stream(gs):
            for _ in range(n):
                self.group.steps(1, stream=gs)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(gs)
                for a in members:
                    a.events.append(ev)
            reports = []
            for a in members:
                a.issued += n
                buf = a.pinned[a.slot]
                a.slot ^= 1
                buf.copy_(a.job.counters, non_blocking=True)
                reports.append((a, buf, a.issued))
            ev = torch.cuda.Event()
            ev.record(gs)
        self.ginflight.append((ev, reports))

    def _group_poll(self):
        """Consume finished group chunks; returns the members that completed."""
        done = []
        while self.ginflight and self.ginflight[0][0].query():
            _, reports = self.ginflight.pop(0)
            for a, buf, issued_at in reports:
                if a.done:
                    continue
                acc = int(buf[0].item())
                a.accepted = acc
                if acc < issued_at:
                    a.rec.stopped = True
                    a.done = True
                elif acc >= a.target:
                    a.done = True
                elif a.refresh_every and acc % a.refresh_every == 0 and acc == issued_at:
                    a.job.refresh(stream=self.gstream)
                    a.refreshed_at = issued_at
                if a.done:
                    done.append(a)
        return done

    # ------------------------------------------------------------------ main loop
    def run(self, jobs, mode="mix", kmax=None, time_scale=1.0):
        """Serve `jobs` (list of workloads.Job).  Returns (results, summary)."""
        import torch
        torch.cuda.init()
        pending = sorted(jobs, key=lambda j: j.arrival)
        slots = self.max_slots if mode == "mix" else 1
        results = []
        active = []
        used = 0.0
        self.members = []                         # grouped jobs (their _Active records)
        self.group = JobGroup([], device=self.device)
        self.gstream = torch.cuda.Stream(device=self.device)
        self.ginflight = []
        self.gdirty = False
        start_ev = torch.cuda.Event(enable_timing=True)
        start_ev.record()
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            # admission
            while pending and pending[0].arrival * time_scale <= now:
                jb = pending[0]
                p = jb.problem
                # a small job joins the group (its own slot count); others need a slot
                grouped = (mode == "mix" and self.group_below and p.ny * p.nx <= self.group_below
                           and len(self.members) < self.group_slots)
                if not grouped and len(active) - len(self.members) >= slots:
                    break
                km = kmax if kmax is not None else p.steps
                fp = footprint(p, km)
                if used + fp > self.budget and active:
                    break
                pending.pop(0)
                used += fp
                rec = Result(jb.job_id, p.name, jb.arrival * time_scale, admitted=now)
                stream = torch.cuda.Stream(device=self.device)
                with torch.cuda.stream(stream):
                    # buffers are zero-filled on the job's own stream, ahead of init_G0
                    job = Job(p, device=self.device, kmax=km, flip_cap=p.steps + 8,
                              delay=self.delay)
                    job.init(stream=stream)
                a = _Active(rec, job, self.gstream if grouped else stream, p.steps,
                            p.refresh_every, self.chunk)
                a.fp = fp
                a.grouped = grouped
                if grouped:
                    stream.synchronize()           # the job is initialised before it joins
                    self.members.append(a)
                    self.gdirty = True
                active.append(a)
            if not active:
                if pending:
                    time.sleep(max(0.0, min(0.001, pending[0].arrival * time_scale - now)))
                continue
            progressed = False
            if self.members:
                for a in self._group_poll():
                    self._finish(a, start_ev, t0)
                    results.append(a.rec)
                    used -= a.fp
                    active.remove(a)
                    self.members.remove(a)
                    self.gdirty = True
                    progressed = True
                if self.members and not self.ginflight:
                    if self.gdirty:
                        self.group.set_jobs([a.job for a in self.members])
                        self.group.build(stream=self.gstream)
                        self.gdirty = False
                if self.members and not self.gdirty and len(self.ginflight) < 2:
                    self._group_issue()
                    progressed = True
            for a in list(active):
                if getattr(a, "grouped", False):
                    continue
                if self._poll(a):
                    self._finish(a, start_ev, t0)
                    results.append(a.rec)
                    used -= a.fp
                    active.remove(a)
                    progressed = True
                    continue
                if len(a.inflight) < 2 and a.issued < a.target:
                    self._issue(a, start_ev)
                    progressed = True
            if not progressed:
                time.sleep(20e-6)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return results, summarize(results, wall)


def summarize(results, wall):
    steps = sum(r.steps for r in results)
    lat = []
    for r in results:
        ts = [r.admitted] + r.step_done
        lat.extend(np.diff(ts[1:]).tolist() if len(ts) > 2 else [])
    job_lat = [r.finished - r.arrival for r in results]
    lat = np.array(lat) if lat else np.array([0.0])
    job_lat = np.array(job_lat) if job_lat else np.array([0.0])
    return dict(jobs=len(results), steps=steps, wall_s=wall, steps_per_s=steps / wall,
                step_p50_ms=1e3 * float(np.percentile(lat, 50)),
                step_p99_ms=1e3 * float(np.percentile(lat, 99)),
                job_p50_s=float(np.percentile(job_lat, 50)),
                job_p99_s=float(np.percentile(job_lat, 99)),
                stopped_early=sum(1 for r in results if r.stopped),
                nonzero_status=sum(1 for r in results if r.status))


def serve_benchmark(n_jobs=64, rate=4.0, seed=0, max_slots=16, chunk=16, time_scale=1.0, delay=64,
                    group_below=96 * 96):
    """The served workload: a seeded Poisson stream of jobs (grid side 24..160,
    wavelength 0.8..1.2, 200..1000 step budget, complex64, refresh every 256),
    served concurrently (per-job streams, and with the jobs of at most
    `group_below` pixels grouped) and, for comparison, one at a time in arrival
    order; then the same jobs all arriving at once (a burst)."""
    import workloads as W
    jobs = W.served_jobs(n_jobs=n_jobs, rate=rate, seed=seed)
    kw = dict(chunk=chunk, delay=delay)
    mix, smix = Server(max_slots=max_slots, **kw).run(jobs, mode="mix", time_scale=time_scale)
    gmix, sgmix = Server(max_slots=max_slots, group_below=group_below, **kw).run(
        jobs, mode="mix", time_scale=time_scale)
    ser, sser = Server(max_slots=1, **kw).run(jobs, mode="serial", time_scale=time_scale)
    # the same jobs all arriving at once: throughput of the device, not of the arrival process
    bmix, sbmix = Server(max_slots=max_slots, **kw).run(jobs, mode="mix", time_scale=0.0)
    bgmix, sbgmix = Server(max_slots=max_slots, group_below=group_below, **kw).run(
        jobs, mode="mix", time_scale=0.0)
    bser, sbser = Server(max_slots=1, **kw).run(jobs, mode="serial", time_scale=0.0)
    ds = {r.job_id: r.digest for r in ser}
    same = sum(1 for rs in (mix, gmix, bmix, bgmix) for r in rs if r.digest == ds.get(r.job_id))
    refreshed = sum(1 for r in ser if r.steps >= 256)
    return dict(jobs=n_jobs, rate_per_s=rate, seed=seed, max_slots=max_slots, delay=delay,
                group_below_pixels=group_below,
                grouped_jobs=sum(1 for j in jobs if j.problem.n <= group_below),
                mix=smix, mix_grouped=sgmix, one_at_a_time=sser, burst_mix=sbmix,
                burst_mix_grouped=sbgmix, burst_one_at_a_time=sbser,
                results_identical=f"{same}/{4 * len(ds)}",
                jobs_reaching_a_refresh=refreshed)
