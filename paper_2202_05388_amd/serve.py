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
"""
from __future__ import annotations

import hashlib
import time
from dataclasses import dataclass, field

import numpy as np

from . import _lib as L
from .hiprt import hip
from .job import Job


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


class Server:
    """delay > 0 serves every job in deferred-update mode (flush every `delay` moves)."""

    def __init__(self, budget_bytes=288e9, max_slots=16, chunk=16, device="cuda:0", delay=0):
        self.budget = float(budget_bytes)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.device = device
        self.delay = int(delay)

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
        H = a.job.history().tobytes()
        rec.digest = hashlib.sha256(E + H).hexdigest()
        del a.job

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
        start_ev = torch.cuda.Event(enable_timing=True)
        start_ev.record()
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            # admission
            while pending and pending[0].arrival * time_scale <= now and len(active) < slots:
                jb = pending[0]
                p = jb.problem
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
                a = _Active(rec, job, stream, p.steps, p.refresh_every, self.chunk)
                a.fp = fp
                active.append(a)
            if not active:
                if pending:
                    time.sleep(max(0.0, min(0.001, pending[0].arrival * time_scale - now)))
                continue
            progressed = False
            for a in list(active):
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


def serve_benchmark(n_jobs=64, rate=4.0, seed=0, max_slots=16, chunk=16, time_scale=1.0, delay=64):
    """The served workload: a seeded Poisson stream of jobs (grid side 24..160,
    wavelength 0.8..1.2, 200..1000 step budget, complex64, refresh every 256),
    served concurrently and, for comparison, one at a time in arrival order."""
    import workloads as W
    jobs = W.served_jobs(n_jobs=n_jobs, rate=rate, seed=seed)
    kw = dict(chunk=chunk, delay=delay)
    mix, smix = Server(max_slots=max_slots, **kw).run(jobs, mode="mix", time_scale=time_scale)
    ser, sser = Server(max_slots=1, **kw).run(jobs, mode="serial", time_scale=time_scale)
    # the same jobs all arriving at once: throughput of the device, not of the arrival process
    bmix, sbmix = Server(max_slots=max_slots, **kw).run(jobs, mode="mix", time_scale=0.0)
    bser, sbser = Server(max_slots=1, **kw).run(jobs, mode="serial", time_scale=0.0)
    dm = {r.job_id: r.digest for r in mix}
    ds = {r.job_id: r.digest for r in ser}
    db = {r.job_id: r.digest for r in bmix}
    same = sum(1 for k in dm if dm[k] == ds.get(k) == db.get(k))
    return dict(jobs=n_jobs, rate_per_s=rate, seed=seed, max_slots=max_slots, delay=delay,
                mix=smix, one_at_a_time=sser, burst_mix=sbmix, burst_one_at_a_time=sbser,
                results_identical=f"{same}/{len(dm)}")
