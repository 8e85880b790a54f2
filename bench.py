#!/usr/bin/env python3
"""Greedy-step throughput of the Green's-function pixel-by-pixel optimiser on one MI355X.

A step is one pass of the hot path: score every candidate flip + select the
argmax (score_candidates) + rank-1 Dyson update of G, E and the FP64
diagonal (apply_flip).  The default workload is the 128x128-pixel grid with 64
monitors, complex64 storage and an FP64 refresh every 256 accepted moves.  The
greedy trajectory of that problem ends after 190 accepted moves (no move
improves the FOM any more), so the benchmark restarts the job (init_G0, inside
the timed region) whenever it stops, and counts accepted moves only.

Prints one JSON line.  The streaming rank-1 kernel is timed alone with HIP
events recorded on its own stream around every launch of the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

MFMA_PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6}     # dense FP32 / FP64 matrix peaks
BF16_PEAK_TFLOPS = 2500.0                           # dense BF16 matrix peak

# HBM traffic per launch from rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE in KiB
# per dispatch), each scaled by what the same counter reports for a device copy of
# exactly 2 GiB (FETCH 1048599.75 KiB -> factor 2.0; WRITE 2097152 KiB -> factor
# 1.0).  A record is valid only for the kernel source and variant it was measured
# on: any change to that source's code (comments and whitespace aside) voids it
# (traffic is then reported as null).
# Counters: profiles/k_rank1_square128_c64.md and profiles/deferred_step_square128_c64.md.
FETCH_SCALE = 2097152.0 / 1048599.75
WRITE_SCALE = 1.0
PMC_TRAFFIC = [
    {"kernel": "k_rank1", "source": "paper_2202_05388_amd/csrc/gfo_rank1.hip", "code_sha256": "a6b6efb2897f6b048c0d7845fc1fb0c76a7153786a46e94aefbd8df1e5a847d9", "workload": "square128_c64", "variant": "2x1x1_nt", "fetch_kib": 1053784.0, "write_kib": 2105344.0},
    # complex64 flush records: one per term bucket (the launcher's kernel for up to 16, 32, 64
    # or 128 pending terms) of the default variant, each taken on flushes that fold the
    # bucket's full term count: the tile kernel, then the pack kernel
    {"kernel": "k_flush_c64", "source": "paper_2202_05388_amd/csrc/gfo_flush.hip", "code_sha256": "467dc02667036d6a9a06a30b399e3413a41a0aeebbb56137dcf67f5f431dbc44", "workload": "square128_c64", "variant": "up_bandseg_s3", "bucket": 16, "tile_kernel": "k_flush_c64_pair<4, 4, true>", "fetch_kib": 539642.0 + 2065.0, "write_kib": 1060921.4 + 4104.0},
    {"kernel": "k_flush_c64", "source": "paper_2202_05388_amd/csrc/gfo_flush.hip", "code_sha256": "467dc02667036d6a9a06a30b399e3413a41a0aeebbb56137dcf67f5f431dbc44", "workload": "square128_c64", "variant": "up_bandseg_s3", "bucket": 32, "tile_kernel": "k_flush_c64_s3<2>", "fetch_kib": 562021.2 + 4135.0, "write_kib": 1060888.1 + 12312.0},
    {"kernel": "k_flush_c64", "source": "paper_2202_05388_amd/csrc/gfo_flush.hip", "code_sha256": "467dc02667036d6a9a06a30b399e3413a41a0aeebbb56137dcf67f5f431dbc44", "workload": "square128_c64", "variant": "up_bandseg_s3", "bucket": 64, "tile_kernel": "k_flush_c64_s3<4>", "fetch_kib": 620708.7 + 8237.0, "write_kib": 1060870.4 + 24624.0},
    {"kernel": "k_flush_c64", "source": "paper_2202_05388_amd/csrc/gfo_flush.hip", "code_sha256": "467dc02667036d6a9a06a30b399e3413a41a0aeebbb56137dcf67f5f431dbc44", "workload": "square128_c64", "variant": "up_bandseg_s3", "bucket": 128, "tile_kernel": "k_flush_c64_s3<8>", "fetch_kib": 1014278.6 + 16452.1, "write_kib": 1060904.5 + 49248.0},
]


def code_hash(path):
    """SHA-256 of a C++/HIP source with its comments and whitespace removed: the
    code a record was measured on, whatever its comments say since."""
    import hashlib
    with open(path, encoding="utf-8") as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return hashlib.sha256(" ".join(text.split()).encode()).hexdigest()


def pmc_traffic(kernel, workload, variant, bucket=None):
    for rec in PMC_TRAFFIC:
        if (rec["kernel"], rec["workload"], rec["variant"]) != (kernel, workload, variant):
            continue
        if rec.get("bucket") != bucket:
            continue
        if code_hash(os.path.join(ROOT, rec["source"])) != rec["code_sha256"]:
            return None
        return 1024.0 * (rec["fetch_kib"] * FETCH_SCALE + rec["write_kib"] * WRITE_SCALE)
    return None


def flush_bucket(terms):
    """Term bucket of a complex64 flush: the launcher runs one kernel for up to
    16, 32, 64 and 128 pending terms."""
    for b in (16, 32, 64):
        if terms <= b:
            return b
    return 128


def flush_traffic(workload, variant, terms):
    """Mean counter traffic per flush over flushes folding `terms` terms each,
    from the bucket records; None if a bucket has no current record."""
    if not terms:
        return None
    vals = [pmc_traffic("k_flush_c64", workload, variant, flush_bucket(t)) for t in terms]
    return None if any(v is None for v in vals) else sum(vals) / len(vals)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


# extra columns of G beyond the minimum leading dimension (--ld-pad)
LD_PAD = 0


def run_steps(job, target, poll, events=None, refresh_every=0, flush_events=None, fused=False):
    """Issue greedy steps until `target` accepted moves; re-init a job that stopped.
    fused: each chunk of steps is one gfo_greedy_steps call.

    flush_events: an EventPool; every flush in the window is timed with a pair
    of its events (the flush a chunk ends with, the flush before a restart and
    the one at the end), and the number of terms it folds (accepted moves since
    the previous flush, refresh or init) is recorded in flush_events.terms.

    Returns (accepted, calls, restarts, accepted_flags) where accepted_flags[i]
    tells whether step call i made a move.
    """
    from paper_2202_05388_amd import _lib as L

    accepted = 0
    calls = 0
    restarts = 0
    flags = []
    in_run_acc = job.n_flips()
    since_flush = 0                         # accepted moves not yet folded into G
    if flush_events is not None and not hasattr(flush_events, "terms"):
        flush_events.terms = []

    def timed_flush():
        nonlocal since_flush
        if job.delay and job.state.pending_calls > 0:
            if flush_events is not None:
                a, b = flush_events.next()
                L.time_next_k1(a, b)
                flush_events.terms.append(since_flush)
            job.flush()
        since_flush = 0

    while accepted < target:
        chunk = min(poll, target - accepted)
        if refresh_every:
            chunk = min(chunk, refresh_every - in_run_acc % refresh_every)
        # every call counts toward the flush interval: a chunk that reaches it
        # launches exactly one flush (chunk <= delay)
        flushes = bool(job.delay) and job.state.pending_calls + chunk >= job.delay
        if fused:
            if flush_events is not None and flushes:
                a, b = flush_events.next()
                L.time_next_k1(a, b)
            job.greedy_steps(chunk)
        else:
            for _ in range(chunk):
                if events is not None:
                    a, b = events.next()
                    L.time_next_k1(a, b)
                elif flush_events is not None and job.state.pending_calls == job.delay - 1:
                    a, b = flush_events.next()       # this step's apply_flip ends with a flush
                    L.time_next_k1(a, b)
                job.step()
        calls += chunk
        n = job.n_flips()                     # host sync
        new = n - in_run_acc
        flags.extend([True] * new + [False] * (chunk - new))
        accepted += new
        in_run_acc = n
        since_flush += new
        if flushes:
            folded = min(job.delay, since_flush)
            if flush_events is not None:
                flush_events.terms.append(folded)
            since_flush -= folded
        if new < chunk:                        # the trajectory ended: restart the job
            timed_flush()                      # apply every accepted move to G before discarding it
            job.init()
            restarts += 1
            in_run_acc = 0
        elif refresh_every and in_run_acc % refresh_every == 0:
            job.refresh()                      # rebuilds G from every accepted move
            since_flush = 0
    timed_flush()                              # no pending update is left outside the timed work
    return accepted, calls, restarts, flags


def flush_triangle(variant):
    """'up': the upper triangle alone is kept current; None: every tile."""
    return "up" if str(variant).startswith("up") else None


def flush_covers_monitors(variant):
    """The pair-interleaved flushes (pair and band forms) update the monitor rows
    in the same kernel."""
    return str(variant).startswith(("up_pair", "up_band"))


def flush_alg_bytes(variant, dtype, N, ld, n_mon=0):
    """Minimal HBM bytes of one flush of the N x ld design block.  complex64:
    the whole block read and written (16 N ld) or, keeping only the upper
    triangle, half of it (8 N ld); plus the monitor rows (16 n_mon ld) for a
    variant that updates them in the same kernel.  complex128 (FP64 flush of the
    upper triangle and the monitor rows): 16 N ld + 32 n_mon ld."""
    if dtype != "c64":
        return 16 * N * ld + 32 * n_mon * ld
    mon = 16 * n_mon * ld if flush_covers_monitors(variant) else 0
    return {"up": 8, None: 16}[flush_triangle(variant)] * N * ld + mon


def flush_split(variant, dtype, terms):
    """True when the flush of `terms` terms runs the split-product kernel (FP32
    products as six BF16 part products; the launcher takes it for 17 to 128
    terms and the pair flush for up to 16)."""
    return dtype == "c64" and str(variant) == "up_bandseg_s3" and 16 < terms <= 128


def flush_mfma_flops(variant, dtype, N, ld, n_mon, terms):
    """Matrix-core flops of one flush that folds `terms` pending terms: real
    flops of the complex products over the 64 x 64 tiles the kernel computes
    (for the triangle variants and the complex128 flush, the tiles on and above
    the diagonal of the design block, plus the monitor rows where the kernel
    covers them), 2 flops per real product and three real products per complex
    one in the _3m variants (four otherwise); the split-product kernel issues
    four real products per complex one, each as six BF16 part products.  Only
    the terms actually folded count, not the zero padding up to the kernel's
    term bucket."""
    nb = (N + 63) // 64
    if dtype != "c64":
        tiles = nb * (nb + 1) // 2 + (n_mon + 63) // 64 * (ld // 64)
        per = 8
    else:
        tri = flush_triangle(variant)
        tiles = nb * (nb + 1) // 2 if tri else nb * (ld // 64)
        if flush_covers_monitors(variant):
            tiles += (n_mon + 63) // 64 * (ld // 64)
        # the split variant runs the three-product pair flush for up to 16 terms
        three = "3m" in str(variant) or str(variant) == "up_bandseg_s3"
        per = 48 if flush_split(variant, dtype, terms) else 6 if three else 8
    return float(per) * 64 * 64 * tiles * terms


def flush_mfma_peak(variant, dtype, terms):
    """Dense matrix peak (TFLOP/s) of the instructions the flush of `terms` terms issues."""
    return BF16_PEAK_TFLOPS if flush_split(variant, dtype, terms) else MFMA_PEAK_TFLOPS[dtype]


def flush_roofline(variant, dtype, N, ld, n_mon, terms, ms):
    """Roofline of the flushes of a timed window: every flush's matrix-core
    flops (from the terms it folds) and minimal HBM bytes, summed, against the
    summed kernel time; the bound is the larger of the two ideal times."""
    if not ms:
        return None
    fl = [flush_mfma_flops(variant, dtype, N, ld, n_mon, r) for r in terms]
    flops = sum(fl)
    nbytes = flush_alg_bytes(variant, dtype, N, ld, n_mon) * len(ms)
    secs = sum(ms) * 1e-3
    # each flush's matrix work at the peak of the instructions it issues
    t_mfma = sum(f / (flush_mfma_peak(variant, dtype, r) * 1e12) for f, r in zip(fl, terms))
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    peak = flops / t_mfma / 1e12 if t_mfma > 0 else MFMA_PEAK_TFLOPS[dtype]
    common = dict(avg_launch_us=1e6 * secs / len(ms), launches=len(ms),
                  mean_terms=sum(terms) / len(terms), mfma_flops_per_launch=flops / len(ms),
                  algorithmic_bytes_per_launch=nbytes / len(ms), variant=variant)
    if t_hbm >= t_mfma:
        a = nbytes / secs / 1e9
        return dict(bound="hbm", achieved=a, peak=HBM_PEAK_GBS, unit="GB/s", frac=a / HBM_PEAK_GBS,
                    **common)
    a = flops / secs / 1e12
    return dict(bound="mfma", achieved=a, peak=peak, unit="TFLOP/s", frac=a / peak, **common)


def copy_ceiling(nbytes=2 << 30, reps=10):
    """Device-to-device copy bandwidth (read + write bytes / time) with torch's copy kernel."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def time_workload(problem, steps, warmup, poll, with_events=True, autotune=True, upper=False):
    import torch
    from paper_2202_05388_amd.hiprt import EventPool
    from paper_2202_05388_amd.job import Job
    from paper_2202_05388_amd import autotune as at

    kmax = max(problem.refresh_every, 0) * 2 if problem.refresh_every else 0
    job = Job(problem, device="cuda:0", kmax=kmax, ld_pad=LD_PAD, upper=upper)
    job.init()
    tuned = None
    if autotune:
        tuned = at.tune(job, reps=6, save=False)
        _log(f"[bench] autotune {problem.dtype}: {tuned['name']} {tuned['us']:.1f} us "
             f"({tuned['gbs']:.0f} GB/s) in {tuned['seconds']:.1f} s")
        job.init()
    if warmup:
        run_steps(job, warmup, poll, refresh_every=problem.refresh_every)
    job.init()
    torch.cuda.synchronize()
    events = EventPool(steps + poll + 8) if with_events else None
    t0 = time.perf_counter()
    acc, calls, restarts, flags = run_steps(job, steps, poll, events, problem.refresh_every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k1_ms = None
    if events is not None:
        d = events.elapsed_ms()
        sel = [x for x, f in zip(d, flags) if f]
        k1_ms = sum(sel) / len(sel)
        events.close()
    st = job.status()
    fom = job.fom()
    hist = job.history()
    del job
    torch.cuda.empty_cache()
    return dict(accepted=acc, calls=calls, restarts=restarts, seconds=t1 - t0, k1_ms=k1_ms,
                status=st, fom_last=fom, last_run_pixels=[int(x) for x in hist[:, 0]],
                k1_variant=None if tuned is None else tuned["name"])


def time_deferred_graph(problem, steps, warmup, delay, fused=True):
    """Deferred mode with every window of `delay` steps replayed from a HIP graph
    (captured from gfo_greedy_steps when fused)."""
    import torch
    from paper_2202_05388_amd.job import Job

    kmax = 2 * problem.refresh_every if problem.refresh_every else 0
    job = Job(problem, device="cuda:0", kmax=kmax, delay=delay, ld_pad=LD_PAD)
    job.init()
    g, s = job.capture_steps(delay, fused=fused)
    re = problem.refresh_every

    def run(target):
        job.init()
        acc = restarts = 0
        while acc < target:
            before = job.n_flips()
            g.replay()
            now = job.n_flips()
            acc += now - before
            if now - before < delay:
                job.flush()
                job.init()
                restarts += 1
            elif re and now % re == 0:
                job.refresh()
        return acc, restarts

    run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc, restarts = run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = dict(delay=delay, fused=fused, storage=problem.dtype, graph_window=delay, accepted=acc,
               restarts=restarts, steps_per_s=acc / dt, ms_per_step=1e3 * dt / acc,
               fom_last=job.fom(), status=job.status())
    del job, g
    torch.cuda.empty_cache()
    return out


def time_deferred(problem, steps, warmup, poll, delay, fused=True, tune=True, packed=False):
    """Greedy steps with deferred rank-1 updates: E, the FP64 diagonal and the monitor
    rows every step, the design block by one rank-`delay` matrix-core product per
    `delay` steps.  fused: gfo_greedy_steps (one kernel per move), else
    score_candidates + apply_flip per move.  Times the flush kernel with HIP
    events on its stream."""
    import torch
    from paper_2202_05388_amd.hiprt import EventPool
    from paper_2202_05388_amd.job import Job

    from paper_2202_05388_amd import autotune as at

    kmax = 2 * problem.refresh_every if problem.refresh_every else 0
    job = Job(problem, device="cuda:0", kmax=kmax, delay=delay or 64, ld_pad=LD_PAD, packed=packed)
    job.init()
    g_bytes = job.G.numel() * job.G.element_size()
    delay_tuned = None
    if delay is None:
        # the flush interval from the trajectory this workload runs (autotuner)
        delay_tuned = at.tune_delay(job, moves=256, refresh_every=problem.refresh_every,
                                    save=False)
        delay = job.delay
        _log(f"[bench] flush interval autotune {problem.name}: {delay_tuned}")
    flush_tuned = None
    if problem.dtype == "c64":
        from paper_2202_05388_amd import _lib as L
        from paper_2202_05388_amd import autotune as at
        # the library's default flush runs the timed window (the variant whose
        # counter traffic is recorded); the others are timed here for the record
        flush_tuned = dict(name=L.flush_variants()[L.flush_get_variant()])
        if tune:
            flush_tuned["variants_us"] = {r["name"]: round(r["us"], 1)
                                          for r in at.time_flush_variants(job)}
            _log(f"[bench] flush variants: {flush_tuned}")
            job.init()
    run_steps(job, warmup, poll, refresh_every=problem.refresh_every, fused=fused)
    job.init()
    torch.cuda.synchronize()
    fev = EventPool(steps // delay + 64)
    t0 = time.perf_counter()
    acc, calls, restarts, flags = run_steps(job, steps, poll, None, problem.refresh_every,
                                            flush_events=fev, fused=fused)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fl = fev.elapsed_ms()
    terms = list(getattr(fev, "terms", []))
    fev.close()
    assert len(terms) == len(fl), (len(terms), len(fl))
    hist = job.history()
    N = problem.n
    ld = (N + 63) // 64 * 64
    variant = None if flush_tuned is None else flush_tuned["name"]
    roof = flush_roofline(variant, problem.dtype, N, ld, problem.n_mon, terms, fl)
    out = dict(delay=delay, delay_autotune=None if delay_tuned is None else delay_tuned["all"],
               fused=fused, storage=problem.dtype, accepted=acc, restarts=restarts,
               steps_per_s=acc / dt, ms_per_step=1e3 * dt / acc, flushes_timed=len(fl),
               flush_terms=terms, flush_variant=variant,
               flush_variants_us=None if flush_tuned is None else flush_tuned.get("variants_us"),
               flush_us=None if not fl else 1e3 * sum(fl) / len(fl),
               flush_roofline=roof, fom_last=job.fom(), status=job.status(),
               storage_layout="band-packed" if packed else "dense", g_bytes=g_bytes,
               last_run_pixels=[int(x) for x in hist[:, 0]])
    del job
    torch.cuda.empty_cache()
    return out


def eps_greedy_study(runs=20, eps_list=(0.0, 0.1, 0.2, 0.3), with_oracle=True):
    """Epsilon-greedy on the 21x21 lens (the 2-D analogue of the paper's Sec. V
    study): `runs` seeded trajectories per eps, each to termination.  Reports the
    terminal FOM statistics and the GPU step rate; one trajectory is also run by
    the oracle on the host and compared move for move."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2202_05388_amd.job import Job

    p = W.SQUARE_21
    job = Job(p, device="cuda:0")
    out = {}
    steps_total, t_total = 0, 0.0
    for eps in eps_list:
        foms, lens = [], []
        for seed in range(runs):
            draws = W.eps_greedy_draws(2000, seed)
            job.init()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n = job.run_eps_greedy(eps, draws, poll_every=64)
            torch.cuda.synchronize()
            t_total += time.perf_counter() - t0
            steps_total += n
            foms.append(job.fom())
            lens.append(n)
        out[f"eps_{eps}"] = dict(fom_mean=float(np.mean(foms)), fom_std=float(np.std(foms)),
                                 fom_max=float(np.max(foms)), moves_mean=float(np.mean(lens)))
    greedy_fom = out["eps_0.0"]["fom_mean"]
    for k, v in out.items():
        v["vs_greedy"] = v["fom_mean"] / greedy_fom
    cpu = None
    if with_oracle:
        # CPU baseline: one trajectory on the oracle (host cores), compared with the GPU's
        from oracle import greedy as og
        draws = W.eps_greedy_draws(2000, 0)
        t0 = time.perf_counter()
        ref = og.eps_greedy(p, 0.1, draws, tier="T2")
        t_cpu = time.perf_counter() - t0
        job.init()
        job.run_eps_greedy(0.1, draws, poll_every=64)
        same = [tuple(map(int, h)) for h in job.history()] == [(s.pixel, s.eps_idx)
                                                                for s in ref.steps]
        cpu = dict(kind="oracle", eps=0.1, seed=0, moves=len(ref.steps), seconds=t_cpu,
                   moves_per_s=len(ref.steps) / t_cpu, gpu_matches=bool(same))
    del job
    torch.cuda.empty_cache()
    return dict(workload=p.name, runs_per_eps=runs, by_eps=out,
                gpu_moves_per_s=steps_total / t_total, cpu_baseline=cpu)


def time_eps_greedy(problem, steps, eps, delay, fused=True):
    """Epsilon-greedy steps (top-4 scores, drawn choice, rank-1 apply; deferred
    updates when delay > 0) until `steps` moves, restarting finished trajectories.
    fused: the steps that do not explore run through gfo_greedy_steps; otherwise
    every step takes the top-4 path (the same moves and state)."""
    import torch
    import workloads as W
    from paper_2202_05388_amd.job import Job

    job = Job(problem, device="cuda:0", delay=delay, ld_pad=LD_PAD)
    job.init()
    job.run_eps_greedy(eps, W.eps_greedy_draws(64, 99), poll_every=64, fused=fused)   # warm-up
    job.init()
    torch.cuda.synchronize()
    moves, restarts, seed = 0, 0, 0
    t0 = time.perf_counter()
    while moves < steps:
        n = job.run_eps_greedy(eps, W.eps_greedy_draws(min(2000, steps - moves), seed),
                               poll_every=32, fused=fused)
        moves += n
        seed += 1
        if job.delay:
            job.flush()
        job.init()
        restarts += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del job
    torch.cuda.empty_cache()
    return dict(eps=eps, delay=delay, fused=fused, moves=moves, restarts=restarts,
                moves_per_s=moves / dt, ms_per_move=1e3 * dt / moves)


def time_regions(problem, steps, delay, apply):
    """Greedy 2x2-region moves (score_regions, pixel moves, then four rank-1
    updates in deferred mode or one joint rank-k step) until `steps` region moves,
    restarting finished trajectories; every pending term is flushed before a
    restart and at the end."""
    import torch
    from paper_2202_05388_amd.job import Job

    job = Job(problem, device="cuda:0", delay=delay, ld_pad=LD_PAD)
    job.init()
    job.run_region_greedy(16, poll_every=16, apply=apply)            # warm-up
    job.flush()
    job.init()
    torch.cuda.synchronize()
    moves, restarts = 0, 0
    t0 = time.perf_counter()
    while moves < steps:
        want = steps - moves
        n, made = job.run_region_greedy(want, poll_every=32, apply=apply)
        moves += n
        if n < want:                               # the trajectory ended: restart
            job.flush()
            job.init()
            restarts += 1
    job.flush()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = dict(workload=problem.name, region="2x2", delay=delay, apply=apply, moves=moves,
               restarts=restarts, moves_per_s=moves / dt, ms_per_move=1e3 * dt / moves,
               status=job.status())
    del job
    torch.cuda.empty_cache()
    return out


def regions_cpu_baseline(problem, steps=20):
    """The oracle's region greedy (flipped-set tier) for a bounded number of moves."""
    from oracle import regions as orr
    t0 = time.perf_counter()
    tr = orr.region_greedy(problem, 2, steps=steps, tier="T2")
    dt = time.perf_counter() - t0
    return dict(kind="oracle", value=len(tr.steps) / dt, unit="region moves/s",
                sample=f"first {len(tr.steps)} region moves of {problem.name} (T2), {dt:.1f} s",
                cores=os.cpu_count())


def time_rank_k(problem, steps, warmup, precision, upper=False):
    """Rank-k steps as the batched workload specifies them: score with top-k and
    the spacing rule, one joint Woodbury update, and the FP64 refresh after every
    `problem.refresh_every` rank-k steps (kmax covers every pixel those steps can
    flip).  `steps` counts rank-k steps that accepted at least one move; a job
    whose step accepts none is restarted.  Polls the move counter after every
    step (a rank-k step is ~1 ms).

    Reports moves/s and steps/s over the whole window (refreshes included), the
    mean time of the matrix-core update kernel, the refresh time, the FOM after
    every step against the cumulative number of flips, and at every refresh the
    FOM error of the FP32/BF16 path: |FOM before - FOM after| / FOM after, the
    refresh being the FP64 re-solve of the same structure.

    upper: keep only the upper triangle of the symmetric design block current
    (state.lower_stale): the refresh's product and the rank-k update leave out
    the blocks wholly below the diagonal, and the update's bytes are those of
    the triangle with its diagonal and the monitor rows."""
    import torch
    from paper_2202_05388_amd import _lib as L
    from paper_2202_05388_amd.hiprt import EventPool
    from paper_2202_05388_amd.job import Job

    from paper_2202_05388_amd import autotune as at

    prec = L.GFO_FP32 if precision == "fp32" else L.GFO_BF16
    re = problem.refresh_every
    kmax = min(problem.n, problem.rank_k * max(steps, warmup))
    job = Job(problem, device="cuda:0", kmax=kmax, upper=upper)
    job.init()
    tuned = at.tune_rank_k(job, rank=problem.rank_k, precision=prec, save=False)
    _log(f"[bench] rank-k update autotune ({precision}): "
         + ", ".join(f"{r['name']} {r['us']:.0f} us" for r in tuned["all"]))

    def run(n, events):
        job.init()
        done = moves = restarts = in_run = 0
        durations_ok, curve, errs, refresh_s = [], [(0, job.fom())], [], 0.0
        last = 0
        while done < n:
            if events is not None:
                a, b = events.next()
                L.time_next_k1(a, b)
            job.score(topk=problem.rank_k, min_spacing=problem.min_spacing)
            job.apply_rank_k(problem.rank_k, precision=prec)
            now = job.n_flips()
            durations_ok.append(now > last)
            if now == last:
                job.init()
                restarts += 1
                last = in_run = 0
                continue
            moves += now - last
            last = now
            done += 1
            in_run += 1
            curve.append((moves, job.fom()))
            if re and in_run % re == 0:
                f0 = job.fom()
                t0 = time.perf_counter()
                job.refresh()
                f1 = job.fom()                     # synchronises
                refresh_s += time.perf_counter() - t0
                errs.append(abs(f0 - f1) / f1)
        return moves, restarts, durations_ok, curve, errs, refresh_s

    run(warmup, None)
    torch.cuda.synchronize()
    ev = EventPool(4 * steps + 16)
    t0 = time.perf_counter()
    moves, restarts, ok, curve, errs, refresh_s = run(steps, ev)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    d = [x for x, f in zip(ev.elapsed_ms(), ok) if f]
    ev.close()
    N, R = problem.n, problem.rows
    # algorithmic bytes of one update: G read and written once (complex64), the
    # whole block or the upper triangle with its diagonal plus the monitor rows
    nbytes = 8 * N * job.ld + 16 * (R - N) * job.ld if upper else 16 * N * R
    k_ms = sum(d) / len(d)
    flipped = int((job.eps_idx.cpu().numpy() != 0).sum())
    best = max(curve, key=lambda c: c[1])
    out = dict(precision=precision, rank=problem.rank_k, min_spacing=problem.min_spacing,
               storage="upper triangle" if upper else "full", refresh_every_steps=re, kmax=kmax,
               steps=steps, moves=moves, restarts=restarts,
               moves_per_s=moves / dt, steps_per_s=steps / dt, seconds=dt,
               refreshes=len(errs), refresh_seconds=refresh_s, flipped_at_end=flipped,
               update_us=k_ms * 1e3, update_bytes=nbytes, update_gbs=nbytes / (k_ms * 1e-3) / 1e9,
               update_hbm_frac=nbytes / (k_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
               fom_last=job.fom(), fom_best=best[1], flips_at_best=best[0],
               fom_err_at_refresh_max=max(errs) if errs else None,
               fom_err_at_refresh_mean=sum(errs) / len(errs) if errs else None,
               fom_vs_flips=_sample_curve(curve), update_variant=tuned["name"],
               update_variants_us={r["name"]: round(r["us"], 1) for r in tuned["all"]},
               status=job.status())
    del job
    torch.cuda.empty_cache()
    return out


def _sample_curve(curve, n=25):
    """At most n (flips, FOM) points of a curve, its ends included."""
    if len(curve) <= n:
        return [[int(a), float(b)] for a, b in curve]
    idx = sorted({round(i * (len(curve) - 1) / (n - 1)) for i in range(n)})
    return [[int(curve[i][0]), float(curve[i][1])] for i in idx]


def greedy_fom_curve(problem):
    """FOM after every move of one rank-1 greedy trajectory to its end (the
    predicted FOM each pick records, which the move reaches exactly)."""
    import torch
    from paper_2202_05388_amd import _lib as L
    from paper_2202_05388_amd.job import Job

    job = Job(problem, device="cuda:0", kmax=2 * problem.refresh_every, delay=64)
    job.init()
    cap = 4096
    buf = torch.zeros(cap * L.PICK_BYTES, dtype=torch.uint8, device="cuda:0")
    curve, done = [(0, job.fom())], 0
    while done < cap:
        n = min(64, cap - done)
        job.greedy_steps(n, out=buf.data_ptr() + done * L.PICK_BYTES)
        raw = buf[done * L.PICK_BYTES:(done + n) * L.PICK_BYTES].cpu().numpy().tobytes()
        recs = (L.Pick * n).from_buffer_copy(raw)
        made = [r for r in recs if r.pixel >= 0]
        curve.extend((done + i + 1, float(r.fom_new)) for i, r in enumerate(made))
        done += n
        if len(made) < n:
            break
    job.flush()
    torch.cuda.synchronize()
    del job
    torch.cuda.empty_cache()
    return curve


def time_refresh(problem):
    """One FP64 refresh of the state the greedy trajectory ends in."""
    import torch
    from paper_2202_05388_amd.job import Job
    job = Job(problem, device="cuda:0", kmax=max(2 * problem.steps, 512))
    job.init()
    k = job.run_greedy(problem.steps, poll_every=64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    job.refresh()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    N, R = problem.n, problem.rows
    flips = int((job.eps_idx.cpu().numpy() != 0).sum())
    kp = (flips + 3) // 4 * 4
    # FP64 flops of the two products as computed: G = G0 + Z U_D^T on the design
    # block's upper triangle and the monitor rows, Z = U M (R x kp x kp); the
    # rate is over the whole refresh (the inverse and the gathers included)
    product_flops = 8.0 * kp * (N * (N + 1) / 2 + (R - N) * N) + 8.0 * R * kp * kp
    out = dict(flipped_pixels=flips, ms=dt * 1e3, product_flops=product_flops,
               product_tflops_over_refresh=product_flops / dt / 1e12, status=job.status())
    del job
    torch.cuda.empty_cache()
    return out


def host_info():
    """CPU model, logical CPUs, RAM and the BLAS library numpy uses (threadpoolctl)."""
    info = dict(cpu_model=None, logical_cpus=os.cpu_count(), ram_gb=None, blas=None,
                blas_threads=None)
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["ram_gb"] = round(int(line.split()[1]) / 1024**2, 1)
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if blas:
            info["blas"] = f"{blas[0].get('internal_api')} {blas[0].get('version')}"
            info["blas_threads"] = int(blas[0].get("num_threads", 1))
    except Exception:  # pragma: no cover
        pass
    return info


def cpu_baseline(problem, max_steps):
    """The FP64 oracle (flipped-set tier) on the same workload, host cores."""
    from oracle import greedy as og

    host = host_info()
    t0 = time.perf_counter()
    tr = og.greedy(problem.replace(tau=1e-9), steps=max_steps, tier="T2")
    dt = time.perf_counter() - t0
    n = len(tr.steps)
    return dict(value=n / dt, unit="steps/s", cores=int(host["blas_threads"] or os.cpu_count()),
                kind="oracle",
                sample=f"oracle greedy trajectory, flipped-set tier (FP64), {n} steps "
                       f"({'to termination' if tr.stopped else 'capped'}) of {problem.name}, "
                       f"{dt:.1f} s", host=host), [s.pixel for s in tr.steps], tr


def cpu_dense_resolve_baseline(steps=10):
    """The oracle's dense re-solve tier (T1: one direct solve of the 1024-pixel
    system per step) on the 32x32 FP64 workload, its first `steps` steps."""
    import workloads as W
    from oracle import greedy as og
    p = W.SMALL_32
    t0 = time.perf_counter()
    tr = og.greedy(p, steps=steps, tier="T1")
    dt = time.perf_counter() - t0
    return dict(kind="oracle", tier="T1", workload=p.name, value=len(tr.steps) / dt,
                unit="steps/s", sample=f"first {len(tr.steps)} greedy steps, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--poll", type=int, default=32)
    ap.add_argument("--workload", default="square128_c64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-plain", action="store_true")
    ap.add_argument("--no-eager-upper", action="store_true",
                    help="skip the eager leg that keeps the upper triangle of the design block alone")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-rank-k", action="store_true")
    ap.add_argument("--no-deferred", action="store_true")
    ap.add_argument("--delay", type=int, default=None,
                    help="deferred-mode flush interval (default: chosen by the autotuner from the "
                         "workload's trajectory)")
    ap.add_argument("--no-refresh-timing", action="store_true")
    ap.add_argument("--no-eps-greedy", action="store_true")
    ap.add_argument("--no-regions", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=64,
                    help="jobs in the served stream (0 = skip the serving measurement)")
    ap.add_argument("--serve-rate", type=float, default=4.0, help="job arrivals per second")
    ap.add_argument("--ld-pad", type=int, default=0,
                    help="extra columns of G (a multiple of 64) beyond the minimum leading dimension")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also time a plain 2 GiB device copy (HBM ceiling, counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU row sharding "
                                   "is a design only", "n_gpus": args.gpus}))
        sys.exit(2)

    import workloads as W

    global LD_PAD
    LD_PAD = args.ld_pad
    problem = W.WORKLOADS[args.workload]
    _log(f"[bench] {problem.name}: {problem.ny}x{problem.nx}, {problem.n_mon} monitors, "
         f"{problem.dtype}, steps={args.steps} warmup={args.warmup}")
    copy_gbs = None
    if args.calib_copy:
        copy_gbs = copy_ceiling()
        _log(f"[bench] device copy ceiling {copy_gbs:.0f} GB/s")
    res = time_workload(problem, args.steps, args.warmup, args.poll,
                        autotune=not args.no_autotune)
    N, R = problem.n, problem.rows
    elem = 8 if problem.dtype == "c64" else 16
    bytes_per_launch = 2 * elem * N * R            # one read + one write of every stored entry
    k1_s = res["k1_ms"] / 1e3
    achieved = bytes_per_launch / k1_s / 1e9
    value = res["accepted"] / res["seconds"]
    _log(f"[bench] {res['accepted']} moves, {res['restarts']} restarts, {res['seconds']:.3f} s, "
         f"K1 {res['k1_ms'] * 1e3:.1f} us = {achieved:.0f} GB/s")

    # eager updates of the upper triangle alone (the design block is symmetric):
    # minimal traffic = the triangle with its diagonal and the monitor rows, read
    # and written once
    eager_upper = None
    if not args.no_eager_upper:
        _log("[bench] eager, upper triangle of the design block alone")
        # the variant timed on the triangle itself (its skipped tiles change the best shape)
        ru = time_workload(problem, args.steps, args.warmup, args.poll,
                           autotune=not args.no_autotune, upper=True)
        up_bytes = 2 * elem * (N * (N + 1) // 2 + problem.n_mon * N)
        up_gbs = up_bytes / (ru["k1_ms"] / 1e3) / 1e9
        eager_upper = dict(value=ru["accepted"] / ru["seconds"], unit="steps/s",
                           ms_per_step=1e3 * ru["seconds"] / ru["accepted"], restarts=ru["restarts"],
                           k1_us=ru["k1_ms"] * 1e3, algorithmic_bytes_per_launch=up_bytes,
                           achieved_gbs=up_gbs, frac=up_gbs / HBM_PEAK_GBS,
                           variant=ru["k1_variant"] or res["k1_variant"], status=ru["status"])
        _log(f"[bench] eager upper {eager_upper}")

    plain = None
    if not args.no_fp64_plain and problem.dtype == "c64" and problem.name.startswith("square128"):
        pp = W.SQUARE_128_FP64
        _log(f"[bench] plain FP64 loop {pp.name}")
        r2 = time_workload(pp, args.steps, args.warmup, args.poll, autotune=not args.no_autotune)
        plain = dict(workload=pp.name, value=r2["accepted"] / r2["seconds"], unit="steps/s",
                     ms_per_step=1e3 * r2["seconds"] / r2["accepted"],
                     k1_us=r2["k1_ms"] * 1e3,
                     k1_gbs=2 * 16 * N * R / (r2["k1_ms"] / 1e3) / 1e9)

    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        _log("[bench] cpu baseline (oracle)")
        cpu, ref_pixels, tr = cpu_baseline(problem, max_steps=200)
        if problem.name == "square128_c64":
            cpu["dense_resolve_square32"] = cpu_dense_resolve_baseline()
        gpu_pixels = res["last_run_pixels"]
        n = min(len(ref_pixels), len(gpu_pixels))
        match = sum(1 for a, b in zip(ref_pixels, gpu_pixels) if a == b)
        if tr.stopped and len(gpu_pixels) == len(ref_pixels):
            fom_ref = tr.steps[-1].fom
            accuracy = dict(trajectory_steps=len(ref_pixels), pixels_matching=match,
                            fom_gpu=res["fom_last"], fom_oracle=fom_ref,
                            fom_rel_err=abs(res["fom_last"] - fom_ref) / fom_ref)
        else:
            accuracy = dict(pixels_matching=match, compared=n)

    deferred = None
    if not args.no_deferred:
        deferred = {}
        forms = [problem]
        if problem.name == "square128_c64":
            forms.append(W.SQUARE_128_FP64)
        for pf in forms:
            _log(f"[bench] deferred updates, {pf.name}, delay {args.delay or 'autotuned'}")
            deferred[pf.name] = time_deferred(pf, args.steps, args.warmup, args.poll, args.delay)
            _log(f"[bench] deferred {pf.name}: {deferred[pf.name]}")
            d_pf = deferred[pf.name]["delay"]
            key = pf.name + "_per_call"
            deferred[key] = time_deferred(pf, args.steps, args.warmup, args.poll, d_pf,
                                          fused=False, tune=False)
            _log(f"[bench] deferred {key}: {deferred[key]}")
            key = pf.name + "_graph"
            deferred[key] = time_deferred_graph(pf, args.steps, args.warmup, d_pf)
            _log(f"[bench] deferred {key}: {deferred[key]}")
            # the same fused loop on band-packed storage (about half of G's bytes)
            key = pf.name + "_packed"
            deferred[key] = time_deferred(pf, args.steps, args.warmup, args.poll, d_pf,
                                          tune=False, packed=True)
            _log(f"[bench] deferred {key}: {deferred[key]}")
    if args.delay is None:
        # the other deferred legs use the interval chosen for the headline workload
        args.delay = deferred[problem.name]["delay"] if deferred else 64

    rank_k = None
    if not args.no_rank_k and problem.name == "square128_c64":
        rk = W.SQUARE_128_RANK16
        rank_k = {}
        for prec in ("fp32", "bf16"):
            _log(f"[bench] rank-{rk.rank_k} steps ({prec})")
            rank_k[prec] = time_rank_k(rk, steps=rk.steps, warmup=16, precision=prec)
            _log(f"[bench] rank-{rk.rank_k} {prec}: {rank_k[prec]}")
        # the same steps keeping the design block's upper triangle alone
        rank_k["fp32_upper"] = time_rank_k(rk, steps=rk.steps, warmup=16, precision="fp32", upper=True)
        _log(f"[bench] rank-{rk.rank_k} fp32, upper triangle: {rank_k['fp32_upper']}")
        g = greedy_fom_curve(problem)
        rank_k["rank1_greedy"] = dict(moves=len(g) - 1, fom_last=g[-1][1],
                                      fom_vs_flips=_sample_curve(g))
        # flips the rank-16 form needs to reach the greedy trajectory's final FOM
        for prec in ("fp32", "bf16", "fp32_upper"):
            reach = [f for f, v in rank_k[prec]["fom_vs_flips"] if v >= g[-1][1]]
            rank_k[prec]["flips_to_greedy_fom"] = reach[0] if reach else None

    eps_greedy = None
    if not args.no_eps_greedy and problem.name == "square128_c64":
        _log("[bench] epsilon-greedy study (21x21 lens) and rate at 128^2")
        eps_greedy = dict(study=eps_greedy_study(with_oracle=not args.no_cpu_baseline),
                          square128_c64=time_eps_greedy(problem, min(args.steps, 1000), 0.1,
                                                        args.delay),
                          square128_c64_per_step=time_eps_greedy(problem, min(args.steps, 1000),
                                                                 0.1, args.delay, fused=False))
        _log(f"[bench] epsilon-greedy {eps_greedy}")

    regions = None
    if not args.no_regions and problem.name == "square128_c64":
        rp = W.SQUARE_128_REGIONS
        _log(f"[bench] region moves ({rp.name})")
        regions = dict(deferred=time_regions(rp, 500, args.delay, "sequential"),
                       rank_k=time_regions(rp, 100, 0, "rank_k"))
        if not args.no_cpu_baseline:
            regions["cpu_baseline"] = regions_cpu_baseline(rp)
        _log(f"[bench] regions {regions}")

    refresh = None
    if not args.no_refresh_timing and problem.refresh_every:
        _log("[bench] FP64 refresh at the end of the trajectory")
        refresh = time_refresh(problem.replace(steps=min(problem.steps, 500)))
        _log(f"[bench] refresh {refresh}")

    serving = None
    if args.serve_jobs > 0:
        from paper_2202_05388_amd.serve import serve_benchmark
        _log(f"[bench] serving {args.serve_jobs} jobs at {args.serve_rate}/s (mix, then one at a time)")
        serving = serve_benchmark(n_jobs=args.serve_jobs, rate=args.serve_rate, delay=args.delay)
        for k in ("mix", "mix_grouped", "one_at_a_time", "burst_mix", "burst_mix_grouped",
                  "burst_one_at_a_time"):
            _log(f"[bench] serving {k} {serving[k]}")

    N, R, ld = problem.n, problem.rows, (problem.n + 63) // 64 * 64
    eager_roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": achieved / HBM_PEAK_GBS,
                  "traffic": pmc_traffic("k_rank1", problem.name, res["k1_variant"]),
                  "traffic_unit": "bytes/launch",
                  "kernel": "k_rank1 (streaming rank-1 update)",
                  "bytes_per_launch": bytes_per_launch, "avg_launch_us": res["k1_ms"] * 1e3,
                  "variant": res["k1_variant"], "copy_ceiling_gbs": copy_gbs}
    eager = dict(value=value, unit="steps/s", ms_per_step=1e3 * res["seconds"] / res["accepted"],
                 restarts=res["restarts"], roofline=eager_roof)
    d = (deferred or {}).get(problem.name)
    if d is not None and d.get("flush_roofline"):
        mode = (f"deferred rank-1 updates, flush every {d['delay']} moves, "
                f"{'fused greedy loop (gfo_greedy_steps)' if d['fused'] else 'per-call'}")
        head_value = d["steps_per_s"]
        head_ms = d["ms_per_step"]
        kind = ("FP64" if problem.dtype != "c64" else
                "FP32 products as BF16 part products on the" if d["flush_variant"] == "up_bandseg_s3"
                else "FP32")
        roofline = dict(d["flush_roofline"])
        # counters per term bucket, averaged over the flushes of the window
        roofline.update(kernel=f"flush of the deferred updates, {kind} MFMA, variant "
                               f"{d['flush_variant']}",
                        traffic=flush_traffic(problem.name, d["flush_variant"], d["flush_terms"])
                        if problem.dtype == "c64" else None,
                        traffic_unit="bytes/launch")
        pix = d["last_run_pixels"]
    else:
        mode = "eager rank-1 updates"
        head_value, head_ms, roofline = value, eager["ms_per_step"], eager_roof
        pix = res["last_run_pixels"]
    if accuracy is not None and not args.no_cpu_baseline:
        m = sum(1 for a, b in zip(ref_pixels, pix) if a == b)
        accuracy["headline_path_pixels_matching"] = f"{m}/{min(len(pix), len(ref_pixels))}"
    if deferred:
        for v in deferred.values():
            v.pop("last_run_pixels", None)

    out = {
        "metric": "greedy steps/s at 128^2 px (% HBM peak) vs FP64 plain; served p50/p99 latency",
        "value": head_value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": problem.dtype,
        "data": "synthetic",
        "config": {"workload": problem.name, "grid": f"{problem.ny}x{problem.nx}",
                   "monitors": problem.n_mon, "storage": problem.dtype, "mode": mode,
                   "refresh_every": problem.refresh_every, "candidates": "eps {1, 12.25}",
                   "restart_when_trajectory_ends": True},
        "roofline": roofline,
        "eager": eager,
        "eager_upper": eager_upper,
        "fp64_plain": plain,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "deferred": deferred,
        "rank_k": rank_k,
        "eps_greedy": eps_greedy,
        "regions": regions,
        "refresh": refresh,
        "serving": serving,
        "device_status": res["status"],
    }
    if plain:
        out["speedup_vs_fp64_plain"] = head_value / plain["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
