"""Autotuner: kernel variants and the deferred-update schedule, on the live shape.

  * the streaming rank-1 kernel of apply_flip (tile variants, bit-identical);
  * the complex64 flush of the deferred terms (tile variants);
  * the matrix-core update of apply_flips_rank_k (tile and epilogue variants),
    per input precision;
  * the flush interval of deferred mode, from the trajectory the job runs.

Kernels are timed with HIP events recorded around the kernel alone; the flush
interval by the wall clock of the fused greedy loop.  Choices are cached as JSON
keyed by (architecture, N, R, storage type, ...).

Cache path: $GFO_AUTOTUNE_CACHE, else ~/.cache/gfo/autotune.json.
"""
from __future__ import annotations

import json
import os
import time

from . import _lib as L

ARCH = "gfx950"


def cache_path() -> str:
    return os.environ.get("GFO_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gfo", "autotune.json"))


def _key(N: int, R: int, dtype: str) -> str:
    return f"{ARCH}/N{N}/R{R}/{dtype}"


def load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(d: dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_k1_variants(job, reps: int = 10, warm: int = 2, variants=None) -> list:
    """Average kernel time (us) of each variant on `job`'s shape.

    Uses two alternating moves on pixel 0 (to material 1 and back), so the job's
    structure is unchanged after an even number of calls.
    """
    import torch
    from .hiprt import EventPool

    code = L.GFO_C64 if job.dtype_name == "c64" else L.GFO_C128
    names = L.k1_variants(code)
    idxs = range(len(names)) if variants is None else variants
    base = job.picks.data_ptr()
    job.set_pick(0, 1, slot=0)
    job.set_pick(0, 0, slot=1)
    torch.cuda.synchronize()
    old = L.k1_get_variant(code)
    out = []
    try:
        for vi in idxs:
            L.k1_set_variant(code, vi)
            for i in range(warm):
                job.apply(pick_ptr=base + (i % 2) * L.PICK_BYTES)
            ev = EventPool(reps)
            for i in range(reps):
                a, b = ev.next()
                L.time_next_k1(a, b)
                job.apply(pick_ptr=base + ((warm + i) % 2) * L.PICK_BYTES)
            if (warm + reps) % 2:
                job.apply(pick_ptr=base + L.PICK_BYTES)
            ms = ev.elapsed_ms()
            ev.close()
            out.append(dict(variant=vi, name=names[vi], us=1e3 * sum(ms) / len(ms),
                            us_min=1e3 * min(ms)))
    finally:
        L.k1_set_variant(code, old)
    return out


def tune(job, reps: int = 10, save: bool = True, variants=None) -> dict:
    """Time the variants (default all; else a list of names) on this job's
    shape, select and cache the fastest."""
    t0 = time.time()
    code = L.GFO_C64 if job.dtype_name == "c64" else L.GFO_C128
    idxs = None if variants is None else [L.k1_variants(code).index(v) for v in variants]
    res = time_k1_variants(job, reps=reps, variants=idxs)
    elem = 8 if job.dtype_name == "c64" else 16
    bytes_per = 2 * elem * job.N * job.R
    for r in res:
        r["gbs"] = bytes_per / (r["us"] * 1e-6) / 1e9
    best = min(res, key=lambda r: r["us"])
    L.k1_set_variant(code, best["variant"])
    entry = dict(variant=best["variant"], name=best["name"], us=best["us"], gbs=best["gbs"],
                 seconds=time.time() - t0, all=res)
    if save:
        d = load_cache()
        d[_key(job.N, job.R, job.dtype_name)] = entry
        save_cache(d)
    return entry


def time_flush_variants(job, reps: int = 2, variants=None) -> list:
    """Mean flush-kernel time (us) of each complex64 flush variant on `job`'s shape
    (deferred job, delay d): each measurement runs d greedy steps, whose last apply
    ends with the flush; the job restarts when its trajectory ends.  `variants`:
    names to time (default all)."""
    import torch
    from .hiprt import EventPool

    if not job.delay or job.dtype_name != "c64":
        raise L.GfoError("flush tuning needs a complex64 job in deferred mode")
    names = L.flush_variants()
    idxs = range(len(names)) if variants is None else [names.index(v) for v in variants]
    old = L.flush_get_variant()
    out = []
    try:
        for vi in idxs:
            L.flush_set_variant(vi)
            ev = EventPool(reps + 1)
            for rep in range(reps + 1):
                job.flush()
                start = job.n_flips()
                for i in range(job.delay):
                    if i == job.delay - 1 and rep > 0:
                        a, b = ev.next()
                        L.time_next_k1(a, b)
                    job.step()
                if job.n_flips() - start < job.delay:
                    job.init()
            ms = ev.elapsed_ms()
            ev.close()
            out.append(dict(variant=vi, name=names[vi], us=1e3 * sum(ms) / max(len(ms), 1)))
    finally:
        L.flush_set_variant(old)
    torch.cuda.synchronize()
    return out


def tune_flush(job, reps: int = 2) -> dict:
    res = time_flush_variants(job, reps)
    best = min(res, key=lambda r: r["us"])
    L.flush_set_variant(best["variant"])
    return dict(variant=best["variant"], name=best["name"], us=best["us"], all=res)


def time_rk_variants(job, rank: int = 16, precision: int = None, reps: int = 4,
                     warm: int = 2, variants=None) -> list:
    """Mean time (us) of the matrix-core update of apply_flips_rank_k for each
    variant on `job`'s shape (complex64, eager).  Each measurement applies
    `rank` spaced pixels to material 1 and then back to their material, so the
    structure is unchanged after every pair (G up to FP32 rounding)."""
    import torch
    from .hiprt import EventPool

    if job.dtype_name != "c64" or job.delay:
        raise L.GfoError("rank-k tuning needs a complex64 job in eager mode")
    precision = L.GFO_FP32 if precision is None else precision
    p = job.problem
    N = job.N
    cur = job.eps_idx.cpu().numpy()
    step = max(1, N // rank)
    pix = [min(N - 1, i * step + (i * 7) % max(step, 1)) for i in range(rank)]
    there = [(j, 1 if int(cur[j]) == 0 else 0) for j in pix]
    back = [(j, int(cur[j])) for j in pix]
    base = job.picks.data_ptr()

    def apply(moves):
        for t, (j, e) in enumerate(moves):
            job.set_pick(j, e, slot=t)
        job.apply_rank_k(rank, precision=precision, pick_ptr=base)

    names = L.rk_variants()
    idxs = range(len(names)) if variants is None else [names.index(v) for v in variants]
    old = L.rk_get_variant()
    out = []
    try:
        for vi in idxs:
            L.rk_set_variant(vi)
            for i in range(warm):
                apply(there if i % 2 == 0 else back)
            if warm % 2:
                apply(back)
            ev = EventPool(2 * reps)
            for i in range(2 * reps):
                a, b = ev.next()
                L.time_next_k1(a, b)
                apply(there if i % 2 == 0 else back)
            ms = ev.elapsed_ms()
            ev.close()
            out.append(dict(variant=vi, name=names[vi], us=1e3 * sum(ms) / len(ms),
                            us_min=1e3 * min(ms)))
    finally:
        L.rk_set_variant(old)
    torch.cuda.synchronize()
    return out


def tune_rank_k(job, rank: int = 16, precision: int = None, reps: int = 4,
                save: bool = True) -> dict:
    """Time the rank-k update variants on this job's shape, select and cache the
    fastest (key: shape, rank padding, input precision)."""
    t0 = time.time()
    precision = L.GFO_FP32 if precision is None else precision
    res = time_rk_variants(job, rank=rank, precision=precision, reps=reps)
    bytes_per = 16 * job.N * job.R
    for r in res:
        r["gbs"] = bytes_per / (r["us"] * 1e-6) / 1e9
    best = min(res, key=lambda r: r["us"])
    L.rk_set_variant(best["variant"])
    prec = "fp32" if precision == L.GFO_FP32 else "bf16"
    entry = dict(variant=best["variant"], name=best["name"], us=best["us"], gbs=best["gbs"],
                 seconds=time.time() - t0, all=res)
    if save:
        d = load_cache()
        d[f"{_key(job.N, job.R, job.dtype_name)}/rk{16 if rank <= 16 else 32}/{prec}"] = entry
        save_cache(d)
    return entry


def tune_delay(job, moves: int = 256, candidates=(32, 64, 128), chunk: int = 32,
               refresh_every: int = 0, save: bool = True) -> dict:
    """Choose the flush interval (pending terms per flush) of a deferred-mode
    job from its own trajectory: for each candidate, start from init_G0 and time
    the fused greedy loop (gfo_greedy_steps in chunks of `chunk` moves, the
    flushes it launches and a final one) over the first `moves` moves, or to the
    trajectory's end if it ends earlier.  Longer trajectories favour more terms
    per flush (a flush is one pass over the design block, shared by more
    moves); short ones pay for a partial last flush.  Sets the fastest on the
    job (job.delay and its state) and caches it by shape and trajectory length."""
    import torch

    if job.dtype_name not in ("c64", "c128"):
        raise L.GfoError("unknown storage type")
    res = []
    for d in candidates:
        if not 1 <= d <= L.GFO_MAX_DELAY:
            continue
        job.delay = d
        job.state.delay = d
        job.init()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = job.run_greedy(moves, poll_every=chunk, refresh_every=refresh_every, fused=True)
        job.flush()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res.append(dict(delay=d, moves=n, us_per_move=1e6 * dt / max(n, 1)))
    best = min(res, key=lambda r: r["us_per_move"])
    job.delay = best["delay"]
    job.state.delay = best["delay"]
    job.init()
    entry = dict(delay=best["delay"], moves=best["moves"], all=res)
    if save:
        d = load_cache()
        d[f"{_key(job.N, job.R, job.dtype_name)}/delay/{best['moves']}"] = entry
        save_cache(d)
    return entry


def apply_cached(job) -> bool:
    """Select the cached variant for this job's shape, if any.  Returns True if found."""
    e = load_cache().get(_key(job.N, job.R, job.dtype_name))
    if not e:
        return False
    code = L.GFO_C64 if job.dtype_name == "c64" else L.GFO_C128
    names = L.k1_variants(code)
    if e["variant"] < len(names) and names[e["variant"]] == e["name"]:
        L.k1_set_variant(code, e["variant"])
        return True
    return False


if __name__ == "__main__":
    # Times the variants of one kernel family on a named workload and prints one
    # line per variant (mean kernel time from HIP events), e.g.
    #   python -m paper_2202_05388_amd.autotune --kernel flush --delay 64
    #   python -m paper_2202_05388_amd.autotune --kernel rank-k --variants pre128_r4
    import argparse
    import sys

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W
    from .job import Job

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="square128_c64")
    ap.add_argument("--kernel", choices=["k1", "flush", "rank-k"], default="k1")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--delay", type=int, default=64, help="pending terms per flush (--kernel flush)")
    ap.add_argument("--rank", type=int, default=16, help="pixels per move (--kernel rank-k)")
    ap.add_argument("--bf16", action="store_true", help="BF16 operands (--kernel rank-k)")
    ap.add_argument("--variants", default=None, help="comma-separated variant names (default all)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy 2 GiB device to device (a kernel of known traffic, to scale counters)")
    args = ap.parse_args()
    if args.calib_copy:
        import torch
        src = torch.empty(1 << 29, dtype=torch.float32, device="cuda:0").fill_(1.0)
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        del src
    p = W.WORKLOADS[args.workload]
    sel = args.variants.split(",") if args.variants else None
    if args.kernel == "k1":
        job = Job(p, device="cuda:0")
        job.init()
        e = tune(job, reps=args.reps, save=False, variants=sel)
        for r in sorted(e["all"], key=lambda r: r["us"]):
            print(f"{r['name']:>20s} {r['us']:9.1f} us {r['gbs']:7.0f} GB/s", flush=True)
        print(json.dumps({k: v for k, v in e.items() if k != "all"}))
    elif args.kernel == "flush":
        job = Job(p, device="cuda:0", delay=args.delay)
        job.init()
        for r in time_flush_variants(job, reps=args.reps, variants=sel):
            print(f"{r['name']:>20s} {r['us']:9.1f} us", flush=True)
    else:
        job = Job(p, device="cuda:0")
        job.init()
        prec = L.GFO_BF16 if args.bf16 else L.GFO_FP32
        for r in time_rk_variants(job, rank=args.rank, precision=prec, reps=args.reps, variants=sel):
            gbs = 16 * job.N * job.R / (r["us"] * 1e-6) / 1e9
            print(f"{r['name']:>20s} {r['us']:9.1f} us {gbs:7.0f} GB/s", flush=True)
