"""Serving loop on the GPU: jobs of different sizes and wavelengths overlap on the
device, and each job's result (final fields and move history) is bit-identical to
the same job run alone."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _jobs():
    js = W.served_jobs(n_jobs=8, rate=50.0, seed=3, side_range=(12, 40), steps_range=(20, 90))
    # a short refresh cadence so that refreshes happen inside the mix
    return [W.Job(j.job_id, j.arrival, j.problem.replace(refresh_every=16)) for j in js]


@pytest.mark.parametrize("delay", [0, 16])
def test_mixed_results_equal_alone(delay):
    from paper_2202_05388_amd.serve import Server
    jobs = _jobs()
    print(f"[case] serving {len(jobs)} jobs, delay {delay}: " +
          ", ".join(f"{j.problem.ny}x{j.problem.nx}/{j.problem.steps}" for j in jobs), flush=True)
    mix, smix = Server(max_slots=4, chunk=8, delay=delay).run(jobs, mode="mix")
    alone, salone = Server(max_slots=1, chunk=8, delay=delay).run(jobs, mode="serial")
    dm = {r.job_id: r for r in mix}
    da = {r.job_id: r for r in alone}
    assert set(dm) == set(da) == {j.job_id for j in jobs}
    for k in dm:
        assert dm[k].steps == da[k].steps > 0
        assert dm[k].digest == da[k].digest, k
        assert dm[k].status == 0
    print("mix", smix, "\nalone", salone, flush=True)
    assert smix["steps"] == salone["steps"]
    assert smix["step_p99_ms"] >= smix["step_p50_ms"] > 0


def test_budget_admission_limits_residency():
    from paper_2202_05388_amd.serve import Server, footprint
    jobs = _jobs()[:4]
    big = max(footprint(j.problem, j.problem.steps) for j in jobs)
    res, summ = Server(budget_bytes=1.5 * big, max_slots=4, chunk=8).run(jobs, mode="mix")
    assert len(res) == 4 and summ["nonzero_status"] == 0


def test_table_steps_equal_per_job_calls():
    """gfo_greedy_steps_table moves every job of a group with one launch per
    move; each job's moves and state are bit for bit those of its own
    gfo_greedy_steps calls: jobs of different sizes and materials, one whose
    trajectory ends inside the run, term buffers that fill at different steps
    (one job starts with pending terms), chunks of several lengths."""
    import torch
    from paper_2202_05388_amd.job import Job, JobGroup
    probs = [W.tiny(24, 24, n_mon=16, dtype="c64", tau=1e-6),
             W.tiny(30, 26, n_mon=8, dtype="c64", tau=1e-6, wavelength=1.1),
             W.tiny(12, 12, n_mon=4, dtype="c64", tau=1e-6),
             W.tiny(40, 36, n_mon=16, dtype="c64", tau=1e-6, eps_table=(1.0, 12.25, 4.0),
                    cand_mask=0b111)]
    print("[case] job table: " + ", ".join(f"{p.ny}x{p.nx}" for p in probs), flush=True)

    def make():
        js = [Job(p, device="cuda:0", delay=16, flip_cap=400) for p in probs]
        for j in js:
            j.init()
        js[1].greedy_steps(5)                     # five pending terms before the group starts
        return js

    alone, grouped = make(), make()
    chunks = [7, 16, 1, 9, 24]
    for n in chunks:
        for j in alone:
            j.greedy_steps(n)
    group = JobGroup(grouped, device="cuda:0")
    group.build()
    for n in chunks:
        group.steps(n)
    torch.cuda.synchronize()
    assert any(j.n_flips() < j.steps_issued for j in alone)      # a trajectory ended
    for a, b in zip(alone, grouped):
        assert a.state.pending_calls == b.state.pending_calls
        assert np.array_equal(a.history(), b.history()) and a.status() == b.status() == 0
        Ga, Ea, da, ia = a.host_state()
        Gb, Eb, db, ib = b.host_state()
        assert np.array_equal(Ga, Gb) and np.array_equal(Ea, Eb)
        assert np.array_equal(da, db) and np.array_equal(ia, ib)


def test_grouped_serving_equals_alone_and_follows_the_oracle():
    """The served mix with small jobs grouped (one launch per move for all of
    them) gives every job the result it gets alone, bit for bit; one served job's
    move sequence and FOM are checked against the FP64 oracle's greedy
    trajectory (certified ties, FOM to 1e-4)."""
    from oracle import greedy as og
    from paper_2202_05388_amd.serve import Server
    from parity import certify_sequence
    jobs = _jobs()
    mix, smix = Server(max_slots=4, chunk=8, delay=16, group_below=32 * 32).run(jobs, mode="mix")
    alone, _ = Server(max_slots=1, chunk=8, delay=16).run(jobs, mode="serial")
    dm = {r.job_id: r for r in mix}
    da = {r.job_id: r for r in alone}
    assert set(dm) == set(da) == {j.job_id for j in jobs}
    small = [j for j in jobs if j.problem.n <= 32 * 32]
    assert len(small) >= 2
    for k in dm:
        assert dm[k].digest == da[k].digest, k
        assert dm[k].steps == da[k].steps > 0 and dm[k].status == 0
    print("grouped mix", smix, flush=True)
    # one small served job against the oracle
    j = small[0]
    p = j.problem
    ref = og.greedy(p.replace(tau=1e-9), steps=p.steps, tier="T2")
    got = [(int(a), int(b)) for a, b in dm[j.job_id].history]
    t = certify_sequence(p, [(s.pixel, s.eps_idx) for s in ref.steps], got)
    print(f"served job {p.name}: {len(got)} moves, oracle {len(ref.steps)}, identical for {t}",
          flush=True)
    fom_ref = ref.steps[-1].fom if len(got) == len(ref.steps) else None
    if fom_ref is not None:
        assert abs(dm[j.job_id].fom - fom_ref) <= 1e-4 * fom_ref
