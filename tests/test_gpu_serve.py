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
