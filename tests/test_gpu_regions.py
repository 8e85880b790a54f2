"""Multi-pixel region moves on the GPU (2x2 pixels; paper Sec. II with N_V = 4):
region scores against the oracle's, region greedy trajectories equal to the
oracle's, deferred = eager, the joint rank-k application = the sequential one."""
import numpy as np
import pytest

from oracle import regions as orr
from oracle import state as ost
import workloads as W
from parity import c64_drift_tol, rel_elem

pytestmark = pytest.mark.gpu


def _job(p, **kw):
    from paper_2202_05388_amd.job import Job
    print(f"[case] {p.name} {p.ny}x{p.nx} {p.dtype} {kw}", flush=True)
    return Job(p, device="cuda:0", **kw)


def _lens(n, dtype="c128", **kw):
    return W.tiny(n, n, n_mon=4, cand_mask=W.MASK_BOTH, pitch=0.025, mon_distance=0.5,
                  dtype=dtype, tau=1e-9 if dtype == "c128" else 1e-6, region=2, **kw)


def _gpu_region_scores(job):
    K = orr.n_regions(job.problem, 2)
    n_eps = len(job.problem.eps_table)
    return job.scores().reshape(-1)[: K * n_eps].reshape(K, n_eps)


@pytest.mark.parametrize("delay", [0, 16])
def test_region_scores_match_oracle_on_a_random_structure(delay):
    """Random mixed structure (uploaded), then in deferred mode a few pixel moves
    so that pending terms enter the in-block entries."""
    p = _lens(12)
    idx = W.random_eps_idx(p, 0.35, seed=21)
    job = _job(p, delay=delay)
    job.init()                                            # workspace, no pending terms
    G, E = ost.dense_state(p, ost.eps_of(p, idx))
    job.upload_state(G, E, np.diagonal(G[: p.n]).copy(), idx)
    if delay:
        job.run_greedy(9, poll_every=9)                  # 9 pending rank-1 terms
        idx = job.eps_idx.cpu().numpy()
    job.region_step(apply="sequential")                   # scores, pick, pixel moves, apply
    F_gpu = _gpu_region_scores(job).copy()
    ev = orr._RegionEvaluator(p, 2, "T1")
    Eo, row, G_VV = ev(idx)
    F = orr.region_scores(p, 2, Eo, G_VV, row, idx)
    fin = np.isfinite(F)
    assert np.array_equal(np.isfinite(F_gpu), fin)
    assert np.allclose(F_gpu[fin], F[fin], rtol=1e-10, atol=0)


def test_region_greedy_matches_oracle_trajectory():
    p = _lens(16)
    ref = orr.region_greedy(p, 2, steps=200, tier="T2")
    assert ref.stopped and len(ref.steps) >= 10
    job = _job(p)
    job.init()
    n, moves = job.run_region_greedy(200, poll_every=8)
    assert moves == [(s.pixel, s.eps_idx) for s in ref.steps]
    assert abs(job.fom() - ref.steps[-1].fom) <= 1e-9 * ref.steps[-1].fom
    E = job.E.cpu().numpy()
    assert rel_elem(E, ref.E) <= 1e-9 and job.status() == 0


@pytest.mark.parametrize("dtype,delay", [("c128", 16), ("c64", 64)])
def test_region_greedy_deferred_equals_eager(dtype, delay):
    p = _lens(24, dtype=dtype)
    a = _job(p)
    a.init()
    na, ma = a.run_region_greedy(300, poll_every=16)
    b = _job(p, delay=delay)
    b.init()
    nb, mb = b.run_region_greedy(300, poll_every=16)
    assert ma == mb and na >= 10
    Ga, Ea, _, _ = a.host_state()
    Gb, Eb, _, _ = b.host_state()
    tol = 1e-12 if dtype == "c128" else c64_drift_tol(b.n_flips())
    assert rel_elem(Gb, Ga) <= tol
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, b.eps_idx.cpu().numpy()))
    assert rel_elem(Eb, Ed) <= (1e-11 if dtype == "c128" else 2e-5)


@pytest.mark.parametrize("delay", [0, 16])
def test_region_rank_k_application_equals_sequential(delay):
    """Joint rank-k application of the region moves equals the pixel moves one by
    one; with delay > 0 the rank-k step follows flushes that leave the lower
    triangle of the design block out of date, so it reads the upper one."""
    p = _lens(24, dtype="c64")
    a = _job(p)
    a.init()
    na, ma = a.run_region_greedy(300, poll_every=16, apply="sequential")
    b = _job(p, delay=delay)
    b.init()
    nb, mb = b.run_region_greedy(300, poll_every=16, apply="rank_k")
    assert ma == mb and na >= 10
    Ga, Ea, _, _ = a.host_state()
    Gb, Eb, _, _ = b.host_state()
    tol = c64_drift_tol(b.n_flips())
    assert rel_elem(Gb, Ga) <= tol
    assert rel_elem(Eb, Ea) <= tol


def _lens3(n, dtype="c128"):
    """The lens with a three-entry permittivity table, every material a candidate."""
    return _lens(n, dtype).replace(eps_table=(1.0, 12.25, 2.25), cand_mask=0b111)


def test_region_scores_three_materials():
    """Regions of mixed materials: a candidate is any material that changes at
    least one of the region's pixels."""
    p = _lens3(12)
    idx = W.random_material_idx(p, seed=5)
    job = _job(p)
    job.init()
    G, E = ost.dense_state(p, ost.eps_of(p, idx))
    job.upload_state(G, E, np.diagonal(G[: p.n]).copy(), idx)
    job.region_step(apply="sequential")
    F_gpu = _gpu_region_scores(job).copy()
    ev = orr._RegionEvaluator(p, 2, "T1")
    Eo, row, G_VV = ev(idx)
    F = orr.region_scores(p, 2, Eo, G_VV, row, idx)
    assert F.shape == F_gpu.shape and F.shape[1] == 3
    fin = np.isfinite(F)
    assert np.array_equal(np.isfinite(F_gpu), fin)
    assert np.allclose(F_gpu[fin], F[fin], rtol=1e-10, atol=0)


def test_region_greedy_three_materials_matches_oracle():
    p = _lens3(16)
    ref = orr.region_greedy(p, 2, steps=200, tier="T2")
    assert ref.stopped and len(ref.steps) >= 10
    job = _job(p)
    job.init()
    n, moves = job.run_region_greedy(200, poll_every=8)
    assert moves == [(s.pixel, s.eps_idx) for s in ref.steps]
    E = job.E.cpu().numpy()
    assert rel_elem(E, ref.E) <= 1e-9 and job.status() == 0


def test_region_moves_on_an_odd_grid_are_refused():
    """2x2 regions need an even grid: EINVAL before any launch, state untouched."""
    from paper_2202_05388_amd import _lib as L
    p = _lens(12).replace(nx=13)
    job = _job(p)
    job.init()
    with pytest.raises(L.GfoError):
        job.region_step(apply="sequential")
    assert job.n_flips() == 0 and job.status() == 0
