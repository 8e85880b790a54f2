"""GPU parity of the greedy step (init_G0, score_candidates, apply_flip) against the
FP64 oracle, through the C ABI.

Tolerances: complex128 storage is compared at 1e-12 relative for single
operations and 1e-9 along trajectories (fields, FOM); complex64 storage at
3e-7 relative for init (one rounding) and 1e-4 along trajectories.
"""
import json
import os

import numpy as np
import pytest

from oracle import greens, greedy as og, state as ost
import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _job(p, **kw):
    import torch
    from paper_2202_05388_amd.job import Job
    print(f"[case] {p.name} {p.ny}x{p.nx} mon={p.n_mon} {kw.get('dtype', p.dtype)}", flush=True)
    j = Job(p, device="cuda:0", **kw)
    return j


# element-wise relative error with an absolute floor of 1e-3 x the largest entry
from parity import c64_drift_tol, rel_elem as _rel  # noqa: E402


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(6, 8, 4), (5, 7, 3), (1, 1, 1), (3, 70, 2)])
def test_init_G0_matches_oracle(dtype, shape):
    ny, nx, nm = shape
    p = W.tiny(ny, nx, n_mon=nm, dtype=dtype)
    job = _job(p)
    job.init()
    G, E, diag, eps_idx = job.host_state()
    G0 = greens.build_G0(p)
    Einc = greens.incident_field(p)
    tol = 1e-13 if dtype == "c128" else 3e-7
    assert np.max(np.abs(G - G0)) <= tol * np.max(np.abs(G0))
    assert np.max(np.abs(E - Einc)) <= tol
    st = greens.self_term(p.pitch, greens.k0_of(p))
    assert np.allclose(diag, st, rtol=1e-14, atol=0)
    assert np.all(eps_idx == 0) and job.n_flips() == 0 and job.status() == 0
    # padding columns are zero
    import torch
    pad = job.G[:, job.N:].abs().max().item() if job.ld > job.N else 0.0
    assert pad == 0.0


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_scores_and_selection_on_random_state(seed, dtype):
    p = W.tiny(9, 11, n_mon=6, dtype=dtype, cand_mask=W.MASK_BOTH)
    N = p.n
    idx = W.random_eps_idx(p, 0.3, seed)
    G, E = ost.dense_state(p, ost.eps_of(p, idx))
    job = _job(p)
    job.upload_state(G, E, np.diagonal(G[:N]), idx)
    job.score(topk=1, tau=1e-9)
    F_gpu = job.scores()
    F_ref = og.scores_closed_form(p, E, np.diagonal(G[:N]), G[N + p.fom_monitor], idx)
    fin = np.isfinite(F_ref)
    assert np.array_equal(fin, np.isfinite(F_gpu))
    tol = 1e-12 if dtype == "c128" else 1e-6
    assert np.allclose(F_gpu[fin], F_ref[fin], rtol=tol, atol=0)
    pick = job.read_picks(1)[0]
    ref = og.select_greedy(F_ref, ost.fom_of_state(p, E), 1e-9)
    assert (pick[0], pick[1]) == (ref.pixel, ref.eps_idx)
    assert abs(pick[2] - ref.fom_new) <= tol * ref.fom_new


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_apply_flip_equals_paper_update_and_resolve(dtype):
    p = W.tiny(8, 9, n_mon=5, dtype=dtype)
    N = p.n
    idx = W.random_eps_idx(p, 0.25, 3)
    eps = ost.eps_of(p, idx)
    G, E = ost.dense_state(p, eps)
    job = _job(p)
    job.upload_state(G, E, np.diagonal(G[:N]), idx)
    j = 37
    new = 1 - int(idx[j])
    job.set_pick(j, new)
    job.apply()
    G1, E1, d1, idx1 = job.host_state()
    Gu, Eu = ost.update_region(p, G, E, eps, [j], [p.eps_table[new]])
    idx2 = idx.copy()
    idx2[j] = new
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx2))
    tol = 1e-12 if dtype == "c128" else 2e-6
    assert _rel(G1, Gu) <= tol and _rel(G1, Gd) <= tol
    assert _rel(E1, Eu) <= tol and _rel(E1, Ed) <= tol
    assert _rel(d1, np.diagonal(Gd[:N])) <= (1e-12 if dtype == "c128" else 2e-6)
    assert idx1[j] == new and job.n_flips() == 1
    assert [tuple(r) for r in job.history()] == [(j, new)]


def test_sentinel_and_invalid_picks_are_noops():
    p = W.tiny(4, 6, n_mon=4)
    job = _job(p)
    job.init()
    G0, E0, d0, i0 = job.host_state()
    for pix, e in [(-1, 1), (p.n, 1), (3, 0), (3, 7)]:
        job.set_pick(pix, e)
        job.apply()
    G1, E1, d1, i1 = job.host_state()
    assert np.array_equal(G0, G1) and np.array_equal(E0, E1) and np.array_equal(d0, d1)
    assert job.n_flips() == 0 and job.status() == 0


def test_greedy_stops_when_nothing_improves():
    """Add-only flips on a grid where every pixel is already material: no candidate."""
    p = W.tiny(3, 4, n_mon=2, cand_mask=W.MASK_ADD_ONLY)
    N = p.n
    idx = np.ones(N, np.uint8)
    G, E = ost.dense_state(p, ost.eps_of(p, idx))
    job = _job(p)
    job.upload_state(G, E, np.diagonal(G[:N]), idx)
    job.score()
    pk = job.read_picks(1)[0]
    assert pk[0] == -1
    assert np.all(np.isneginf(job.scores()))


def test_square32_fp64_trajectory_matches_stored_oracle():
    """32x32 FP64: 50 greedy steps; pixel sequence exact, FOM and fields 1e-9."""
    gold = json.load(open(os.path.join(HERE, "golden", "square32_fp64.json")))
    p = W.SMALL_32
    job = _job(p)
    job.init()
    n = job.run_greedy(p.steps, poll_every=10)
    hist = job.history()
    assert n == len(gold["steps"])
    assert [int(x) for x in hist[:, 0]] == [s["pixel"] for s in gold["steps"]]
    assert [int(x) for x in hist[:, 1]] == [s["eps_idx"] for s in gold["steps"]]
    G, E, d, idx = job.host_state()
    N = p.n
    Emon = np.array([complex(*z) for z in gold["final"]["E_mon"]])
    Epix = np.array([complex(*z) for z in gold["final"]["E_pix"]])
    assert _rel(E[N:], Emon) <= 1e-9
    assert _rel(E[gold["sample_pixels"]], Epix) <= 1e-9
    assert abs(job.fom() - gold["steps"][-1]["fom"]) <= 1e-9 * gold["steps"][-1]["fom"]
    assert job.status() == 0


def test_square32_fp64_state_matches_dense_resolve():
    """After 20 steps the whole G (design + monitor rows) equals the T1 re-solve."""
    p = W.SMALL_32
    job = _job(p)
    job.init()
    job.run_greedy(20, poll_every=20)
    G, E, d, idx = job.host_state()
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx))
    assert _rel(G, Gd) <= 1e-11
    assert _rel(E, Ed) <= 1e-11
    assert _rel(d, np.diagonal(Gd[: p.n])) <= 1e-11


def test_k1_variants_bitwise_identical():
    from paper_2202_05388_amd import _lib as L
    for dtype, code in (("c64", L.GFO_C64), ("c128", L.GFO_C128)):
        p = W.tiny(7, 9, n_mon=5, dtype=dtype)
        N = p.n
        idx = W.random_eps_idx(p, 0.3, 5)
        G, E = ost.dense_state(p, ost.eps_of(p, idx))
        outs = []
        old = L.k1_get_variant(code)
        try:
            for v in range(len(L.k1_variants(code))):
                L.k1_set_variant(code, v)
                job = _job(p)
                job.upload_state(G, E, np.diagonal(G[:N]), idx)
                job.set_pick(20, 1 - int(idx[20]))
                job.apply()
                outs.append(job.host_state()[0])
        finally:
            L.k1_set_variant(code, old)
        for o in outs[1:]:
            assert np.array_equal(o, outs[0])


def test_run_is_deterministic():
    p = W.tiny(12, 12, n_mon=4, dtype="c64", steps=30)
    res = []
    for _ in range(2):
        job = _job(p)
        job.init()
        job.run_greedy(30, poll_every=8)
        res.append(job.host_state())
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype,refresh_every", [("c64", 0), ("c128", 0), ("c64", 50)])
def test_eager_upper_triangle_equals_full(dtype, refresh_every):
    """Eager rank-1 updates that keep only the upper triangle of the design block
    (lower_stale = 1 before init_G0 and refresh_G; the update skips the tiles
    below the diagonal) make the same moves as full eager updates and, with the
    lower triangle copied back, leave the same state."""
    from paper_2202_05388_amd.job import Job
    p = W.tiny(40, 44, n_mon=8, dtype=dtype, cand_mask=W.MASK_BOTH)
    print(f"[case] eager upper {dtype} refresh {refresh_every}", flush=True)
    full = Job(p, device="cuda:0", kmax=256)
    full.init()
    n_full = full.run_greedy(150, poll_every=25, refresh_every=refresh_every)
    up = Job(p, device="cuda:0", kmax=256, upper=True)
    up.init()
    assert up.state.lower_stale == 1
    n_up = up.run_greedy(150, poll_every=25, refresh_every=refresh_every)
    assert n_up == n_full > 100
    assert up.state.lower_stale == 1
    assert np.array_equal(up.history(), full.history())
    Gf, Ef, df, i_f = full.host_state()
    Gu, Eu, du, iu = up.host_state()
    tol = 1e-12 if dtype == "c128" else c64_drift_tol(n_full)
    assert _rel(Gu, Gf) <= tol and _rel(Eu, Ef) <= tol and _rel(du, df) <= tol
    assert np.array_equal(iu, i_f) and up.status() == 0


@pytest.mark.parametrize("delay", [0, 16])
def test_invalid_arguments_are_refused_before_any_launch(delay):
    """An empty candidate mask (also one with only bits past the table), a tie band
    outside [0, 1), topk outside 1..GFO_MAX_RANK_K, a negative spacing or step
    count: EINVAL, and the state is left as it was."""
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(8, 9, n_mon=5, dtype="c64", cand_mask=W.MASK_BOTH)
    job = _job(p, delay=delay)
    job.init()
    E0 = job.E.cpu().clone()
    bad_scores = [dict(cand_mask=0), dict(cand_mask=0b100), dict(tau=-1e-9), dict(tau=1.0),
                  dict(tau=float("nan")), dict(topk=0), dict(topk=L.GFO_MAX_RANK_K + 1),
                  dict(min_spacing=-1)]
    for kw in bad_scores:
        with pytest.raises(L.GfoError):
            job.score(**kw)
    for kw in (dict(cand_mask=0), dict(tau=float("inf"))):
        with pytest.raises(L.GfoError):
            job.greedy_steps(4, **kw)
    with pytest.raises(L.GfoError):
        job.greedy_steps(-1)
    job.greedy_steps(0)
    assert job.n_flips() == 0 and job.status() == 0
    assert job.state.pending_calls == 0
    assert bool((job.E.cpu() == E0).all())
