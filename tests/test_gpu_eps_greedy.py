"""Epsilon-greedy policy on the GPU (paper Sec. V): top-4 scores, the drawn
choice, rank-1 apply.  The move sequence must be the oracle's, draw for draw."""
import numpy as np
import pytest

from oracle import greedy as og
from oracle import state as ost
import workloads as W
from parity import c64_drift_tol, rel_elem

pytestmark = pytest.mark.gpu


def _job(p, **kw):
    from paper_2202_05388_amd.job import Job
    print(f"[case] {p.name} {p.ny}x{p.nx} {p.dtype} {kw}", flush=True)
    return Job(p, device="cuda:0", **kw)


@pytest.mark.parametrize("eps,seed", [(0.1, 7), (0.3, 8), (1.0, 9)])
def test_eps_greedy_square21_matches_oracle(eps, seed):
    p = W.SQUARE_21
    draws = W.eps_greedy_draws(400, seed)
    ref = og.eps_greedy(p, eps, draws, tier="T2")
    assert ref.stopped
    job = _job(p)
    job.init()
    n = job.run_eps_greedy(eps, draws, poll_every=16)
    hist = [(int(a), int(b)) for a, b in job.history()]
    assert hist == [(s.pixel, s.eps_idx) for s in ref.steps] and n == len(ref.steps)
    assert abs(job.fom() - ref.steps[-1].fom) <= 1e-9 * ref.steps[-1].fom
    E = job.E.cpu().numpy()
    assert rel_elem(E, ref.E) <= 1e-9
    assert job.status() == 0


def test_eps_zero_is_the_greedy_path():
    p = W.SQUARE_21
    a = _job(p)
    a.init()
    a.run_greedy(400, poll_every=16)
    b = _job(p)
    b.init()
    b.run_eps_greedy(0.0, W.eps_greedy_draws(400, 1), poll_every=16)
    assert np.array_equal(a.history(), b.history())


@pytest.mark.parametrize("dtype,delay", [("c128", 16), ("c64", 8)])
def test_eps_greedy_deferred_equals_eager(dtype, delay):
    p = W.SQUARE_21.replace(dtype=dtype, tau=1e-9 if dtype == "c128" else 1e-6)
    draws = W.eps_greedy_draws(400, 4)
    a = _job(p)
    a.init()
    a.run_eps_greedy(0.2, draws, poll_every=16)
    b = _job(p, delay=delay)
    b.init()
    b.run_eps_greedy(0.2, draws, poll_every=16)
    assert np.array_equal(a.history(), b.history())
    Ga, Ea, _, _ = a.host_state()
    Gb, Eb, _, _ = b.host_state()
    tol = 1e-12 if dtype == "c128" else c64_drift_tol(b.n_flips())
    assert rel_elem(Gb, Ga) <= tol
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, b.eps_idx.cpu().numpy()))
    assert rel_elem(Eb, Ed) <= (1e-11 if dtype == "c128" else 2e-5)


@pytest.mark.parametrize("eps,seed", [(0.3, 11), (1.0, 12)])
def test_eps_greedy_three_materials_matches_oracle(eps, seed):
    """With three materials a pixel has two candidate moves, so the exploration set
    (the best move at each of the four best distinct pixels) differs from the four
    best moves."""
    p = W.SQUARE_21.replace(eps_table=(1.0, 12.25, 2.25), cand_mask=0b111)
    draws = W.eps_greedy_draws(600, seed)
    ref = og.eps_greedy(p, eps, draws, tier="T2", steps=600)
    assert ref.stopped and len({s.eps_idx for s in ref.steps}) == 3
    job = _job(p)
    job.init()
    n = job.run_eps_greedy(eps, draws, poll_every=16)
    hist = [(int(a), int(b)) for a, b in job.history()]
    assert hist == [(s.pixel, s.eps_idx) for s in ref.steps] and n == len(ref.steps)
    E = job.E.cpu().numpy()
    assert rel_elem(E, ref.E) <= 1e-9
    assert job.status() == 0


@pytest.mark.parametrize("dtype,delay,eps", [("c128", 0, 0.3), ("c64", 8, 0.3), ("c64", 16, 0.1),
                                             ("c64", 0, 0.5)])
def test_eps_greedy_fused_runs_equal_per_step_path(dtype, delay, eps):
    """Steps whose draw does not explore go through gfo_greedy_steps in runs; the
    moves and the whole state equal, bit for bit, those of every step taken
    through the top-4 selection, the drawn choice and apply_flip."""
    p = W.tiny(40, 40, n_mon=8, dtype=dtype, cand_mask=W.MASK_BOTH,
               tau=1e-9 if dtype == "c128" else 1e-6)
    draws = W.eps_greedy_draws(600, 11)
    out = []
    for fused in (False, True):
        job = _job(p, delay=delay)
        job.init()
        n = job.run_eps_greedy(eps, draws, poll_every=24, fused=fused)
        G, E, d, idx = job.host_state()
        out.append((n, job.history(), G, E, d, idx, job.status()))
    (n0, h0, G0, E0, d0, i0, s0), (n1, h1, G1, E1, d1, i1, s1) = out
    assert n0 == n1 > 50 and np.array_equal(h0, h1)
    assert np.array_equal(G0, G1) and np.array_equal(E0, E1) and np.array_equal(d0, d1)
    assert np.array_equal(i0, i1) and s0 == s1 == 0
