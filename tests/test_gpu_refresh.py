"""GPU parity of refresh_G (FP64 re-solve from G0 and the flipped set) and of the
128x128 trajectories (complex128 plain loop; complex64 with refresh) against the
stored FP64 oracle trajectory."""
import json
import os

import numpy as np
import pytest

from oracle import greens, greedy as og, state as ost
import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _job(p, **kw):
    from paper_2202_05388_amd.job import Job
    print(f"[case] {p.name} {p.ny}x{p.nx} mon={p.n_mon} {p.dtype} {kw}", flush=True)
    return Job(p, device="cuda:0", **kw)


# element-wise relative error with an absolute floor of 1e-3 x the largest entry
from parity import c64_drift_tol, certify_sequence, rel_elem as _rel  # noqa: E402


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("fill,seed", [(0.0, 0), (0.05, 1), (0.3, 2)])
def test_refresh_equals_dense_resolve(dtype, fill, seed):
    p = W.tiny(9, 13, n_mon=6, dtype=dtype)
    N = p.n
    idx = W.random_eps_idx(p, fill, seed)
    k = int(idx.sum())
    job = _job(p, kmax=max(k, 1))
    job.init()
    # garbage in G/E/diag, the structure only in eps_idx: refresh must rebuild everything
    rng = np.random.default_rng(seed)
    junk = rng.standard_normal((p.rows, N)) + 1j * rng.standard_normal((p.rows, N))
    job.upload_state(junk, junk[:, 0], junk[:N, 1], idx)
    job.refresh()
    G, E, d, idx2 = job.host_state()
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx))
    tol = 1e-12 if dtype == "c128" else 3e-7
    assert _rel(G, Gd) <= tol
    assert _rel(E, Ed) <= tol
    assert _rel(d, np.diagonal(Gd[:N])) <= 1e-12          # diag64 is FP64 in both modes
    assert np.array_equal(idx, idx2) and job.status() == 0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("upper", [False, True])
def test_refresh_large_flipped_set_equals_dense_resolve(dtype, upper):
    """301 flipped pixels of 624 (kp = 304): each Gauss-Jordan step spans two
    256-column chunks and 38 row groups, the products have ragged 128-row tiles
    and a partial chunk of 8 terms.  With the upper triangle kept alone the
    product leaves out the tiles below the diagonal; the lower triangle copied
    back gives the same state.

    Tolerance: two FP64 solves of one system differ by up to a modest multiple
    of u kappa, u = 2^-53 and kappa the 2-norm condition number of the core
    diag(1/alpha) - G0[V,V] (here about 1.1e3).  LAPACK's own inverse put
    through the same Woodbury formula lands 21 u kappa from the dense solve;
    the bound is 100 u kappa (complex64: plus one rounding)."""
    p = W.tiny(24, 26, n_mon=6, dtype=dtype)
    N = p.n
    rng = np.random.default_rng(7)
    idx = np.zeros(N, np.uint8)
    idx[rng.choice(N, 301, replace=False)] = 1
    job = _job(p, kmax=301, upper=upper)
    job.init()
    junk = rng.standard_normal((p.rows, N)) + 1j * rng.standard_normal((p.rows, N))
    job.upload_state(junk, junk[:, 0], junk[:N, 1], idx)
    job.state.lower_stale = int(upper)
    job.refresh()
    assert job.state.lower_stale == int(upper)
    G, E, d, idx2 = job.host_state()
    eps = ost.eps_of(p, idx)
    Gd, Ed = ost.dense_state(p, eps)
    G0 = greens.build_G0(p)
    alpha = greens.alpha_of(p, eps)
    V = np.nonzero(alpha != 0)[0]
    kappa = np.linalg.cond(np.diag(1.0 / alpha[V]) - G0[np.ix_(V, V)])
    tol64 = max(1e-12, 100 * 2.0 ** -53 * kappa)
    tol = tol64 if dtype == "c128" else 3e-7 + tol64
    print(f"kappa {kappa:.3g}: G {_rel(G, Gd):.3g}, E {_rel(E, Ed):.3g} (bound {tol:.3g})", flush=True)
    assert _rel(G, Gd) <= tol
    assert _rel(E, Ed) <= tol
    assert _rel(d, np.diagonal(Gd[:N])) <= tol64
    assert np.array_equal(idx, idx2) and job.status() == 0


def test_refresh_overflow_sets_status_and_changes_nothing():
    """More flipped pixels than kmax: GFO_ERANGE, the status bit, and the state
    exactly as it was."""
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(6, 6, n_mon=4)
    idx = W.random_eps_idx(p, 0.5, 3)
    job = _job(p, kmax=4)
    job.init()
    G0, E0, d0, _ = job.host_state()
    import torch
    job.eps_idx.copy_(torch.from_numpy(idx))
    with pytest.raises(L.GfoError) as err:
        job.refresh()
    assert err.value.code == L.GFO_ERANGE
    G1, E1, d1, _ = job.host_state()
    assert job.status() & L.GFO_STATUS_REFRESH_OVERFLOW
    assert np.array_equal(G0, G1) and np.array_equal(E0, E1) and np.array_equal(d0, d1)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_refresh_overflow_in_deferred_mode_keeps_pending_terms(dtype):
    """Deferred mode with pending terms and a flipped set larger than kmax: the
    refused refresh keeps the pending terms and the pending count, so the state
    after the next flush is still the dense re-solve of the structure."""
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(10, 12, n_mon=4, dtype=dtype)
    job = _job(p, kmax=3, delay=16)
    job.init()
    n = job.run_greedy(9, poll_every=9)
    assert n == 9 and job.state.pending_calls == 9
    with pytest.raises(L.GfoError) as err:
        job.refresh()
    assert err.value.code == L.GFO_ERANGE
    assert job.state.pending_calls == 9
    assert job.status() & L.GFO_STATUS_REFRESH_OVERFLOW
    G, E, d, idx = job.host_state()                 # flushes the nine pending terms
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx))
    tol = 1e-11 if dtype == "c128" else c64_drift_tol(9)
    assert _rel(G, Gd) <= tol and _rel(E, Ed) <= tol
    assert _rel(d, np.diagonal(Gd[:p.n])) <= (1e-11 if dtype == "c128" else 2e-6)


def test_refresh_is_idempotent_and_removes_drift_c64():
    p = W.tiny(20, 20, n_mon=8, dtype="c64", steps=60)
    job = _job(p, kmax=64)
    job.init()
    job.run_greedy(60, poll_every=20)
    G_b, E_b, d_b, idx = job.host_state()
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx))
    before = _rel(G_b, Gd)
    job.refresh()
    G1, E1, d1, _ = job.host_state()
    job.refresh()
    G2, E2, d2, _ = job.host_state()
    after = _rel(G1, Gd)
    assert after <= 3e-7 and after <= before
    assert np.array_equal(G1, G2) and np.array_equal(E1, E2)
    assert _rel(E1, Ed) <= 3e-7


def _gold128():
    return json.load(open(os.path.join(HERE, "golden", "square128_fp64.json")))


def _c(z):
    return np.array([complex(*v) for v in z])


def test_square128_fp64_trajectory_matches_oracle():
    """Plain complex128 loop: exact pixel sequence to termination, fields/FOM 1e-9."""
    gold = _gold128()
    p = W.SQUARE_128_FP64
    N = p.n
    job = _job(p)
    job.init()
    n100 = job.run_greedy(100, poll_every=50)
    assert n100 == 100
    _, E, _, _ = job.host_state()
    ck = gold["checkpoints"]["100"]
    assert _rel(E[N:], _c(ck["E_mon"])) <= 1e-9
    assert _rel(E[gold["sample_pixels"]], _c(ck["E_pix"])) <= 1e-9
    n = 100 + job.run_greedy(2000, poll_every=64)
    assert n == len(gold["steps"])
    hist = job.history()
    assert [int(x) for x in hist[:, 0]] == [s["pixel"] for s in gold["steps"]]
    _, E, _, _ = job.host_state()
    assert _rel(E[N:], _c(gold["final"]["E_mon"])) <= 1e-9
    assert abs(job.fom() - gold["steps"][-1]["fom"]) <= 1e-9 * gold["steps"][-1]["fom"]


@pytest.mark.parametrize("refresh_every", [0, 64])
def test_square128_c64_trajectory_matches_oracle(refresh_every):
    """complex64 storage, FP64 denominators, optional FP64 refresh: same pixel
    sequence as the FP64 oracle except at certified ties; fields and FOM within
    1e-4 at step 100 and at the end."""
    gold = _gold128()
    p = W.SQUARE_128
    N = p.n
    job = _job(p, kmax=256)
    job.init()
    n100 = job.run_greedy(100, poll_every=32, refresh_every=refresh_every)
    assert n100 == 100
    _, E, _, _ = job.host_state()
    ck = gold["checkpoints"]["100"]
    assert _rel(E[N:], _c(ck["E_mon"])) <= 1e-4
    assert _rel(E[gold["sample_pixels"]], _c(ck["E_pix"])) <= 1e-4
    n = 100 + job.run_greedy(2000, poll_every=32, refresh_every=refresh_every)
    hist = [(int(a), int(b)) for a, b in job.history()]
    gp = [(s["pixel"], s["eps_idx"]) for s in gold["steps"]]
    _, E, _, _ = job.host_state()
    seen = {}
    t = certify_sequence(p, gp, hist, checkpoints=[len(hist)],
                         on_state=lambda step, Ex: seen.setdefault(step, Ex))
    print(f"c64 sequence: {n} moves, identical for the first {t}, oracle {len(gp)}", flush=True)
    assert t >= 150
    if t == len(gp) == len(hist):
        assert _rel(E[N:], _c(gold["final"]["E_mon"])) <= 1e-4
        assert _rel(E[gold["sample_pixels"]], _c(gold["final"]["E_pix"])) <= 1e-4
    else:
        # the final fields against the oracle's state of the GPU's own structure
        Ex = seen[len(hist)]
        assert _rel(E[N:], Ex[N:]) <= 1e-4
        assert _rel(E[gold["sample_pixels"]], Ex[gold["sample_pixels"]]) <= 1e-4
    assert abs(job.fom() - gold["steps"][-1]["fom"]) <= 1e-4 * gold["steps"][-1]["fom"]
    assert job.status() == 0
