"""Deferred rank-1 updates (state.delay > 0): pending terms, eager E / diagonal /
monitor rows, rank-r matrix-core flush.  The move sequence and the state after a
flush must equal eager mode and the oracle."""
import json
import os

import numpy as np
import pytest

from oracle import state as ost
import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _job(p, **kw):
    from paper_2202_05388_amd.job import Job
    print(f"[case] {p.name} {p.ny}x{p.nx} {p.dtype} {kw}", flush=True)
    return Job(p, device="cuda:0", **kw)


# element-wise relative error with an absolute floor of 1e-3 x the largest entry
from parity import c64_drift_tol, rel_elem as _rel  # noqa: E402


@pytest.mark.parametrize("dtype,delay", [("c128", 16), ("c128", 64), ("c64", 16), ("c64", 64),
                                         ("c64", 7), ("c64", 128), ("c128", 100)])
def test_deferred_equals_eager(dtype, delay):
    p = W.tiny(24, 28, n_mon=8, dtype=dtype, cand_mask=W.MASK_BOTH)
    eager = _job(p)
    eager.init()
    n1 = eager.run_greedy(150, poll_every=25)
    lazy = _job(p, delay=delay)
    lazy.init()
    n2 = lazy.run_greedy(150, poll_every=25)
    assert n1 == n2
    assert np.array_equal(eager.history(), lazy.history())
    Ge, Ee, de, ie = eager.host_state()
    Gl, El, dl, il = lazy.host_state()
    tol = 1e-12 if dtype == "c128" else c64_drift_tol(n1)
    assert _rel(Gl, Ge) <= tol and _rel(El, Ee) <= tol and _rel(dl, de) <= tol
    assert np.array_equal(ie, il) and lazy.status() == 0
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, il))
    assert _rel(Gl, Gd) <= (1e-11 if dtype == "c128" else c64_drift_tol(n1))


def test_deferred_square32_fp64_matches_stored_oracle():
    gold = json.load(open(os.path.join(HERE, "golden", "square32_fp64.json")))
    p = W.SMALL_32
    job = _job(p, delay=8)
    job.init()
    n = job.run_greedy(p.steps, poll_every=10)
    hist = job.history()
    assert n == len(gold["steps"])
    assert [int(x) for x in hist[:, 0]] == [s["pixel"] for s in gold["steps"]]
    _, E, _, _ = job.host_state()
    Emon = np.array([complex(*z) for z in gold["final"]["E_mon"]])
    assert _rel(E[p.n:], Emon) <= 1e-9


@pytest.mark.parametrize("fused", [False, True])
def test_deferred_square128_c64_matches_oracle(fused):
    """128 x 128 pixels, complex64, deferred rank-1 updates flushed every 64 moves,
    chunks of 32 moves, refresh every 256 (the benchmark's configuration); fused:
    gfo_greedy_steps (one kernel per move), else score_candidates + apply_flip.
    The fields at the monitors and at sampled pixels after 100 moves, the move
    sequence (up to certified ties) and the final FOM match the FP64 oracle."""
    from parity import certify_sequence
    gold = json.load(open(os.path.join(HERE, "golden", "square128_fp64.json")))
    p = W.SQUARE_128
    N = p.n
    job = _job(p, delay=64, kmax=512)
    job.init()
    assert job.run_greedy(100, poll_every=32, refresh_every=256, fused=fused) == 100
    E = job.E.cpu().numpy().astype(np.complex128)      # E is current in deferred mode
    ck = gold["checkpoints"]["100"]
    Em = np.array([complex(*z) for z in ck["E_mon"]])
    assert _rel(E[N:], Em) <= 1e-4
    Ep = np.array([complex(*z) for z in ck["E_pix"]])
    assert _rel(E[gold["sample_pixels"]], Ep) <= 1e-4
    job.run_greedy(2000, poll_every=32, refresh_every=256, fused=fused)
    hist = [(int(a), int(b)) for a, b in job.history()]
    gp = [(s["pixel"], s["eps_idx"]) for s in gold["steps"]]
    t = certify_sequence(p, gp, hist)
    print(f"deferred c64 sequence identical for {t} of {len(gp)}", flush=True)
    assert t >= 150
    assert abs(job.fom() - gold["steps"][-1]["fom"]) <= 1e-4 * gold["steps"][-1]["fom"]


def test_flush_on_demand_and_partial_pending():
    p = W.tiny(16, 18, n_mon=6, dtype="c128")
    job = _job(p, delay=64)
    job.init()
    job.run_greedy(23, poll_every=23)                 # 23 pending terms, no automatic flush yet
    assert job.state.pending_calls == 23
    G, E, d, idx = job.host_state()                   # flushes
    assert job.state.pending_calls == 0
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx))
    assert _rel(G, Gd) <= 1e-11 and _rel(E, Ed) <= 1e-11 and _rel(d, np.diagonal(Gd[: p.n])) <= 1e-11


def test_refresh_discards_pending_and_rank_k_flushes_first():
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(16, 18, n_mon=6, dtype="c64")
    job = _job(p, delay=16, kmax=64)
    job.init()
    job.run_greedy(10, poll_every=10)
    job.refresh()                                     # pending terms dropped, G rebuilt in FP64
    G, E, d, idx = job.host_state()
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx))
    assert _rel(G, Gd) <= 3e-7
    job.run_greedy(5, poll_every=5)                   # five pending terms
    idx0 = job.eps_idx.cpu().numpy()
    job.score(topk=4, min_spacing=3)
    picks = [(a, b) for a, b, _, _ in job.read_picks(4) if a >= 0]
    job.apply_rank_k(4, precision=L.GFO_FP32)
    G, E, d, idx = job.host_state()
    idx1 = idx0.copy()
    for a, b in picks:
        idx1[a] = b
    assert np.array_equal(idx, idx1)
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx))
    assert _rel(G, Gd) <= 2e-5 and _rel(E, Ed) <= 2e-5


@pytest.mark.parametrize("dtype,delay,fused", [("c128", 16, False), ("c64", 16, False),
                                               ("c64", 16, True), ("c128", 8, True)])
def test_graph_replays_equal_stream_launches(dtype, delay, fused):
    """A captured window of steps, replayed with host polls and device work between
    replays, gives the same moves and state as launching every step on a stream."""
    p = W.tiny(20, 22, n_mon=6, dtype=dtype, cand_mask=W.MASK_BOTH)
    ref = _job(p, delay=delay)
    ref.init()
    n_ref = ref.run_greedy(5 * delay, poll_every=delay)
    job = _job(p, delay=delay)
    job.init()
    n = job.run_greedy_graph(5 * delay, window=delay, fused=fused)
    assert n == n_ref
    assert np.array_equal(job.history(), ref.history())
    Gr, Er, dr, ir = ref.host_state()
    G, E, d, i = job.host_state()
    assert np.array_equal(G, Gr) and np.array_equal(E, Er) and np.array_equal(d, dr)


@pytest.mark.parametrize("delay", [64, 128])
def test_flush_variants_agree(delay):
    """Every complex64 flush variant gives the eager move sequence and state."""
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(40, 44, n_mon=8, dtype="c64", cand_mask=W.MASK_BOTH)
    eager = _job(p)
    eager.init()
    n_ref = eager.run_greedy(150, poll_every=25)
    Ge, Ee, de, ie = eager.host_state()
    names = L.flush_variants()
    old = L.flush_get_variant()
    states = {}
    try:
        for vi, name in enumerate(names):
            L.flush_set_variant(vi)
            print(f"[flush variant] {name}", flush=True)
            job = _job(p, delay=delay)
            job.init()
            assert job.run_greedy(150, poll_every=25) == n_ref
            assert np.array_equal(job.history(), eager.history())
            G, E, d, i = job.host_state()
            tol = c64_drift_tol(n_ref)
            assert _rel(G, Ge) <= tol and _rel(E, Ee) <= tol and np.array_equal(i, ie)
            states[name] = G
    finally:
        L.flush_set_variant(old)
    assert len(states) == len(names)




@pytest.mark.parametrize("ny,nx,n_mon,steps", [(60, 62, 20, 20), (60, 62, 20, 50), (64, 64, 70, 40),
                                               (24, 26, 8, 60), (64, 64, 70, 64), (60, 62, 20, 100),
                                               (64, 64, 70, 127), (24, 26, 8, 90)])
def test_split_flush_matches_pair_flush(ny, nx, n_mon, steps):
    """The split-product flush (17 to 128 pending terms; each FP32 product summed
    from six BF16 part products on the matrix cores) against the FP32 pair flush
    after the same moves.  Both sum the same K terms onto G in FP32, each within
    about K u max|G| of the exact sum (a term reaches at most max|G|), so the
    upper triangle and the monitor rows agree to 4 K u max|G|; the fields,
    diagonal and materials are not touched by the flush and agree bit for bit.
    Cases: 20 terms (two chunks of 16), 40 to 64 (four), 90 to 127 (eight, one
    workgroup per compute unit); ragged last band, one and two monitor bands,
    fewer tiles than workgroups."""
    import torch
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(ny, nx, n_mon=n_mon, dtype="c64", cand_mask=W.MASK_BOTH, tau=1e-6)
    names = L.flush_variants()
    old = L.flush_get_variant()
    out = {}
    try:
        for name in ("up_pair4_3m_nt", "up_bandseg_s3"):
            L.flush_set_variant(names.index(name))
            print(f"[case] {ny}x{nx} n_mon {n_mon}: {steps} pending terms, flush {name}", flush=True)
            job = _job(p, delay=128)
            job.init()
            job.run_greedy(steps, poll_every=steps)
            K = job.state.pending_calls
            assert 17 <= K <= 128, K
            job.flush()
            torch.cuda.synchronize()
            N = p.n
            G = job.G[:, :N].cpu().numpy()
            iu = np.triu_indices(N)
            out[name] = (K, G[:N][iu].copy(), G[N:].copy(), job.history(), job.host_state()[1:])
    finally:
        L.flush_set_variant(old)
    Ka, ua, ma, ha, sa = out["up_pair4_3m_nt"]
    Kb, ub, mb, hb, sb = out["up_bandseg_s3"]
    assert Ka == Kb and np.array_equal(ha, hb)
    tol = 4 * Ka * 2.0 ** -24
    assert _rel(ub, ua, floor=1.0) <= tol
    assert _rel(mb, ma, floor=1.0) <= tol
    for x, y in zip(sa, sb):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("ny,nx,n_mon,steps", [(60, 62, 20, 50), (64, 64, 70, 40), (24, 26, 8, 60),
                                               (60, 62, 20, 100)])
def test_band_flush_equals_pair_flush_bitwise(ny, nx, n_mon, steps):
    """The persistent band flushes (33 to 64 pending terms; row-major and
    column-segment tile orders) run the pair flush's matrix steps in the same
    order: after the same moves, G (upper triangle and monitor rows, then the
    mirrored block) is bit for bit that of the pair flush.  Cases: runs of
    several tiles that cross row bands and column segments, a ragged last band,
    one and two monitor bands (the second ragged), fewer tiles than
    workgroups."""
    import torch
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(ny, nx, n_mon=n_mon, dtype="c64", cand_mask=W.MASK_BOTH, tau=1e-6)
    names = L.flush_variants()
    old = L.flush_get_variant()
    out = {}
    try:
        for name in ("up_pair4_3m_nt", "up_band4_3m_nt", "up_bandseg4_3m_nt"):
            L.flush_set_variant(names.index(name))
            print(f"[case] {ny}x{nx} n_mon {n_mon}: {steps} pending terms, flush {name}", flush=True)
            job = _job(p, delay=128)
            job.init()
            n = job.run_greedy(steps, poll_every=steps)
            assert 33 <= job.state.pending_calls <= 128, (n, job.state.pending_calls)
            job.flush()
            torch.cuda.synchronize()
            N = p.n
            G = job.G[:, :N].cpu().numpy()
            iu = np.triu_indices(N)
            out[name] = (G[:N][iu].copy(), G[N:].copy(), job.host_state())
    finally:
        L.flush_set_variant(old)
    ua, ma, sa = out["up_pair4_3m_nt"]
    for name in ("up_band4_3m_nt", "up_bandseg4_3m_nt"):
        ub, mb, sb = out[name]
        assert np.array_equal(ua, ub) and np.array_equal(ma, mb), name
        for x, y in zip(sa, sb):
            assert np.array_equal(x, y), name

@pytest.mark.parametrize("dtype,delay,poll,form,n_mon", [
    ("c128", 16, 25, 0, 8), ("c64", 64, 32, 0, 8), ("c64", 7, 10, 0, 8), ("c64", 0, 20, 0, 8),
    ("c128", 16, 25, 1, 8), ("c64", 64, 32, 1, 8), ("c64", 7, 10, 1, 8),
    ("c64", 16, 10, 0, 150), ("c128", 16, 10, 1, 150),
    ("c64", 128, 40, 0, 8), ("c64", 100, 30, 1, 8), ("c128", 128, 50, 0, 150)])
def test_greedy_steps_equal_per_call_path(dtype, delay, poll, form, n_mon):
    """gfo_greedy_steps (fused kernels in deferred mode) makes the same moves and
    leaves bit for bit the same state as score_candidates + apply_flip per move,
    including the flushes, the stop and the refresh boundary.  form 0: one kernel
    per move on this grid; form 1: the two-kernel loop of larger grids.  150
    monitors: three monitor workgroups, the FOM monitor (75) in the second."""
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(40, 44, n_mon=n_mon, dtype=dtype, cand_mask=W.MASK_BOTH)   # ~130 moves
    ref = _job(p, delay=delay, kmax=256)
    ref.init()
    n_ref = ref.run_greedy(400, poll_every=poll, refresh_every=50)
    job = _job(p, delay=delay, kmax=256)
    job.init()
    old = L.loop_get_form()
    L.loop_set_form(form)
    try:
        n = job.run_greedy(400, poll_every=poll, refresh_every=50, fused=True)
    finally:
        L.loop_set_form(old)
    assert n == n_ref and n > 100
    assert np.array_equal(job.history(), ref.history())
    assert job.state.pending_calls == ref.state.pending_calls
    Gr, Er, dr, ir = ref.host_state()
    G, E, d, i = job.host_state()
    assert np.array_equal(G, Gr) and np.array_equal(E, Er) and np.array_equal(d, dr)
    assert np.array_equal(i, ir) and job.status() == ref.status() == 0


@pytest.mark.parametrize("form", [0, 1])
def test_greedy_steps_history_full(form):
    """Past the history capacity the fused loop flags GFO_STATUS_HISTORY_FULL,
    keeps counting moves, and still makes the per-call path's moves and state."""
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(40, 44, n_mon=8, dtype="c64", cand_mask=W.MASK_BOTH)   # ~130 moves
    ref = _job(p, delay=16, flip_cap=10)
    ref.init()
    for _ in range(30):
        ref.step()
    job = _job(p, delay=16, flip_cap=10)
    job.init()
    old = L.loop_get_form()
    L.loop_set_form(form)
    try:
        job.greedy_steps(30)
    finally:
        L.loop_set_form(old)
    assert job.n_flips() == ref.n_flips() == 30
    assert job.status() == ref.status() == L.GFO_STATUS_HISTORY_FULL
    assert np.array_equal(job.history(), ref.history()) and len(job.history()) == 10
    Gr, Er, dr, ir = ref.host_state()
    G, E, d, i = job.host_state()
    assert np.array_equal(G, Gr) and np.array_equal(E, Er) and np.array_equal(d, dr)
    assert np.array_equal(i, ir)


def test_greedy_steps_picks_record_and_stop():
    """The per-step pick records of gfo_greedy_steps match the history; after the
    stop rule refuses a move every later record is the sentinel."""
    import torch
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(12, 14, n_mon=6, dtype="c128", cand_mask=W.MASK_BOTH)   # stops after 24 moves
    job = _job(p, delay=16)
    job.init()
    n_steps = 60
    out = torch.zeros(n_steps * L.PICK_BYTES, dtype=torch.uint8, device="cuda:0")
    job.greedy_steps(n_steps, out=out.data_ptr())
    raw = out.cpu().numpy().tobytes()
    picks = [(q.pixel, q.eps_idx) for q in (L.Pick * n_steps).from_buffer_copy(raw)]
    n = job.n_flips()
    assert 0 < n < n_steps
    assert [tuple(map(int, h)) for h in job.history()] == picks[:n]
    assert all(pk == (-1, -1) for pk in picks[n:])
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, job.eps_idx.cpu().numpy()))
    G, E, _, _ = job.host_state()
    assert _rel(G, Gd) <= 1e-11 and _rel(E, Ed) <= 1e-11


def test_upper_only_flush_then_sync_lower():
    """The default complex64 flush brings only the upper triangle of the design
    block up to date and marks the lower one out of date.  The moves are those
    of eager mode, the upper triangle and the monitor rows match eager G, and
    gfo_sync_lower then makes the whole block match (lower = upper exactly)."""
    import torch
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(40, 44, n_mon=8, dtype="c64", cand_mask=W.MASK_BOTH)
    eager = _job(p)
    eager.init()
    n_ref = eager.run_greedy(150, poll_every=25)
    Ge, Ee, de, ie = eager.host_state()
    assert L.flush_variants()[L.flush_get_variant()] == "up_bandseg_s3"
    job = _job(p, delay=64)
    job.init()
    assert job.state.lower_stale == 1               # init_G0 filled the upper triangle only
    assert job.run_greedy(150, poll_every=25) == n_ref
    assert np.array_equal(job.history(), eager.history())
    job.flush()
    assert job.state.lower_stale == 1
    torch.cuda.synchronize()
    N = p.n
    G = job.G[:, :N].cpu().to(torch.complex128).numpy()
    iu, il = np.triu_indices(N), np.tril_indices(N, -1)
    D, De = G[:N], Ge[:N]
    tol = c64_drift_tol(n_ref)
    assert _rel(D[iu], De[iu]) <= tol
    assert not _rel(D[il], De[il]) <= 1e-1         # the lower triangle was left behind
    assert _rel(G[N:], Ge[N:]) <= tol              # monitor rows are current
    job.sync_lower()
    assert job.state.lower_stale == 0
    G2, E2, d2, i2 = job.host_state()
    D2 = G2[:N]
    assert np.array_equal(D2[iu], D[iu]) and np.array_equal(D2[il], D2.T[il])
    assert _rel(G2, Ge) <= tol and _rel(E2, Ee) <= tol and np.array_equal(i2, ie)
    job.sync_lower()                                # current: a no-op
    assert np.array_equal(job.host_state()[0], G2)


def test_eager_moves_after_an_upper_only_flush():
    """A job switched to eager updates while its lower triangle is out of date
    reads design entries from the upper triangle: same moves and state as a job
    that was eager throughout."""
    p = W.tiny(40, 44, n_mon=8, dtype="c64", cand_mask=W.MASK_BOTH)
    ref = _job(p)
    ref.init()
    assert ref.run_greedy(80, poll_every=16) == 80
    job = _job(p, delay=16)
    job.init()
    assert job.run_greedy(48, poll_every=16) == 48
    assert job.state.pending_calls == 0 and job.state.lower_stale == 1
    job.delay = 0
    job.state.delay = 0
    assert job.run_greedy(32, poll_every=16) == 32
    assert job.state.lower_stale == 1
    assert np.array_equal(job.history(), ref.history())
    G, E, d, i = job.host_state()
    Gr, Er, dr, ir = ref.host_state()
    tol = c64_drift_tol(80)
    assert _rel(G, Gr) <= tol and _rel(E, Er) <= tol and np.array_equal(i, ir)
