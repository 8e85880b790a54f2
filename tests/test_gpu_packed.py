"""Band-packed storage of G (the design block's upper triangle in bands of 64
rows, then the monitor rows): every deferred-mode path gives, bit for bit, the
moves and the state of the same job in dense storage (whose deferred mode is
held to the oracle at full size elsewhere), and a small packed run follows the
oracle directly."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _pair(p, delay, kmax=0):
    from paper_2202_05388_amd.job import Job
    print(f"[case] {p.ny}x{p.nx} n_mon {p.n_mon} {p.dtype} delay {delay} kmax {kmax}", flush=True)
    dense = Job(p, device="cuda:0", delay=delay, kmax=kmax)
    packed = Job(p, device="cuda:0", delay=delay, kmax=kmax, packed=True)
    for j in (dense, packed):
        j.init()
    return dense, packed


def _same(a, b):
    import torch
    torch.cuda.synchronize()
    assert np.array_equal(a.history(), b.history())
    assert a.status() == b.status() == 0
    assert a.state.pending_calls == b.state.pending_calls
    Ga, Ea, da, ia = a.host_state()
    Gb, Eb, db, ib = b.host_state()
    N = a.N
    iu = np.triu_indices(N)
    assert np.array_equal(Ga[:N][iu], Gb[:N][iu])          # the design block's upper triangle
    assert np.array_equal(Ga[N:], Gb[N:])                   # the monitor rows
    assert np.array_equal(Ea, Eb) and np.array_equal(da, db) and np.array_equal(ia, ib)


@pytest.mark.parametrize("ny,nx,n_mon,dtype,delay", [
    (60, 62, 20, "c64", 64), (64, 64, 70, "c64", 128), (24, 26, 8, "c64", 16),
    (60, 62, 20, "c128", 64), (9, 11, 3, "c128", 7)])
def test_packed_equals_dense_bitwise(ny, nx, n_mon, dtype, delay):
    """Fused greedy loop (chunks of several lengths, flushes of every term
    bucket on the way), the per-call path, a refresh in the middle and the moves
    after it: packed == dense bit for bit (ragged last band; one, two and three
    monitor bands)."""
    p = W.tiny(ny, nx, n_mon=n_mon, dtype=dtype, cand_mask=W.MASK_BOTH,
               tau=1e-6 if dtype == "c64" else 1e-9)
    dense, packed = _pair(p, delay, kmax=256)
    for n in (7, 40, 1, 90):
        for j in (dense, packed):
            j.greedy_steps(n)
    _same(dense, packed)
    for j in (dense, packed):
        j.refresh()
    _same(dense, packed)
    for _ in range(25):                                    # per-call path
        for j in (dense, packed):
            j.score()
            j.apply()
    for j in (dense, packed):
        j.greedy_steps(33)
    _same(dense, packed)


@pytest.mark.parametrize("variant", ["up_pair4_3m_nt", "up_pair4_3m_nt_x8", "up_band4_3m_nt",
                                     "up_bandseg4_3m_nt", "up_bandseg_s3", "w32_3m"])
def test_packed_flush_variants(variant):
    """Every complex64 flush variant on packed storage (the non-symmetric one
    falls back to the pair kernel there) gives the dense result of the same
    variant bit for bit, at 32, 64 and 128 terms (for the split-product default,
    its two-, four- and eight-chunk forms)."""
    from paper_2202_05388_amd import _lib as L
    names = L.flush_variants()
    old = L.flush_get_variant()
    try:
        L.flush_set_variant(names.index(variant))
        p = W.tiny(40, 44, n_mon=40, dtype="c64", cand_mask=W.MASK_BOTH, tau=1e-6)
        for delay in (32, 64, 128):
            dense, packed = _pair(p, delay)
            for j in (dense, packed):
                j.greedy_steps(delay + 10)
            if variant == "w32_3m":
                # the dense non-symmetric form keeps the whole block current: moves equal,
                # states within FP32 rounding of the pair form's
                for a in (dense, packed):
                    assert a.status() == 0
                assert np.array_equal(dense.history(), packed.history())
            else:
                _same(dense, packed)
    finally:
        L.flush_set_variant(old)


def test_packed_region_moves_equal_dense():
    """2x2 region moves (joint solves on in-block entries read through the upper
    triangle, applied as deferred rank-1 terms) on packed storage."""
    p = W.tiny(24, 24, n_mon=8, dtype="c64", cand_mask=W.MASK_BOTH, tau=1e-6)
    dense, packed = _pair(p, 32)
    for j in (dense, packed):
        j.run_region_greedy(30, poll_every=10)
    _same(dense, packed)


def test_packed_job_table_equals_own_calls():
    """Grouped serving (one launch per move for every job of a table) with
    packed and dense jobs side by side: each job bit for bit as its own calls."""
    import torch
    from paper_2202_05388_amd.job import Job, JobGroup
    probs = [W.tiny(24, 24, n_mon=16, dtype="c64", tau=1e-6),
             W.tiny(30, 26, n_mon=8, dtype="c64", tau=1e-6, wavelength=1.1)]

    def make():
        js = [Job(probs[0], device="cuda:0", delay=16, packed=True),
              Job(probs[1], device="cuda:0", delay=16),
              Job(probs[1], device="cuda:0", delay=16, packed=True)]
        for j in js:
            j.init()
        return js

    alone, grouped = make(), make()
    for n in (9, 16, 30):
        for j in alone:
            j.greedy_steps(n)
    group = JobGroup(grouped, device="cuda:0")
    group.build()
    for n in (9, 16, 30):
        group.steps(n)
    torch.cuda.synchronize()
    for a, b in zip(alone, grouped):
        _same(a, b)
    _same(alone[1], alone[2])                               # dense == packed in the table too


def test_packed_follows_the_oracle():
    """A small packed complex128 run against the oracle's greedy trajectory
    (dense re-solve tier): the same pixels, fields to 1e-9."""
    import torch
    from oracle import greedy as og
    from paper_2202_05388_amd.job import Job
    p = W.tiny(8, 10, n_mon=4, cand_mask=W.MASK_BOTH, dtype="c128", steps=20)
    ref = og.greedy(p, tier="T1")
    job = Job(p, device="cuda:0", delay=6, packed=True)
    job.init()
    n = job.run_greedy(p.steps, poll_every=5, fused=True)
    torch.cuda.synchronize()
    assert n == len(ref.steps)
    assert [int(x) for x in job.history()[:, 0]] == ref.pixels()
    _, E, _, _ = job.host_state()
    from parity import rel_elem
    assert rel_elem(E, ref.E) < 1e-9


def test_packed_footprint_at_128():
    """At 128 x 128 pixels the packed G takes about half the bytes, and a
    deferred run equals the dense one (200 fused moves, flushes and a restart)."""
    import torch
    p = W.SQUARE_128
    dense, packed = _pair(p, 64)
    assert packed.G.numel() * packed.G.element_size() < 0.52 * dense.G.numel() * dense.G.element_size()
    for j in (dense, packed):
        j.run_greedy(200, poll_every=32, fused=True)
    torch.cuda.synchronize()
    _same(dense, packed)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_packed_two_kernel_loop_equals_dense(dtype):
    """The fused loop's two-kernel form (grids above 65,536 pixels; forced here
    on a small grid) on packed storage, bit for bit as dense."""
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(40, 42, n_mon=30, dtype=dtype, cand_mask=W.MASK_BOTH,
               tau=1e-6 if dtype == "c64" else 1e-9)
    L.loop_set_form(1)
    try:
        dense, packed = _pair(p, 64)
        for n in (33, 70, 5):
            for j in (dense, packed):
                j.greedy_steps(n)
        _same(dense, packed)
    finally:
        L.loop_set_form(0)


def test_packed_strip_equals_dense_at_sampled_entries():
    """The 48 x 2048 strip (98,304 pixels, 256 monitors): packed G takes 38.9 GB
    beside the dense 77.5 GB.  120 fused moves at 128 terms per flush (the
    two-kernel loop), then a flush: the same moves, fields, diagonal and FOM
    monitor row, and the same upper-triangle entries at 4096 sampled positions,
    bit for bit."""
    import torch
    p = W.STRIP_48x2048
    dense, packed = _pair(p, 128)
    assert packed.G.numel() * packed.G.element_size() < 39.0e9
    for j in (dense, packed):
        j.greedy_steps(60)
        j.greedy_steps(60)
        j.flush()
    torch.cuda.synchronize()
    assert np.array_equal(dense.history(), packed.history())
    assert dense.status() == packed.status() == 0
    for a, b in ((dense.E, packed.E), (dense.diag64, packed.diag64), (dense.eps_idx, packed.eps_idx)):
        assert torch.equal(a, b)
    N, ld = p.n, dense.ld
    rng = np.random.default_rng(0)
    r = rng.integers(0, N, 4096)
    c = rng.integers(0, N, 4096)
    r, c = np.minimum(r, c), np.maximum(r, c)                 # upper-triangle positions
    b = r // 64
    off = 64 * (b * ld - 32 * b * (b - 1)) + (r % 64) * (ld - 64 * b) + (c - 64 * b)
    idx = torch.from_numpy(off.astype(np.int64)).to(packed.G.device)
    got = packed.G[idx]
    want = dense.G[torch.from_numpy(r).to(dense.G.device), torch.from_numpy(c).to(dense.G.device)]
    assert torch.equal(got, want)
    nb = (N + 63) // 64
    mon0 = 64 * (nb * ld - 32 * nb * (nb - 1))
    m0 = p.fom_monitor
    assert torch.equal(packed.G[mon0 + m0 * ld: mon0 + (m0 + 1) * ld], dense.G[N + m0])
