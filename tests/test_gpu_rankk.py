"""GPU parity of the rank-k path: spaced top-k selection (score_candidates with
topk > 1) against the oracle's rank-k rule, and apply_flips_rank_k (FP64 Woodbury
core + matrix-core rank-k update) against the dense re-solve of the new structure.

Tolerances (element by element, tests/parity.py): E and the FP64 diagonal come
from the FP64 Woodbury core, 5e-6; FP32 matrix-core inputs round U and W once to
FP32, so G is held to the complex64 drift bound of k updates; BF16 inputs (8-bit
mantissa) are held to 1e-2 of the largest update entry and reported.  Along the
128x128 rank-16 trajectory the fields and the FOM agree with the exact state of
the GPU's structure to 1e-4.
"""
import numpy as np
import pytest

from oracle import greedy as og, state as ost
import workloads as W

pytestmark = pytest.mark.gpu


def _job(p, **kw):
    from paper_2202_05388_amd.job import Job
    print(f"[case] {p.name} {p.ny}x{p.nx} mon={p.n_mon} {p.dtype} {kw}", flush=True)
    return Job(p, device="cuda:0", **kw)


# element-wise relative error with an absolute floor of 1e-3 x the largest entry
from parity import c64_drift_tol, certify_rank_k_set, rel_elem as _rel  # noqa: E402


@pytest.mark.parametrize("k,spacing,seed", [(16, 3, 0), (5, 0, 1), (32, 2, 2)])
def test_topk_selection_matches_oracle(k, spacing, seed):
    p = W.tiny(24, 26, n_mon=8, dtype="c64", cand_mask=W.MASK_BOTH)
    N = p.n
    idx = W.random_eps_idx(p, 0.2, seed)
    G, E = ost.dense_state(p, ost.eps_of(p, idx))
    job = _job(p)
    job.upload_state(G, E, np.diagonal(G[:N]), idx)
    job.score(topk=k, min_spacing=spacing, tau=1e-6)
    got = job.read_picks(k)
    F = og.scores_closed_form(p, E, np.diagonal(G[:N]), G[N + p.fom_monitor], idx)
    ref = og.select_rank_k(F, ost.fom_of_state(p, E), 1e-6, k, spacing, p.nx)
    gp = [(a, b) for a, b, _, _ in got if a >= 0]
    assert gp == [(r.pixel, r.eps_idx) for r in ref]
    assert all(a < 0 for a, _, _, _ in got[len(ref):])


@pytest.mark.parametrize("n_eps", [3, 8])
@pytest.mark.parametrize("k,spacing,seed", [(12, 0, 3), (20, 2, 4)])
def test_topk_selection_many_materials_matches_oracle(n_eps, k, spacing, seed):
    """The spaced top-k selection over (pixel, material) with 3- and 8-entry
    tables on 624 pixels: three score chunks of 256 pixels, up to 2048 scores per
    chunk, each pick's excluded window summarised again; equal to the oracle's
    rule, sentinels after the last improving move."""
    table = {3: (1.0, 12.25, 2.25), 8: (1.0, 12.25, 2.25, 4.0, 6.25, 9.0, 3.0, 1.5)}[n_eps]
    p = W.tiny(24, 26, n_mon=8, dtype="c64", cand_mask=(1 << n_eps) - 1, eps_table=table)
    N = p.n
    idx = W.random_material_idx(p, seed)
    G, E = ost.dense_state(p, ost.eps_of(p, idx))
    job = _job(p)
    job.upload_state(G, E, np.diagonal(G[:N]), idx)
    job.score(topk=k, min_spacing=spacing, tau=1e-6)
    got = job.read_picks(k)
    F = og.scores_closed_form(p, E, np.diagonal(G[:N]), G[N + p.fom_monitor], idx)
    ref = og.select_rank_k(F, ost.fom_of_state(p, E), 1e-6, k, spacing, p.nx)
    assert len(ref) >= 4
    gp = [(a, b) for a, b, _, _ in got if a >= 0]
    assert gp == [(r.pixel, r.eps_idx) for r in ref]
    assert all(a < 0 for a, _, _, _ in got[len(ref):])


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("s", [1, 7, 16, 24])
def test_rank_k_update_equals_resolve(precision, s):
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(20, 24, n_mon=8, dtype="c64")
    N = p.n
    idx = W.random_eps_idx(p, 0.15, 4)
    G, E = ost.dense_state(p, ost.eps_of(p, idx))
    rng = np.random.default_rng(s)
    pix = rng.choice(N, s, replace=False)
    job = _job(p)
    job.upload_state(G, E, np.diagonal(G[:N]), idx)
    for t, j in enumerate(pix):
        job.set_pick(int(j), 1 - int(idx[j]), slot=t)
    prec = L.GFO_FP32 if precision == "fp32" else L.GFO_BF16
    job.apply_rank_k(s, precision=prec)
    G1, E1, d1, idx1 = job.host_state()
    idx2 = idx.copy()
    idx2[pix] = 1 - idx2[pix]
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx2))
    assert np.array_equal(idx1, idx2) and job.n_flips() == s and job.status() == 0
    upd = np.linalg.norm(Gd - G)
    err_G = np.linalg.norm(G1 - Gd)
    print(f"rank-{s} {precision}: |dG|/|G| {err_G / np.linalg.norm(Gd):.2e}, "
          f"|dG|/|update| {err_G / upd:.2e}", flush=True)
    # diag64 and E come from the FP64 Woodbury core in both precisions
    assert _rel(d1, np.diagonal(Gd[:N])) <= 5e-6
    assert _rel(E1, Ed) <= 5e-6
    if precision == "fp32":
        assert _rel(G1, Gd) <= c64_drift_tol(s)
    else:
        # each entry against the largest update entry: both BF16 factors of a
        # product are rounded (unit roundoff 2^-8), so a product is off by up to
        # 2 * 2^-8 = 7.8e-3 of |U_ri W_iq|, which cancellation can leave far above
        # the entry's own update
        assert _rel(G1 - G, Gd - G, floor=1.0) <= 1e-2


def test_rank_k_skips_sentinels_duplicates_and_noops():
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(10, 12, n_mon=4, dtype="c64")
    N = p.n
    idx = np.zeros(N, np.uint8)
    G, E = ost.dense_state(p, ost.eps_of(p, idx))
    job = _job(p)
    job.upload_state(G, E, np.diagonal(G[:N]), idx)
    picks = [(5, 1), (-1, 1), (5, 1), (7, 0), (9, 1)]      # (7, 0) is already material 0
    for t, (j, e) in enumerate(picks):
        job.set_pick(j, e, slot=t)
    job.apply_rank_k(len(picks), precision=L.GFO_FP32)
    G1, E1, d1, idx1 = job.host_state()
    idx2 = idx.copy()
    idx2[[5, 9]] = 1
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx2))
    assert np.array_equal(idx1, idx2) and job.n_flips() == 2
    assert _rel(G1, Gd) <= 5e-6 and _rel(E1, Ed) <= 5e-6


def test_rank_k_trajectory_matches_oracle_policy():
    """Rank-16 steps with spacing 3 on a 40x40 grid: the chosen sets and the FOM
    follow the oracle's rank-k policy (tier T1 state each step)."""
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(40, 40, n_mon=8, dtype="c64", cand_mask=W.MASK_BOTH, rank_k=16, min_spacing=3,
               steps=4, tau=1e-6)
    ref = og.rank_k_trajectory(p, steps=4, tier="T2")
    job = _job(p)
    job.init()
    for t, group in enumerate(ref.steps):
        job.score(topk=16, min_spacing=3, tau=1e-6)
        got = [(a, b) for a, b, _, _ in job.read_picks(16) if a >= 0]
        assert got == [(s.pixel, s.eps_idx) for s in group], t
        job.apply_rank_k(16, precision=L.GFO_FP32)
        fom = job.fom()
        assert abs(fom - group[0].fom) <= 1e-4 * group[0].fom


def test_rank_k_upper_triangle_trajectory_with_refresh():
    """The rank-16 trajectory with only the upper triangle kept (state.lower_stale:
    the rank-k update and the refresh's product leave out the blocks below the
    diagonal, every read goes to the upper triangle) and an FP64 refresh after
    every two steps: the chosen sets and the FOM follow the oracle's policy, and
    the final state with its lower triangle copied back is the dense re-solve's."""
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(40, 40, n_mon=8, dtype="c64", cand_mask=W.MASK_BOTH, rank_k=16, min_spacing=3,
               steps=6, tau=1e-6)
    ref = og.rank_k_trajectory(p, steps=6, tier="T2")
    job = _job(p, kmax=256, upper=True)
    job.init()
    assert job.state.lower_stale == 1
    for t, group in enumerate(ref.steps):
        job.score(topk=16, min_spacing=3, tau=1e-6)
        got = [(a, b) for a, b, _, _ in job.read_picks(16) if a >= 0]
        assert got == [(s.pixel, s.eps_idx) for s in group], t
        job.apply_rank_k(16, precision=L.GFO_FP32)
        if t % 2 == 1:
            job.refresh()
        assert job.state.lower_stale == 1
        assert abs(job.fom() - group[0].fom) <= 1e-4 * group[0].fom, t
    G1, E1, d1, idx1 = job.host_state()
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx1))
    assert _rel(G1, Gd) <= 3e-7 and _rel(E1, Ed) <= 3e-7   # the last step was refreshed
    assert job.status() == 0


def test_rank_k_three_materials_follows_oracle_policy():
    """Spaced top-k over (pixel, material) with a three-entry table: at most one
    move per pixel, the chosen sets and the FOM follow the oracle's policy."""
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(32, 32, n_mon=8, dtype="c64", cand_mask=0b111, eps_table=(1.0, 12.25, 2.25),
               rank_k=16, min_spacing=3, steps=3, tau=1e-6)
    ref = og.rank_k_trajectory(p, steps=3, tier="T2")
    assert len({s.eps_idx for g in ref.steps for s in g}) >= 2
    job = _job(p)
    job.init()
    for t, group in enumerate(ref.steps):
        job.score(topk=16, min_spacing=3, tau=1e-6)
        got = [(a, b) for a, b, _, _ in job.read_picks(16) if a >= 0]
        assert got == [(s.pixel, s.eps_idx) for s in group], t
        assert len({a for a, _ in got}) == len(got)
        job.apply_rank_k(16, precision=L.GFO_FP32)
        assert abs(job.fom() - group[0].fom) <= 1e-4 * group[0].fom
    assert job.status() == 0


@pytest.mark.timeout(300)
def test_rank16_square128_follows_oracle_policy():
    """The 128x128 rank-16 workload (spacing 3, FP32 matrix-core inputs), 8 steps:
    each step's set equals the oracle's rank-k rule up to certified ties, judged
    on the exact (FP64 flipped-set) scores of the structure the GPU chose it at;
    after each step the FOM and the fields at the monitors and at sampled pixels
    agree element by element with the exact state of the GPU's structure to 1e-4,
    and while the sets agree the FOM follows the oracle's own rank-k trajectory."""
    from paper_2202_05388_amd import _lib as L
    p = W.SQUARE_128_RANK16
    N, steps = p.n, 8
    m0 = N + p.fom_monitor
    ref = og.rank_k_trajectory(p, steps=steps, tier="T2")
    assert len(ref.steps) == steps
    fs = ost.FlippedSet(p)
    sample = np.random.default_rng(0).choice(N, 256, replace=False)
    job = _job(p)
    job.init()
    idx = np.zeros(N, np.uint8)
    same = 0
    E, diag, rows = fs.state(ost.eps_of(p, idx), rows=[m0])
    for t in range(steps):
        job.score(topk=p.rank_k, min_spacing=p.min_spacing, tau=p.tau)
        got = [(a, b) for a, b, _, _ in job.read_picks(p.rank_k) if a >= 0]
        F = og.scores_closed_form(p, E, diag, rows[m0], idx)
        common = certify_rank_k_set(F, ost.fom_of_state(p, E), got, p.rank_k, p.min_spacing,
                                    p.nx, tol=1e-4)
        if same == t and got == [(s.pixel, s.eps_idx) for s in ref.steps[t]]:
            same += 1
        print(f"  step {t}: {len(got)} picks, {common} equal to the oracle rule's prefix",
              flush=True)
        job.apply_rank_k(p.rank_k, precision=L.GFO_FP32)
        for j, e in got:
            idx[j] = e
        E, diag, rows = fs.state(ost.eps_of(p, idx), rows=[m0])
        fom = ost.fom_of_state(p, E)
        assert abs(job.fom() - fom) <= 1e-4 * fom
        if same == t + 1:
            assert abs(job.fom() - ref.steps[t][0].fom) <= 1e-4 * ref.steps[t][0].fom
        Eg = job.E.cpu().numpy().astype(np.complex128)
        assert _rel(Eg[N:], E[N:]) <= 1e-4
        assert _rel(Eg[sample], E[sample]) <= 1e-4
        assert np.array_equal(job.eps_idx.cpu().numpy(), idx)
    print(f"rank-16 at 128x128: sets equal to the oracle's for {same} of {steps} steps", flush=True)
    assert job.status() == 0


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("s", [16, 24])
def test_rank_k_update_variants(precision, s):
    """Every matrix-core update variant gives the dense re-solve's G; the
    streaming variants (products summed from zero, G added once) agree bit for
    bit.  30 x 70 pixels: ld = 2112 leaves a 64-column remainder of the
    128-column workgroup tiles, and R = 2108 rows a ragged last row block."""
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(30, 70, n_mon=8, dtype="c64")
    N = p.n
    idx = W.random_eps_idx(p, 0.15, 6)
    G, E = ost.dense_state(p, ost.eps_of(p, idx))
    pix = np.random.default_rng(s).choice(N, s, replace=False)
    idx2 = idx.copy()
    idx2[pix] = 1 - idx2[pix]
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx2))
    prec = L.GFO_FP32 if precision == "fp32" else L.GFO_BF16
    names = L.rk_variants()
    old = L.rk_get_variant()
    out = {}
    try:
        for vi, name in enumerate(names):
            L.rk_set_variant(vi)
            job = _job(p)
            job.upload_state(G, E, np.diagonal(G[:N]), idx)
            for t, j in enumerate(pix):
                job.set_pick(int(j), int(idx2[j]), slot=t)
            job.apply_rank_k(s, precision=prec)
            G1, E1, d1, i1 = job.host_state()
            assert np.array_equal(i1, idx2) and job.status() == 0
            if precision == "fp32":
                assert _rel(G1, Gd) <= c64_drift_tol(s), name
            else:
                assert _rel(G1 - G, Gd - G, floor=1.0) <= 1e-2, name
            assert _rel(E1, Ed) <= 5e-6, name
            out[name] = G1
    finally:
        L.rk_set_variant(old)
    streaming = [n for n in names if n != "acc64"]
    assert len(streaming) >= 2
    for n in streaming[1:]:
        assert np.array_equal(out[n], out[streaming[0]]), n


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_rank_k_upper_triangle_equals_full(precision):
    """With state.lower_stale set the rank-k update leaves out the blocks of
    design rows wholly below the diagonal; every entry it keeps (the upper
    triangle with its diagonal, the monitor rows), E and the FP64 diagonal equal
    the full update's bit for bit, in every variant, and the state with its lower
    triangle copied back is the dense re-solve's."""
    from paper_2202_05388_amd import _lib as L
    p = W.tiny(30, 70, n_mon=8, dtype="c64")
    N, s = p.n, 16
    idx = W.random_eps_idx(p, 0.15, 6)
    G, E = ost.dense_state(p, ost.eps_of(p, idx))
    pix = np.random.default_rng(3).choice(N, s, replace=False)
    idx2 = idx.copy()
    idx2[pix] = 1 - idx2[pix]
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, idx2))
    prec = L.GFO_FP32 if precision == "fp32" else L.GFO_BF16
    upper = np.triu(np.ones((N, N), bool))
    old = L.rk_get_variant()
    try:
        for vi, name in enumerate(L.rk_variants()):
            L.rk_set_variant(vi)
            out = []
            for lower_stale in (0, 1):
                job = _job(p)
                job.upload_state(G, E, np.diagonal(G[:N]), idx)
                job.state.lower_stale = lower_stale
                for t, j in enumerate(pix):
                    job.set_pick(int(j), int(idx2[j]), slot=t)
                job.apply_rank_k(s, precision=prec)
                assert job.status() == 0 and job.state.lower_stale == lower_stale
                raw = job.dense_G()[:, :N].cpu().numpy()
                out.append((job, raw, job.E.cpu().numpy(), job.diag64.cpu().numpy()))
            (_, Gf, Ef, df), (up, Gu, Eu, du) = out
            assert np.array_equal(Gu[:N][upper], Gf[:N][upper]), name
            assert np.array_equal(Gu[N:], Gf[N:]), name
            assert np.array_equal(Eu, Ef) and np.array_equal(du, df), name
            # rows 1920..2047 x columns 0..127 lie below the diagonal in every
            # variant's row groups (128, 256 or 512 rows): left as uploaded
            G64 = G[:N].astype(np.complex64)
            assert np.array_equal(Gu[1920:2048, :128], G64[1920:2048, :128]), name
            assert not np.array_equal(Gf[1920:2048, :128], G64[1920:2048, :128]), name
            G1, E1, d1, i1 = up.host_state()
            assert np.array_equal(i1, idx2)
            if precision == "fp32":
                assert _rel(G1, Gd) <= c64_drift_tol(s), name
            else:
                assert _rel(G1 - G, Gd - G, floor=1.0) <= 1e-2, name
            assert _rel(E1, Ed) <= 5e-6, name
    finally:
        L.rk_set_variant(old)
