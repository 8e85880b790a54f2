"""Pins of the oracle's structure state (T1 dense, T2 flipped set, T0 brute force)
and of the paper's update equations, on small seeded grids.

The identities used are exact in exact arithmetic and independent of the code
paths they check: the solve residual, reciprocity, the imaginary-part identity
for real contrast, E = Einc + G B Einc, T2 = T1, update = re-solve, involution
and commutativity of flips, and the closed form of a single flip in vacuum.
"""
import math

import numpy as np
import pytest

from oracle import greens, greedy, state
import workloads as W


def _random_state(ny=5, nx=6, fill=0.35, seed=0, n_mon=4):
    p = W.tiny(ny, nx, n_mon=n_mon)
    idx = W.random_eps_idx(p, fill, seed)
    return p, idx, state.eps_of(p, idx)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dense_state_residual_and_reciprocity(seed):
    p, idx, eps = _random_state(seed=seed)
    N = p.n
    G0 = greens.build_G0(p)
    G, E = state.dense_state(p, eps, G0)
    alpha = greens.alpha_of(p, eps)
    res = (np.eye(N) - G0[:N] * alpha[None, :]) @ G[:N] - G0[:N]
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(G0[:N])
    assert np.linalg.norm(G[:N] - G[:N].T) <= 1e-12 * np.linalg.norm(G[:N])
    # monitor rows obey G_M = G0_MD + G0_MD B G_D
    resM = G0[N:] + (G0[N:] * alpha[None, :]) @ G[:N] - G[N:]
    assert np.linalg.norm(resM) <= 1e-12 * np.linalg.norm(G[N:])


@pytest.mark.parametrize("seed", [0, 3])
def test_imaginary_part_identity(seed):
    """Im G = (I + conj(G) B) Im G0 (I + B G) for real contrast B."""
    p, idx, eps = _random_state(seed=seed)
    N = p.n
    G0 = greens.build_G0(p)
    G, _ = state.dense_state(p, eps, G0)
    B = np.diag(greens.alpha_of(p, eps))
    I = np.eye(N)
    lhs = G[:N].imag
    rhs = ((I + np.conj(G[:N]) @ B) @ G0[:N].imag @ (I + B @ G[:N])).real
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(lhs)


def test_field_is_green_applied_to_source():
    """E_D = Einc_D + G_D B Einc_D and E_M = Einc_M + G_M B Einc_D."""
    p, idx, eps = _random_state(seed=5)
    N = p.n
    G, E = state.dense_state(p, eps)
    Einc = greens.incident_field(p)
    a = greens.alpha_of(p, eps)
    assert np.allclose(E[:N], Einc[:N] + G[:N] @ (a * Einc[:N]), rtol=0, atol=1e-12)
    assert np.allclose(E[N:], Einc[N:] + G[N:] @ (a * Einc[:N]), rtol=0, atol=1e-12)


def test_single_flip_in_vacuum_closed_form():
    """G'_pp = G0_pp / (1 - alpha G0_pp) for one flipped pixel (eq. form14, N_V = 1)."""
    p = W.tiny(3, 3, n_mon=2)
    k0 = greens.k0_of(p)
    eps = np.ones(9)
    eps[4] = 12.25
    G, _ = state.dense_state(p, eps)
    g0 = greens.self_term(p.pitch, k0)
    alpha = k0**2 * 11.25
    assert abs(G[4, 4] - g0 / (1 - alpha * g0)) <= 1e-13 * abs(G[4, 4])


@pytest.mark.parametrize("seed", [0, 1])
def test_flipped_set_equals_dense(seed):
    p, idx, eps = _random_state(ny=6, nx=8, fill=0.3, seed=seed)
    N = p.n
    G, E = state.dense_state(p, eps)
    fs = state.FlippedSet(p)
    E2, diag2, rows = fs.state(eps, rows=[N + 1, 3])
    assert np.allclose(E2, E, rtol=0, atol=1e-12)
    assert np.allclose(diag2, np.diagonal(G[:N]), rtol=0, atol=1e-15)
    assert np.allclose(rows[N + 1], G[N + 1], rtol=0, atol=1e-15)
    assert np.allclose(rows[3], G[3], rtol=0, atol=1e-15)


def test_empty_flipped_set_is_vacuum():
    p = W.tiny(3, 4)
    E, diag, rows = state.FlippedSet(p).state(np.ones(p.n), rows=[p.n])
    assert np.allclose(E, greens.incident_field(p))
    assert np.allclose(diag, greens.self_term(p.pitch, greens.k0_of(p)))


def test_paper_update_single_pixel_equals_resolve():
    p, idx, eps = _random_state(seed=7)
    G, E = state.dense_state(p, eps)
    j = 11
    new = 12.25 if eps[j] == 1.0 else 1.0
    G1, E1 = state.update_region(p, G, E, eps, [j], [new])
    eps2 = eps.copy()
    eps2[j] = new
    G2, E2 = state.dense_state(p, eps2)
    assert np.linalg.norm(G1 - G2) <= 1e-12 * np.linalg.norm(G2)
    assert np.linalg.norm(E1 - E2) <= 1e-12 * np.linalg.norm(E2)


def test_paper_update_region_equals_sequential_and_resolve():
    """Woodbury over a region (eq. form14) = sequential single flips = re-solve."""
    p, idx, eps = _random_state(seed=8)
    G, E = state.dense_state(p, eps)
    region = [2, 9, 17, 23]
    new = [12.25 if eps[j] == 1.0 else 1.0 for j in region]
    Gr, Er = state.update_region(p, G, E, eps, region, new)
    Gs, Es, es = G, E, eps.copy()
    for j, v in zip(region, new):
        Gs, Es = state.update_region(p, Gs, Es, es, [j], [v])
        es[j] = v
    Gd, Ed = state.dense_state(p, es)
    for Gx, Ex in ((Gr, Er), (Gs, Es)):
        assert np.linalg.norm(Gx - Gd) <= 1e-12 * np.linalg.norm(Gd)
        assert np.linalg.norm(Ex - Ed) <= 1e-12 * np.linalg.norm(Ed)


def test_flip_unflip_involution_and_commutativity():
    p, idx, eps = _random_state(seed=9)
    G, E = state.dense_state(p, eps)
    j, l = 4, 20
    vj = 12.25 if eps[j] == 1.0 else 1.0
    vl = 12.25 if eps[l] == 1.0 else 1.0
    G1, E1 = state.update_region(p, G, E, eps, [j], [vj])
    e1 = eps.copy(); e1[j] = vj
    G2, E2 = state.update_region(p, G1, E1, e1, [j], [eps[j]])
    assert np.linalg.norm(G2 - G) <= 1e-12 * np.linalg.norm(G)
    assert np.linalg.norm(E2 - E) <= 1e-12 * np.linalg.norm(E)
    # a then b == b then a
    Ga, Ea = state.update_region(p, G1, E1, e1, [l], [vl])
    Gb, Eb = state.update_region(p, G, E, eps, [l], [vl])
    eb = eps.copy(); eb[l] = vl
    Gb, Eb = state.update_region(p, Gb, Eb, eb, [j], [vj])
    assert np.linalg.norm(Ga - Gb) <= 1e-12 * np.linalg.norm(Ga)


def test_brute_force_scores_equal_closed_form():
    """Tier T0 (full solve per candidate) = eqs. form4-form9 with N_V = 1 at the monitor."""
    p, idx, eps = _random_state(ny=4, nx=5, fill=0.4, seed=4, n_mon=3)
    N = p.n
    G, E = state.dense_state(p, eps)
    F0 = state.brute_force_scores(p, idx)
    F1 = greedy.scores_closed_form(p, E, np.diagonal(G[:N]), G[N + p.fom_monitor], idx)
    fin = np.isfinite(F0)
    assert np.array_equal(fin, np.isfinite(F1))
    assert fin.sum() == N          # two materials, both allowed: one candidate per pixel
    assert np.allclose(F1[fin], F0[fin], rtol=1e-12, atol=0)


@pytest.mark.parametrize("table", [(1.0, 12.25), (1.0, 12.25, 4.0)])
def test_walking_tier_equals_flipped_set_tier_along_moves(table):
    """Tier T2u (diagonal carried by the paper's one-pixel update, E and the FOM
    row from the flipped set) equals tier T2 at every structure of a random move
    sequence that also un-flips and re-flips pixels."""
    from oracle import greedy as og
    p = W.tiny(7, 9, n_mon=4, eps_table=table, cand_mask=(1 << len(table)) - 1)
    rng = np.random.default_rng(5)
    walk = og._Evaluator(p, "T2u")
    full = og._Evaluator(p, "T2")
    idx = np.zeros(p.n, np.uint8)
    for t in range(30):
        if t:
            j = int(rng.integers(0, p.n)) if t % 4 else int(np.flatnonzero(idx)[0])
            idx[j] = (idx[j] + 1 + int(rng.integers(0, len(table) - 1))) % len(table)
        Ew, dw, rw = walk(idx)
        Ef, df, rf = full(idx)
        assert np.max(np.abs(Ew - Ef)) <= 1e-12 * np.max(np.abs(Ef))
        assert np.max(np.abs(dw - df)) <= 1e-12 * np.max(np.abs(df))
        assert np.max(np.abs(rw - rf)) <= 1e-12 * np.max(np.abs(rf))
    # two pixels changed at once: a full evaluation
    idx[:2] = 1 - np.minimum(idx[:2], 1)
    Ew, dw, _ = walk(idx)
    Ef, df, _ = full(idx)
    assert np.allclose(dw, df, rtol=1e-12, atol=0) and np.allclose(Ew, Ef, rtol=1e-12, atol=0)


def test_replay_final_record_reports_the_end_state():
    """replay(final=True) of a whole greedy trajectory ends at a state where no
    move improves the FOM, the same FOM as the trajectory's last step."""
    from oracle import greedy as og
    p = W.tiny(5, 6, n_mon=4, steps=200)
    tr = og.greedy(p, tier="T2")
    assert tr.stopped
    rep = og.replay(p, [(s.pixel, s.eps_idx) for s in tr.steps], tier="T2u", final=True)
    assert len(rep) == len(tr.steps) + 1
    for r, s in zip(rep, tr.steps):
        assert (r["oracle_pixel"], r["oracle_eps"]) == (s.pixel, s.eps_idx)
    last = rep[-1]
    assert last["F_taken"] is None and last["oracle_pixel"] is None
    assert abs(last["fom_before"] - tr.steps[-1].fom) <= 1e-12 * tr.steps[-1].fom
    assert not last["Fstar"] > last["fom_before"] * (1 + p.tau)
