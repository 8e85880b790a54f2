"""Pins of the oracle's greedy policy: brute-force argmax, tie rule on mirror-symmetric
grids, monotone FOM (Sec. IV), T1 = T2 trajectories, rank-k selection rules."""
import numpy as np
import pytest

from oracle import greens, greedy, state
import workloads as W


def test_greedy_matches_brute_force_argmax():
    p = W.tiny(4, 5, n_mon=3, cand_mask=W.MASK_BOTH, steps=6)
    G0 = greens.build_G0(p)
    traj = greedy.greedy(p, tier="T1")
    idx = np.zeros(p.n, np.uint8)
    for s in traj.steps:
        F = state.brute_force_scores(p, idx, G0)
        _, E = state.dense_state(p, state.eps_of(p, idx), G0)
        fom = state.fom_of_state(p, E)
        Fstar = F.max()
        assert Fstar > fom
        # chosen candidate is within the tie band of the brute-force max and is its lowest index
        band = np.flatnonzero(F.ravel() >= Fstar * (1 - p.tau))
        assert band[0] == s.pixel * F.shape[1] + s.eps_idx
        idx[s.pixel] = s.eps_idx
        _, E = state.dense_state(p, state.eps_of(p, idx), G0)
        assert abs(state.fom_of_state(p, E) - s.fom) <= 1e-12 * s.fom


def test_greedy_fom_monotone_and_prediction_exact():
    p = W.tiny(6, 6, n_mon=4, cand_mask=W.MASK_BOTH, steps=25)
    traj = greedy.greedy(p, tier="T1")
    foms = [traj.fom0] + [s.fom for s in traj.steps]
    assert all(b > a for a, b in zip(foms, foms[1:]))
    for s in traj.steps:
        assert abs(s.fom_pred - s.fom) <= 1e-11 * s.fom


def test_mirror_symmetry_gives_exact_ties_and_lowest_index_wins():
    p = W.tiny(4, 6, n_mon=4, cand_mask=W.MASK_BOTH)
    N = p.n
    idx = W.mirror_symmetric_eps_idx(p, 0.3, seed=2)
    G, E = state.dense_state(p, state.eps_of(p, idx))
    F = greedy.scores_closed_form(p, E, np.diagonal(G[:N]), G[N + p.fom_monitor], idx)
    # mirror symmetry x -> -x maps pixel (iy, ix) to (iy, nx-1-ix); scores are equal up to rounding
    Fm = F.reshape(p.ny, p.nx, -1)[:, ::-1, :].reshape(N, -1)
    fin = np.isfinite(F)
    assert np.array_equal(fin, np.isfinite(Fm))
    assert np.allclose(F[fin], Fm[fin], rtol=1e-12, atol=0)
    pick = greedy.select_greedy(F, state.fom_of_state(p, E), p.tau)
    assert pick is not None and pick.n_tied >= 2
    assert pick.pixel % p.nx < p.nx / 2          # lowest index of the mirror pair


def test_select_greedy_tie_band_and_stop_rule():
    F = np.array([[-np.inf, 1.0], [-np.inf, 1.0 + 5e-10], [-np.inf, 0.5]])
    pk = greedy.select_greedy(F, 0.9, 1e-9)
    assert (pk.pixel, pk.eps_idx, pk.n_tied) == (0, 1, 2)
    assert greedy.select_greedy(F, 1.0 + 5e-10, 1e-9) is None     # no strict improvement
    assert greedy.select_greedy(np.full((3, 2), -np.inf), 0.1, 1e-9) is None


def test_T1_and_T2_trajectories_agree():
    p = W.tiny(8, 8, n_mon=4, cand_mask=W.MASK_BOTH, steps=12)
    t1 = greedy.greedy(p, tier="T1")
    t2 = greedy.greedy(p, tier="T2")
    assert t1.pixels() == t2.pixels()
    for a, b in zip(t1.steps, t2.steps):
        assert abs(a.fom - b.fom) <= 1e-11 * a.fom
    assert np.allclose(t1.E, t2.E, rtol=0, atol=1e-11)


def test_rank_k_selection_rules():
    p = W.tiny(12, 12, n_mon=4, cand_mask=W.MASK_BOTH, rank_k=5, min_spacing=3)
    N = p.n
    idx = W.random_eps_idx(p, 0.2, seed=3)
    G, E = state.dense_state(p, state.eps_of(p, idx))
    fom = state.fom_of_state(p, E)
    F = greedy.scores_closed_form(p, E, np.diagonal(G[:N]), G[N + p.fom_monitor], idx)
    picks = greedy.select_rank_k(F, fom, p.tau, 5, 3, p.nx)
    assert 1 <= len(picks) <= 5
    assert picks[0].pixel == greedy.select_greedy(F, fom, p.tau).pixel
    for i, a in enumerate(picks):
        assert a.fom_new > fom
        for b in picks[:i]:
            d = max(abs(a.pixel // p.nx - b.pixel // p.nx), abs(a.pixel % p.nx - b.pixel % p.nx))
            assert d >= 3
    # scores are non-increasing along the picks (each is the best still eligible)
    vals = [pk.fom_new for pk in picks]
    assert all(b <= a * (1 + p.tau) for a, b in zip(vals, vals[1:]))


def test_rank_k_trajectory_joint_state_is_exact():
    p = W.tiny(10, 10, n_mon=4, cand_mask=W.MASK_BOTH, rank_k=4, min_spacing=3, steps=3)
    tr = greedy.rank_k_trajectory(p, tier="T1")
    idx = np.zeros(p.n, np.uint8)
    for group in tr.steps:
        for s in group:
            idx[s.pixel] = s.eps_idx
    _, E = state.dense_state(p, state.eps_of(p, idx))
    assert abs(state.fom_of_state(p, E) - tr.steps[-1][0].fom) <= 1e-12 * state.fom_of_state(p, E)


def test_replay_certifies_own_sequence():
    p = W.tiny(6, 6, n_mon=4, cand_mask=W.MASK_BOTH, steps=8)
    tr = greedy.greedy(p, tier="T1")
    rep = greedy.replay(p, [(s.pixel, s.eps_idx) for s in tr.steps], tier="T2")
    for r, s in zip(rep, tr.steps):
        assert r["oracle_pixel"] == s.pixel
        assert abs(r["F_taken"] - r["Fstar"]) <= 1e-9 * r["Fstar"]


def test_stored_square32_trajectory_reproduced_by_flipped_set_tier():
    """The stored 32x32 trajectory (written by tier T1) is reproduced by tier T2."""
    import json, os
    path = os.path.join(os.path.dirname(__file__), "golden", "square32_fp64.json")
    gold = json.load(open(path))
    p = W.SMALL_32
    tr = greedy.greedy(p, tier="T2")
    assert [s.pixel for s in tr.steps] == [s["pixel"] for s in gold["steps"]]
    for a, b in zip(tr.steps, gold["steps"]):
        assert abs(a.fom - b["fom"]) <= 1e-11 * b["fom"]


# ---------------------------------------------------------------- epsilon-greedy (Sec. V)
def test_eps_greedy_with_eps_zero_is_the_greedy_trajectory():
    p = W.tiny(6, 7, n_mon=4, cand_mask=W.MASK_BOTH, steps=60)
    g = greedy.greedy(p, tier="T2")
    e = greedy.eps_greedy(p, 0.0, W.eps_greedy_draws(60, seed=3), tier="T2")
    assert [(s.pixel, s.eps_idx) for s in e.steps] == [(s.pixel, s.eps_idx) for s in g.steps]
    assert e.stopped == g.stopped and np.allclose([s.fom for s in e.steps], [s.fom for s in g.steps])


def test_eps_greedy_explore_choice_is_the_drawn_rank_by_brute_force():
    """With eps = 1 every step explores: the move taken must be the
    floor(u * n)-th best of the n <= 4 FOM-increasing moves, ranking every
    candidate structure by a full re-solve (tier T0) and sorting."""
    p = W.tiny(4, 5, n_mon=4, cand_mask=W.MASK_BOTH, steps=12)
    idx0 = W.random_eps_idx(p, 0.3, seed=11)              # breaks the mirror ties
    draws = W.eps_greedy_draws(12, seed=5)
    tr = greedy.eps_greedy(p, 1.0, draws, tier="T1", eps_idx0=idx0)
    assert len(tr.steps) >= 4
    G0 = greens.build_G0(p)
    cur = idx0.copy()
    for t, s in enumerate(tr.steps):
        F = state.brute_force_scores(p, cur, G0)
        _, E = state.dense_state(p, state.eps_of(p, cur), G0)
        fom = state.fom_of_state(p, E)
        # best move of each pixel (two materials: one candidate per pixel), improving only
        best = F.max(axis=1)
        order = [int(q) for q in np.argsort(-best, kind="stable") if best[q] > fom * (1 + p.tau)]
        top = order[:4]
        vals = best[top]
        assert np.all(np.diff(vals) < 0) and np.all(-np.diff(vals) > 1e-9 * vals[0])  # no ties here
        want = top[min(int(draws[t][1] * len(top)), len(top) - 1)]
        assert s.pixel == want and s.eps_idx == int(np.argmax(F[want]))
        cur[s.pixel] = s.eps_idx


def test_eps_greedy_fom_rises_and_ends_without_an_improving_move():
    p = W.tiny(6, 6, n_mon=4, cand_mask=W.MASK_BOTH, steps=400)
    tr = greedy.eps_greedy(p, 0.5, W.eps_greedy_draws(400, seed=2), tier="T2")
    assert tr.stopped
    foms = [tr.fom0] + [s.fom for s in tr.steps]
    assert all(b > a for a, b in zip(foms, foms[1:]))
    G0 = greens.build_G0(p)
    F = state.brute_force_scores(p, tr.eps_idx, G0)
    assert not F.max() > foms[-1] * (1 + p.tau)


# ---------------------------------------------------------------- rank-k selection vs brute force
def spaced_top_k_brute_force(F, fom, tau, k, spacing, nx):
    """Independent statement of the rank-k rule (eq. form14 moves with a
    minimum-spacing set): list every candidate, sort by (-FOM', pixel,
    material), walk the list and accept a candidate iff it improves the FOM by
    more than the band, its pixel is not yet chosen and its Chebyshev distance
    to EVERY accepted pixel is at least `spacing` (checked pair by pair), until
    k are accepted.  Equal to the band rule only where tied scores are exactly
    equal, which the callers arrange."""
    N, ne = F.shape
    cands = sorted((-F[p, e], p, e) for p in range(N) for e in range(ne) if np.isfinite(F[p, e]))
    chosen = []
    for negf, p, e in cands:
        if len(chosen) == k or not -negf > fom * (1.0 + tau):
            break
        ok = True
        for q, _ in chosen:
            cheb = max(abs(p // nx - q // nx), abs(p % nx - q % nx))
            if q == p or cheb < spacing:
                ok = False
                break
        if ok:
            chosen.append((p, e))
    return chosen


def rank_k_case(kind, seed=0):
    """(problem, F, fom) of a state on a 14x14 grid whose scores are computed by
    the closed form on the exact (tier T1) state.  'random': a random mask;
    'mirror': a mirror-symmetric mask with the score array symmetrised so that
    mirror pairs tie exactly; 'three': a three-material table (so one pixel has
    two candidates)."""
    if kind == "three":
        p = W.tiny(14, 14, n_mon=4, cand_mask=0b111, eps_table=(1.0, 12.25, 4.0))
        idx = W.random_material_idx(p, seed)
    else:
        p = W.tiny(14, 14, n_mon=4, cand_mask=W.MASK_BOTH)
        idx = (W.mirror_symmetric_eps_idx(p, 0.25, seed) if kind == "mirror"
               else W.random_eps_idx(p, 0.25, seed))
    N = p.n
    G, E = state.dense_state(p, state.eps_of(p, idx))
    F = greedy.scores_closed_form(p, E, np.diagonal(G[:N]), G[N + p.fom_monitor], idx)
    if kind == "mirror":
        Fm = F.reshape(p.ny, p.nx, -1)[:, ::-1, :].reshape(N, -1)
        F = np.maximum(F, Fm)
    fom = state.fom_of_state(p, E)
    return p, F, fom


def _distinct_scores_separated(F, tau):
    v = np.unique(F[np.isfinite(F)])
    return v.size < 2 or np.min(np.diff(v) / v[1:]) > 4 * tau


@pytest.mark.parametrize("kind", ["random", "mirror", "three"])
@pytest.mark.parametrize("spacing", [0, 2, 3])
def test_rank_k_selection_equals_brute_force_spaced_top_k(kind, spacing):
    p, F, fom = rank_k_case(kind, seed=4)
    # band tau on scores whose distinct values lie further apart than the band (then
    # the band holds exact ties only), and tau = 0 on the same scores
    tau = 1e-9
    assert _distinct_scores_separated(F, tau)
    for t in (0.0, tau):
        for k in (1, 5, 16, 40):
            got = [(pk.pixel, pk.eps_idx) for pk in greedy.select_rank_k(F, fom, t, k, spacing, p.nx)]
            want = spaced_top_k_brute_force(F, fom, t, k, spacing, p.nx)
            assert got == want, (kind, spacing, t, k)
    # the case exercises the rule: with k = 40 the spacing rule, not k, ends the set
    # (spacing >= 2), and the accepted set is strictly smaller than without it
    full = spaced_top_k_brute_force(F, fom, tau, 40, spacing, p.nx)
    if spacing >= 2:
        assert len(full) < 40
        assert len(spaced_top_k_brute_force(F, fom, tau, 40, 0, p.nx)) > len(full)


def test_rank_k_band_takes_the_lowest_index_among_near_ties():
    """Near-ties within the band (not exact ties): the lowest (pixel, material)
    of the band is accepted first, then the rule repeats over what is left."""
    nx = 10
    F = np.full((30, 2), -np.inf)
    F[25, 1] = 2.0 + 1e-9          # the largest score
    F[3, 1] = 2.0                  # within tau = 1e-9 * 2 of it: tied, lower index wins
    F[28, 1] = 1.5                 # (2, 8): far from pixels 3 (0, 3) and 25 (2, 5)
    F[4, 1] = 1.9                  # Chebyshev distance 1 from pixel 3: excluded at spacing 2
    picks = greedy.select_rank_k(F, 1.0, 1e-9, 4, 2, nx)
    assert [(pk.pixel, pk.eps_idx) for pk in picks] == [(3, 1), (25, 1), (28, 1)]
    # spacing 1 keeps pixel 4 (distance 1 >= 1), ordered by score after the band
    picks = greedy.select_rank_k(F, 1.0, 1e-9, 4, 1, nx)
    assert [pk.pixel for pk in picks] == [3, 25, 4, 28]
    # nothing above fom (1 + tau) is accepted
    assert greedy.select_rank_k(F, 2.0 + 1e-9, 1e-9, 4, 0, nx) == []
