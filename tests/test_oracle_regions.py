"""Pins of the oracle's multi-pixel region moves (paper Sec. II with N_V > 1;
Sec. IV's pillar moves): closed-form region scores against a full re-solve of
every candidate structure, the one-pixel reduction, the greedy rule against the
brute-force argmax, T1 = T2 trajectories."""
import numpy as np

from oracle import greedy, greens, regions, state
import workloads as W


def test_region_scores_match_brute_force_resolve():
    p = W.tiny(4, 6, n_mon=4, cand_mask=W.MASK_BOTH)
    idx = W.random_eps_idx(p, 0.4, seed=3)               # mixed regions included
    ev = regions._RegionEvaluator(p, 2, "T1")
    E, row, G_VV = ev(idx)
    F = regions.region_scores(p, 2, E, G_VV, row, idx)
    F0 = regions.brute_force_region_scores(p, 2, idx)
    assert np.array_equal(np.isfinite(F), np.isfinite(F0))
    fin = np.isfinite(F0)
    assert np.allclose(F[fin], F0[fin], rtol=1e-10, atol=0)


def test_one_pixel_regions_are_the_single_pixel_scores():
    p = W.tiny(4, 5, n_mon=4, cand_mask=W.MASK_BOTH)
    idx = W.random_eps_idx(p, 0.5, seed=4)
    ev = regions._RegionEvaluator(p, 1, "T1")
    E, row, G_VV = ev(idx)
    F = regions.region_scores(p, 1, E, G_VV, row, idx)
    G, E2 = state.dense_state(p, state.eps_of(p, idx))
    N = p.n
    F1 = greedy.scores_closed_form(p, E2, np.diagonal(G[:N]), G[N + p.fom_monitor], idx)
    fin = np.isfinite(F1)
    assert np.array_equal(np.isfinite(F), fin) and np.allclose(F[fin], F1[fin], rtol=1e-12)


def test_flipped_set_block_entries_match_dense():
    p = W.tiny(6, 6, n_mon=4)
    idx = W.random_eps_idx(p, 0.3, seed=5)
    E1, r1, B1 = regions._RegionEvaluator(p, 2, "T1")(idx)
    E2, r2, B2 = regions._RegionEvaluator(p, 2, "T2")(idx)
    assert np.allclose(E1, E2, rtol=1e-12, atol=1e-14)
    assert np.allclose(r1, r2, rtol=1e-12, atol=1e-14)
    assert np.allclose(B1, B2, rtol=1e-12, atol=1e-14)


def _lens(n, steps):
    """Grid at lambda/40 with the monitors half a wavelength out: 2x2 region moves
    improve the FOM here (at lambda/20 no 2x2 silicon block does, from vacuum)."""
    return W.tiny(n, n, n_mon=4, cand_mask=W.MASK_BOTH, steps=steps, pitch=0.025,
                  mon_distance=0.5)


def test_region_greedy_is_brute_force_argmax_and_monotone():
    p = _lens(8, 8)
    tr = regions.region_greedy(p, 2, tier="T1")
    assert len(tr.steps) >= 3
    G0 = greens.build_G0(p)
    cur = np.zeros(p.n, np.uint8)
    fom = tr.fom0
    for s in tr.steps:
        F0 = regions.brute_force_region_scores(p, 2, cur, G0)
        Fstar = F0.max()
        band = np.flatnonzero(F0.ravel() >= Fstar * (1 - p.tau))
        assert Fstar > fom and band[0] == s.pixel * F0.shape[1] + s.eps_idx
        cur[regions.region_pixels(p, 2, s.pixel)] = s.eps_idx
        assert s.fom > fom
        fom = s.fom


def test_region_trajectories_T1_equal_T2():
    p = _lens(16, 40)
    a = regions.region_greedy(p, 2, tier="T1")
    b = regions.region_greedy(p, 2, tier="T2")
    assert [(s.pixel, s.eps_idx) for s in a.steps] == [(s.pixel, s.eps_idx) for s in b.steps]
    assert a.stopped == b.stopped and len(a.steps) >= 10
    assert np.allclose([s.fom for s in a.steps], [s.fom for s in b.steps], rtol=1e-10)


def test_region_update_by_paper_formula_equals_resolve():
    """The move applied by eqs. form10-form14 on the region equals the re-solve."""
    p = W.tiny(4, 6, n_mon=4)
    idx = W.random_eps_idx(p, 0.3, seed=6)
    G, E = state.dense_state(p, state.eps_of(p, idx))
    V = regions.region_pixels(p, 2, 3)
    eps_cur = state.eps_of(p, idx)
    G2, E2 = state.update_region(p, G, E, eps_cur, V, np.full(V.size, p.eps_table[1]))
    idx2 = idx.copy()
    idx2[V] = 1
    Gd, Ed = state.dense_state(p, state.eps_of(p, idx2))
    assert np.allclose(E2, Ed, rtol=1e-11, atol=1e-13) and np.allclose(G2, Gd, rtol=1e-10, atol=1e-13)
