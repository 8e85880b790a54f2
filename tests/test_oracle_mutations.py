"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin catches each.

Each case patches one oracle function with a typical slip (dropped term, wrong
sign, transposed operand, wrong tie direction) and re-runs the relevant pin
body; the pin must fail.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import greens, greedy, state
import workloads as W


def _self_term_pin_holds():
    k0 = 2 * math.pi
    h = 0.05
    a = h / math.sqrt(math.pi)
    re = integrate.quad(lambda r: 2 * math.pi * r * greens.g2d(r, k0).real, 0, a, limit=200)[0]
    im = integrate.quad(lambda r: 2 * math.pi * r * greens.g2d(r, k0).imag, 0, a, limit=200)[0]
    st = greens.self_term(h, k0)
    return abs(st - complex(re, im)) <= 1e-8 * abs(st)


def _dense_pins_hold():
    p = W.tiny(4, 5, n_mon=2)
    eps = state.eps_of(p, W.random_eps_idx(p, 0.4, 1))
    N = p.n
    G0 = greens.build_G0(p)
    G, _ = state.dense_state(p, eps, G0)
    a = greens.alpha_of(p, eps)
    res = (np.eye(N) - G0[:N] * a[None, :]) @ G[:N] - G0[:N]
    ok_res = np.linalg.norm(res) <= 1e-12 * np.linalg.norm(G0[:N])
    ok_sym = np.linalg.norm(G[:N] - G[:N].T) <= 1e-12 * np.linalg.norm(G[:N])
    return ok_res and ok_sym


def _score_pin_holds():
    p = W.tiny(3, 4, n_mon=2)
    idx = W.random_eps_idx(p, 0.4, 2)
    G, E = state.dense_state(p, state.eps_of(p, idx))
    N = p.n
    F0 = state.brute_force_scores(p, idx)
    F1 = greedy.scores_closed_form(p, E, np.diagonal(G[:N]), G[N + p.fom_monitor], idx)
    fin = np.isfinite(F0)
    return np.allclose(F1[fin], F0[fin], rtol=1e-10, atol=0)


def _mirror_tie_pin_holds():
    p = W.tiny(4, 6, n_mon=4)
    idx = W.mirror_symmetric_eps_idx(p, 0.3, seed=2)
    G, E = state.dense_state(p, state.eps_of(p, idx))
    N = p.n
    F = greedy.scores_closed_form(p, E, np.diagonal(G[:N]), G[N + p.fom_monitor], idx)
    pick = greedy.select_greedy(F, state.fom_of_state(p, E), p.tau)
    return pick.pixel % p.nx < p.nx / 2


def test_unpatched_pins_hold():
    assert _self_term_pin_holds() and _dense_pins_hold() and _score_pin_holds()
    assert _mirror_tie_pin_holds()


def test_pin_catches_dropped_static_term(monkeypatch):
    def bad(h, k0):
        a = h / np.sqrt(np.pi)
        return complex(1j * np.pi * a / (2 * k0) * special.hankel1(1, k0 * a))   # "-1/k0^2" dropped
    monkeypatch.setattr(greens, "self_term", bad)
    assert not _self_term_pin_holds()


def test_pin_catches_transposed_contrast_product(monkeypatch):
    orig = state.dense_state

    def bad(problem, eps, G0=None):
        if G0 is None:
            G0 = greens.build_G0(problem)
        N = problem.n
        a = greens.alpha_of(problem, eps)
        A = np.eye(N) - a[:, None] * G0[:N]          # B G0 instead of G0 B
        G_D = np.linalg.solve(A, G0[:N])
        return np.concatenate([G_D, G0[N:]]), None
    monkeypatch.setattr(state, "dense_state", bad)
    assert not _dense_pins_hold()
    monkeypatch.setattr(state, "dense_state", orig)


def test_pin_catches_wrong_contrast_sign(monkeypatch):
    orig = greens.k0_of

    def scores_bad(problem, E, diag, g_mon_row, eps_idx):
        N = problem.n
        k0 = orig(problem)
        table = np.asarray(problem.eps_table)
        eps_cur = table[np.asarray(eps_idx, np.int64)]
        out = np.full((N, table.size), -np.inf)
        for e in range(table.size):
            alpha = k0**2 * (eps_cur - table[e])        # sign slip
            En = E[N + problem.fom_monitor] + alpha * g_mon_row * E[:N] / (1 - alpha * diag)
            out[:, e] = np.where(np.asarray(eps_idx) == e, -np.inf, np.abs(En) ** 2)
        return out
    monkeypatch.setattr(greedy, "scores_closed_form", scores_bad)
    assert not _score_pin_holds()


def test_pin_catches_highest_index_tie_break(monkeypatch):
    def bad(F, fom_now, tau):
        Fstar = float(np.max(F))
        tied = np.flatnonzero(F.ravel() >= Fstar - tau * Fstar)
        flat = int(tied[-1])
        return greedy.Pick(flat // F.shape[1], flat % F.shape[1], float(F.ravel()[flat]))
    monkeypatch.setattr(greedy, "select_greedy", bad)
    assert not _mirror_tie_pin_holds()


def _eps_greedy_pin_holds():
    """Explore steps take the drawn rank of the brute-force ordering (eps = 1)."""
    p = W.tiny(4, 5, n_mon=4, cand_mask=W.MASK_BOTH, steps=6)
    idx0 = W.random_eps_idx(p, 0.3, seed=11)
    draws = W.eps_greedy_draws(6, seed=5)
    tr = greedy.eps_greedy(p, 1.0, draws, tier="T1", eps_idx0=idx0)
    G0 = greens.build_G0(p)
    cur = idx0.copy()
    for t, s in enumerate(tr.steps):
        F = state.brute_force_scores(p, cur, G0)
        _, E = state.dense_state(p, state.eps_of(p, cur), G0)
        fom = state.fom_of_state(p, E)
        best = F.max(axis=1)
        top = [int(q) for q in np.argsort(-best, kind="stable") if best[q] > fom * (1 + p.tau)][:4]
        if s.pixel != top[min(int(draws[t][1] * len(top)), len(top) - 1)]:
            return False
        cur[s.pixel] = s.eps_idx
    return len(tr.steps) > 0


def test_pin_catches_eps_greedy_rank_slip(monkeypatch):
    assert _eps_greedy_pin_holds()

    def bad(F, fom_now, tau, eps, u_explore, u_choice, nx, n_top=4):
        top = greedy.select_rank_k(F, fom_now, tau, n_top, 0, nx)
        if not top:
            return None
        i = min(int(u_choice * (len(top) - 1)), len(top) - 1) if u_explore < eps else 0  # never the last
        return top[i]
    monkeypatch.setattr(greedy, "select_eps_greedy", bad)
    assert not _eps_greedy_pin_holds()


def _region_score_pin_holds():
    from oracle import regions
    p = W.tiny(4, 6, n_mon=4, cand_mask=W.MASK_BOTH)
    idx = W.random_eps_idx(p, 0.4, seed=3)
    E, row, G_VV = regions._RegionEvaluator(p, 2, "T1")(idx)
    F = regions.region_scores(p, 2, E, G_VV, row, idx)
    F0 = regions.brute_force_region_scores(p, 2, idx)
    fin = np.isfinite(F0)
    return np.allclose(F[fin], F0[fin], rtol=1e-10, atol=0)


def test_pin_catches_region_solve_with_B_on_the_wrong_side(monkeypatch):
    from oracle import regions
    assert _region_score_pin_holds()
    orig_solve = np.linalg.solve

    def scores_bad(problem, b, E, G_VV, g_mon_row, eps_idx):
        K = regions.n_regions(problem, b)
        k0 = greens.k0_of(problem)
        table = np.asarray(problem.eps_table)
        cur = np.asarray(eps_idx, np.int64)
        Em0 = E[problem.n + problem.fom_monitor]
        out = np.full((K, table.size), -np.inf)
        for k in range(K):
            V = regions.region_pixels(problem, b, k)
            for e in range(table.size):
                if not (problem.cand_mask >> e) & 1 or np.all(cur[V] == e):
                    continue
                bv = k0**2 * (table[e] - table[cur[V]])
                A = np.eye(V.size) - bv[:, None] * G_VV[k]          # B G instead of G B
                x = orig_solve(A, E[V])
                En = Em0 + g_mon_row[V] @ (bv * x)
                out[k, e] = abs(En) ** 2
        return out
    monkeypatch.setattr(regions, "region_scores", scores_bad)
    assert not _region_score_pin_holds()


# ---------------------------------------------------------------- rank-k selection (spaced top-k)
def _rank_k_pin_holds():
    """select_rank_k equals the brute-force spaced top-k on every case of the pin."""
    from test_oracle_greedy import rank_k_case, spaced_top_k_brute_force
    for kind in ("random", "mirror", "three"):
        p, F, fom = rank_k_case(kind, seed=4)
        for spacing in (0, 2, 3):
            for t in (0.0, 1e-9):
                for k in (5, 16, 40):
                    got = [(pk.pixel, pk.eps_idx)
                           for pk in greedy.select_rank_k(F, fom, t, k, spacing, p.nx)]
                    if got != spaced_top_k_brute_force(F, fom, t, k, spacing, p.nx):
                        return False
    return True


def _rank_k_with(mask_fn):
    """A select_rank_k whose exclusion after each pick is mask_fn(dy, dx, spacing, pixel, q)."""
    def bad(F, fom_now, tau, k, min_spacing, nx):
        F = F.copy()
        picks = []
        N = F.shape[0]
        q = np.arange(N)
        while len(picks) < k:
            pk = greedy.select_greedy(F, fom_now, tau)
            if pk is None:
                break
            picks.append(pk)
            dy = np.abs(q // nx - pk.pixel // nx)
            dx = np.abs(q % nx - pk.pixel % nx)
            F[mask_fn(dy, dx, min_spacing, pk.pixel, q), :] = -np.inf
        return picks
    return bad


@pytest.mark.parametrize("name,mask_fn", [
    # one more than the spacing asks for (over-strict)
    ("spacing_plus_1", lambda dy, dx, s, p, q: np.maximum(dy, dx) < max(s, 1) + 1),
    # one less (a neighbour at distance spacing - 1 accepted)
    ("spacing_minus_1", lambda dy, dx, s, p, q: np.maximum(dy, dx) < max(s - 1, 1)),
    # an eligible candidate skipped: the next pixel in row-major order is dropped too
    ("skips_next_pixel", lambda dy, dx, s, p, q: (np.maximum(dy, dx) < max(s, 1)) | (q == p + 1)),
    # Manhattan distance in place of Chebyshev
    ("manhattan", lambda dy, dx, s, p, q: dy + dx < max(s, 1)),
    # only the chosen pixel's row is checked (the column offset ignored)
    ("row_only", lambda dy, dx, s, p, q: (dy == 0) & (dx < max(s, 1))),
])
def test_pin_catches_rank_k_exclusion_slip(monkeypatch, name, mask_fn):
    assert _rank_k_pin_holds()
    monkeypatch.setattr(greedy, "select_rank_k", _rank_k_with(mask_fn))
    assert not _rank_k_pin_holds(), name


def test_pin_catches_rank_k_that_ignores_the_improvement_rule(monkeypatch):
    """A set filled up to k with candidates that do not improve the FOM."""
    assert _rank_k_pin_holds()
    orig = greedy.select_rank_k

    def bad(F, fom_now, tau, k, min_spacing, nx):
        return orig(F, -1.0, tau, k, min_spacing, nx)     # every finite score "improves"
    monkeypatch.setattr(greedy, "select_rank_k", bad)
    assert not _rank_k_pin_holds()
