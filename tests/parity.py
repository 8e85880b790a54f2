"""Shared parity checks of the GPU tests against the FP64 oracle.

Element-wise relative error: |got_i - want_i| / max(|want_i|, floor * max_j |want_j|).
Every value of a field is held to the tolerance on its own; the floor keeps an
entry that is near zero (a node of the field) from demanding more than the
largest entries' absolute accuracy times `floor`.  The whole-array norm ratio
is kept as a diagnostic.

Certified ties (reduced-precision runs): the GPU's move sequence equals the
oracle's up to a step t; from t on the oracle replays the GPU's own moves and
each must be a certified tie, its exact FP64 score within `tol` of the best
exact score at that state.
"""
from __future__ import annotations

import numpy as np

FLOOR = 1e-3
C64_U = 2.0 ** -24            # unit roundoff of complex64 storage (FP32 parts)


def c64_drift_tol(n_updates):
    """Element-wise tolerance (with the 1e-3 floor) for complex64 state that went
    through n rank-1 (or rank-k) updates on two different paths, or on one path
    against the exact state.  Each update adds a term c u_r v_q whose size can
    reach max|G|, rounded once to FP32, so the absolute error of an entry grows
    like sqrt(n) u max|G| for independent roundings; three times that, against
    the floor 1e-3 max|G|, is 3 sqrt(n) u / 1e-3 (2.2e-3 at n = 150).  The
    fields against the FP64 oracle are held to the stated 1e-4 instead."""
    return 3.0 * np.sqrt(max(int(n_updates), 1)) * C64_U / FLOOR


def rel_elem(got, want, floor=FLOOR):
    """Largest element-wise relative error (with the absolute floor)."""
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (got.shape, want.shape)
    if want.size == 0:
        return 0.0
    top = float(np.max(np.abs(want)))
    if top == 0.0:
        return float(np.max(np.abs(got)))
    scale = np.maximum(np.abs(want), floor * top)
    return float(np.max(np.abs(got - want) / scale))


def rel_norm(got, want):
    got = np.asarray(got)
    want = np.asarray(want)
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300))


def report(what, got, want, floor=FLOOR):
    """Element-wise error (returned) and a one-line record of both measures."""
    e = rel_elem(got, want, floor)
    print(f"[parity] {what}: elementwise {e:.3e}, norm {rel_norm(got, want):.3e}", flush=True)
    return e


def assert_close(what, got, want, tol, floor=FLOOR):
    got = np.asarray(got)
    want = np.asarray(want)
    e = report(what, got, want, floor)
    if not e <= tol:
        top = float(np.max(np.abs(want)))
        scale = np.maximum(np.abs(want), floor * top)
        i = int(np.argmax(np.abs(got - want) / scale))
        raise AssertionError(f"{what}: element {np.unravel_index(i, want.shape)} relative error "
                             f"{e:.3e} > {tol:.1e} (got {got.flat[i]}, want {want.flat[i]})")


def first_divergence(a, b):
    t = 0
    while t < min(len(a), len(b)) and a[t] == b[t]:
        t += 1
    return t


def certify_sequence(p, oracle_moves, gpu_moves, tol=1e-4, checkpoints=(), on_state=None):
    """Parity of a reduced-precision move sequence against the FP64 greedy sequence.

    The sequences agree up to a step t; from t on, the oracle replays the GPU's
    own moves (tier T2u) and every move must be a certified tie.  If the GPU
    stops first, the best remaining exact score must improve the FOM by less
    than tol.  on_state(step, E) is called with the oracle's exact field of the
    GPU's structure after `step` moves for every step in `checkpoints` beyond t,
    and for the last step when it is listed (also when the GPU stopped at t).
    Returns t, the index of the first divergence.
    """
    from oracle import greedy as og

    t = first_divergence(oracle_moves, gpu_moves)
    if t == len(oracle_moves) == len(gpu_moves):
        return t
    idx0 = np.zeros(p.n, np.uint8)
    for j, e in gpu_moves[:t]:
        idx0[j] = e
    n = len(gpu_moves)
    want = {int(c) for c in checkpoints if int(c) > t or int(c) == n}
    given = set()

    def cb(u, eps_idx, E):
        if on_state is not None and t + u + 1 in want:
            given.add(t + u + 1)
            on_state(t + u + 1, E)

    rep = og.replay(p, gpu_moves[t:], tier="T2u", eps_idx0=idx0, callback=cb, final=True)
    if on_state is not None and n in want and n not in given:
        on_state(n, rep[-1]["E"])            # no move replayed: the end state is step t
    for r in rep[:-1]:
        u = t + r["step"]
        assert r["F_taken"] >= (1 - tol) * r["Fstar"], \
            f"step {u}: move {gpu_moves[u]} is not a certified tie ({r['F_taken']} vs {r['Fstar']})"
    last = rep[-1]
    if len(gpu_moves) < len(oracle_moves):
        assert last["Fstar"] <= last["fom_before"] * (1 + tol), "stopped before the oracle"
    print(f"[parity] certified {len(gpu_moves) - t} moves after the divergence at step {t}",
          flush=True)
    return t


def certify_rank_k_set(F, fom, gpu_set, k, spacing, nx, tol=1e-4):
    """A rank-k set chosen in reduced precision against the exact scores F of
    the state it was chosen at: the sets are built in the same order, and pick
    i must be eligible given picks 0..i-1 (pixel new, Chebyshev distance >=
    spacing to each of them) and a certified tie of the best eligible exact
    score.  If the GPU's set is shorter than k, no eligible candidate may be
    left that improves the FOM by more than tol.  Returns the number of picks
    that equal the oracle's own rule (the length of the common prefix)."""
    from oracle import greedy as og

    F = np.array(F, dtype=np.float64)
    nx = int(nx)
    own = [(pk.pixel, pk.eps_idx) for pk in og.select_rank_k(F, fom, 0.0, k, spacing, nx)]
    common = first_divergence(own, list(gpu_set))
    iy = np.arange(F.shape[0]) // nx
    ix = np.arange(F.shape[0]) % nx
    for i, (j, e) in enumerate(gpu_set):
        Fstar = float(np.max(F))
        assert np.isfinite(F[j, e]), f"pick {i} ({j}, {e}) is not eligible"
        assert F[j, e] >= (1 - tol) * Fstar, f"pick {i} ({j}, {e}): {F[j, e]} vs best {Fstar}"
        assert F[j, e] > fom * (1 - tol), f"pick {i} does not improve the FOM"
        cheb = np.maximum(np.abs(iy - iy[j]), np.abs(ix - ix[j]))
        F[cheb < max(spacing, 1), :] = -np.inf
    if len(gpu_set) < k:
        assert not np.max(F) > fom * (1 + tol), "set ended while an eligible move improves the FOM"
    return common
