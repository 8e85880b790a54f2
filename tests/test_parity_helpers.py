"""CPU checks of the GPU tests' parity helpers (tests/parity.py): the element-wise
measure, sequence certification and rank-k set certification, on oracle states
with planted deviations."""
import numpy as np
import pytest

from oracle import greedy as og, state as ost
import workloads as W
import parity


def test_rel_elem_sees_one_bad_entry_that_the_norm_hides():
    want = np.ones(10000, np.complex128)
    want[7] = 1e-2                          # a weak entry
    got = want.copy()
    got[7] *= 1 + 1e-2                      # 1 % off on the weak entry only
    assert parity.rel_norm(got, want) < 2e-6
    assert parity.rel_elem(got, want) == pytest.approx(1e-2, rel=1e-9)
    # below the floor, the error is measured against floor * max|want|
    got = want.copy()
    got[7] = 0.0
    want[7] = 1e-9
    assert parity.rel_elem(got, want) == pytest.approx(1e-9 / 1e-3, rel=1e-6)


def test_certify_sequence_accepts_the_oracle_and_rejects_a_worse_move():
    p = W.tiny(6, 7, n_mon=4, steps=40, tau=1e-9)
    tr = og.greedy(p, tier="T2")
    moves = [(s.pixel, s.eps_idx) for s in tr.steps]
    assert parity.certify_sequence(p, moves, moves) == len(moves)
    # the GPU stops early: refused, since an improving move is left
    with pytest.raises(AssertionError):
        parity.certify_sequence(p, moves, moves[:-3])
    # at step 5 the GPU takes a clearly worse move: refused
    idx = np.zeros(p.n, np.uint8)
    for j, e in moves[:5]:
        idx[j] = e
    E, diag, rows = ost.FlippedSet(p).state(ost.eps_of(p, idx), rows=[p.n + p.fom_monitor])
    F = og.scores_closed_form(p, E, diag, rows[p.n + p.fom_monitor], idx)
    flat = np.argsort(F.ravel())
    fin = flat[np.isfinite(F.ravel()[flat])]
    worse = int(fin[len(fin) // 2])
    bad = moves[:5] + [(worse // F.shape[1], worse % F.shape[1])] + moves[6:]
    with pytest.raises(AssertionError, match="certified tie"):
        parity.certify_sequence(p, moves, bad)


def test_certify_rank_k_set_rules():
    from test_oracle_greedy import rank_k_case
    p, F, fom = rank_k_case("random", seed=4)
    own = [(pk.pixel, pk.eps_idx) for pk in og.select_rank_k(F, fom, 0.0, 16, 3, p.nx)]
    assert parity.certify_rank_k_set(F, fom, own, 16, 3, p.nx) == len(own)
    # a set that breaks the spacing rule
    j0 = own[0][0]
    close = j0 + 1 if (j0 + 1) % p.nx else j0 - 1
    with pytest.raises(AssertionError):
        parity.certify_rank_k_set(F, fom, own[:1] + [(close, 1 - 0)] + own[2:], 16, 3, p.nx)
    # a set cut short while eligible improving moves remain
    if len(own) == 16:
        pytest.skip("case fills the set")
    with pytest.raises(AssertionError, match="set ended"):
        parity.certify_rank_k_set(F, fom, own[:-1], 16, 3, p.nx)
