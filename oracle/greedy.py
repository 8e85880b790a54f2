"""Candidate scores, greedy / rank-k selection, trajectories and replay (FP64).

Score of a candidate (p, eps'): the FOM of the structure with pixel p set to
eps'.  For N_V = 1 the paper's flipped-region solve (eqs. form6-form9) is a
scalar division, and eq. form4 evaluated at the monitor (eq. para1) gives

    alpha  = k0^2 (eps' - eps_p)
    E'_m0  = E_m0 + alpha G[m0, p] E_p / (1 - alpha G_pp)
    FOM'   = |E'_m0|^2.

The tier-T0 brute force (oracle.state.brute_force_scores) pins this closed form.

Greedy policy (Sec. IV; Sec. V): take the move with the largest FOM increase,
stop when no move increases the FOM.  The paper gives no rule for equal
scores; every workload here is mirror symmetric about x = 0, so exact ties are
common.  Reading adopted: with F* the largest candidate FOM, every candidate
with FOM' >= F* - tau F* is tied and the lowest (pixel, material index) wins;
the move is accepted iff F* > FOM (1 + tau).

Rank-k selection: repeat the greedy rule over the candidates that still
improve the FOM individually, whose pixel is not yet chosen and whose
Chebyshev distance to every chosen pixel is at least `min_spacing`, until k
pixels are chosen or none is eligible.  The chosen set is then applied jointly
(eq. form14 with V = the set).

Epsilon-greedy policy (Sec. V): with probability 1 - eps the agent takes the
greedy move; otherwise it explores, choosing at random among the top four
FOM-increasing moves; it runs until no FOM-increasing move is left.  Readings
adopted: the top four are the first four picks of the rank-k rule with no
spacing (distinct pixels; for a two-material table these are the four best
moves), the greedy move among them; random numbers are inputs, one pair
(u_explore, u_choice) per step: the step explores iff u_explore < eps and then
takes entry floor(u_choice * n) of the n (<= 4) improving moves.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

from . import greens, state


def scores_closed_form(problem, E, diag, g_mon_row, eps_idx) -> np.ndarray:
    """(N, n_eps) candidate FOMs; -inf where (p, e) is not a candidate."""
    N = problem.n
    k0 = greens.k0_of(problem)
    table = np.asarray(problem.eps_table, dtype=np.float64)
    eps_idx = np.asarray(eps_idx, dtype=np.int64)
    eps_cur = table[eps_idx]
    E_m0 = E[N + problem.fom_monitor]
    E_D = E[:N]
    out = np.full((N, table.size), -np.inf)
    for e in range(table.size):
        if not (problem.cand_mask >> e) & 1:
            continue
        alpha = k0**2 * (table[e] - eps_cur)
        E_new = E_m0 + alpha * g_mon_row * E_D / (1.0 - alpha * diag)
        F = E_new.real**2 + E_new.imag**2
        out[:, e] = np.where(eps_idx == e, -np.inf, F)
    return out


@dataclass
class Pick:
    pixel: int
    eps_idx: int
    fom_new: float
    n_tied: int = 1


def select_greedy(F: np.ndarray, fom_now: float, tau: float):
    """Greedy choice with the tie rule; None when no candidate improves the FOM."""
    Fstar = float(np.max(F))
    if not np.isfinite(Fstar) or not Fstar > fom_now * (1.0 + tau):
        return None
    tied = np.flatnonzero(F.ravel() >= Fstar - tau * Fstar)
    flat = int(tied[0])                       # lowest (pixel, material) in row-major order
    return Pick(flat // F.shape[1], flat % F.shape[1], float(F.ravel()[flat]), int(tied.size))


def select_rank_k(F: np.ndarray, fom_now: float, tau: float, k: int, min_spacing: int, nx: int):
    """Up to k picks: greedy rule restricted to spaced, individually improving candidates."""
    F = F.copy()
    picks = []
    N = F.shape[0]
    iy = np.arange(N) // nx
    ix = np.arange(N) % nx
    while len(picks) < k:
        p = select_greedy(F, fom_now, tau)
        if p is None:
            break
        picks.append(p)
        cheb = np.maximum(np.abs(iy - iy[p.pixel]), np.abs(ix - ix[p.pixel]))
        F[cheb < max(min_spacing, 1), :] = -np.inf
    return picks


@dataclass
class Step:
    step: int
    pixel: int
    eps_idx: int
    fom_pred: float        # candidate FOM computed before the move
    fom: float             # FOM of the new structure (exact state)
    n_tied: int


@dataclass
class Trajectory:
    problem_name: str
    steps: list = field(default_factory=list)
    fom0: float = 0.0
    stopped: bool = False
    eps_idx: np.ndarray = None
    E: np.ndarray = None

    def pixels(self):
        return [s.pixel for s in self.steps]


class _Evaluator:
    """Exact state of the current structure by tier T1, T2 or T2u.

    T2u walks a sequence of one-pixel moves: E and the FOM monitor's row come
    from the flipped set (tier T2, O(k N) once the k x k system is solved), and
    diag(G) is carried from the previous structure by the paper's update
    (eq. form10 with a one-pixel region, restricted to the diagonal):
        diag'[q] = diag[q] + c G[q, j] G[j, q],  c = alpha / (1 - alpha G[j, j]),
    with column j of the previous structure's G taken exactly from the flipped
    set and G[j, q] = G[q, j] (reciprocity).  Any other change of structure
    (the first call, or more than one pixel changed) is a full T2 evaluation.
    It avoids the O(k^2 N) diagonal of T2 at every step of a long replay; the
    tests pin it against T2 along random move sequences.
    """

    def __init__(self, problem, tier):
        self.problem = problem
        self.tier = tier
        N = problem.n
        self.m0_row = N + problem.fom_monitor
        if tier == "T1":
            self.G0 = greens.build_G0(problem)
        else:
            self.fs = state.FlippedSet(problem)
        self.prev = None

    def __call__(self, eps_idx):
        eps = state.eps_of(self.problem, eps_idx)
        if self.tier == "T1":
            G, E = state.dense_state(self.problem, eps, self.G0)
            N = self.problem.n
            return E, np.diagonal(G[:N]).copy(), G[self.m0_row]
        if self.tier == "T2u":
            return self._walk(np.asarray(eps_idx).copy(), eps)
        E, diag, rows = self.fs.state(eps, rows=[self.m0_row])
        return E, diag, rows[self.m0_row]

    def _walk(self, eps_idx, eps):
        N = self.problem.n
        changed = None if self.prev is None else np.flatnonzero(eps_idx != self.prev[0])
        if changed is not None and changed.size == 0:
            return self.prev[2:]
        if changed is None or changed.size > 1:
            E, diag, rows = self.fs.state(eps, rows=[self.m0_row])
        else:
            j = int(changed[0])
            eps_prev, diag_prev = self.prev[1], self.prev[3]
            col = self.fs.column_of(eps_prev, j)[:N]
            alpha = greens.k0_of(self.problem) ** 2 * (eps[j] - eps_prev[j])
            c = alpha / (1.0 - alpha * col[j])
            diag = diag_prev + c * col * col
            E, _, rows = self.fs.state(eps, rows=[self.m0_row], with_diag=False)
        row = rows[self.m0_row]
        self.prev = (eps_idx, eps, E, diag, row)
        return E, diag, row


def greedy(problem, steps=None, tier="T1", eps_idx0=None, tau=None, callback=None) -> Trajectory:
    """Canonical greedy trajectory: exact state each step, closed-form scores, tie rule."""
    steps = problem.steps if steps is None else steps
    tau = problem.tau if tau is None else tau
    ev = _Evaluator(problem, tier)
    eps_idx = (np.zeros(problem.n, np.uint8) if eps_idx0 is None
               else np.asarray(eps_idx0, np.uint8).copy())
    E, diag, row = ev(eps_idx)
    fom = state.fom_of_state(problem, E)
    traj = Trajectory(problem.name, fom0=fom)
    for t in range(steps):
        F = scores_closed_form(problem, E, diag, row, eps_idx)
        pick = select_greedy(F, fom, tau)
        if pick is None:
            traj.stopped = True
            break
        eps_idx[pick.pixel] = pick.eps_idx
        E, diag, row = ev(eps_idx)
        fom = state.fom_of_state(problem, E)
        traj.steps.append(Step(t, pick.pixel, pick.eps_idx, pick.fom_new, fom, pick.n_tied))
        if callback is not None:
            callback(t, eps_idx, E)
    traj.eps_idx = eps_idx
    traj.E = E
    return traj


def replay(problem, moves, tier="T2", eps_idx0=None, check_every=1, callback=None, final=False):
    """Follow a given move sequence [(pixel, eps_idx), ...] and certify each choice.

    At each checked step returns the oracle's best candidate FOM F*, the oracle
    FOM of the move actually taken, and the oracle's own greedy pick.  final:
    one more record (step = len(moves), F_taken None) with F*, the FOM and the
    field E of the structure the sequence ends in, so a caller can check that
    no move is left that improves the FOM.  tier "T2u" suits long sequences (check_every = 1).
    """
    ev = _Evaluator(problem, tier)
    eps_idx = (np.zeros(problem.n, np.uint8) if eps_idx0 is None
               else np.asarray(eps_idx0, np.uint8).copy())
    E, diag, row = ev(eps_idx)
    out = []
    for t, (p, e) in enumerate(moves):
        if t % check_every == 0:
            F = scores_closed_form(problem, E, diag, row, eps_idx)
            best = select_greedy(F, state.fom_of_state(problem, E), problem.tau)
            out.append(dict(step=t, Fstar=float(np.max(F)), F_taken=float(F[p, e]),
                            oracle_pixel=None if best is None else best.pixel,
                            oracle_eps=None if best is None else best.eps_idx,
                            fom_before=state.fom_of_state(problem, E)))
        eps_idx[p] = e
        if (t + 1) % check_every == 0 or t + 1 == len(moves):
            E, diag, row = ev(eps_idx)
            if callback is not None:
                callback(t, eps_idx, E)
    if final:
        if not moves:
            E, diag, row = ev(eps_idx)
        F = scores_closed_form(problem, E, diag, row, eps_idx)
        best = select_greedy(F, state.fom_of_state(problem, E), problem.tau)
        out.append(dict(step=len(moves), Fstar=float(np.max(F)), F_taken=None,
                        oracle_pixel=None if best is None else best.pixel,
                        oracle_eps=None if best is None else best.eps_idx,
                        fom_before=state.fom_of_state(problem, E), E=E))
    return out


def rank_k_trajectory(problem, steps=None, tier="T2", tau=None) -> Trajectory:
    """Rank-k policy: each step applies up to k spaced picks jointly."""
    steps = problem.steps if steps is None else steps
    tau = problem.tau if tau is None else tau
    ev = _Evaluator(problem, tier)
    eps_idx = np.zeros(problem.n, np.uint8)
    E, diag, row = ev(eps_idx)
    fom = state.fom_of_state(problem, E)
    traj = Trajectory(problem.name, fom0=fom)
    for t in range(steps):
        F = scores_closed_form(problem, E, diag, row, eps_idx)
        picks = select_rank_k(F, fom, tau, problem.rank_k, problem.min_spacing, problem.nx)
        if not picks:
            traj.stopped = True
            break
        for pk in picks:
            eps_idx[pk.pixel] = pk.eps_idx
        E, diag, row = ev(eps_idx)
        fom = state.fom_of_state(problem, E)
        traj.steps.append([Step(t, pk.pixel, pk.eps_idx, pk.fom_new, fom, pk.n_tied)
                           for pk in picks])
    traj.eps_idx = eps_idx
    traj.E = E
    return traj


def select_eps_greedy(F: np.ndarray, fom_now: float, tau: float, eps: float, u_explore: float,
                      u_choice: float, nx: int, n_top: int = 4):
    """Epsilon-greedy choice; None when no candidate improves the FOM."""
    top = select_rank_k(F, fom_now, tau, n_top, 0, nx)
    if not top:
        return None
    i = 0
    if u_explore < eps:
        i = min(int(u_choice * len(top)), len(top) - 1)
    return top[i]


def eps_greedy(problem, eps, draws, steps=None, tier="T2", eps_idx0=None, tau=None,
               n_top=4) -> Trajectory:
    """Epsilon-greedy trajectory; step t uses draws[t] = (u_explore, u_choice)."""
    steps = problem.steps if steps is None else steps
    tau = problem.tau if tau is None else tau
    ev = _Evaluator(problem, tier)
    eps_idx = (np.zeros(problem.n, np.uint8) if eps_idx0 is None
               else np.asarray(eps_idx0, np.uint8).copy())
    E, diag, row = ev(eps_idx)
    fom = state.fom_of_state(problem, E)
    traj = Trajectory(problem.name, fom0=fom)
    for t in range(min(steps, len(draws))):
        F = scores_closed_form(problem, E, diag, row, eps_idx)
        pick = select_eps_greedy(F, fom, tau, eps, float(draws[t][0]), float(draws[t][1]),
                                 problem.nx, n_top)
        if pick is None:
            traj.stopped = True
            break
        eps_idx[pick.pixel] = pick.eps_idx
        E, diag, row = ev(eps_idx)
        fom = state.fom_of_state(problem, E)
        traj.steps.append(Step(t, pick.pixel, pick.eps_idx, pick.fom_new, fom, pick.n_tied))
    traj.eps_idx = eps_idx
    traj.E = E
    return traj
