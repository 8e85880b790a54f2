"""Multi-pixel candidate regions (FP64).  Test infrastructure, like all of oracle/.

The paper's moves may flip a region V of several pixels at once (Sec. II with
N_V > 1; Sec. IV flips through-thickness pillars of 2x2 pixels).  Here blocks of
b x b pixels tile the design grid (ny and nx multiples of b); region
k = by * (nx / b) + bx, its pixels in row-major order.  A region move sets every
pixel of the region to material e.

Score of the move (region k, material e), from eqs. form4, form6-form9 at the
monitor (eq. para1), with the area-included G:
    B    = diag(b_i),  b_i = k0^2 (eps_e - eps_cur_i)   (0 where pixel i is at e)
    x    = (I - G_VV B)^-1 E_V                          (fields on V after the move)
    E'   = E_m0 + G[m0, V] B x
    FOM' = |E'|^2
A candidate is any material of the candidate mask that changes at least one
pixel of the region.  The greedy rule is the single-pixel one with (region,
material) in place of (pixel, material): the lowest index within the relative
band tau of the best wins, and the move is taken only if the best exceeds
FOM (1 + tau).
"""
from __future__ import annotations

import numpy as np

from . import greens, state
from .greedy import Step, Trajectory, select_greedy


def n_regions(problem, b: int) -> int:
    if problem.ny % b or problem.nx % b:
        raise ValueError("the grid must be a multiple of the block size")
    return (problem.ny // b) * (problem.nx // b)


def region_pixels(problem, b: int, k: int) -> np.ndarray:
    """Pixel indices of region k, row-major inside the block."""
    rx = problem.nx // b
    by, bx = divmod(k, rx)
    iy = by * b + np.arange(b)
    ix = bx * b + np.arange(b)
    return (iy[:, None] * problem.nx + ix[None, :]).reshape(-1)


def region_scores(problem, b, E, G_VV, g_mon_row, eps_idx) -> np.ndarray:
    """(n_regions, n_eps) FOM' of every region move; -inf for non-candidates.

    G_VV: (n_regions, b*b, b*b) in-block entries of the current G; g_mon_row:
    the FOM monitor row of G over the design pixels; E: the current field (R).
    """
    K = n_regions(problem, b)
    k0 = greens.k0_of(problem)
    table = np.asarray(problem.eps_table, dtype=np.float64)
    cur = np.asarray(eps_idx, dtype=np.int64)
    Em0 = E[problem.n + problem.fom_monitor]
    out = np.full((K, table.size), -np.inf)
    for k in range(K):
        V = region_pixels(problem, b, k)
        for e in range(table.size):
            if not (problem.cand_mask >> e) & 1 or np.all(cur[V] == e):
                continue
            bvec = k0**2 * (table[e] - table[cur[V]])
            A = np.eye(V.size, dtype=np.complex128) - G_VV[k] * bvec[None, :]
            x = np.linalg.solve(A, E[V])
            En = Em0 + g_mon_row[V] @ (bvec * x)
            out[k, e] = float(En.real**2 + En.imag**2)
    return out


def brute_force_region_scores(problem, b, eps_idx, G0=None) -> np.ndarray:
    """Tier T0: FOM of every region-move structure by a full T1 solve."""
    if G0 is None:
        G0 = greens.build_G0(problem)
    K = n_regions(problem, b)
    cur = np.asarray(eps_idx, dtype=np.int64)
    n_eps = len(problem.eps_table)
    out = np.full((K, n_eps), -np.inf)
    for k in range(K):
        V = region_pixels(problem, b, k)
        for e in range(n_eps):
            if not (problem.cand_mask >> e) & 1 or np.all(cur[V] == e):
                continue
            trial = cur.copy()
            trial[V] = e
            _, E = state.dense_state(problem, state.eps_of(problem, trial), G0)
            out[k, e] = state.fom_of_state(problem, E)
    return out


class _RegionEvaluator:
    """E, the FOM monitor row and the in-block entries of G for a structure,
    by tier T1 (dense solve) or T2 (flipped set)."""

    def __init__(self, problem, b, tier):
        self.problem, self.b, self.tier = problem, b, tier
        self.K = n_regions(problem, b)
        self.pix = np.stack([region_pixels(problem, b, k) for k in range(self.K)])   # K x b^2
        self.m0_row = problem.n + problem.fom_monitor
        if tier == "T1":
            self.G0 = greens.build_G0(problem)
        else:
            self.fs = state.FlippedSet(problem)
            # G0 inside a block depends only on the offsets: the same for every block
            p0 = self.pix[0]
            self.G0_VV = greens.G0_block(problem, p0, p0)

    def __call__(self, eps_idx):
        p = self.problem
        eps = state.eps_of(p, eps_idx)
        N = p.n
        if self.tier == "T1":
            G, E = state.dense_state(p, eps, self.G0)
            G_VV = G[self.pix[:, :, None], self.pix[:, None, :]]
            return E, G[self.m0_row, :N], G_VV
        E, _, rows = self.fs.state(eps, rows=[self.m0_row])
        V, U, Q = self.fs.solve(eps)
        G_VV = np.broadcast_to(self.G0_VV, (self.K,) + self.G0_VV.shape).copy()
        if V.size:
            UQ = U[:N] @ Q                                  # N x k
            A = UQ[self.pix]                                # K x b^2 x k
            Bm = U[:N][self.pix]                            # K x b^2 x k (U[q] = G0[V, q])
            G_VV = G_VV + np.einsum("kia,kja->kij", A, Bm)
        return E, rows[self.m0_row], G_VV


def region_greedy(problem, b, steps=None, tier="T2", eps_idx0=None, tau=None) -> Trajectory:
    """Greedy trajectory over region moves; Step.pixel holds the region index."""
    steps = problem.steps if steps is None else steps
    tau = problem.tau if tau is None else tau
    ev = _RegionEvaluator(problem, b, tier)
    eps_idx = (np.zeros(problem.n, np.uint8) if eps_idx0 is None
               else np.asarray(eps_idx0, np.uint8).copy())
    E, row, G_VV = ev(eps_idx)
    fom = state.fom_of_state(problem, E)
    traj = Trajectory(problem.name, fom0=fom)
    for t in range(steps):
        F = region_scores(problem, b, E, G_VV, row, eps_idx)
        pick = select_greedy(F, fom, tau)
        if pick is None:
            traj.stopped = True
            break
        eps_idx[region_pixels(problem, b, pick.pixel)] = pick.eps_idx
        E, row, G_VV = ev(eps_idx)
        fom = state.fom_of_state(problem, E)
        traj.steps.append(Step(t, pick.pixel, pick.eps_idx, pick.fom_new, fom, pick.n_tied))
    traj.eps_idx = eps_idx
    traj.E = E
    return traj
