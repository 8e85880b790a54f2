"""Field and Green's matrix of a structure, FP64 (tiers T0/T1/T2 + the paper's updates).

A structure is a permittivity per design pixel.  With B = diag(alpha_p),
alpha_p = k0^2 (eps_p - 1), the discretised Dyson equation (eq. form2) and
Lippmann-Schwinger equation (eq. form3) over the design region D and the
monitors M read

    G_D = G0_DD + G0_DD B G_D          E_D = Einc_D + G0_DD B E_D
    G_M = G0_MD + G0_MD B G_D          E_M = Einc_M + G0_MD B E_D

(rows of G: design pixels then monitors; columns: design pixels).  Tier T1
solves these directly; it *is* the definition of the state of a structure.
Tier T2 uses that B vanishes off the flipped set V, so (push-through identity)

    G = G0 + G0[:, V] (I - B_V G0[V, V])^-1 B_V G0[V, :]
    E = Einc + G0[:, V] (I - B_V G0[V, V])^-1 B_V Einc[V],

which costs O(k^2 N) for k = |V| instead of O(N^3).  Tier T0 (brute force) is
T1 applied to every candidate structure.

``update_region`` is the paper's own update (eqs. form4-form9 for the field,
eqs. form10-form14 for G) for a selected region V, written out plainly so that
the tests can pin it against T1.

Pins (tests/test_oracle_state.py): the residual of the T1 solve; reciprocity
G_D = G_D^T; the imaginary-part identity Im G = (I + conj(G) B) Im G0 (I + B G)
(real B); E_D = Einc_D + G_D B Einc_D; T2 = T1; the paper's update = T1 for
single pixels and regions, flip followed by un-flip returns the original, and
two flips commute; the Mie series of a dielectric disk (oracle.mie).
"""
from __future__ import annotations

import numpy as np

from . import greens


def eps_of(problem, eps_idx) -> np.ndarray:
    table = np.asarray(problem.eps_table, dtype=np.float64)
    return table[np.asarray(eps_idx, dtype=np.int64)]


# --------------------------------------------------------------------------- T1
def dense_state(problem, eps, G0=None):
    """Tier T1: (G, E) of the structure with per-pixel permittivity `eps` (length N).

    Direct dense solve of the discretised Dyson / Lippmann-Schwinger equations.
    """
    N = problem.n
    if G0 is None:
        G0 = greens.build_G0(problem)
    Einc = greens.incident_field(problem)
    alpha = greens.alpha_of(problem, eps)
    G0_DD = G0[:N]
    G0_MD = G0[N:]
    A = np.eye(N, dtype=np.complex128) - G0_DD * alpha[None, :]   # I - G0_DD B
    G_D = np.linalg.solve(A, G0_DD)
    E_D = np.linalg.solve(A, Einc[:N])
    G_M = G0_MD + (G0_MD * alpha[None, :]) @ G_D
    E_M = Einc[N:] + (G0_MD * alpha[None, :]) @ E_D
    return np.concatenate([G_D, G_M], axis=0), np.concatenate([E_D, E_M])


def field_at(problem, eps, points, E_D=None):
    """Total field at arbitrary points outside the pixels, eq. form4 with V = D.

    E(r) = Einc(r) + sum_q h^2 g(|r - r_q|) alpha_q E_q.
    """
    if E_D is None:
        _, E = dense_state(problem, eps)
        E_D = E[: problem.n]
    k0 = greens.k0_of(problem)
    h = problem.pitch
    alpha = greens.alpha_of(problem, eps)
    pxy = greens.pixel_xy(problem)
    pts = np.asarray(points, dtype=np.float64)
    d = pts[:, None, :] - pxy[None, :, :]
    r = np.hypot(d[..., 0], d[..., 1])
    Einc = np.exp(1j * k0 * pts[:, 1])
    return Einc + (h * h * greens.g2d(r, k0)) @ (alpha * E_D)


# --------------------------------------------------------------------------- T2
class FlippedSet:
    """Tier T2: exact state from G0 and the flipped set only.

    Columns G0[:, p] are evaluated on first use and cached per pixel.
    """

    def __init__(self, problem):
        self.problem = problem
        self.N = problem.n
        self.R = problem.rows
        self.cols = {}
        self.Einc = greens.incident_field(problem)
        self.G0_diag = greens.self_term(problem.pitch, greens.k0_of(problem))
        self._all_rows = np.arange(self.R)

    def column(self, p: int) -> np.ndarray:
        c = self.cols.get(p)
        if c is None:
            c = greens.G0_block(self.problem, self._all_rows, [p])[:, 0]
            self.cols[p] = c
        return c

    def solve(self, eps):
        """Return (V, U = G0[:, V], Q = (I - B_V G0[V,V])^-1 B_V), V in the order
        of U's columns (any order of the flipped set gives the same state).  The
        last structure's solve is kept, so consecutive calls on one structure
        solve once; U is a view that the next solve of another structure changes."""
        key = np.asarray(eps, dtype=np.float64).tobytes()
        if getattr(self, "_last_key", None) == key:
            return self._last
        self._last = self._solve(eps)
        self._last_key = key
        return self._last

    def _columns(self, Vset):
        """U = G0[:, V] for the flipped set, as a view of a persistent R x cap
        buffer whose columns are kept in slot order: a pixel that leaves the set
        frees its slot (the last slot's column moves into it), a new pixel takes
        the next slot.  A one-pixel change of V then moves one column instead of
        restacking k of them.  Returns (V in slot order, U)."""
        if not hasattr(self, "_slots"):
            self._slots, self._pos = [], {}
            self._U = np.zeros((self.R, 16), np.complex128)
        for q in [q for q in self._slots if q not in Vset]:
            i, last = self._pos.pop(q), self._slots.pop()
            if last != q:
                self._slots[i] = last
                self._pos[last] = i
                self._U[:, i] = self._U[:, len(self._slots)]
        for q in sorted(Vset - set(self._pos)):
            if len(self._slots) == self._U.shape[1]:
                grown = np.zeros((self.R, 2 * self._U.shape[1]), np.complex128)
                grown[:, : len(self._slots)] = self._U[:, : len(self._slots)]
                self._U = grown
            self._pos[q] = len(self._slots)
            self._U[:, len(self._slots)] = self.column(q)
            self._slots.append(q)
        return np.array(self._slots, dtype=np.int64), self._U[:, : len(self._slots)]

    def _solve(self, eps):
        alpha = greens.alpha_of(self.problem, eps)
        V, U = self._columns({int(q) for q in np.flatnonzero(alpha != 0.0)})   # U: R x k
        k = V.size
        if k == 0:
            return V, np.zeros((self.R, 0), np.complex128), np.zeros((0, 0), np.complex128)
        aV = alpha[V]
        A = np.eye(k, dtype=np.complex128) - aV[:, None] * U[V, :]     # I - B_V G0[V,V]
        Q = np.linalg.solve(A, np.diag(aV).astype(np.complex128))
        return V, U, Q

    def column_of(self, eps, j: int) -> np.ndarray:
        """Column j (a design pixel) of G of the structure `eps`, all R rows:
        G[:, j] = G0[:, j] + U Q G0[V, j], with G0[V, j] = U[j, :] (symmetry)."""
        V, U, Q = self.solve(eps)
        col = self.column(j).copy()
        if V.size:
            col = col + U @ (Q @ U[j, :])
        return col

    def state(self, eps, rows=(), with_diag=True):
        """E (R), diag(G) over design pixels (N), and the requested full rows of G.

        G0 is symmetric on the design block (reciprocity of the free-space
        kernel), so G0[V, q] for design q equals U[q, :].  with_diag=False
        skips the O(k^2 N) diagonal (returned as None).
        """
        V, U, Q = self.solve(eps)
        N = self.N
        E = self.Einc.copy()
        diag = np.full(N, self.G0_diag, dtype=np.complex128) if with_diag else None
        out_rows = {}
        if V.size:
            E = E + U @ (Q @ self.Einc[V])
            if with_diag:
                U_D = U[:N]
                diag = diag + np.einsum("qa,qa->q", U_D @ Q, U_D)
        for r in rows:
            base = greens.G0_block(self.problem, [r], np.arange(N))[0]
            if V.size:
                base = base + (U[r] @ Q) @ U[:N].T
            out_rows[int(r)] = base
        return E, diag, out_rows


# --------------------------------------------------------------------------- paper's update
def update_region(problem, G, E, eps_cur, region, eps_new):
    """Paper's update of (G, E) when the pixels `region` change to `eps_new`.

    b_i = k0^2 (eps_new_i - eps_cur_i) for each pixel of the region (the
    paper's b with dV absorbed into the area-included G).
      field:  [1 - G_VV b] E_V^new = E_V^old          (eqs. form6, form9)
              E^new = E^old + G^old[:, V] b E_V^new   (eq. form4)
      Green:  [1 - G_VV b] G_V^new(r') = G_V^old(r')  (eqs. form12, form14)
              G^new = G^old + G^old[:, V] b G_V^new   (eq. form10)
    """
    region = np.asarray(region, dtype=np.int64)
    k0 = greens.k0_of(problem)
    b = k0**2 * (np.asarray(eps_new, dtype=np.float64) - np.asarray(eps_cur)[region])
    G_VV = G[region][:, region]
    A = np.eye(region.size, dtype=np.complex128) - G_VV * b[None, :]
    E_V_new = np.linalg.solve(A, E[region])
    G_V_new = np.linalg.solve(A, G[region, :])
    E_out = E + G[:, region] @ (b * E_V_new)
    G_out = G + G[:, region] @ (b[:, None] * G_V_new)
    return G_out, E_out


# --------------------------------------------------------------------------- T0
def fom_of_state(problem, E) -> float:
    """|E|^2 at the figure-of-merit monitor."""
    e = E[problem.n + problem.fom_monitor]
    return float(e.real**2 + e.imag**2)


def brute_force_scores(problem, eps_idx, G0=None) -> np.ndarray:
    """Tier T0: FOM of every candidate structure by a full T1 solve.

    Returns an (N, n_eps) array; entries that are not candidates (the pixel's
    current material, or a material outside the candidate mask) are -inf.
    """
    if G0 is None:
        G0 = greens.build_G0(problem)
    eps_idx = np.asarray(eps_idx, dtype=np.int64)
    n_eps = len(problem.eps_table)
    out = np.full((problem.n, n_eps), -np.inf)
    for p in range(problem.n):
        for e in range(n_eps):
            if not (problem.cand_mask >> e) & 1 or e == eps_idx[p]:
                continue
            trial = eps_idx.copy()
            trial[p] = e
            _, E = dense_state(problem, eps_of(problem, trial), G0)
            out[p, e] = fom_of_state(problem, E)
    return out
