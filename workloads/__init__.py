"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module holds problem *inputs* only: grid sizes, wavelength, pixel pitch,
monitor coordinates, the material table, step counts and seeded random draws
(random permittivity masks, the served job stream).  It contains none of the
method's arithmetic (no Green's functions, no solves, no scores), so that the
FP64 oracle and the GPU path can both consume it without sharing any code that
computes a result.

Geometry conventions (2-D TM, scalar E_z, background vacuum eps_bg = 1):
  * design grid of ny rows (along the propagation axis y) by nx columns (x);
    pixel p = iy * nx + ix;
  * a line of n_mon monitor points at y = ny*h/2 + d (d beyond the exit face),
    x_m = (m - n_mon/2) * s with s = nx*h/n_mon, so that monitor n_mon/2 sits
    on the mirror axis x = 0 and is the figure-of-merit monitor.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

EPS_VACUUM = 1.0
EPS_SILICON = 12.25   # refractive index 3.5

# candidate masks: bit i set <=> table entry i may be proposed
MASK_ADD_ONLY = 0b10  # only eps_table[1] (add material)
MASK_BOTH = 0b11      # add or remove material


@dataclass(frozen=True)
class Problem:
    """One optimisation problem: geometry, materials and run length."""

    name: str
    ny: int
    nx: int
    n_mon: int
    wavelength: float = 1.0
    pitch: float = 0.05
    mon_distance: float = 2.0
    eps_table: tuple = (EPS_VACUUM, EPS_SILICON)
    cand_mask: int = MASK_BOTH
    dtype: str = "c128"          # storage of G and E on the GPU: "c64" | "c128"
    steps: int = 50
    refresh_every: int = 0       # 0 = never
    rank_k: int = 1
    min_spacing: int = 0
    tau: float = 1e-9            # relative tie band of the greedy selection
    region: int = 1              # side of the square regions a move flips (1 = one pixel)

    @property
    def n(self) -> int:
        return self.ny * self.nx

    @property
    def rows(self) -> int:
        return self.ny * self.nx + self.n_mon

    @property
    def fom_monitor(self) -> int:
        return self.n_mon // 2

    @property
    def mon_spacing(self) -> float:
        return self.nx * self.pitch / self.n_mon

    def monitor_xy(self) -> np.ndarray:
        """(n_mon, 2) float64 monitor coordinates (x, y)."""
        m = np.arange(self.n_mon, dtype=np.float64)
        x = (m - self.n_mon / 2) * self.mon_spacing
        y = np.full(self.n_mon, self.ny * self.pitch / 2 + self.mon_distance)
        return np.ascontiguousarray(np.stack([x, y], axis=1))

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)

    def storage_bytes(self) -> int:
        """Bytes of the stored (rows x n) complex matrix."""
        per = 8 if self.dtype == "c64" else 16
        return per * self.rows * self.n


# The five named workloads ---------------------------------------------------
# 32x32 plain FP64 run: add-only flips, 16 monitors 2 wavelengths past the grid.
SMALL_32 = Problem("square32_fp64", 32, 32, 16, pitch=0.05, mon_distance=2.0,
                   cand_mask=MASK_ADD_ONLY, dtype="c128", steps=50)
# 128x128 headline: complex64 storage + FP64 refresh every 256 steps.
SQUARE_128 = Problem("square128_c64", 128, 128, 64, pitch=0.05, mon_distance=2.0,
                     cand_mask=MASK_BOTH, dtype="c64", steps=2000, refresh_every=256,
                     tau=1e-6)
# the same grid in plain FP64 (complex128, no refresh): the baseline loop.
SQUARE_128_FP64 = SQUARE_128.replace(name="square128_fp64", dtype="c128",
                                     refresh_every=0, tau=1e-9)
# 48x2048 high-NA strip lens at h = lambda/16, 256 monitors at 20 wavelengths.
STRIP_48x2048 = Problem("strip48x2048_c64", 48, 2048, 256, pitch=1.0 / 16,
                        mon_distance=20.0, cand_mask=MASK_BOTH, dtype="c64",
                        steps=500, refresh_every=256, tau=1e-6)
# rank-16 moves on the 128x128 grid, Chebyshev spacing >= 3.
SQUARE_128_RANK16 = SQUARE_128.replace(name="square128_rank16", steps=300, rank_k=16,
                                       min_spacing=3, refresh_every=16)

# 21x21 focusing lens for the exploration study: the 2-D analogue of the paper's
# small epsilon-greedy demonstration (21x21 pixels at lambda/20, silicon eps 12,
# focus at NA 0.7: half-aperture 0.525 lambda, focal distance 0.525/tan(asin 0.7)
# = 0.536 lambda past the exit face).
SQUARE_21 = Problem("square21_fp64", 21, 21, 8, pitch=0.05, mon_distance=0.536,
                    eps_table=(EPS_VACUUM, 12.0), cand_mask=MASK_BOTH, dtype="c128",
                    steps=2000)

# 2x2-pixel region moves (pillars) on a 128x128 grid at lambda/40, so that a
# region has the lambda/20 footprint of one pixel of the other workloads.
SQUARE_128_REGIONS = Problem("square128_regions_c64", 128, 128, 64, pitch=0.025,
                             mon_distance=1.0, cand_mask=MASK_BOTH, dtype="c64", steps=2000,
                             refresh_every=256, tau=1e-6, region=2)

WORKLOADS = {p.name: p for p in (SMALL_32, SQUARE_128, SQUARE_128_FP64, STRIP_48x2048,
                                 SQUARE_128_RANK16, SQUARE_21, SQUARE_128_REGIONS)}


def tiny(ny: int, nx: int, n_mon: int = 4, **kw) -> Problem:
    """A small problem for unit tests (default pitch lambda/20, monitors 1 lambda out)."""
    base = dict(pitch=0.05, mon_distance=1.0, cand_mask=MASK_BOTH, dtype="c128", steps=10)
    base.update(kw)
    return Problem(f"tiny{ny}x{nx}", ny, nx, n_mon, **base)


# Seeded random draws ----------------------------------------------------------
def random_eps_idx(problem: Problem, fill: float, seed: int) -> np.ndarray:
    """uint8 material index per pixel; each pixel is material 1 with prob `fill`."""
    rng = np.random.default_rng(seed)
    return (rng.random(problem.n) < fill).astype(np.uint8)


def random_material_idx(problem: Problem, seed: int) -> np.ndarray:
    """uint8 material index per pixel, uniform over the permittivity table."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, len(problem.eps_table), problem.n).astype(np.uint8)


def mirror_symmetric_eps_idx(problem: Problem, fill: float, seed: int) -> np.ndarray:
    """Random material mask that is symmetric under ix -> nx-1-ix."""
    rng = np.random.default_rng(seed)
    half = (problem.nx + 1) // 2
    m = (rng.random((problem.ny, half)) < fill).astype(np.uint8)
    full = np.concatenate([m, m[:, : problem.nx - half][:, ::-1]], axis=1)
    return np.ascontiguousarray(full.reshape(-1))


def eps_greedy_draws(n_steps: int, seed: int) -> np.ndarray:
    """(n_steps, 2) float64 uniforms in [0, 1): for step t, the draw that decides
    whether the step explores, and the draw that chooses among the top moves."""
    return np.random.default_rng(seed).random((n_steps, 2))


@dataclass
class Job:
    """One served optimisation job."""

    job_id: int
    arrival: float      # seconds after the stream starts
    problem: Problem


def served_jobs(n_jobs: int = 64, rate: float = 4.0, seed: int = 0,
                side_range=(24, 160), wl_range=(0.8, 1.2), steps_range=(200, 1000),
                pitch: float = 0.05, n_mon: int = 16) -> list:
    """Poisson stream of jobs (inter-arrival ~ Exp(rate)), drawn in a fixed order per job:
    inter-arrival, grid side (uniform integer), wavelength (uniform), step count."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += float(rng.exponential(1.0 / rate))
        side = int(rng.integers(side_range[0], side_range[1] + 1))
        wl = float(rng.uniform(*wl_range))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        prob = Problem(f"job{j}_{side}", side, side, n_mon, wavelength=wl, pitch=pitch,
                       mon_distance=2.0 * wl, cand_mask=MASK_BOTH, dtype="c64",
                       steps=steps, refresh_every=256, tau=1e-6)
        jobs.append(Job(j, t, prob))
    return jobs
