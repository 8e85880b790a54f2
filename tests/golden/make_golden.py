"""Write the stored oracle trajectories under tests/golden/.

Calls only the oracle and the shared workload definitions.  Usage:

    python tests/golden/make_golden.py square32          # 32x32 FP64, 50 steps, tier T1
    python tests/golden/make_golden.py square128 [steps] # 128x128, tier T2 (long: O(k^2 N)/step)

Each file records the problem, the move sequence with the predicted and exact
FOM of every step, and sampled exact fields at checkpoints.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import greedy  # noqa: E402
import workloads as W  # noqa: E402


def _c(z):
    return [float(np.real(z)), float(np.imag(z))]


def _problem_dict(p):
    return dict(name=p.name, ny=p.ny, nx=p.nx, n_mon=p.n_mon, wavelength=p.wavelength,
                pitch=p.pitch, mon_distance=p.mon_distance, eps_table=list(p.eps_table),
                cand_mask=p.cand_mask, tau=p.tau)


def write(problem, tier, steps, path, checkpoint_every, sample_pixels):
    t0 = time.time()
    ckpt = {}
    N = problem.n

    def cb(t, eps_idx, E):
        if (t + 1) % checkpoint_every == 0:
            ckpt[t + 1] = dict(E_mon=[_c(z) for z in E[N:]],
                               E_pix=[_c(E[q]) for q in sample_pixels])
            print(f"  step {t + 1}: {time.time() - t0:.1f}s", flush=True)

    traj = greedy.greedy(problem, steps=steps, tier=tier, callback=cb)
    out = dict(problem=_problem_dict(problem), tier=tier, fom0=traj.fom0, stopped=traj.stopped,
               steps=[dict(pixel=s.pixel, eps_idx=s.eps_idx, fom_pred=s.fom_pred, fom=s.fom,
                           n_tied=s.n_tied) for s in traj.steps],
               sample_pixels=[int(q) for q in sample_pixels],
               checkpoints={str(k): v for k, v in ckpt.items()},
               final=dict(E_mon=[_c(z) for z in traj.E[N:]],
                          E_pix=[_c(traj.E[q]) for q in sample_pixels],
                          eps_idx=[int(v) for v in traj.eps_idx]),
               seconds=time.time() - t0)
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {path}: {len(traj.steps)} steps in {time.time() - t0:.1f}s")


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "square32"
    if which == "square32":
        p = W.SMALL_32
        write(p, "T1", p.steps, os.path.join(HERE, "square32_fp64.json"), 10,
              np.arange(0, p.n, 7))
    elif which == "square128":
        p = W.SQUARE_128_FP64
        steps = int(sys.argv[2]) if len(sys.argv) > 2 else p.steps
        rng = np.random.default_rng(0)
        sample = np.sort(rng.choice(p.n, 64, replace=False))
        write(p, "T2", steps, os.path.join(HERE, "square128_fp64.json"), 100, sample)
    elif which == "strip":
        p = W.STRIP_48x2048.replace(tau=1e-9)
        steps = int(sys.argv[2]) if len(sys.argv) > 2 else p.steps
        rng = np.random.default_rng(0)
        sample = np.sort(rng.choice(p.n, 64, replace=False))
        write(p, "T2", steps, os.path.join(HERE, "strip48x2048_fp64.json"), 50, sample)
    else:
        raise SystemExit(f"unknown golden {which}")


if __name__ == "__main__":
    main()
