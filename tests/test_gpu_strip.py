"""GPU parity on the 48x2048-pixel high-NA strip (98304 pixels, 256 monitors at 20
wavelengths, complex64 G of 77.5 GB resident in HBM, FP64 refresh every 256 moves)
against the stored FP64 oracle trajectory (flipped-set tier, 500 steps).

The move sequence must match the oracle's until a step t; from t on, every move
of the GPU's sequence must be a certified tie (its exact FP64 score within 1e-4
of the best exact score at that state, the oracle replaying the GPU's own
moves).  The fields at the monitors and at the sampled pixels agree with the
oracle element by element to 1e-4 at every stored checkpoint: the stored
trajectory's fields up to t, the oracle's fields of the GPU's own structure
after t.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from parity import assert_close, certify_sequence, first_divergence

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _c(z):
    return np.array([complex(*v) for v in z])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("delay,fused", [(0, False), (64, False), (64, True)])
def test_strip48x2048_c64_matches_oracle(delay, fused):
    """fused: gfo_greedy_steps, as the benchmark drives the strip (two kernels per
    move on a grid of this size), else score_candidates + apply_flip per move."""
    import torch
    from paper_2202_05388_amd.job import Job
    gold = json.load(open(os.path.join(HERE, "golden", "strip48x2048_fp64.json")))
    p = W.STRIP_48x2048
    N = p.n
    sample = gold["sample_pixels"]
    print(f"[case] {p.name}: G {p.storage_bytes() / 1e9:.1f} GB, delay {delay}, fused {fused}",
          flush=True)
    job = Job(p, device="cuda:0", kmax=512, delay=delay)
    job.init()
    fields = {}
    done = 0
    for ck in sorted(int(k) for k in gold["checkpoints"]):
        done += job.run_greedy(ck - done, poll_every=50, refresh_every=256, fused=fused)
        if done < ck:
            break
        E = job.E.cpu().to(torch.complex128).numpy()
        fields[ck] = (E[N:], E[sample])
        print(f"  step {ck} done", flush=True)
    assert job.status() == 0
    hist = [(int(a), int(b)) for a, b in job.history()]
    gp = [(s["pixel"], s["eps_idx"]) for s in gold["steps"]]
    t = first_divergence(gp, hist)
    print(f"strip sequence: GPU {len(hist)} moves, oracle {len(gp)}, identical for {t}", flush=True)
    checked = []
    for ck, (Em, Ep) in fields.items():
        if ck <= t:
            g = gold["checkpoints"][str(ck)]
            assert_close(f"E_mon step {ck}", Em, _c(g["E_mon"]), 1e-4)
            assert_close(f"E_pix step {ck}", Ep, _c(g["E_pix"]), 1e-4)
            checked.append(ck)

    def on_state(step, E):
        Em, Ep = fields[step]
        assert_close(f"E_mon step {step} (oracle replay)", Em, E[N:], 1e-4)
        assert_close(f"E_pix step {step} (oracle replay)", Ep, E[sample], 1e-4)
        checked.append(step)

    # every move after the divergence is a certified tie, and the fields of the
    # GPU's own structure are checked at the checkpoints past it
    certify_sequence(p, gp, hist, tol=1e-4,
                     checkpoints=[c for c in fields if c > t and c <= len(hist)],
                     on_state=on_state)
    assert sorted(checked) == sorted(c for c in fields if c <= len(hist)), (checked, list(fields))
    assert len(checked) >= 1
