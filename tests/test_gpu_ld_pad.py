"""A leading dimension above the minimum (state.ldG: a multiple of 64 past
ceil64(N)).  Every entry's arithmetic is independent of the row stride, so a
padded job makes the same moves and leaves bit for bit the state of an unpadded
one, and its padding columns stay zero (eager and deferred modes, the fused loop,
the flush, the refresh)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _job(p, **kw):
    from paper_2202_05388_amd.job import Job
    print(f"[case] {p.name} {p.ny}x{p.nx} {p.dtype} {kw}", flush=True)
    return Job(p, device="cuda:0", **kw)


@pytest.mark.parametrize("dtype,delay,fused,ld_pad", [
    ("c64", 64, True, 64), ("c128", 16, True, 128), ("c64", 0, False, 64), ("c64", 16, False, 192)])
def test_padded_leading_dimension_equals_minimal(dtype, delay, fused, ld_pad):
    p = W.tiny(40, 44, n_mon=8, dtype=dtype, cand_mask=W.MASK_BOTH)     # N = 1760, min ld 1792, ~130 moves
    ref = _job(p, delay=delay, kmax=256)
    job = _job(p, delay=delay, kmax=256, ld_pad=ld_pad)
    assert job.ld == ref.ld + ld_pad
    for j in (ref, job):
        j.init()
    n_ref = ref.run_greedy(300, poll_every=20, refresh_every=40, fused=fused)
    n = job.run_greedy(300, poll_every=20, refresh_every=40, fused=fused)
    assert n == n_ref and n > 100
    assert np.array_equal(job.history(), ref.history())
    Gr, Er, dr, ir = ref.host_state()
    G, E, d, i = job.host_state()
    assert np.array_equal(G, Gr) and np.array_equal(E, Er) and np.array_equal(d, dr)
    assert np.array_equal(i, ir) and job.status() == ref.status() == 0
    pad = job.G[:, job.N:].cpu()
    assert pad.shape[1] == job.ld - job.N and not pad.abs().amax().item()
