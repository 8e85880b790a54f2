"""score_candidates_static, the scoring entry point for callers that cannot
allocate device memory, against score_candidates on the same states through
the C ABI: two calls in a row, the second on a smaller problem, each giving the
same records (pixel, material, predicted FOM, FOM gain) bit for bit."""
import ctypes as C

import numpy as np
import pytest

from oracle import state as ost
import workloads as W

pytestmark = pytest.mark.gpu


def _static_picks(job, p, topk, spacing):
    """The records of score_candidates_static, called with the job's state but
    no workspace, on a fresh stream-ordered output buffer."""
    import torch
    from paper_2202_05388_amd import _lib as L
    st = L.State.from_buffer_copy(job.state)
    st.work = None
    st.work_bytes = 0
    out = torch.full((topk * L.PICK_BYTES,), 0xAB, dtype=torch.uint8, device=job.device)
    stream = torch.cuda.current_stream().cuda_stream
    L.score_candidates_static(job.prob, st, p.cand_mask, p.tau, topk, spacing, out.data_ptr(),
                              stream)
    raw = out.cpu().numpy().tobytes()
    return [(r.pixel, r.eps_idx, r.fom_new, r.dfom) for r in (L.Pick * topk).from_buffer_copy(raw)]


@pytest.mark.parametrize("order", ["large_then_small"])
def test_static_scores_equal_workspace_scores(order):
    from paper_2202_05388_amd.job import Job
    cases = [  # (problem, fill, seed, topk, spacing): the second is smaller
        (W.tiny(40, 44, n_mon=8, dtype="c64", tau=1e-6), 0.2, 3, 16, 3),
        (W.tiny(9, 11, n_mon=4, dtype="c128"), 0.3, 5, 1, 0),
    ]
    for p, fill, seed, topk, spacing in cases:
        print(f"[case] static scores {p.ny}x{p.nx} {p.dtype} topk {topk} spacing {spacing}",
              flush=True)
        N = p.n
        idx = W.random_eps_idx(p, fill, seed)
        G, E = ost.dense_state(p, ost.eps_of(p, idx))
        job = Job(p, device="cuda:0")
        job.upload_state(G, E, np.diagonal(G[:N]), idx)
        job.score(topk=topk, min_spacing=spacing)
        ref = job.read_picks(topk)
        got = _static_picks(job, p, topk, spacing)
        assert got == ref
        assert ref[0][0] >= 0 and job.status() == 0
