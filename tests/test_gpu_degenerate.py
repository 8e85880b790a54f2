"""Degenerate shapes: one monitor (the FOM monitor alone, whose pending terms are
zero), a single row of pixels, a single pixel.  The fused loop equals the
per-call path bit for bit, deferred equals eager, and the final state equals
the oracle's dense re-solve of the final structure (Sec. II, Eq. form2)."""
import numpy as np
import pytest

from oracle import state as ost
import workloads as W

pytestmark = pytest.mark.gpu


def _job(p, **kw):
    from paper_2202_05388_amd.job import Job
    print(f"[case] {p.name} {p.ny}x{p.nx} n_mon={p.n_mon} {p.dtype} {kw}", flush=True)
    return Job(p, device="cuda:0", **kw)


# element-wise relative error with an absolute floor of 1e-3 x the largest entry
from parity import c64_drift_tol, rel_elem as _rel  # noqa: E402


@pytest.mark.parametrize("ny,nx,n_mon,dtype,delay", [
    (1, 64, 1, "c64", 16), (1, 64, 1, "c128", 7), (8, 8, 1, "c64", 64), (3, 5, 2, "c128", 4),
    (1, 1, 1, "c64", 4), (1, 1, 1, "c128", 4), (2, 97, 3, "c64", 128)])
def test_degenerate_shapes(ny, nx, n_mon, dtype, delay):
    p = W.tiny(ny, nx, n_mon=n_mon, dtype=dtype, cand_mask=W.MASK_BOTH)
    eager = _job(p)
    eager.init()
    n_e = eager.run_greedy(200, poll_every=16)
    per_call = _job(p, delay=delay)
    per_call.init()
    n_p = per_call.run_greedy(200, poll_every=16)
    fused = _job(p, delay=delay)
    fused.init()
    n_f = fused.run_greedy(200, poll_every=16, fused=True)
    print(f"[moves] {n_e} {n_p} {n_f}", flush=True)
    assert n_e == n_p == n_f and n_e < 200
    assert np.array_equal(fused.history(), per_call.history())
    assert np.array_equal(per_call.history(), eager.history())
    Gp, Ep, dp, ip = per_call.host_state()
    Gf, Ef, df, i_f = fused.host_state()
    assert np.array_equal(Gf, Gp) and np.array_equal(Ef, Ep) and np.array_equal(df, dp)
    assert np.array_equal(i_f, ip)
    Ge, Ee, de, ie = eager.host_state()
    tol = 1e-12 if dtype == "c128" else c64_drift_tol(n_e)
    assert np.array_equal(ie, ip) and _rel(Gp, Ge) <= tol and _rel(Ep, Ee) <= tol
    Gd, Ed = ost.dense_state(p, ost.eps_of(p, ip))
    dense_tol = 1e-11 if dtype == "c128" else c64_drift_tol(n_e)
    assert _rel(Gp, Gd) <= dense_tol and _rel(Ep, Ed) <= dense_tol
    assert eager.status() == per_call.status() == fused.status() == 0
